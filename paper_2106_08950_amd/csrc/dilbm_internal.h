// dilbm_internal.h -- device-visible structures of libdilbm (internal to the library).
//
// Memory layout of one solve in HBM:
//   pop[2]        two population buffers, structure of arrays [9][ny][pitch] of shifted,
//                 scaled populations g_i = 36 (f_i - w_i rho0) in FP32 (or FP16 times
//                 2^k); the factor 36 makes the D2Q9 weights exact integers.  What is
//                 stored at step t is g_i - 3 K_i c_i.V_t (K_i = 36 w_i): the populations
//                 seen from a reference frame moving with a small pseudo-random uniform
//                 velocity V_t drawn afresh every step (see ref_velocity), which keeps
//                 FP32/FP16 rounding from accumulating a bias.  The pull scheme keeps
//                 post-collision values: node x at time t_n finds f_i in
//                 pop[p][i][x - c_i].  Rows are `pitch` values apart (row_pitch: nx
//                 rounded up to whole 128-byte lines); the padding is never touched.
//   tile_head[2]  two list sets; per tile two words: the number of bodies whose phi
//                 support (plus the skin kBinSkin) may touch the tile, and the first of
//                 their list entries (one 8-byte scalar load per tile, from a dense array)
//   tile_list[2]  per tile, `list_cap` entries: body index and four-wave mask (entry 0
//                 lives in the tile's head; its slot here is unused).  The lists are kept
//                 across steps: lsel[p] names the set the steps of parity p read, and a
//                 rebuild fills the other set (see kBinSkin)
//   bstate[2]     body state SoA [5][nb]: x, y, ux, uy, omega (FP64)
//   bconst        body constants SoA [5][nb]: radius, rho_s, mass, inertia, fixed
//   bsnap[2]      per body, what the collide kernel reads of it (BodySnap, 32 B): written
//                 with every body update, so that a tile reads one listed body in one
//                 dependent load
//   bxy[2]        per body, (x, y) rounded to FP32, written with the snapshot: the pair
//                 search reads 8 bytes per partner and takes the FP64 state only for
//                 partners within reach
//   acc[2]        FP64 force accumulators: Fx, Fy, T per body ([nb * 3]), then the wall
//                 force in kWallSlots slots of one 128-byte line each (acc_words)
//   err           sticky error bits
// Everything else double-buffered is indexed by the step parity p: a step with parity p
// reads slot p and writes slot 1 - p (bodies, snapshots, force sums) or both (populations).
#pragma once

#include <stdint.h>

namespace dilbm {

constexpr int kQ = 9;
// Tile shapes (nodes): 0-4 hold 256 nodes, one per lane; 5 is a 512-node row segment with
// two neighbouring nodes per lane, for FP16 populations on lattices of even width.
constexpr int kNumTileShapes = 6;
constexpr int kTileTX[kNumTileShapes] = {64, 128, 256, 32, 16, 512};
constexpr int kTileTY[kNumTileShapes] = {4, 2, 1, 8, 16, 1};
constexpr int kPairShape = 5;
constexpr int kBlockThreads = 256;       // threads of every collide block
constexpr int kMaxListCap = 1024;
// A tile-list entry: the body index in the low 27 bits and, in bits 27-30, which of the
// tile's four waves hold a node within the body's support (set by the binning; a wave
// skips a body whose bit is clear).
constexpr int kListIndexBits = 27;
constexpr int32_t kListIndexMask = (1 << kListIndexBits) - 1;

// Register budget of the collide kernel, per population storage: it is compiled for at
// least this many waves per SIMD (512 / N VGPRs per lane).  The step streams populations,
// so waves in flight are bytes in flight, but a tighter budget costs scheduling freedom.
// Measured on the 4096^2 suspension: FP32 (256 x 1 tiles) 6 waves (80 VGPRs) against 7:
// 0.5% faster with discs, 2% without; FP16 7 waves (72 VGPRs) against 6: 3-4% faster;
// 8 waves (64 VGPRs) makes both slower and spills in the FP16 instances.
// Population bytes (both buffers, all solves of a launch) above which the collide kernels
// store with the non-temporal hint: MI355X's last-level cache (Infinity Cache) holds 256 MB.
#ifndef DILBM_STORE_NT_MIN_MB
#define DILBM_STORE_NT_MIN_MB 256
#endif
constexpr uint64_t kStoreNtMinBytes = (uint64_t)DILBM_STORE_NT_MIN_MB << 20;

#ifndef DILBM_COLLIDE_WAVES_F32
#define DILBM_COLLIDE_WAVES_F32 6
#endif
#ifndef DILBM_COLLIDE_WAVES_F16
#define DILBM_COLLIDE_WAVES_F16 7
#endif
// the same for the FP16 instance with two nodes per lane (512-node tiles)
#ifndef DILBM_COLLIDE_WAVES_X2
#define DILBM_COLLIDE_WAVES_X2 5
#endif
// Persistent collide grid: each block walks one contiguous chunk of about this many tiles,
// per population storage type (0 = one block per tile); the grid never drops below one
// resident wave.  Shorter chunks keep the tiles in flight closer together, longer ones
// pay the per-block set-up less often.  Measured on the 4096^2 suspension and the
// 4096 x 2048 channel: FP32 best at 3 tiles, FP16 at 6.
#ifndef DILBM_CHUNK_FP32
#define DILBM_CHUNK_FP32 3
#endif
#ifndef DILBM_CHUNK_FP16
#define DILBM_CHUNK_FP16 6
#endif

enum ErrBits : int32_t { kErrUnstable = 1, kErrCapacity = 2, kErrInternal = 4 };

// Neighbour lists of the Eq. (28) pair search.  Each body keeps the partners that were
// within r_i + r_j + xi + kNbrSkin of it when the lists were last built; while no body of
// the solve has moved more than kNbrSkin / 2 since then, every pair within reach is on
// them.  A body that has moved that far raises the solve's rebuild flag, and at the next
// step every body rebuilds its list by the full sweep.  A list that would pass
// kNbrCap entries is marked -1: that body sweeps every step until the next rebuild.
constexpr int kNbrCap = 64;
constexpr double kNbrSkin = 2.0;
// Tile lists are built with the reach R + support + kBinSkin and rebuilt only once some
// body of the solve has moved half that skin since: a body moves well under half of it
// per step, so until the rebuild every node within R + support of it lies in a listed
// tile.
constexpr double kBinSkin = 2.0;

// The force on the walls is summed over kWallSlots accumulators, one 128-byte line each,
// chosen by the block index: with a single accumulator every wave of a walled solve adds
// to one address and the atomics serialize (a 256^3 duct with walls across y and z took
// 1450 us per collide launch instead of 450).  wall_base(w): the first word of the slots
// after w per-body words; acc_words(nb, k): one accumulator buffer for nb bodies of k
// words each.
constexpr int kWallSlots = 64;
constexpr int kWallSlotWords = 16;
__host__ __device__ constexpr int64_t wall_base(int64_t body_words) {
  return (body_words + kWallSlotWords - 1) / kWallSlotWords * kWallSlotWords;
}
__host__ __device__ constexpr int64_t acc_words(int64_t nb, int k) {
  return wall_base(nb * k) + (int64_t)kWallSlots * kWallSlotWords;
}

// One body as the collide kernel sees it at a step: position (FP64, so that node - centre
// differences keep FP64 accuracy before they are rounded), rigid velocity, spin and radius.
struct BodySnap {
  double x, y;
  float u, v, w, r;
};

// Row pitch of the population planes, in populations: nx rounded up to whole 128-byte
// lines (32 FP32 or 64 FP16 values), so every row starts on a line.  Rows that start
// mid-line cost the pooled ensemble of 256 solves of arbitrary width 23% of its
// throughput, and a 4090-wide FP32 lattice 16% per node against a 4096-wide one; the
// padding columns are never read or written by a step.
inline int32_t row_pitch(int32_t nx, int32_t storage) {
  const int32_t a = storage == 1 ? 64 : 32;
  return (nx + a - 1) / a * a;
}

struct SolveDesc {
  // geometry and tiling
  int32_t nx, ny;
  int32_t pitch;               // row stride of the population planes (row_pitch)
  int32_t tx, ty;              // tile extent in nodes
  int32_t tiles_x, tiles_y;
  int64_t tile_base;           // first global tile index of this solve
  int32_t body_base;           // first global body index of this solve
  int32_t nbodies;
  int32_t list_cap;
  uint32_t wall_mask;
  // chunk control (rewritten by the host before every chunk)
  int64_t step0;               // steps the solve has taken at the chunk start
  int32_t active_steps;        // step k of the chunk runs iff k < active_steps
  int32_t parity0;             // parity of the solve's state at the chunk start
  // FP32 node constants
  float omega;                 // 1 / tau
  float khalf;                 // 1 - 1 / (2 tau)
  float rho0;
  float rho36;                 // 36 rho0
  float Gx, Gy;
  // per-solve constants of the collision (uniform; formed on the host so the kernels take
  // them as scalar operands): 9 c.G and 3 c.G for the direction pairs (1,3), (2,4),
  // (5,7), (6,8), and khalf K for K = 4 and 16
  float g9[4], g3[4];
  float khk4, khk16;
  float phi_k;                 // 4 / eps * log2(e): phi = 1 / (1 + 2^(-l * phi_k))
  float lcut;                  // -cutoff * eps
  float wall_h;
  int32_t wall_y_lo, wall_y_hi;  // rows outside [lo, hi) are within a y-wall's support
  int32_t wall_x_lo, wall_x_hi;
  float kappa;                 // force scale of Eqs. (18)-(19)
  // open ends in x (non-equilibrium extrapolation at the columns x = 0 and x = nx - 1)
  int32_t xbc, inlet_kind, inlet_profile, outlet_kind;
  float u_in_x, u_in_y;        // prescribed inlet velocity (peak of a parabolic profile)
  float rho36_in, rho36_out;   // 36 x prescribed inlet / outlet density
  float prof_y0, prof_inv_h;   // parabolic profile: s = (y + 1/2 - prof_y0) * prof_inv_h
  float store_scale, store_inv;
  int32_t storage;
  int32_t store_nt;            // population stores carry the non-temporal hint
  // FP64 body constants
  double rho0_d;
  double gx, gy;
  double inv_eps_p, inv_eps_p1, inv_eps_w, inv_eps_w1, xi;  // Eqs. (28)-(29)
  double wall_h_d;
  double support;              // cutoff * eps: phi support beyond the radius
  double rmax;                 // largest body radius of the solve (pair search reach)
  // device buffers
  void *pop[2];
  int32_t *tile_head[2];
  int32_t *tile_list[2];
  double *bstate[2];
  const double *bconst;
  BodySnap *bsnap[2];
  float *bxy[2];               // per body (x, y) in FP32, interleaved: coarse pair search
  double *acc[2];
  int32_t *err;
  // neighbour lists of the pair search: count per body (-1: sweep every step), kNbrCap
  // partner indices per body, the position each body had when its list was built, and the
  // rebuild flags (by step parity: a step reads flag[p], raises flag[p ^ 1]; the collide
  // kernel of the next step clears flag[p])
  int32_t *nbr_cnt;
  int32_t *nbr_list;
  double *nbr_ref;
  int32_t *nl_flag;
  // tile lists kept across steps: lsel[p] names the list set (0 or 1) the steps of parity
  // p read; rb_flag[p] asks the body step of parity p to rebin every body (into the other
  // set, with the reach R + support + kBinSkin); bin_ref holds each body's position when
  // it was last binned
  int32_t *lsel;
  int32_t *rb_flag;
  double *bin_ref;
};

// A rectangle of nodes [x, x + w) x [y, y + h) inside one solve.
struct Region {
  int32_t x, y, w, h;
};

// Per-launch batch header, read by every kernel of a step.
struct BatchHeader {
  int64_t total_tiles;
  int32_t total_bodies;
  int32_t nsolves;
  int32_t solo_slot;           // descriptor slot of the only member, or -1
  int32_t natural;             // collide order: 1 = tile b to block b (grid-stride), 0 = chunks
};

}  // namespace dilbm
