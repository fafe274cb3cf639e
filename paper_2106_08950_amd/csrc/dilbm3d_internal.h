// dilbm3d_internal.h -- device-visible structures of the three-dimensional DI-LBM path of
// libdilbm (internal to the library).
//
// Memory layout of one 3-D solve in HBM:
//   pop[2]        two population buffers, structure of arrays [q][nz][ny][pitch] (q = 19
//                 or 27; pitch = row_pitch3, whole 128-byte lines) of FP32
//                 g_i = S (f_i - w_i rho0), S = 36 or 216, stored in the moving frame of
//                 ref_velocity3, or of FP16 g_i 2^k (no frame: the stochastic rounding of
//                 the stores keeps FP16 free of drift).  Pull scheme: node x at time t_n
//                 finds f_i in pop[p][i][x - c_i].
//   tile_head[2]  two list sets; per tile (64 x 4 x 1 or 256 x 1 x 1 nodes) two words:
//                 the number of spheres whose phi support (plus the skin kBinSkin3) may
//                 touch it and the first list entry; tile_list[2]: `list_cap` entries per
//                 tile (sphere index and four-wave mask; entry 0 lives in the head).  The
//                 lists are kept across steps: lsel[p] names the set the steps of parity p
//                 read, and a rebuild fills the other set
//   bstate[2]     sphere state SoA [9][nb]: x, y, z, u, v, w, omega_x, omega_y, omega_z
//   bconst        sphere constants SoA [5][nb]: radius, rho_s, mass, inertia, fixed
//   bsnap[2]      per sphere, what the collide kernel reads of it (SphereSnap, 64 B),
//                 written with every sphere update
//   acc[2]        FP64 accumulators [acc_words(nb, 6)]: force (3) and torque (3) per sphere,
//                 then the wall force in the last slot
//   err           sticky error bits (kErrUnstable, kErrCapacity, kErrInternal)
// Everything else double-buffered is indexed by the step parity p: a step with parity p
// reads slot p and writes slot 1 - p.
#pragma once

#include <stdint.h>

namespace dilbm {

constexpr int kQ3 = 19;      // D3Q19
constexpr int kQ3Max = 27;   // D3Q27

// Directions: rest, the six axis directions, the twelve edge directions (D3Q19), then the
// eight corner directions (D3Q27); opposite directions are neighbours (i, i + 1) for odd i.
constexpr int C3X[kQ3Max] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                             1, -1, 1, -1, 1, -1, -1, 1};
constexpr int C3Y[kQ3Max] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                             1, -1, 1, -1, -1, 1, 1, -1};
constexpr int C3Z[kQ3Max] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                             1, -1, -1, 1, 1, -1, 1, -1};
// Tiles are tile_x x (256 / tile_x) x 1 nodes, 256 threads: tile_x = 256 (a whole row of
// up to 256 nodes per block) when nx >= DILBM3D_WIDE_MIN, else 64 (64 x 4 x 1).
#ifndef DILBM3D_WIDE_MIN
#define DILBM3D_WIDE_MIN 192
#endif
constexpr int kMaxListCap3 = 1024;

// Row pitch of the population planes (populations per row): whole 128-byte lines, 32 FP32
// or 64 FP16 values.
inline int32_t row_pitch3(int32_t nx, int32_t storage) {
  const int32_t a = storage == 1 ? 64 : 32;
  return (nx + a - 1) / a * a;
}

// Tile lists are built with the reach R + support + kBinSkin3 and rebuilt once some sphere
// has moved half that skin since its last binning.
constexpr double kBinSkin3 = 2.0;

// A multi-step call checks the sticky error flags every this many steps.
constexpr int64_t kPollSteps3 = 32;

// Population bytes (both buffers) above which the collide kernel stores with the
// non-temporal hint: MI355X's last-level cache (Infinity Cache) holds 256 MB.
constexpr uint64_t kStoreNtMinBytes3 = 256ull << 20;

// Register budget of the collide kernel: compiled for at least this many waves per SIMD.
#ifndef DILBM3D_COLLIDE_WAVES
#define DILBM3D_COLLIDE_WAVES 5
#endif
// the same for the D3Q27 instances (27 populations per node)
#ifndef DILBM3D27_COLLIDE_WAVES
#define DILBM3D27_COLLIDE_WAVES 5
#endif
// the same for FP16 populations on either lattice.  The LDS of a block (the population
// stash and the force rows) allows six per SIMD.  Measured on the 256^3 suspension: six
// against five, D3Q19 FP16 393 -> 372 us per launch (79 VGPRs, no spills), D3Q27 FP16
// 464 -> 454 us (80 VGPRs, 12 bytes of spills in the sphere loop); the FP32 instances
// spill at six and lose 3% (D3Q19) and 8% (D3Q27).
#ifndef DILBM3D_COLLIDE_WAVES_F16
#define DILBM3D_COLLIDE_WAVES_F16 6
#endif

// Chunk of tiles each collide block sweeps (the grid never drops below one resident
// wave while tiles last).  On the 256^3 suspension: 2 tiles 546 us, 3 549 us, 4 (one row
// of 64-wide tiles) 548 us, 8 558 us.
#ifndef DILBM3D_CHUNK
#define DILBM3D_CHUNK 2
#endif

// One sphere as the collide kernel sees it at a step: centre in FP64 (node - centre
// differences keep FP64 accuracy before they are rounded), velocity, spin and radius.
struct SphereSnap {
  double x, y, z;
  float u, v, w;
  float ox, oy, oz;
  float r;
  float pad[2];
};

struct Desc3 {
  int32_t nx, ny, nz;
  int32_t pitch;      // row stride of the population planes: nx rounded up to 32 (whole
                      // 128-byte lines, as in the 2-D planes); padding is never touched
  int32_t tile_x;     // 64 or 256
  int32_t tiles_x, tiles_y;
  int64_t ntiles;
  // a member of a batch (dilbm3d_batch_*): its first tile and first sphere in the batch's
  // concatenation, and the parity and step count of its state when the batch call began
  int64_t tile_base;
  int32_t body_base;
  int32_t parity0;
  int64_t step0;
  int32_t nbodies;
  int32_t list_cap;
  // FP32 node-update constants
  float omega;        // 1 / tau
  float khalf;        // 1 - 1/(2 tau)
  float inv_khalf;    // 1 / khalf
  float rho0;
  float Gx, Gy, Gz;
  float cg[kQ3Max / 2];  // c_i.G for the direction pairs (2k + 1, 2k + 2)
  float kappa;        // force scale of Eq. (18): 1 or 1 - 1/(2 tau)
  float lcut;         // -cutoff * eps
  float phi_k;        // 4 / eps * log2(e)
  float wall_h;
  uint32_t wall_mask; // bit 0 y, bit 1 x, bit 2 z
  int32_t store_nt;   // population stores carry the non-temporal hint
  int32_t storage;    // 0: FP32 populations; 1: FP16, g 2^k, stochastically rounded
  float store_scale, store_inv;  // 2^k and 2^-k (1 for FP32)
  // nodes within h + cutoff*eps of a walled seam: [0, lo) and [hi, n) on each axis
  int32_t wall_lo[3], wall_hi[3];  // axis order x, y, z
  // open ends in x (non-equilibrium extrapolation at the planes x = 0 and x = nx - 1)
  int32_t xbc, inlet_kind, inlet_profile, outlet_kind;
  float u_in[3];      // prescribed inlet velocity (peak of a parabolic profile)
  float drho_in, drho_out;  // prescribed inlet / outlet density minus rho0
  // parabolic inlet: s = (c + 1/2 - c0) * inv_h across y (and z for a duct)
  float prof_y0, prof_inv_hy, prof_z0, prof_inv_hz;
  // FP64 sphere constants
  double rho0_d;
  double gx, gy, gz;
  double inv_eps_p, inv_eps_p1, inv_eps_w, inv_eps_w1, xi;
  double wall_h_d;
  double support;     // cutoff * eps
  // device buffers
  float *pop[2];
  int32_t *tile_head[2];
  int32_t *tile_list[2];
  double *bstate[2];
  const double *bconst;
  SphereSnap *bsnap[2];
  double *acc[2];
  // tile lists kept across steps (as in two dimensions): the list set the steps of parity
  // p read, the per-parity rebin requests, and each sphere's position at its last binning
  int32_t *lsel;
  int32_t *rb_flag;
  double *bin_ref;
  int32_t *err;
};

}  // namespace dilbm
