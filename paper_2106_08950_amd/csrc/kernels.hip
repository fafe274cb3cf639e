// kernels.hip -- gfx950 kernels of the DI-LBM time step.
//
// k_collide   one fused pass over every node of every member solve: pull the 9 shifted
//             populations (streaming, Eq. (13) left-hand side), take the moments
//             (Eqs. (5), (16)), rebuild the diffuse solid field of the bodies listed for
//             the node's tile (Eq. (14)), correct the velocity (Eq. (17)), collide with the
//             Eq. (15) force term (Eq. (13)) and write the 9 populations back at the node.
//             Per listed body, each wave sums its nodes' force and torque contributions
//             in FP64 (a transpose through the wave's own LDS rows) and adds the totals
//             with one atomic instruction (Eqs. (18)-(19)).
// k_bodies    one wave per body, FP64: repulsion (Eqs. (28)-(29)), Newton-Euler update
//             (Eqs. (22)-(24)) and binning of the moved body into the tile lists of the
//             next step.
// k_fields    rho and corrected u of the current state (no collision).
//
// The stencil is bandwidth bound (about 3 FLOP per byte of population traffic), so the
// kernel is built for HBM streaming: structure-of-arrays planes, one node per lane, 64
// consecutive nodes of a row per wave.  FP32 whole-row tiles (256 x 1) run one tile per
// block in natural order, so neighbouring row segments stream on the eight XCDs at
// once; other shapes sweep contiguous chunks of each XCD's eighth of the tiles
// (neighbouring tiles share L2 lines at their edges).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.h"
#include "dilbm_internal.h"
#include "kernels.h"

namespace dilbm {

namespace {

// D2Q9 velocities of Eq. (3).  The populations are kept as g_i = 36 (f_i - w_i rho0), so
// the weights of Eq. (4) enter as the exact integers K_i = 36 w_i = 16, 4, 1: with 1/9 and
// 1/36 rounded to FP32 the equilibrium's first moment would be rho u (1 + 7.5e-9), a
// momentum source of that relative size in every collision that compounds over
// thousands of steps.  Every constant on the mass and momentum path is exact in binary;
// what remains is unbiased round-to-nearest.
constexpr int CX[kQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY[kQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr float KQ[kQ] = {16.0f, 4.0f, 4.0f, 4.0f, 4.0f, 1.0f, 1.0f, 1.0f, 1.0f};


struct StoreF32 {
  static constexpr int kWaves = DILBM_COLLIDE_WAVES_F32;  // register budget, waves per SIMD
  using T = float;
  static constexpr bool kFrame = true;  // stored in the moving frame of ref_velocity
  static constexpr int kRefLog2 = -17;  // |V_t| < 2^-17
  static constexpr bool kStochastic = false;
  static constexpr bool kScaled = false;  // stored values are g_i itself
  static __device__ __forceinline__ float ldb(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                              uint32_t soff, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  }
  template <bool NT = false>
  static __device__ __forceinline__ void stb(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                             uint32_t soff, float v, float) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff,
                                          NT ? kStoreNT : 0);
  }
  static __device__ __forceinline__ float ld(const T *p, int64_t i, float) { return p[i]; }
  template <bool NT = false>
  static __device__ __forceinline__ void st(T *p, int64_t i, float v, float) {
    put<NT>(v, p + i);
  }
  static __device__ __forceinline__ float ldo(const T *plane, uint32_t byte_off, float) {
    return *(const DILBM_GLOBAL T *)((const DILBM_GLOBAL char *)plane + byte_off);
  }
  template <bool NT = false>
  static __device__ __forceinline__ void sto(T *plane, uint32_t byte_off, float v, float) {
    put<NT>(v, (DILBM_GLOBAL T *)((DILBM_GLOBAL char *)plane + byte_off));
  }
};

// FP16 storage keeps 11 significant bits of g_i 2^k.  Rounded to nearest, a population
// whose per-step change is under half an FP16 ulp never changes at all: a slowly
// accelerating flow stalls.  The collide write-back therefore rounds stochastically:
// random bits below the 10 kept mantissa bits are added to the FP32 pattern, which is
// then truncated; the stored value rounds up with probability equal to its distance
// from the lower neighbour in ulps, so it is right on average at every magnitude
// (values that are already representable, zero included, are stored exactly).  Host
// conversions in and out round to nearest.  FP16 needs no moving frame: its storage
// rounding dwarfs the FP32 arithmetic drift the frame removes.
struct StoreF16 {
  static constexpr int kWaves = DILBM_COLLIDE_WAVES_F16;  // register budget, waves per SIMD
  using T = _Float16;
  static constexpr bool kFrame = false;
  static constexpr int kRefLog2 = 0;
  static constexpr bool kStochastic = true;
  // the collide kernel works on the stored scale g_i 2^k directly (no multiply by 2^-k
  // after each load or by 2^k before each store)
  static constexpr bool kScaled = true;
  // v * scale rounded stochastically to FP16.  The gfx950 conversion v_cvt_sr_f16_f32 adds
  // the top 13 bits of its random operand to the 13 FP32 mantissa bits that FP16 drops,
  // then truncates (normal range), so with 13 uniform random bits the stored value rounds
  // up with exactly its distance from the lower neighbour: unbiased for every FP32 input.
  // (Eight random bits leave a bias of up to 1/512 ulp that depends on where the value
  // sits between its neighbours; in a slowly varying flow it repeats from step to step,
  // and it moved the settling disc of the FP16 tests by 9e-3 lattice units in 20 000
  // steps, against 1.6e-3 with 13 bits.)  h supplies 32 random bits; odd k take the word
  // rotated by 13, so one word serves two populations with disjoint bits.
  static __device__ __forceinline__ uint16_t round_bits(float v, float scale, uint32_t h,
                                                        int k) {
    return sr_half(v * scale, (k & 1) ? __builtin_amdgcn_alignbit(h, h, 13) : h);
  }
  template <bool NT = false>
  static __device__ __forceinline__ void stb_bits(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                  uint32_t soff, uint16_t h) {
    __builtin_amdgcn_raw_buffer_store_b16(h, r, voff, soff, NT ? kStoreNT : 0);
  }
  template <bool NT = false>
  static __device__ __forceinline__ void st_bits(T *p, int64_t i, uint16_t h) {
    put<NT>(h, (uint16_t *)p + i);
  }
  template <bool NT = false>
  static __device__ __forceinline__ void sto_bits(T *plane, uint32_t byte_off, uint16_t h) {
    put<NT>(h, (DILBM_GLOBAL uint16_t *)((DILBM_GLOBAL char *)plane + byte_off));
  }
  static __device__ __forceinline__ float ldb(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                              uint32_t soff, float inv) {
    const uint16_t h = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
    return (float)__builtin_bit_cast(_Float16, h) * inv;
  }
  template <bool NT = false>
  static __device__ __forceinline__ void stb(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                             uint32_t soff, float v, float scale) {
    const _Float16 h = (_Float16)(v * scale);  // round to nearest even
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, h), r, voff, soff,
                                          NT ? kStoreNT : 0);
  }
  static __device__ __forceinline__ float ld(const T *p, int64_t i, float inv) {
    return (float)p[i] * inv;
  }
  template <bool NT = false>
  static __device__ __forceinline__ void st(T *p, int64_t i, float v, float scale) {
    put<NT>((_Float16)(v * scale), p + i);  // round to nearest even
  }
  static __device__ __forceinline__ float ldo(const T *plane, uint32_t byte_off, float inv) {
    return (float)*(const DILBM_GLOBAL T *)((const DILBM_GLOBAL char *)plane + byte_off) * inv;
  }
  template <bool NT = false>
  static __device__ __forceinline__ void sto(T *plane, uint32_t byte_off, float v, float scale) {
    put<NT>((_Float16)(v * scale), (DILBM_GLOBAL T *)((DILBM_GLOBAL char *)plane + byte_off));
  }
};

constexpr float kInv36 = 1.0f / 36.0f;

// x / 36 to within the round-off of the correctly rounded quotient: one product with the
// rounded reciprocal and one exact-residual correction.  Unlike x * fl(1/36) alone it
// carries no constant relative bias.
__device__ __forceinline__ float div36(float x) {
  const float q = x * kInv36;
  return fmaf(fmaf(-36.0f, q, x), kInv36, q);
}

// Reference frame of the stored populations.  Step t has a uniform velocity V_t, and
// what is stored is g_i - 3 K_i c_i.V_t.  The step computes the same update in that
// frame: the equilibrium's linear term takes the momentum relative to V_t, the
// second-order, forcing and solid terms the true velocity.  Only the rounding changes.
// In a smooth, steadily driven flow a node gains nearly the same increment every step,
// and rounding a fixed increment onto the FP32 (or FP16) grid of a slowly changing value
// makes the same error every step: a drift that grows with the step count (about 6e-5
// of the momentum after 1000 steps of uniform acceleration at tau = 0.6).  With V_t
// pseudo-random those roundings see a different offset every step and average out.
// V_t has 20 significant bits on the binary grid 2^(L-19), |V_t| < 2^L, so every frame
// constant 3 K_i c_i.V_t, its changes and short sums of them are exact in FP32: a fluid
// at rest stays exactly at rest.  V_t is the SplitMix64 finaliser (Steele, Lea and
// Flood, OOPSLA 2014) of t, the solve's own step count: the same sequence whether a
// solve runs alone or batched.

template <int L>
__device__ __forceinline__ float2 ref_velocity(int64_t t) {
  const uint64_t z = splitmix64((uint64_t)t);
  const int kx = (int)(z & 0xFFFFFu) - (1 << 19);
  const int ky = (int)((z >> 20) & 0xFFFFFu) - (1 << 19);
  constexpr float q = (float)(1.0 / (double)(1ull << (19 - L)));  // 2^(L-19)
  return make_float2((float)kx * q, (float)ky * q);
}

template <class ST>
__device__ __forceinline__ float2 frame_velocity(int64_t t) {
  if constexpr (ST::kFrame)
    return ref_velocity<ST::kRefLog2>(t);
  else
    return make_float2(0.0f, 0.0f);
}

// 3 K_i c_i.V: the frame offset of direction i
__device__ __forceinline__ double frame_offset(int i, float2 V) {
  return 3.0 * (double)KQ[i] * ((double)CX[i] * V.x + (double)CY[i] * V.y);
}

// A body snapshot through the constant address space (scalar loads: the index is
// wave-uniform and no kernel writes snapshots while the collide kernel reads them).
__device__ __forceinline__ BodySnap load_snap(const DILBM_CONST BodySnap *q) {
  return BodySnap{q->x, q->y, q->u, q->v, q->w, q->r};
}





enum TileMode { kModeStep = 0, kModeFields = 1 };

// How population planes are addressed: one buffer resource per population buffer with
// scalar plane offsets (buffer under 4 GB), a scalar plane base with 32-bit byte offsets
// (plane under 2 GB), or 64-bit addresses.
enum AddrMode { kAddrBuf = 0, kAddrG32 = 1, kAddrWide = 2 };

// Per-node inputs of the collision, all in g units (36 x physical) except where noted.
struct NodeState {
  float drho, rho;        // physical
  float ux, uy;           // corrected velocity, Eq. (17)
  float momx, momy;       // rho u - V: momentum relative to the storage frame, physical
  float Px, Py;           // rho (A - Phi u*), physical
  float Qxx, Qxy, Qyy;    // rho (M - Phi u* u*), physical
};

// Eq. (13) for one node, over the four pairs of opposite directions (c_j = -c_i) so that
// each pair shares its even part: the post-collision g_i is
//   g_i + omega (geq_i - g_i) + khalf K_i S_i,
//   geq_i = K_i [drho + 3 c.(rho u - V) + rho (4.5 (c.u)^2 - 1.5 u^2)]   (frame V),
//   S_i   = 3 (c - u).G + 9 (c.u)(c.G)                          (body-force forcing)
//         + 3 c.P + 4.5 c.Q.c - 1.5 tr Q   when the tile has solid (Eq. (15) summed).
template <bool SOLID, bool SCALED = false>
__device__ __forceinline__ void collide_node(const float f[kQ], float out[kQ], const NodeState &n,
                                             const SolveDesc &d, float inv = 1.0f,
                                             float scale = 1.0f) {
  // SCALED: f and out are at the storage scale (g_i 2^k, as FP16 stores them); the update
  // is formed in g units and applied at that scale (inv = 2^-k, scale = 2^k, both exact)
  const float Gx = d.Gx, Gy = d.Gy, om = d.omega;
  const float usq = n.ux * n.ux + n.uy * n.uy;
  const float even0 = fmaf(-1.5f * n.rho, usq, n.drho);
  const float r45 = 4.5f * n.rho;
  float se0 = -3.0f * (n.ux * Gx + n.uy * Gy);
  if (SOLID) se0 = fmaf(-1.5f, n.Qxx + n.Qyy, se0);
  // each output is f + (small update): the update's own roundings are tiny, and the one
  // rounding at the scale of f sees an addend that changes from step to step
  if (SCALED)
    out[0] = fmaf(scale, fmaf(om, fmaf(-inv, f[0], 16.0f * even0), d.khk16 * se0), f[0]);
  else
    out[0] = f[0] + fmaf(om, 16.0f * even0 - f[0], d.khk16 * se0);
  auto pair = [&](int i, int j, float K, float khK, float g9, float g3, float cu, float cm,
                  float cP, float cQc) {
    const float E = fmaf(r45, cu * cu, even0);
    const float O = 3.0f * cm;
    float Se = fmaf(g9, cu, se0);
    float So = g3;
    if (SOLID) {
      Se = fmaf(4.5f, cQc, Se);
      So = fmaf(3.0f, cP, So);
    }
    if (SCALED) {
      out[i] = fmaf(scale, fmaf(om, fmaf(-inv, f[i], K * (E + O)), khK * (Se + So)), f[i]);
      out[j] = fmaf(scale, fmaf(om, fmaf(-inv, f[j], K * (E - O)), khK * (Se - So)), f[j]);
    } else {
      out[i] = f[i] + fmaf(om, K * (E + O) - f[i], khK * (Se + So));
      out[j] = f[j] + fmaf(om, K * (E - O) - f[j], khK * (Se - So));
    }
  };
  // (1,0)/(-1,0), (0,1)/(0,-1), (1,1)/(-1,-1), (-1,1)/(1,-1)
  pair(1, 3, 4.0f, d.khk4, d.g9[0], d.g3[0], n.ux, n.momx, n.Px, n.Qxx);
  pair(2, 4, 4.0f, d.khk4, d.g9[1], d.g3[1], n.uy, n.momy, n.Py, n.Qyy);
  pair(5, 7, 1.0f, d.khalf, d.g9[2], d.g3[2], n.ux + n.uy, n.momx + n.momy, n.Px + n.Py,
       n.Qxx + 2.0f * n.Qxy + n.Qyy);
  pair(6, 8, 1.0f, d.khalf, d.g9[3], d.g3[3], n.uy - n.ux, n.momy - n.momx, n.Py - n.Px,
       n.Qxx - 2.0f * n.Qxy + n.Qyy);
}

// Change of storage frame V_t -> V_{t+1} of one node's populations: g_i -= 3 K_i c_i.dV
// (axis directions 12 dV, diagonals 3 (dVx +- dVy); exact constants).
struct FrameShift {
  float a, b, c5, c6;
  __device__ __forceinline__ void apply(float g[kQ]) const {
    g[1] -= a;
    g[3] += a;
    g[2] -= b;
    g[4] += b;
    g[5] -= c5;
    g[7] += c5;
    g[6] -= c6;
    g[8] += c6;
  }
};

// 36 (f^eq_i - w_i rho0) in the storage frame V for density R/36 and velocity u, with
// mom = rho u - V given separately (physical units).
__device__ __forceinline__ void geq_frame(float R, float rho36, float ux, float uy, float momx,
                                          float momy, float geq[kQ]) {
  const float rho = R * kInv36;
  const float drho = (R - rho36) * kInv36;
  const float even0 = fmaf(-1.5f * rho, ux * ux + uy * uy, drho);
  const float r45 = 4.5f * rho;
  geq[0] = 16.0f * even0;
#pragma unroll
  for (int i = 1; i < kQ; ++i) {
    const float cu = (float)CX[i] * ux + (float)CY[i] * uy;
    const float cm = (float)CX[i] * momx + (float)CY[i] * momy;
    geq[i] = KQ[i] * (fmaf(r45, cu * cu, even0) + 3.0f * cm);
  }
}

// Non-equilibrium extrapolation (Guo, Zheng & Shi 2002), the paper's treatment of its
// physical boundaries (Section 3), at an inlet (x = 0) or outlet (x = nx - 1) node:
// f*_b = f^eq(rho_b, u_b) + (1 - 1/tau) (f_nb - f^eq(rho_nb, u_nb)), from the populations
// the neighbouring column pulls at this step.  u_nb carries half the body force, as in the
// neighbour's own collision; the storage frame cancels in the non-equilibrium part.
template <class ST>
__device__ void nee_node(const SolveDesc &d, const typename ST::T *src, int64_t plane, int x,
                         int y, const FrameShift &fs, float V36x, float V36y, float out[kQ],
                         float &rho_b, float &uxb, float &uyb) {
  const int nx = d.nx, ny = d.ny;
  const bool inlet = x == 0;
  const int xn = inlet ? 1 : nx - 2;  // the neighbour; its pulls stay inside [0, nx)
  float g[kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    int ys = y - CY[i];
    ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
    g[i] = ST::ld(src, i * plane + (int64_t)ys * d.pitch + (xn - CX[i]), d.store_inv);
  }
  fs.apply(g);
  const float D = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
  const float Jx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
  const float Jy = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
  const float R = d.rho36 + D;
  const float Jgx = Jx + (V36x + 18.0f * d.Gx), Jgy = Jy + (V36y + 18.0f * d.Gy);
  const float ux = Jgx / R, uy = Jgy / R;
  const float momx = div36(Jgx - V36x), momy = div36(Jgy - V36y);
  float Rb = R;
  float bx = ux, by = uy;
  if (inlet) {
    if (d.inlet_kind == 0) {  // velocity inlet
      float sh = 1.0f;
      if (d.inlet_profile) {
        const float sv = ((float)y + 0.5f - d.prof_y0) * d.prof_inv_h;
        sh = (sv > 0.0f && sv < 1.0f) ? 4.0f * sv * (1.0f - sv) : 0.0f;
      }
      bx = sh * d.u_in_x;
      by = sh * d.u_in_y;
    } else {
      Rb = d.rho36_in;
    }
  } else if (d.outlet_kind == 0) {
    Rb = d.rho36_out;
  }
  const bool same = Rb == R && bx == ux && by == uy;
  const float mbx = same ? momx : div36(fmaf(Rb, bx, -V36x));
  const float mby = same ? momy : div36(fmaf(Rb, by, -V36y));
  float eb[kQ], en[kQ];
  geq_frame(Rb, d.rho36, bx, by, mbx, mby, eb);
  geq_frame(R, d.rho36, ux, uy, momx, momy, en);
  const float keep = 1.0f - d.omega;
#pragma unroll
  for (int i = 0; i < kQ; ++i) out[i] = fmaf(keep, g[i] - en[i], eb[i]);
  rho_b = Rb * kInv36;
  uxb = bx;
  uyb = by;
}

// One tile of one solve.  MODE kModeStep: full step; kModeFields: moments only.
template <class ST, int TX, int TY, int MODE, int AM, bool OPEN>
__device__ __forceinline__ void process_tile(const SolveDesc &d, const int lt, const int p,
                                             const int64_t t, float (*red)[3][64],
                                             double *__restrict__ out_rho,
                                             double *__restrict__ out_ux,
                                             double *__restrict__ out_uy,
                                             const Region region, const int xoff) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int nx = d.nx, ny = d.ny;
  const int tyi = lt / d.tiles_x;
  const int txi = lt - tyi * d.tiles_x;
  const int x0 = txi * TX, y0 = tyi * TY;
  // xoff: the second half of a 512-node tile, read by the fields pass in two halves
  const int x = x0 + xoff + (tid % TX);
  // a wave covers part of one row when the tile is at least 64 wide: its row is uniform
  const int y = TX >= 64 ? __builtin_amdgcn_readfirstlane(y0 + tid / TX) : y0 + tid / TX;
  const bool valid = (x < nx) && (y < ny);
  // an inlet / outlet node (open ends in x): its state comes from its neighbour
  const bool bnd = OPEN && d.xbc && valid && (x == 0 || x == nx - 1);
  const int xc = min(x, nx - 1);  // clamped coordinates keep loads in bounds
  const int yc = min(y, ny - 1);

  // ---- pull streaming: f_i(x, t) = f_i*(x - c_i, t - 1) --------------------------------
  // (issued before anything else of the tile waits on memory: the population stream is
  // what the kernel is bound by)
  using T = typename ST::T;
  const T *__restrict__ src = (const T *)d.pop[p];
  T *__restrict__ dst = (T *)d.pop[p ^ 1];
  const int pitch = d.pitch;  // row stride of the planes (rows start on 128-byte lines)
  const int64_t plane = (int64_t)pitch * ny;
  const int xm = (xc == 0) ? nx - 1 : xc - 1;
  const int xp = (xc + 1 == nx) ? 0 : xc + 1;
  const int ym = (yc == 0) ? ny - 1 : yc - 1;
  const int yp = (yc + 1 == ny) ? 0 : yc + 1;
  const float inv = d.store_inv;
  const float sc = d.store_scale;
  // scaled storage: f holds the stored values g_i 2^k (the loads skip the multiply)
  const float ld_inv = ST::kScaled ? 1.0f : inv;
  float f[kQ];
  // byte offsets inside a plane: 32-bit unless the plane reaches 2 GB
  uint32_t o_r0 = 0, o_rm = 0, o_rp = 0, o_x0 = 0, o_xm = 0, o_xp = 0;
  constexpr uint32_t es = sizeof(T);
  if (AM != kAddrWide) {
    o_r0 = (uint32_t)(yc * pitch) * es;
    o_rm = (uint32_t)(ym * pitch) * es;
    o_rp = (uint32_t)(yp * pitch) * es;
    o_x0 = (uint32_t)xc * es;
    o_xm = (uint32_t)xm * es;
    o_xp = (uint32_t)xp * es;
  }
  const uint32_t pb = (uint32_t)plane * es;  // plane bytes (buffer mode only)
  if (AM == kAddrBuf && TX >= 64) {
    // rows are wave-uniform: plane and row offsets go in the scalar offset, and every
    // load needs one of three per-lane column offsets
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)src, (short)0, (int)(kQ * pb), kBufferFlags);
    const uint32_t s0 = __builtin_amdgcn_readfirstlane(o_r0);
    const uint32_t sm = __builtin_amdgcn_readfirstlane(o_rm);
    const uint32_t sp = __builtin_amdgcn_readfirstlane(o_rp);
    f[0] = ST::ldb(rs, o_x0, 0 * pb + s0, ld_inv);
    f[1] = ST::ldb(rs, o_xm, 1 * pb + s0, ld_inv);
    f[2] = ST::ldb(rs, o_x0, 2 * pb + sm, ld_inv);
    f[3] = ST::ldb(rs, o_xp, 3 * pb + s0, ld_inv);
    f[4] = ST::ldb(rs, o_x0, 4 * pb + sp, ld_inv);
    f[5] = ST::ldb(rs, o_xm, 5 * pb + sm, ld_inv);
    f[6] = ST::ldb(rs, o_xp, 6 * pb + sm, ld_inv);
    f[7] = ST::ldb(rs, o_xp, 7 * pb + sp, ld_inv);
    f[8] = ST::ldb(rs, o_xm, 8 * pb + sp, ld_inv);
  } else if (AM == kAddrBuf) {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)src, (short)0, (int)(kQ * pb), kBufferFlags);
    f[0] = ST::ldb(rs, o_r0 + o_x0, 0 * pb, ld_inv);
    f[1] = ST::ldb(rs, o_r0 + o_xm, 1 * pb, ld_inv);
    f[2] = ST::ldb(rs, o_rm + o_x0, 2 * pb, ld_inv);
    f[3] = ST::ldb(rs, o_r0 + o_xp, 3 * pb, ld_inv);
    f[4] = ST::ldb(rs, o_rp + o_x0, 4 * pb, ld_inv);
    f[5] = ST::ldb(rs, o_rm + o_xm, 5 * pb, ld_inv);
    f[6] = ST::ldb(rs, o_rm + o_xp, 6 * pb, ld_inv);
    f[7] = ST::ldb(rs, o_rp + o_xp, 7 * pb, ld_inv);
    f[8] = ST::ldb(rs, o_rp + o_xm, 8 * pb, ld_inv);
  } else if (AM == kAddrG32) {
    f[0] = ST::ldo(src + 0 * plane, o_r0 + o_x0, ld_inv);
    f[1] = ST::ldo(src + 1 * plane, o_r0 + o_xm, ld_inv);
    f[2] = ST::ldo(src + 2 * plane, o_rm + o_x0, ld_inv);
    f[3] = ST::ldo(src + 3 * plane, o_r0 + o_xp, ld_inv);
    f[4] = ST::ldo(src + 4 * plane, o_rp + o_x0, ld_inv);
    f[5] = ST::ldo(src + 5 * plane, o_rm + o_xm, ld_inv);
    f[6] = ST::ldo(src + 6 * plane, o_rm + o_xp, ld_inv);
    f[7] = ST::ldo(src + 7 * plane, o_rp + o_xp, ld_inv);
    f[8] = ST::ldo(src + 8 * plane, o_rp + o_xm, ld_inv);
  } else {
    const int64_t r0 = (int64_t)yc * pitch, rm = (int64_t)ym * pitch, rp = (int64_t)yp * pitch;
    f[0] = ST::ld(src, 0 * plane + r0 + xc, ld_inv);
    f[1] = ST::ld(src, 1 * plane + r0 + xm, ld_inv);
    f[2] = ST::ld(src, 2 * plane + rm + xc, ld_inv);
    f[3] = ST::ld(src, 3 * plane + r0 + xp, ld_inv);
    f[4] = ST::ld(src, 4 * plane + rp + xc, ld_inv);
    f[5] = ST::ld(src, 5 * plane + rm + xm, ld_inv);
    f[6] = ST::ld(src, 6 * plane + rm + xp, ld_inv);
    f[7] = ST::ld(src, 7 * plane + rp + xp, ld_inv);
    f[8] = ST::ld(src, 8 * plane + rp + xm, ld_inv);
  }

  // the tile's head (body count and first list entry, one scalar load) and that body's
  // snapshot, in flight with the populations.  The first entry is used before the count
  // is known: it is clamped into range for the snapshot load and used only when the
  // count lists it.  An overflowed list (count > capacity) is flagged by the binning:
  // read only what fits.
  const int ls = *(const DILBM_CONST int32_t *)(d.lsel + p);  // the list set of this step
  const uint64_t hv = *(const DILBM_CONST uint64_t *)(d.tile_head[ls] + 2 * (int64_t)lt);
  const int32_t raw0 = (int32_t)(hv >> 32);
  const int nb = min((int32_t)(uint32_t)hv, d.list_cap);
  const int nbs = d.nbodies;
  const DILBM_CONST int32_t *list =
      (const DILBM_CONST int32_t *)(d.tile_list[ls] + (int64_t)lt * d.list_cap);
  const DILBM_CONST BodySnap *snap = (const DILBM_CONST BodySnap *)d.bsnap[p];
  BodySnap s0{0.0, 0.0, 0.f, 0.f, 0.f, 0.f};
  if (nbs > 0) s0 = load_snap(snap + min(raw0 & kListIndexMask, nbs - 1));
  if (MODE == kModeStep) {
    // the body step after this one rebins into the other set: it starts empty
    if (tid == 0 && *(const DILBM_CONST int32_t *)(d.rb_flag + p) != 0)
      d.tile_head[ls ^ 1][2 * (int64_t)lt] = 0;
    if (lt == 0) {
      double *a = d.acc[p ^ 1];
      for (int i = tid, na = (int)acc_words(d.nbodies, 3); i < na; i += kBlockThreads) a[i] = 0.0;
      if (tid == 0) {  // read by the last body step, raised by the next
        d.nl_flag[p ^ 1] = 0;
        d.rb_flag[p ^ 1] = 0;
      }
    }
  }

  // ---- storage frame: populations of step t are stored relative to V_t; a step moves
  // them to the frame of step t + 1 (exact constants, one rounding per population)
  const float2 Vt = frame_velocity<ST>(t);
  float2 Vf = Vt;
  FrameShift fs{0.0f, 0.0f, 0.0f, 0.0f};
  if (MODE == kModeStep && ST::kFrame) {
    Vf = frame_velocity<ST>(t + 1);
    const float dvx = Vf.x - Vt.x, dvy = Vf.y - Vt.y;
    fs = FrameShift{12.0f * dvx, 12.0f * dvy, 3.0f * (dvx + dvy), 3.0f * (dvy - dvx)};
    fs.apply(f);
  }
  const float V36x = 36.0f * Vf.x, V36y = 36.0f * Vf.y;  // frame momentum, g units (exact)

  // ---- moments, Eqs. (5) and (16); u* carries half the fluid body force ----------------
  // (in g units: D = 36 delta rho, J = 36 j - 36 V, R = 36 rho; the frame carries no mass)
  float D = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  float Jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  float Jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
  if (ST::kScaled) {  // back to g units (exact: a power of two)
    D *= inv;
    Jx *= inv;
    Jy *= inv;
  }
  const float R = d.rho36 + D;
  // rho enters only second-order and body terms, drho only the mass term: a constant
  // relative error of 7.5e-9 from fl(1/36) there is harmless
  const float rho = R * kInv36;
  const float drho = D * kInv36;
  // 1/R: hardware reciprocal plus one Newton step (about half an ulp)
  float Rinv = __builtin_amdgcn_rcpf(R);
  Rinv = fmaf(fmaf(-R, Rinv, 1.0f), Rinv, Rinv);
  // 36 rho u* = 36 (j + G/2), back in the fixed frame
  const float Jgx = Jx + (V36x + 18.0f * d.Gx);
  const float Jgy = Jy + (V36y + 18.0f * d.Gy);
  const float usx = Jgx * Rinv;         // u*
  const float usy = Jgy * Rinv;

  // ---- diffuse solid field, Eq. (14), and its sums over the covering bodies ------------
  float Phi = 0.f, Ax = 0.f, Ay = 0.f, Mxx = 0.f, Mxy = 0.f, Myy = 0.f;
  const float lcut = d.lcut;
  const float phik = d.phi_k;
  const float h = d.wall_h;
  // walls: static slabs across the seams; does this tile reach into one's support?
  // (rows [0, wall_lo) and [wall_hi, n) hold the nodes within h + cutoff of a seam)
  const bool wy = (d.wall_mask & 1u) && (y0 < d.wall_y_lo || y0 + TY > d.wall_y_hi);
  const bool wx = (d.wall_mask & 2u) && (x0 < d.wall_x_lo || x0 + TX > d.wall_x_hi);
  const bool any_solid = (nb > 0) || wy || wx;

  if (any_solid) {
    float lwy = -1e30f, lwx = -1e30f;
    if (wy) {
      float dy = (float)yc + 0.5f;
      if (dy >= 0.5f * (float)ny) dy -= (float)ny;
      lwy = h - fabsf(dy);
    }
    if (wx) {
      float dx = (float)xc + 0.5f;
      if (dx >= 0.5f * (float)nx) dx -= (float)nx;
      lwx = h - fabsf(dx);
    }
    const double xnode = (double)xc + 0.5, ynode = (double)yc + 0.5;
    const double dnx = (double)nx, dny = (double)ny;
    // listed body j: its index (checked: a bad entry is flagged and skipped), whether its
    // support reaches this wave's nodes (the entry's wave mask), and its snapshot
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    auto body = [&](const int j, int &e, BodySnap &sj) -> bool {
      const int32_t raw = j == 0 ? raw0 : list[j];
      e = raw & kListIndexMask;
      if (e >= nbs) {
        if (lane == 0) atomicOr(d.err, (int32_t)kErrInternal);
        return false;
      }
      // the wave masks describe the step kernel's waves; the fields pass takes every
      // listed body
      if (MODE == kModeStep && !((raw >> (kListIndexBits + wave)) & 1)) return false;
      if (j == 0)
        sj = s0;
      else
        sj = load_snap(snap + e);
      return true;
    };
    // One pass over the listed bodies with unit weights.  The weights of several
    // overlapping supports are w_b = phi_b min(1, 1/S), S = sum of phi over the bodies
    // and walls; every sum below is linear in the weights, so the node-local sums are
    // scaled once afterwards, and the force sums, already added, are corrected by a
    // second pass only in waves where some node has S > 1.
    const float kap = d.kappa;
    double *__restrict__ acc = d.acc[p];
    const bool own = valid && !bnd;  // a node whose solid field this tile computes
    float S = 0.f;
    if (own && wy && lwy >= lcut) S += phi_of(lwy, phik);
    if (own && wx && lwx >= lcut) S += phi_of(lwx, phik);
    // the wave's three sums of one body's force and torque, by a transpose through its own
    // LDS rows: each lane stores its three values, lanes 8k..8k+7 add the 64 values of
    // component k (eight each, in FP64), three DPP steps combine the eight, and one atomic
    // instruction with three active lanes adds the totals
    auto reduce3 = [&](const int e, const float fx, const float fy, const float tq) {
      float(*r)[64] = red[tid >> 6];
      r[0][lane] = fx;
      r[1][lane] = fy;
      r[2][lane] = tq;
      __builtin_amdgcn_wave_barrier();
      double part = 0.0;
      if (lane < 24) {
        const float *q = &r[lane >> 3][(lane & 7) * 8];
#pragma unroll
        for (int k = 0; k < 8; ++k) part += (double)q[k];
      }
      __builtin_amdgcn_wave_barrier();
      part += dpp_f64<0xB1>(part);   // quad_perm [1, 0, 3, 2]
      part += dpp_f64<0x4E>(part);   // quad_perm [2, 3, 0, 1]
      part += dpp_f64<0x141>(part);  // row_half_mirror: the eight lanes of a group
      if (lane < 24 && (lane & 7) == 0) unsafeAtomicAdd(&acc[3 * e + (lane >> 3)], part);
    };
    for (int j = 0; j < nb; ++j) {
      int e;
      BodySnap sj;
      if (!body(j, e, sj)) continue;
      const float rx = (float)min_image(xnode - sj.x, dnx);
      const float ry = (float)min_image(ynode - sj.y, dny);
      const float l = sj.r - __builtin_amdgcn_sqrtf(rx * rx + ry * ry);  // within 1 ulp
      float fx = 0.f, fy = 0.f, tq = 0.f;
      if (own && l >= lcut) {
        const float w = phi_of(l, phik);
        S += w;
        // rigid-body solid velocity U + omega x r
        const float ux_s = sj.u - sj.w * ry;
        const float uy_s = sj.v + sj.w * rx;
        Phi += w;
        Ax += w * ux_s;
        Ay += w * uy_s;
        Mxx += w * ux_s * ux_s;
        Mxy += w * ux_s * uy_s;
        Myy += w * uy_s * uy_s;
        // force on the body: -w rho (u_s - u*) (times the Eq. (18) scale)
        fx = -kap * w * rho * (ux_s - usx);
        fy = -kap * w * rho * (uy_s - usy);
        tq = rx * fy - ry * fx;
      }
      if (MODE == kModeStep && __ballot(fx != 0.f || fy != 0.f) != 0) reduce3(e, fx, fy, tq);
    }
    const float scale = S > 1.0f ? 1.0f / S : 1.0f;
    Phi *= scale;
    Ax *= scale;
    Ay *= scale;
    Mxx *= scale;
    Mxy *= scale;
    Myy *= scale;
    // where S > 1 the forces above took phi_b for w_b: add (scale - 1) times them
    if (MODE == kModeStep && __ballot(own && S > 1.0f) != 0) {
      const float c = scale - 1.0f;  // 0 where S <= 1
      for (int j = 0; j < nb; ++j) {
        int e;
        BodySnap sj;
        if (!body(j, e, sj)) continue;
        const float rx = (float)min_image(xnode - sj.x, dnx);
        const float ry = (float)min_image(ynode - sj.y, dny);
        const float l = sj.r - __builtin_amdgcn_sqrtf(rx * rx + ry * ry);
        float fx = 0.f, fy = 0.f, tq = 0.f;
        if (own && c != 0.0f && l >= lcut) {
          const float w = phi_of(l, phik);
          const float ux_s = sj.u - sj.w * ry;
          const float uy_s = sj.v + sj.w * rx;
          fx = c * (-kap * w * rho * (ux_s - usx));
          fy = c * (-kap * w * rho * (uy_s - usy));
          tq = rx * fy - ry * fx;
        }
        if (__ballot(fx != 0.f || fy != 0.f) != 0) reduce3(e, fx, fy, tq);
      }
    }

    // wall slabs: solid velocity 0; their force goes to the last accumulator slot
    if (wy || wx) {
      float fx = 0.f, fy = 0.f;
      if (valid && !bnd && wy && lwy >= lcut) {
        const float w = scale * phi_of(lwy, phik);
        Phi += w;
        fx += kap * w * rho * usx;
        fy += kap * w * rho * usy;
      }
      if (valid && !bnd && wx && lwx >= lcut) {
        const float w = scale * phi_of(lwx, phik);
        Phi += w;
        fx += kap * w * rho * usx;
        fy += kap * w * rho * usy;
      }
      if (MODE == kModeStep && __ballot(fx != 0.f || fy != 0.f) != 0) {
        const double sx = wave_sum((double)fx);
        const double sy = wave_sum((double)fy);
        if (lane == 0) {
          double *wa = acc + wall_base(3 * nbs) + (blockIdx.x % kWallSlots) * kWallSlotWords;
          unsafeAtomicAdd(wa, sx);
          unsafeAtomicAdd(wa + 1, sy);
        }
      }
    }
  }

  // ---- corrected velocity, Eq. (17): u = u* + (sum_b w_b u_s,b - Phi u*) / 2 ----------
  // P = rho (A - Phi u*) is the momentum the node takes from the bodies; 36 rho u =
  // 36 rho u* + 18 P.  The equilibrium's momentum-carrying term is built from
  // rho u - V = (36 rho u - 36 V) / 36 directly: through u = (36 rho u) / R it would
  // inherit the constant rounding error of 1/R (R is 36 to within 1e-5, a handful of
  // float values), a momentum bias in every collision that compounds over the run.
  const float Px = rho * (Ax - Phi * usx);
  const float Py = rho * (Ay - Phi * usy);
  const float Mx = fmaf(18.0f, Px, Jgx);
  const float My = fmaf(18.0f, Py, Jgy);
  const float ux = Mx * Rinv;
  const float uy = My * Rinv;
  // an inlet / outlet node in this wave (periodic instances compile all of it away)
  const bool any_bnd = OPEN && d.xbc && __ballot(bnd) != 0;

  if (MODE == kModeFields) {
    float rho_r = rho, uxr = ux, uyr = uy;
    if constexpr (OPEN) {
      if (any_bnd && bnd) {
        float tmp[kQ];
        nee_node<ST>(d, src, plane, x, y, fs, V36x, V36y, tmp, rho_r, uxr, uyr);
      }
    }
    // out_* cover the region [rx0, rx0 + rw) x [ry0, ry0 + rh), row stride rw
    const int ox = x - region.x, oy = y - region.y;
    if (valid && ox >= 0 && ox < region.w && oy >= 0 && oy < region.h) {
      const int64_t o = (int64_t)oy * region.w + ox;
      out_rho[o] = (double)rho_r;
      out_ux[o] = (double)uxr;
      out_uy[o] = (double)uyr;
    }
    return;
  }


  // ---- collision, Eq. (13), in g units ----------------------------------------------
  NodeState n;
  n.drho = drho;
  n.rho = rho;
  n.ux = ux;
  n.uy = uy;
  n.momx = div36(Mx - V36x);
  n.momy = div36(My - V36y);
  n.Px = Px;
  n.Py = Py;
  n.Qxx = rho * (Mxx - Phi * usx * usx);
  n.Qxy = rho * (Mxy - Phi * usx * usy);
  n.Qyy = rho * (Myy - Phi * usy * usy);
  float out[kQ];
  if (any_solid)
    collide_node<true, ST::kScaled>(f, out, n, d, inv, sc);
  else
    collide_node<false, ST::kScaled>(f, out, n, d, inv, sc);
  // inlet / outlet nodes replace the result (after the collision: no registers held
  // across it for the few boundary lanes)
  float rho_r = rho, uxr = ux, uyr = uy;
  if constexpr (OPEN) {
    if (any_bnd && bnd) {
      nee_node<ST>(d, src, plane, x, y, fs, V36x, V36y, out, rho_r, uxr, uyr);
      if (ST::kScaled) {  // to the stored scale
#pragma unroll
        for (int i = 0; i < kQ; ++i) out[i] *= sc;
      }
    }
  }
  const float usq = uxr * uxr + uyr * uyr;
  if (__ballot(valid && !(rho_r > 0.0f && usq <= 0.25f)) != 0 && lane == 0)
    atomicOr(d.err, (int32_t)kErrUnstable);
  uint16_t hb[kQ];  // FP16: the stochastically rounded halves
  if constexpr (ST::kStochastic) {
    // 13 random bits per population: five 32-bit words, one hash of (node, step) and four
    // xorshifts, each serving two populations
    const uint32_t tk = lowbias32((uint32_t)t ^ lowbias32((uint32_t)((uint64_t)t >> 32)));
    uint32_t hh[5];
    hh[0] = lowbias32(((uint32_t)yc * (uint32_t)nx + (uint32_t)xc) ^ tk);
#pragma unroll
    for (int r = 1; r < 5; ++r) hh[r] = xorshift32(hh[r - 1]);
#pragma unroll
    for (int i = 0; i < kQ; ++i)
      hb[i] = ST::round_bits(out[i], ST::kScaled ? 1.0f : sc, hh[i >> 1], i & 1);
  }
  // non-temporal stores or not, per solve (the engine's choice); the branch is uniform
  auto put_all = [&](auto nt) {
    constexpr bool NT = decltype(nt)::value;
    if (AM == kAddrBuf && TX >= 64) {
      const __amdgpu_buffer_rsrc_t rd =
          __builtin_amdgcn_make_buffer_rsrc((void *)dst, (short)0, (int)(kQ * pb), kBufferFlags);
      const uint32_t s0 = __builtin_amdgcn_readfirstlane(o_r0);
#pragma unroll
      for (int i = 0; i < kQ; ++i) {
        if constexpr (ST::kStochastic)
          ST::template stb_bits<NT>(rd, o_x0, i * pb + s0, hb[i]);
        else
          ST::template stb<NT>(rd, o_x0, i * pb + s0, out[i], sc);
      }
    } else if (AM == kAddrBuf) {
      const __amdgpu_buffer_rsrc_t rd =
          __builtin_amdgcn_make_buffer_rsrc((void *)dst, (short)0, (int)(kQ * pb), kBufferFlags);
      const uint32_t o = o_r0 + o_x0;
#pragma unroll
      for (int i = 0; i < kQ; ++i) {
        if constexpr (ST::kStochastic)
          ST::template stb_bits<NT>(rd, o, i * pb, hb[i]);
        else
          ST::template stb<NT>(rd, o, i * pb, out[i], sc);
      }
    } else if (AM == kAddrG32) {
      const uint32_t o = o_r0 + o_x0;
#pragma unroll
      for (int i = 0; i < kQ; ++i) {
        if constexpr (ST::kStochastic)
          ST::template sto_bits<NT>(dst + i * plane, o, hb[i]);
        else
          ST::template sto<NT>(dst + i * plane, o, out[i], sc);
      }
    } else {
      const int64_t o = (int64_t)yc * pitch + xc;
#pragma unroll
      for (int i = 0; i < kQ; ++i) {
        if constexpr (ST::kStochastic)
          ST::template st_bits<NT>(dst, i * plane + o, hb[i]);
        else
          ST::template st<NT>(dst, i * plane + o, out[i], sc);
      }
    }
  };
  if (valid) {
    if (d.store_nt)
      put_all(std::true_type{});
    else
      put_all(std::false_type{});
  }
}

// ---- FP16 populations, two nodes per lane --------------------------------------------
// Whole-row tiles of 512 nodes: lane l of a block holds the neighbouring nodes
// x0 + 2l and x0 + 2l + 1.  Every plane's row segment is then 1 KB, as for FP32 in
// 256-node tiles, each lane moves its two populations of a plane in one 4-byte access,
// and a wave keeps twice the bytes in flight of a one-node lane.  Pairs pulled across x
// start at an odd element: those 4-byte loads are 2-byte aligned (gfx9 takes unaligned
// dword loads in the unaligned access mode that the ROCm runtime sets); at the periodic
// row ends the two halves are loaded separately.  Needs an even nx.  Per node the
// arithmetic is that of process_tile.

// Two neighbouring FP16 populations as floats times inv (the lower address first).
__device__ __forceinline__ void unpack2(uint32_t v, float inv, float &a, float &b) {
  a = (float)__builtin_bit_cast(_Float16, (uint16_t)(v & 0xFFFFu)) * inv;
  b = (float)__builtin_bit_cast(_Float16, (uint16_t)(v >> 16)) * inv;
}

// Elements e0 and e1 of a row of FP16 populations as one 32-bit word (e0 in the low half):
// one load when they are neighbours, else two.  Buffer form: `row` is the scalar byte
// offset of the row inside the buffer; pointer form: `base` is the row's first element.
__device__ __forceinline__ uint32_t ld_pair_buf(__amdgpu_buffer_rsrc_t r, uint32_t row, int e0,
                                                int e1) {
  if (e1 == e0 + 1) return __builtin_amdgcn_raw_buffer_load_b32(r, 2u * (uint32_t)e0, row, 0);
  const uint32_t lo = __builtin_amdgcn_raw_buffer_load_b16(r, 2u * (uint32_t)e0, row, 0);
  const uint32_t hi = __builtin_amdgcn_raw_buffer_load_b16(r, 2u * (uint32_t)e1, row, 0);
  return lo | (hi << 16);
}
__device__ __forceinline__ uint32_t ld_pair_ptr(const uint16_t *base, int e0, int e1) {
  if (e1 == e0 + 1) {
    uint32_t v;
    __builtin_memcpy(&v, base + e0, 4);
    return v;
  }
  return (uint32_t)base[e0] | ((uint32_t)base[e1] << 16);
}

template <int AM, bool OPEN>
__device__ __forceinline__ void process_tile_x2(const SolveDesc &d, const int lt, const int p,
                                                const int64_t t, float (*red)[3][64]) {
  using ST = StoreF16;
  constexpr int TX = 512;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int nx = d.nx, ny = d.ny;
  const int tyi = lt / d.tiles_x;
  const int txi = lt - tyi * d.tiles_x;
  const int x0 = txi * TX;
  const int y = __builtin_amdgcn_readfirstlane(tyi);  // one row per tile: wave-uniform
  const int xa = x0 + 2 * tid;                        // the lane's first node
  const bool valid = xa < nx;                         // nx is even: both nodes or neither
  const int xc = min(xa, nx - 2);                     // clamped: loads stay in bounds
  const int ym = (y == 0) ? ny - 1 : y - 1;
  const int yp = (y + 1 == ny) ? 0 : y + 1;
  const float inv = d.store_inv;
  const uint16_t *__restrict__ src = (const uint16_t *)d.pop[p];
  uint16_t *__restrict__ dst = (uint16_t *)d.pop[p ^ 1];
  const int pitch = d.pitch;  // row stride of the planes (a multiple of 64)
  const int64_t plane = (int64_t)pitch * ny;
  // elements pulled across x: c_x = +1 from (xc - 1, xc), c_x = -1 from (xc + 1, xc + 2)
  const int em0 = xc == 0 ? nx - 1 : xc - 1, em1 = xc;
  const int ep0 = xc + 1, ep1 = xc + 2 == nx ? 0 : xc + 2;

  // ---- pull streaming (pairs) --------------------------------------------------------
  uint32_t w[kQ];
  if (AM == kAddrBuf) {
    const uint32_t pb = (uint32_t)plane * 2u;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)src, (short)0, (int)(kQ * pb), kBufferFlags);
    const uint32_t s0 = (uint32_t)(y * pitch) * 2u, sm = (uint32_t)(ym * pitch) * 2u,
                   sp = (uint32_t)(yp * pitch) * 2u;
    w[0] = ld_pair_buf(rs, 0 * pb + s0, xc, xc + 1);
    w[1] = ld_pair_buf(rs, 1 * pb + s0, em0, em1);
    w[2] = ld_pair_buf(rs, 2 * pb + sm, xc, xc + 1);
    w[3] = ld_pair_buf(rs, 3 * pb + s0, ep0, ep1);
    w[4] = ld_pair_buf(rs, 4 * pb + sp, xc, xc + 1);
    w[5] = ld_pair_buf(rs, 5 * pb + sm, em0, em1);
    w[6] = ld_pair_buf(rs, 6 * pb + sm, ep0, ep1);
    w[7] = ld_pair_buf(rs, 7 * pb + sp, ep0, ep1);
    w[8] = ld_pair_buf(rs, 8 * pb + sp, em0, em1);
  } else {
    const int64_t r0 = (int64_t)y * pitch, rm = (int64_t)ym * pitch, rp = (int64_t)yp * pitch;
    w[0] = ld_pair_ptr(src + 0 * plane + r0, xc, xc + 1);
    w[1] = ld_pair_ptr(src + 1 * plane + r0, em0, em1);
    w[2] = ld_pair_ptr(src + 2 * plane + rm, xc, xc + 1);
    w[3] = ld_pair_ptr(src + 3 * plane + r0, ep0, ep1);
    w[4] = ld_pair_ptr(src + 4 * plane + rp, xc, xc + 1);
    w[5] = ld_pair_ptr(src + 5 * plane + rm, em0, em1);
    w[6] = ld_pair_ptr(src + 6 * plane + rm, ep0, ep1);
    w[7] = ld_pair_ptr(src + 7 * plane + rp, ep0, ep1);
    w[8] = ld_pair_ptr(src + 8 * plane + rp, em0, em1);
  }

  // the tile's head and its first body's snapshot, in flight with the populations
  const int ls = *(const DILBM_CONST int32_t *)(d.lsel + p);  // the list set of this step
  const uint64_t hv = *(const DILBM_CONST uint64_t *)(d.tile_head[ls] + 2 * (int64_t)lt);
  const int32_t raw0 = (int32_t)(hv >> 32);
  const int nb = min((int32_t)(uint32_t)hv, d.list_cap);
  const int nbs = d.nbodies;
  const DILBM_CONST int32_t *list =
      (const DILBM_CONST int32_t *)(d.tile_list[ls] + (int64_t)lt * d.list_cap);
  const DILBM_CONST BodySnap *snap = (const DILBM_CONST BodySnap *)d.bsnap[p];
  BodySnap s0{0.0, 0.0, 0.f, 0.f, 0.f, 0.f};
  if (nbs > 0) s0 = load_snap(snap + min(raw0 & kListIndexMask, nbs - 1));
  // the body step after this one rebins into the other set: it starts empty
  if (tid == 0 && *(const DILBM_CONST int32_t *)(d.rb_flag + p) != 0)
    d.tile_head[ls ^ 1][2 * (int64_t)lt] = 0;
  if (lt == 0) {
    double *a = d.acc[p ^ 1];
    for (int i = tid, na = (int)acc_words(d.nbodies, 3); i < na; i += kBlockThreads) a[i] = 0.0;
    if (tid == 0) {  // read by the last body step, raised by the next
      d.nl_flag[p ^ 1] = 0;
      d.rb_flag[p ^ 1] = 0;
    }
  }

  float f[2][kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i) unpack2(w[i], inv, f[0][i], f[1][i]);

  // ---- moments, Eqs. (5) and (16), per node (no storage frame with FP16) -------------
  float rho[2], drho[2], Rinv[2], Jgx[2], Jgy[2], usx[2], usy[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float *g = f[k];
    const float D = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
    const float Jx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    const float Jy = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
    const float R = d.rho36 + D;
    rho[k] = R * kInv36;
    drho[k] = D * kInv36;
    float ri = __builtin_amdgcn_rcpf(R);
    Rinv[k] = fmaf(fmaf(-R, ri, 1.0f), ri, ri);
    Jgx[k] = Jx + 18.0f * d.Gx;
    Jgy[k] = Jy + 18.0f * d.Gy;
    usx[k] = Jgx[k] * Rinv[k];
    usy[k] = Jgy[k] * Rinv[k];
  }

  // ---- diffuse solid field, Eq. (14), per node ----------------------------------------
  float Phi[2] = {0.f, 0.f}, Ax[2] = {0.f, 0.f}, Ay[2] = {0.f, 0.f};
  float Mxx[2] = {0.f, 0.f}, Mxy[2] = {0.f, 0.f}, Myy[2] = {0.f, 0.f};
  const float lcut = d.lcut;
  const float phik = d.phi_k;
  const float h = d.wall_h;
  const bool wy = (d.wall_mask & 1u) && (y < d.wall_y_lo || y + 1 > d.wall_y_hi);
  const bool wx = (d.wall_mask & 2u) && (x0 < d.wall_x_lo || x0 + TX > d.wall_x_hi);
  const bool any_solid = (nb > 0) || wy || wx;
  bool bnd[2] = {false, false};
  if (OPEN && d.xbc && valid) {
    bnd[0] = xa == 0;
    bnd[1] = xa + 1 == nx - 1;
  }

  if (any_solid) {
    float lwy = -1e30f, lwx[2] = {-1e30f, -1e30f};
    if (wy) {
      float dy = (float)y + 0.5f;
      if (dy >= 0.5f * (float)ny) dy -= (float)ny;
      lwy = h - fabsf(dy);
    }
    if (wx) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        float dx = (float)(xc + k) + 0.5f;
        if (dx >= 0.5f * (float)nx) dx -= (float)nx;
        lwx[k] = h - fabsf(dx);
      }
    }
    const double ynode = (double)y + 0.5;
    const double dnx = (double)nx, dny = (double)ny;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    auto body = [&](const int j, int &e, BodySnap &sj) -> bool {
      const int32_t raw = j == 0 ? raw0 : list[j];
      e = raw & kListIndexMask;
      if (e >= nbs) {
        if (lane == 0) atomicOr(d.err, (int32_t)kErrInternal);
        return false;
      }
      if (!((raw >> (kListIndexBits + wave)) & 1)) return false;
      if (j == 0)
        sj = s0;
      else
        sj = load_snap(snap + e);
      return true;
    };
    const float kap = d.kappa;
    double *__restrict__ acc = d.acc[p];
    bool own[2];
    float S[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      own[k] = valid && !bnd[k];
      S[k] = 0.f;
      if (own[k] && wy && lwy >= lcut) S[k] += phi_of(lwy, phik);
      if (own[k] && wx && lwx[k] >= lcut) S[k] += phi_of(lwx[k], phik);
    }
    auto reduce3 = [&](const int e, const float fx, const float fy, const float tq) {
      float(*r)[64] = red[tid >> 6];
      r[0][lane] = fx;
      r[1][lane] = fy;
      r[2][lane] = tq;
      __builtin_amdgcn_wave_barrier();
      double part = 0.0;
      if (lane < 24) {
        const float *q = &r[lane >> 3][(lane & 7) * 8];
#pragma unroll
        for (int k = 0; k < 8; ++k) part += (double)q[k];
      }
      __builtin_amdgcn_wave_barrier();
      part += dpp_f64<0xB1>(part);   // quad_perm [1, 0, 3, 2]
      part += dpp_f64<0x4E>(part);   // quad_perm [2, 3, 0, 1]
      part += dpp_f64<0x141>(part);  // row_half_mirror: the eight lanes of a group
      if (lane < 24 && (lane & 7) == 0) unsafeAtomicAdd(&acc[3 * e + (lane >> 3)], part);
    };
    // one pass with unit weights (see process_tile); a lane's two nodes add their force
    // and torque before the wave's sums
    for (int j = 0; j < nb; ++j) {
      int e;
      BodySnap sj;
      if (!body(j, e, sj)) continue;
      const float ry = (float)min_image(ynode - sj.y, dny);
      float fx = 0.f, fy = 0.f, tq = 0.f;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const float rx = (float)min_image((double)(xc + k) + 0.5 - sj.x, dnx);
        const float l = sj.r - __builtin_amdgcn_sqrtf(rx * rx + ry * ry);
        if (own[k] && l >= lcut) {
          const float wgt = phi_of(l, phik);
          S[k] += wgt;
          const float ux_s = sj.u - sj.w * ry;
          const float uy_s = sj.v + sj.w * rx;
          Phi[k] += wgt;
          Ax[k] += wgt * ux_s;
          Ay[k] += wgt * uy_s;
          Mxx[k] += wgt * ux_s * ux_s;
          Mxy[k] += wgt * ux_s * uy_s;
          Myy[k] += wgt * uy_s * uy_s;
          const float gx = -kap * wgt * rho[k] * (ux_s - usx[k]);
          const float gy = -kap * wgt * rho[k] * (uy_s - usy[k]);
          fx += gx;
          fy += gy;
          tq += rx * gy - ry * gx;
        }
      }
      if (__ballot(fx != 0.f || fy != 0.f) != 0) reduce3(e, fx, fy, tq);
    }
    float scale[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      scale[k] = S[k] > 1.0f ? 1.0f / S[k] : 1.0f;
      Phi[k] *= scale[k];
      Ax[k] *= scale[k];
      Ay[k] *= scale[k];
      Mxx[k] *= scale[k];
      Mxy[k] *= scale[k];
      Myy[k] *= scale[k];
    }
    if (__ballot((own[0] && S[0] > 1.0f) || (own[1] && S[1] > 1.0f)) != 0) {
      for (int j = 0; j < nb; ++j) {
        int e;
        BodySnap sj;
        if (!body(j, e, sj)) continue;
        const float ry = (float)min_image(ynode - sj.y, dny);
        float fx = 0.f, fy = 0.f, tq = 0.f;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const float c = scale[k] - 1.0f;  // 0 where S <= 1
          const float rx = (float)min_image((double)(xc + k) + 0.5 - sj.x, dnx);
          const float l = sj.r - __builtin_amdgcn_sqrtf(rx * rx + ry * ry);
          if (own[k] && c != 0.0f && l >= lcut) {
            const float wgt = phi_of(l, phik);
            const float ux_s = sj.u - sj.w * ry;
            const float uy_s = sj.v + sj.w * rx;
            const float gx = c * (-kap * wgt * rho[k] * (ux_s - usx[k]));
            const float gy = c * (-kap * wgt * rho[k] * (uy_s - usy[k]));
            fx += gx;
            fy += gy;
            tq += rx * gy - ry * gx;
          }
        }
        if (__ballot(fx != 0.f || fy != 0.f) != 0) reduce3(e, fx, fy, tq);
      }
    }
    if (wy || wx) {
      float fx = 0.f, fy = 0.f;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        if (own[k] && wy && lwy >= lcut) {
          const float wgt = scale[k] * phi_of(lwy, phik);
          Phi[k] += wgt;
          fx += kap * wgt * rho[k] * usx[k];
          fy += kap * wgt * rho[k] * usy[k];
        }
        if (own[k] && wx && lwx[k] >= lcut) {
          const float wgt = scale[k] * phi_of(lwx[k], phik);
          Phi[k] += wgt;
          fx += kap * wgt * rho[k] * usx[k];
          fy += kap * wgt * rho[k] * usy[k];
        }
      }
      if (__ballot(fx != 0.f || fy != 0.f) != 0) {
        const double sx = wave_sum((double)fx);
        const double sy = wave_sum((double)fy);
        if (lane == 0) {
          double *wa = acc + wall_base(3 * nbs) + (blockIdx.x % kWallSlots) * kWallSlotWords;
          unsafeAtomicAdd(wa, sx);
          unsafeAtomicAdd(wa + 1, sy);
        }
      }
    }
  }

  // ---- Eq. (17), collision Eq. (13), open ends, checks, per node ----------------------
  const bool any_bnd = OPEN && d.xbc && __ballot(bnd[0] || bnd[1]) != 0;
  const FrameShift fs{0.0f, 0.0f, 0.0f, 0.0f};
  float out[2][kQ];
  bool bad = false;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float Px = rho[k] * (Ax[k] - Phi[k] * usx[k]);
    const float Py = rho[k] * (Ay[k] - Phi[k] * usy[k]);
    const float Mx = fmaf(18.0f, Px, Jgx[k]);
    const float My = fmaf(18.0f, Py, Jgy[k]);
    NodeState n;
    n.drho = drho[k];
    n.rho = rho[k];
    n.ux = Mx * Rinv[k];
    n.uy = My * Rinv[k];
    n.momx = div36(Mx);
    n.momy = div36(My);
    n.Px = Px;
    n.Py = Py;
    n.Qxx = rho[k] * (Mxx[k] - Phi[k] * usx[k] * usx[k]);
    n.Qxy = rho[k] * (Mxy[k] - Phi[k] * usx[k] * usy[k]);
    n.Qyy = rho[k] * (Myy[k] - Phi[k] * usy[k] * usy[k]);
    if (any_solid)
      collide_node<true>(f[k], out[k], n, d);
    else
      collide_node<false>(f[k], out[k], n, d);
    float rho_r = rho[k], uxr = n.ux, uyr = n.uy;
    if constexpr (OPEN) {
      if (any_bnd && bnd[k])
        nee_node<ST>(d, (const _Float16 *)src, plane, xc + k, y, fs, 0.0f, 0.0f, out[k], rho_r,
                     uxr, uyr);
    }
    const float usq = uxr * uxr + uyr * uyr;
    bad = bad || !(rho_r > 0.0f && usq <= 0.25f);
  }
  if (__ballot(valid && bad) != 0 && lane == 0) atomicOr(d.err, (int32_t)kErrUnstable);

  // ---- stochastic FP16 write-back, both nodes' halves in one 4-byte store per plane ---
  const float sc = d.store_scale;
  const uint32_t tk = lowbias32((uint32_t)t ^ lowbias32((uint32_t)((uint64_t)t >> 32)));
  uint32_t hw[kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i) hw[i] = 0u;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    // the same random words per node as process_tile
    uint32_t hh[5];
    hh[0] = lowbias32(((uint32_t)y * (uint32_t)nx + (uint32_t)(xc + k)) ^ tk);
#pragma unroll
    for (int r = 1; r < 5; ++r) hh[r] = xorshift32(hh[r - 1]);
#pragma unroll
    for (int i = 0; i < kQ; ++i)
      hw[i] |= (uint32_t)ST::round_bits(out[k][i], sc, hh[i >> 1], i & 1) << (16 * k);
  }
  auto put_all = [&](auto nt) {
    constexpr bool NT = decltype(nt)::value;
    if (AM == kAddrBuf) {
      const uint32_t pb = (uint32_t)plane * 2u;
      const __amdgpu_buffer_rsrc_t rd =
          __builtin_amdgcn_make_buffer_rsrc((void *)dst, (short)0, (int)(kQ * pb), kBufferFlags);
      const uint32_t s0 = (uint32_t)(y * pitch) * 2u;
#pragma unroll
      for (int i = 0; i < kQ; ++i)
        __builtin_amdgcn_raw_buffer_store_b32(hw[i], rd, 2u * (uint32_t)xc, i * pb + s0,
                                              NT ? kStoreNT : 0);
    } else {
      const int64_t o = (int64_t)y * pitch + xc;
#pragma unroll
      for (int i = 0; i < kQ; ++i) put<NT>(hw[i], (uint32_t *)(dst + i * plane + o));
    }
  };
  if (valid) {
    if (d.store_nt)
      put_all(std::true_type{});
    else
      put_all(std::false_type{});
  }
}

// register budget (waves per SIMD) of a collide instance: two nodes per lane hold twice
// the per-node state
template <class ST, int TX, int TY>
constexpr int collide_waves() {
  return TX * TY > kBlockThreads ? DILBM_COLLIDE_WAVES_X2 : ST::kWaves;
}

template <class ST, int TX, int TY, int AM, bool OPEN>
__global__ __launch_bounds__(kBlockThreads, (collide_waves<ST, TX, TY>())) void k_collide(
    const SolveDesc *__restrict__ descs, const int32_t *__restrict__ tile_solve,
    const BatchHeader *__restrict__ hdr, int k) {
  __shared__ float red[kBlockThreads / 64][3][64];  // per wave: its lanes' force and torque
  const int solo = hdr->solo_slot;  // one member: no per-tile lookup
  auto run = [&](const int64_t t) {
    const int s = solo >= 0 ? solo : __builtin_amdgcn_readfirstlane(tile_solve[t]);
    const SolveDesc &d = descs[s];
    if (k >= d.active_steps) return;
    const int p = (d.parity0 + k) & 1;
    const int lt = (int)(t - d.tile_base);
    if constexpr (TX * TY == 2 * kBlockThreads)
      process_tile_x2<AM, OPEN>(d, lt, p, d.step0 + k, red);
    else
      process_tile<ST, TX, TY, kModeStep, AM, OPEN>(d, lt, p, d.step0 + k, red, nullptr,
                                                    nullptr, nullptr, Region{0, 0, 0, 0}, 0);
  };
  if (hdr->natural) {
    // tile b to block b: consecutive tiles (neighbouring row segments) run on the eight
    // XCDs at once
    for (int64_t t = blockIdx.x; t < hdr->total_tiles; t += gridDim.x) run(t);
    return;
  }
  const WorkSplit ws = xcd_split(hdr->total_tiles);
  // Odd chunks are walked backwards: two neighbouring chunks then reach their common
  // edge at about the same time, so the cache lines the x-shifted loads share across it
  // are still in the XCD's L2 for the second reader.
  const bool rev = (blockIdx.x >> 3) & 1;
  for (int64_t i = ws.begin; i < ws.end; ++i) run(rev ? ws.end - 1 - (i - ws.begin) : i);
}

template <class ST, int TX, int TY>
__global__ __launch_bounds__(kBlockThreads) void k_fields(const SolveDesc *__restrict__ desc,
                                                          int p, Region region,
                                                          double *__restrict__ rho,
                                                          double *__restrict__ ux,
                                                          double *__restrict__ uy) {
  const SolveDesc &d = *desc;
  // tiles that intersect the region
  const int tx0 = region.x / TX, tx1 = (region.x + region.w - 1) / TX;
  const int ty0 = region.y / TY, ty1 = (region.y + region.h - 1) / TY;
  const int ntx = tx1 - tx0 + 1;
  const int64_t n = (int64_t)ntx * (ty1 - ty0 + 1);
  for (int64_t e = blockIdx.x; e < n; e += gridDim.x) {
    const int lt = (int)((ty0 + e / ntx) * d.tiles_x + tx0 + e % ntx);
    // a 512-node tile (one row, two nodes per lane in the step kernel) in two halves
    for (int xoff = 0; xoff < TX * TY; xoff += kBlockThreads)
      process_tile<ST, TX, TY, kModeFields, kAddrWide, true>(d, lt, p, d.step0, nullptr, rho,
                                                             ux, uy, region, xoff);
  }
}

// One wave per body.  BIN_ONLY: bin the bodies of the current state into the lists of
// the current parity (after set_particles or a tile-shape change); otherwise do the body
// step of parity p and bin the moved bodies into the lists of parity p ^ 1.
template <bool BIN_ONLY>
__global__ __launch_bounds__(kBlockThreads) void k_bodies(const SolveDesc *__restrict__ descs,
                                                          const int32_t *__restrict__ body_solve,
                                                          const BatchHeader *__restrict__ hdr,
                                                          int k) {
  const int lane = threadIdx.x & 63;
  const int wpb = kBlockThreads / 64;
  const int total = hdr->total_bodies;
  const int solo = hdr->solo_slot;
  for (int g = blockIdx.x * wpb + (threadIdx.x >> 6); g < total; g += gridDim.x * wpb) {
    const int s = solo >= 0 ? solo : __builtin_amdgcn_readfirstlane(body_solve[g]);
    const SolveDesc &d = descs[s];
    if (!BIN_ONLY && k >= d.active_steps) continue;
    const int p = BIN_ONLY ? (d.parity0 & 1) : ((d.parity0 + k) & 1);
    const int b = g - d.body_base;
    const int nb = d.nbodies;
    if (b < 0 || b >= nb) {  // the tables disagree with the descriptor: never index with b
      if ((threadIdx.x & 63) == 0) atomicOr(d.err, (int32_t)kErrInternal);
      continue;
    }
    const double *st = d.bstate[p];
    const double dnx = (double)d.nx, dny = (double)d.ny;
    double X = st[b], Y = st[nb + b];
    double U = st[2 * nb + b], V = st[3 * nb + b], W = st[4 * nb + b];
    const double R = d.bconst[b], rho_s = d.bconst[nb + b];
    const double m = d.bconst[2 * nb + b], I = d.bconst[3 * nb + b];
    const bool fixed = d.bconst[4 * nb + b] != 0.0;
    int q = p;
    if (BIN_ONLY && b == 0 && lane == 0) d.nl_flag[p] = 1;  // new bodies: build the lists
    // tile lists: the set this step read, and whether this body step rebuilds them (into
    // the other set; a fresh binning writes set 0, emptied by the host)
    const int ls = d.lsel[p];
    const bool rebin = BIN_ONLY || d.rb_flag[p] != 0;
    const int lnew = BIN_ONLY ? 0 : (rebin ? ls ^ 1 : ls);
    if (!BIN_ONLY) {
      // hydrodynamic force and torque of the step (read now: in flight with the pair loads)
      const double *acc = d.acc[p];
      const double hfx = acc[3 * b], hfy = acc[3 * b + 1], T = acc[3 * b + 2];
      // Eq. (28): repulsion from every other body of the solve (minimum image); pairs
      // farther apart than r_i + r_j + xi are rejected on the squared distance.  Partners
      // come from the body's neighbour list (see kNbrCap); when the lists are rebuilt, or
      // this body's overflowed, every other body is swept: first screened on its FP32
      // position (8 bytes each, kU rounds of 64 in flight together) against
      // r_i + max r_j + xi + skin plus a margin far above the FP32 rounding of a position,
      // then tested in FP64, and kept on the list when within r_i + r_j + xi + skin.
      double fx = 0.0, fy = 0.0;
      const double xi = d.xi;
      auto pair = [&](const int j, double &dx, double &dy) -> double {  // d^2, or -1
        dx = min_image(X - st[j], dnx);
        dy = min_image(Y - st[nb + j], dny);
        return dx * dx + dy * dy;
      };
      auto add_force = [&](const int j, const double dx, const double dy, const double d2) {
        const double rr = R + d.bconst[j];
        if (d2 > (rr + xi) * (rr + xi)) return;
        const double dist = sqrt(d2);
        const double kk = dist <= rr ? (rr - dist) * d.inv_eps_p1
                                     : (rr + xi - dist) * (rr + xi - dist) * d.inv_eps_p;
        fx += kk * dx;
        fy += kk * dy;
      };
      int32_t *__restrict__ my_list = d.nbr_list + (int64_t)b * kNbrCap;
      const int cnt0 = d.nbr_cnt[b];
      const bool sweep = d.nl_flag[p] != 0 || cnt0 < 0;
      if (!sweep) {
        // the list: one partner per lane
        if (lane < cnt0) {
          const int j = my_list[lane];
          double dx, dy;
          const double d2 = pair(j, dx, dy);
          add_force(j, dx, dy, d2);
        }
      } else {
        const bool rebuild = d.nl_flag[p] != 0;
        const float *__restrict__ bxy = d.bxy[p];
        const float X32 = (float)X, Y32 = (float)Y;
        const float fnx = (float)d.nx, fny = (float)d.ny;
        const float reach = (float)(R + d.rmax + xi + kNbrSkin) + 0.0625f;
        int cnt = 0;  // list entries kept (wave-uniform)
        constexpr int kU = 16;
        for (int j0 = 0; j0 < nb; j0 += 64 * kU) {
          float2 q32[kU];
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const int j = min(j0 + 64 * u + lane, nb - 1);  // clamped: a valid index
            q32[u] = *(const float2 *)(bxy + 2 * (int64_t)j);
          }
          uint32_t near = 0;  // rounds whose partner is within reach
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            float dx = X32 - q32[u].x, dy = Y32 - q32[u].y;
            if (dx >= 0.5f * fnx) dx -= fnx;
            if (dx < -0.5f * fnx) dx += fnx;
            if (dy >= 0.5f * fny) dy -= fny;
            if (dy < -0.5f * fny) dy += fny;
            if (dx * dx + dy * dy <= reach * reach) near |= 1u << u;
          }
          // rounds in order for every lane, so the list is appended wave by wave
          for (int u = 0; u < kU && j0 + 64 * u < nb; ++u) {
            const int j = j0 + 64 * u + lane;
            bool keep = false;
            if (((near >> u) & 1u) && j < nb && j != b) {
              double dx, dy;
              const double d2 = pair(j, dx, dy);
              const double rs = R + d.bconst[j] + xi + kNbrSkin;
              keep = d2 <= rs * rs;
              add_force(j, dx, dy, d2);
            }
            const uint64_t bal = __ballot(keep);
            if (rebuild && bal != 0) {
              const int slot = cnt + (int)__builtin_amdgcn_mbcnt_hi(
                                         (uint32_t)(bal >> 32),
                                         __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
              if (keep && slot < kNbrCap) my_list[slot] = j;
              cnt += __builtin_popcountll(bal);
            }
          }
        }
        if (rebuild && lane == 0) {
          d.nbr_cnt[b] = cnt <= kNbrCap ? cnt : -1;
          d.nbr_ref[2 * b] = X;
          d.nbr_ref[2 * b + 1] = Y;
        }
      }
      fx = wave_sum(fx);  // every lane now holds the totals
      fy = wave_sum(fy);
      // Eq. (29): the image across the nearer surface of each wall slab
      const double hw = d.wall_h_d;
      for (int wall = 0; wall < 2; ++wall) {
        if (!(d.wall_mask & (1u << wall))) continue;
        const double c = wall == 0 ? Y : X;
        const double n = wall == 0 ? dny : dnx;
        const double dd = (c - hw <= (n - hw) - c) ? 2.0 * (c - hw) : -2.0 * ((n - hw) - c);
        const double dist = fabs(dd);
        double kk = 0.0;
        if (dist > 2.0 * R + xi) {
          kk = 0.0;
        } else if (dist <= 2.0 * R) {
          kk = (2.0 * R - dist) * d.inv_eps_w1;
        } else {
          kk = (2.0 * R + xi - dist) * (2.0 * R + xi - dist) * d.inv_eps_w;
        }
        if (wall == 0)
          fy += kk * dd;
        else
          fx += kk * dd;
      }
      // Eq. (22): hydrodynamic force plus (rho_f / rho_s - 1) m g, rho_f = rho0
      const double gfac = (d.rho0_d / rho_s - 1.0) * m;
      fx += hfx + gfac * d.gx;
      fy += hfy + gfac * d.gy;
      if (fixed) {
        X += U;  // prescribed motion
        Y += V;
      } else {
        // Eqs. (22)-(24), dt = 1: Euler velocity and spin, trapezoidal position
        const double Un = U + fx / m, Vn = V + fy / m, Wn = W + T / I;
        X += 0.5 * (U + Un);
        Y += 0.5 * (V + Vn);
        U = Un;
        V = Vn;
        W = Wn;
      }
      X = X - dnx * floor(X / dnx);
      Y = Y - dny * floor(Y / dny);
      if (X >= dnx) X -= dnx;
      if (Y >= dny) Y -= dny;
      // moved more than half the skin since the lists were built: rebuild them next step
      {
        const double mx = min_image(X - d.nbr_ref[2 * b], dnx);
        const double my = min_image(Y - d.nbr_ref[2 * b + 1], dny);
        if (lane == 0 && !(mx * mx + my * my <= 0.25 * kNbrSkin * kNbrSkin)) d.nl_flag[p ^ 1] = 1;
      }
      // the same for the tile lists, unless this step rebins (from the new position)
      if (!rebin) {
        const double mx = min_image(X - d.bin_ref[2 * b], dnx);
        const double my = min_image(Y - d.bin_ref[2 * b + 1], dny);
        if (lane == 0 && !(mx * mx + my * my <= 0.25 * kBinSkin * kBinSkin)) d.rb_flag[p ^ 1] = 1;
      }
      if (b == 0 && lane == 0) d.lsel[p ^ 1] = lnew;  // the set the next step reads
      q = p ^ 1;
      if (lane == 0) {
        double *sn = d.bstate[q];
        sn[b] = X;
        sn[nb + b] = Y;
        sn[2 * nb + b] = U;
        sn[3 * nb + b] = V;
        sn[4 * nb + b] = W;
      }
    }
    // what the collide kernel of the step reads of this body
    if (lane == 0) {
      d.bsnap[q][b] = BodySnap{X, Y, (float)U, (float)V, (float)W, (float)R};
      *(float2 *)(d.bxy[q] + 2 * (int64_t)b) = make_float2((float)X, (float)Y);
    }
    // a blown-up body is flagged instead of binned (its tile indices would be garbage)
    if (!isfinite(X) || !isfinite(Y) || !isfinite(R)) {
      if (lane == 0) atomicOr(d.err, (int32_t)kErrUnstable);
      continue;
    }
    if (!rebin) continue;  // the lists of the last rebuild still cover this body
    if (lane == 0) {
      d.bin_ref[2 * b] = X;
      d.bin_ref[2 * b + 1] = Y;
    }
    // bin into list set lnew: every tile holding a node within R + support + skin
    const double H = R + d.support + kBinSkin + 1e-3;
    const AxisTiles ax = axis_tiles(X, H, d.nx, d.tx, d.tiles_x);
    const AxisTiles ay = axis_tiles(Y, H, d.ny, d.ty, d.tiles_y);
    const int na = (ax.a1 - ax.a0 + 1) + max(0, ax.b1 - ax.b0 + 1);
    const int nbb = (ay.a1 - ay.a0 + 1) + max(0, ay.b1 - ay.b0 + 1);
    const int na1 = ax.a1 - ax.a0 + 1, nb1 = ay.a1 - ay.a0 + 1;
    int32_t *hd = d.tile_head[lnew];
    int32_t *lst = d.tile_list[lnew];
    for (int e = lane; e < na * nbb; e += 64) {
      const int ia = e % na, ib = e / na;
      const int tx = ia < na1 ? ax.a0 + ia : ax.b0 + (ia - na1);
      const int ty = ib < nb1 ? ay.a0 + ib : ay.b0 + (ib - nb1);
      // which of the tile's four waves hold a node within H of the centre: per wave, the
      // distance from the centre to its rectangle of nodes is bounded from below on each
      // axis by the distance to the rectangle's middle less half its extent (the periodic
      // distance is 1-Lipschitz), so no reached wave is left out
      uint32_t mask = 0;
      const int npw = d.tx * d.ty / 4;  // nodes per wave: 64, or 128 with two per lane
      for (int w = 0; w < 4; ++w) {
        int xa, xb, ya, yb;
        if (d.tx >= npw) {
          ya = yb = ty * d.ty + (npw * w) / d.tx;
          xa = tx * d.tx + (npw * w) % d.tx;
          xb = xa + npw - 1;
        } else {
          ya = ty * d.ty + w * (npw / d.tx);
          yb = ya + npw / d.tx - 1;
          xa = tx * d.tx;
          xb = xa + d.tx - 1;
        }
        const double gx = fmax(fabs(min_image(0.5 * (xa + xb + 1) - X, dnx)) - 0.5 * (xb - xa), 0.0);
        const double gy = fmax(fabs(min_image(0.5 * (ya + yb + 1) - Y, dny)) - 0.5 * (yb - ya), 0.0);
        if (gx * gx + gy * gy <= H * H) mask |= 1u << w;
      }
      if (mask == 0) continue;  // the support misses every node of the tile
      const int tile = ty * d.tiles_x + tx;
      const int32_t entry = b | (int32_t)(mask << kListIndexBits);
      const int slot = atomicAdd(&hd[2 * (int64_t)tile], 1);
      if (slot == 0)
        hd[2 * (int64_t)tile + 1] = entry;  // the first entry sits in the tile's head
      else if (slot < d.list_cap)
        lst[(int64_t)tile * d.list_cap + slot] = entry;
      else
        atomicOr(d.err, (int32_t)kErrCapacity);
    }
  }
}

// Populations in and out (deviations f_i - w_i rho0, FP64, layout [9][ny][nx]) at the
// solve's current step d.step0, stored in that step's frame.
template <class ST>
__global__ void k_set_pops(const SolveDesc *__restrict__ desc, int p,
                           const double *__restrict__ fin) {
  const SolveDesc &d = *desc;
  const int64_t plane = (int64_t)d.nx * d.ny;     // the caller's dense planes
  const int64_t dplane = (int64_t)d.pitch * d.ny;  // the stored planes
  const float2 V = frame_velocity<ST>(d.step0);
  typename ST::T *dst = (typename ST::T *)d.pop[p];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < kQ * plane;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / plane);
    const int64_t n = e - i * plane;
    const int y = (int)(n / d.nx), x = (int)(n - (int64_t)y * d.nx);
    int xs = x - CX[i], ys = y - CY[i];
    if (xs < 0) xs += d.nx;
    if (xs >= d.nx) xs -= d.nx;
    if (ys < 0) ys += d.ny;
    if (ys >= d.ny) ys -= d.ny;
    ST::st(dst, i * dplane + (int64_t)ys * d.pitch + xs,
           (float)(36.0 * fin[e] - frame_offset(i, V)), d.store_scale);
  }
}

template <class ST>
__global__ void k_get_pops(const SolveDesc *__restrict__ desc, int p, double *__restrict__ fout) {
  const SolveDesc &d = *desc;
  const int64_t plane = (int64_t)d.nx * d.ny;     // the caller's dense planes
  const int64_t dplane = (int64_t)d.pitch * d.ny;  // the stored planes
  const float2 V = frame_velocity<ST>(d.step0);
  const typename ST::T *src = (const typename ST::T *)d.pop[p];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < kQ * plane;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / plane);
    const int64_t n = e - i * plane;
    const int y = (int)(n / d.nx), x = (int)(n - (int64_t)y * d.nx);
    int xs = x - CX[i], ys = y - CY[i];
    if (xs < 0) xs += d.nx;
    if (xs >= d.nx) xs -= d.nx;
    if (ys < 0) ys += d.ny;
    if (ys >= d.ny) ys -= d.ny;
    const double g = (double)ST::ld(src, i * dplane + (int64_t)ys * d.pitch + xs, d.store_inv);
    fout[e] = (g + frame_offset(i, V)) / 36.0;
  }
}

// The fluid at rest with rho = rho0 (every deviation zero) at step d.step0, in both
// population buffers.
template <class ST>
__global__ void k_rest_pops(const SolveDesc *__restrict__ desc) {
  const SolveDesc &d = *desc;
  const int64_t plane = (int64_t)d.pitch * d.ny;  // padding columns included
  const float2 V = frame_velocity<ST>(d.step0);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < kQ * plane;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / plane);
    const float v = (float)(-frame_offset(i, V));  // exact
    ST::st((typename ST::T *)d.pop[0], e, v, d.store_scale);
    ST::st((typename ST::T *)d.pop[1], e, v, d.store_scale);
  }
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

__global__ void k_fill_f64(double *p, int64_t n, double v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

__global__ void k_fill_bytes(uint32_t *p, int64_t nwords) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nwords;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = 0u;
}

int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

}  // namespace

// ---------------------------------------------------------------------------------------
// launch wrappers

#define DILBM_SHAPES(X) X(0, 64, 4) X(1, 128, 2) X(2, 256, 1) X(3, 32, 8) X(4, 16, 16)

using CollideKernel = void (*)(const SolveDesc *, const int32_t *, const BatchHeader *, int);

// The k_collide instance for a tile shape, storage format, addressing mode and whether
// any member has open ends in x.
static CollideKernel collide_kernel(int shape, int storage, int addr, bool open) {
#define DILBM_PICK2(ST, tx, ty, A)                             \
  return open ? &k_collide<ST, tx, ty, A, true> : &k_collide<ST, tx, ty, A, false>;
#define DILBM_PICK(ST, tx, ty)                           \
  if (addr == kAddrBuf) { DILBM_PICK2(ST, tx, ty, kAddrBuf) } \
  if (addr == kAddrG32) { DILBM_PICK2(ST, tx, ty, kAddrG32) } \
  DILBM_PICK2(ST, tx, ty, kAddrWide)
#define DILBM_CASE(id, tx, ty)     \
  case id:                         \
    if (storage == 1) {            \
      DILBM_PICK(StoreF16, tx, ty) \
    } else {                       \
      DILBM_PICK(StoreF32, tx, ty) \
    }
  switch (shape) {
    DILBM_SHAPES(DILBM_CASE)
    case 5:  // 512 x 1, two nodes per lane: FP16 populations only
      if (storage == 1) {
        DILBM_PICK(StoreF16, 512, 1)
      }
      return nullptr;
    default:
      return nullptr;
  }
#undef DILBM_CASE
#undef DILBM_PICK
#undef DILBM_PICK2
}

hipError_t launch_collide(int shape, int storage, int addr, bool open, int grid,
                          hipStream_t stream, const SolveDesc *descs, const int32_t *tile_solve,
                          const BatchHeader *hdr, int k) {
  const CollideKernel f = collide_kernel(shape, storage, addr, open);
  if (!f) return hipErrorInvalidValue;
  hipLaunchKernelGGL(f, dim3(grid), dim3(kBlockThreads), 0, stream, descs, tile_solve, hdr, k);
  return hipGetLastError();
}

int collide_blocks_per_cu(int shape, int storage, int addr, bool open) {
  const CollideKernel f = collide_kernel(shape, storage, addr, open);
  int n = 0;
  if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(f),
                                                         kBlockThreads, 0) != hipSuccess)
    return 0;
  return n;
}

hipError_t launch_fields(int shape, int storage, int64_t ntiles, hipStream_t stream,
                         const SolveDesc *desc, int p, Region region, double *rho, double *ux,
                         double *uy) {
  const int grid = grid_for(ntiles, 1);
#define DILBM_CASE(id, tx, ty)                                                               \
  case id:                                                                                   \
    if (storage == 1)                                                                        \
      hipLaunchKernelGGL((k_fields<StoreF16, tx, ty>), dim3(grid), dim3(kBlockThreads), 0,   \
                         stream, desc, p, region, rho, ux, uy);                              \
    else                                                                                     \
      hipLaunchKernelGGL((k_fields<StoreF32, tx, ty>), dim3(grid), dim3(kBlockThreads), 0,   \
                         stream, desc, p, region, rho, ux, uy);                              \
    break;
  switch (shape) {
    DILBM_SHAPES(DILBM_CASE)
    case 5:
      if (storage != 1) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_fields<StoreF16, 512, 1>), dim3(grid), dim3(kBlockThreads), 0,
                         stream, desc, p, region, rho, ux, uy);
      break;
    default:
      return hipErrorInvalidValue;
  }
#undef DILBM_CASE
  return hipGetLastError();
}

hipError_t launch_bodies(bool bin_only, int grid, hipStream_t stream, const SolveDesc *descs,
                         const int32_t *body_solve, const BatchHeader *hdr, int k) {
  if (bin_only)
    hipLaunchKernelGGL((k_bodies<true>), dim3(grid), dim3(kBlockThreads), 0, stream, descs,
                       body_solve, hdr, k);
  else
    hipLaunchKernelGGL((k_bodies<false>), dim3(grid), dim3(kBlockThreads), 0, stream, descs,
                       body_solve, hdr, k);
  return hipGetLastError();
}

hipError_t launch_set_pops(int storage, int64_t count, hipStream_t stream, const SolveDesc *desc,
                           int p, const double *fin) {
  const int grid = grid_for(count, 256);
  if (storage == 1)
    hipLaunchKernelGGL((k_set_pops<StoreF16>), dim3(grid), dim3(256), 0, stream, desc, p, fin);
  else
    hipLaunchKernelGGL((k_set_pops<StoreF32>), dim3(grid), dim3(256), 0, stream, desc, p, fin);
  return hipGetLastError();
}

hipError_t launch_get_pops(int storage, int64_t count, hipStream_t stream, const SolveDesc *desc,
                           int p, double *fout) {
  const int grid = grid_for(count, 256);
  if (storage == 1)
    hipLaunchKernelGGL((k_get_pops<StoreF16>), dim3(grid), dim3(256), 0, stream, desc, p, fout);
  else
    hipLaunchKernelGGL((k_get_pops<StoreF32>), dim3(grid), dim3(256), 0, stream, desc, p, fout);
  return hipGetLastError();
}

hipError_t launch_rest_pops(int storage, int64_t count, hipStream_t stream,
                            const SolveDesc *desc) {
  const int grid = grid_for(count, 256);
  if (storage == 1)
    hipLaunchKernelGGL((k_rest_pops<StoreF16>), dim3(grid), dim3(256), 0, stream, desc);
  else
    hipLaunchKernelGGL((k_rest_pops<StoreF32>), dim3(grid), dim3(256), 0, stream, desc);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, stream, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n, 256)), dim3(256), 0, stream, p, n, v);
  return hipGetLastError();
}

hipError_t launch_zero_bytes(void *p, int64_t bytes, hipStream_t stream) {
  const int64_t words = bytes / 4;
  if (words <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_bytes, dim3(grid_for(words, 256)), dim3(256), 0, stream,
                     (uint32_t *)p, words);
  return hipGetLastError();
}

}  // namespace dilbm
