// kernels3d.hip -- gfx950 kernels of the three-dimensional DI-LBM step (D3Q19 or D3Q27,
// spheres).
//
// The step is the one of kernels.hip carried to three dimensions (Section 2.3 of the
// paper with Eqs. (13)-(19), (22)-(24), (28)-(29)); see dilbm3d.h for the readings.
//
//   k3_collide  one launch per step over all tiles (whole rows of 256 nodes, or 64 x 4 x 1
//               nodes for short rows; 256 threads, one node per lane): pull streaming of
//               the 19 or 27 populations, moments, the solid field of the listed spheres
//               and walls, Eq. (17), the Eq. (13) collision (or, on the planes of open
//               ends, non-equilibrium extrapolation), write-back, and the per-sphere FP64
//               force and torque sums.
//   k3_bodies   one block per sphere: Eq. (28) pair forces, Eq. (29) wall images, the
//               Eqs. (22)-(24) update in FP64 and binning into the next step's tile lists
//               (each entry carries which of the tile's four waves the support reaches).
//   k3_fields   rho and the corrected velocity of Eq. (17) (output only).
//
// Populations are kept as g_i = S (f_i - w_i rho0) in FP32 (or FP16 times 2^k), with S
// making the weights exact integers K_i = S w_i: D3Q19 S = 36 (weights 1/3, 1/18, 1/36 ->
// K = 12, 2, 1), D3Q27 S = 216 (8/27, 2/27, 1/54, 1/216 -> K = 64, 16, 4, 1).  Every
// constant on the mass and momentum path is then exact in binary and what remains is
// unbiased round-to-nearest.  Kernels are instantiated per lattice L (19 or 27
// directions), population storage H (FP16) and, for the collide, open ends in x.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "device_common.h"
#include "dilbm3d_internal.h"
#include "dilbm_internal.h"
#include "kernels3d.h"

namespace dilbm {

namespace {

// The population scale S and the integer weights K_i = S w_i of lattice L.
template <int L>
struct Lat3;
template <>
struct Lat3<19> {
  static constexpr float S = 36.0f;
  static constexpr float K[4] = {12.0f, 2.0f, 1.0f, 0.0f};  // by |c|^2
};
template <>
struct Lat3<27> {
  static constexpr float S = 216.0f;
  static constexpr float K[4] = {64.0f, 16.0f, 4.0f, 1.0f};
};
template <int L>
__host__ __device__ constexpr float kw3(int i) {
  return Lat3<L>::K[(C3X[i] != 0) + (C3Y[i] != 0) + (C3Z[i] != 0)];
}

// x / S correctly rounded: the reciprocal product corrected by one FMA residual step
template <int L>
__device__ __forceinline__ float divS(float x) {
  constexpr float S = Lat3<L>::S, inv = 1.0f / S;
  const float q = x * inv;
  return fmaf(fmaf(-S, q, x), inv, q);
}

__device__ __forceinline__ SphereSnap load_snap3(const DILBM_CONST SphereSnap *q) {
  SphereSnap s;
  s.x = q->x;
  s.y = q->y;
  s.z = q->z;
  s.u = q->u;
  s.v = q->v;
  s.w = q->w;
  s.ox = q->ox;
  s.oy = q->oy;
  s.oz = q->oz;
  s.r = q->r;
  s.pad[0] = s.pad[1] = 0.0f;
  return s;
}

// Reference frame of the stored populations, as in the two-dimensional kernels: after
// step t what is stored is g_i - 3 K_i c_i.V_t with V_t pseudo-random, so the rounding of
// a steady per-step increment onto the FP32 grid does not make the same error every step
// (without it a uniformly driven 64 x 40 x 32 case drifted to 1.8e-5 of the velocity in
// 1000 steps).  Each component of V_t is a multiple of 2^-36 with B significant bits,
// |V_t| < 2^(B-37): B = 18 on D3Q19, 15 on D3Q27.  Every frame constant 3 K_i c_i.V_t is
// then a multiple of 2^-36, and so is every partial sum of them the moments take; those
// sums are bounded by 3 V_max sum_i K_i |c_i|_1 = 3 V_max S (108 V_max < 2^-12.2 on
// D3Q19, 648 V_max < 2^-12.6 on D3Q27), so they hold at most 24 significant bits and are
// exact in FP32, as are the per-step changes of the constants and S V_t: a fluid at rest
// stays exactly at rest.  (With 20 bits the D3Q27 moment sums round: its S is six times
// larger.)  Against the FP32 grid of the populations the offsets stay far above one ulp,
// which is all the decorrelation needs.
template <int L>
__device__ __forceinline__ float3 ref_velocity3(int64_t t) {
  constexpr int B = L == 27 ? 15 : 18;
  constexpr uint32_t mask = (1u << B) - 1u;
  constexpr int half = 1 << (B - 1);
  const uint64_t z = splitmix64((uint64_t)t);
  constexpr float q = 1.0f / 68719476736.0f;  // 2^-36
  return make_float3((float)((int)(z & mask) - half) * q,
                     (float)((int)((z >> 20) & mask) - half) * q,
                     (float)((int)((z >> 40) & mask) - half) * q);
}

// 3 K_i c_i.V: the frame offset of direction i
template <int L>
__device__ __forceinline__ double frame_offset3(int i, float3 V) {
  return 3.0 * (double)kw3<L>(i) *
         ((double)C3X[i] * V.x + (double)C3Y[i] * V.y + (double)C3Z[i] * V.z);
}

__device__ __forceinline__ int wrapi(int k, int n) { return k < 0 ? k + n : (k >= n ? k - n : k); }

enum Mode3 { kStep3 = 0, kFields3 = 1 };

#ifndef DILBM3D27_STASH
#define DILBM3D27_STASH 19
#endif
// populations held in LDS during the sphere loop
template <int L>
constexpr int kStash3 = L == 27 ? DILBM3D27_STASH : L;

// One tile of TX x (256 / TX) x 1 nodes (TX = 64 or 256: a wave is part of one row).
// MODE kStep3: the full step; kFields3: rho and u of the current state.
// OPEN: the instance for open ends in x (d.xbc).  A node of the inlet plane x = 0 or the
// outlet plane x = nx - 1 takes non-equilibrium extrapolation (Guo, Zheng & Shi 2002; the
// treatment the paper gives its physical boundaries, Section 3): its lane pulls the
// populations of its neighbour on the plane x = 1 or nx - 2 instead of its own (the
// neighbour's sources x - c_i stay inside [0, nx), and the lines are those its wave reads
// anyway), so the moments below are the neighbour's, u* carries half the body force as in
// the neighbour's collision, and the lane takes no solid field.  Its output is
//   g_i* = geq_i(boundary) + (1 - 1/tau) (g_i - geq_i(neighbour))
//        = g_i + omega (geq_i(neighbour) - g_i) + [geq_i(boundary) - geq_i(neighbour)],
// the regular update with the bracket in place of the forcing term (the forcing term's
// inputs are set to produce it); the boundary state is prescribed or the neighbour's.  The
// frame constants cancel in the bracket's difference and in the non-equilibrium part.
template <int MODE, int TX, int L, bool H, bool OPEN>
__device__ __forceinline__ void tile3(const Desc3 &d, const int64_t lt, const int p,
                                      const int64_t t, float (*red)[6][64], float *stash,
                                      double *__restrict__ out_rho, double *__restrict__ out_ux,
                                      double *__restrict__ out_uy,
                                      double *__restrict__ out_uz) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // the sizes pass through an empty asm: what is derived from them (the divisions'
  // reciprocals, float copies for the wall distances) is then formed per tile in scalar
  // or short-lived registers, not held in vector registers across the tile loop
  int nx = d.nx, ny = d.ny, nz = d.nz, ntx = d.tiles_x, nty = d.tiles_y, pitch = d.pitch;
  asm volatile("" : "+s"(nx), "+s"(ny), "+s"(nz), "+s"(ntx), "+s"(nty), "+s"(pitch));
  const int64_t trow = lt / ntx;
  const int txi = (int)(lt - trow * ntx);
  const int z = (int)(trow / nty);
  const int tyi = (int)(trow - (int64_t)z * nty);
  constexpr int TY = 256 / TX;
  const int x0 = txi * TX, y0 = tyi * TY;
  const int x = x0 + tid % TX;
  const int y = __builtin_amdgcn_readfirstlane(y0 + tid / TX);  // a wave is part of one row
  const bool valid = x < nx && y < ny;
  const int xc = min(x, nx - 1), yc = min(y, ny - 1);
  // a node of the inlet or outlet plane (see OPEN above)
  const bool bnd = OPEN && d.xbc && valid && (x == 0 || x == nx - 1);
  const bool own = valid && !bnd;  // a node whose solid field this tile computes

  // ---- pull streaming: f_i(x, t) = f_i*(x - c_i, t - 1) ------------------------------
  // one buffer resource per population buffer; the row of every direction is
  // wave-uniform (scalar offset), the column is one of three per-lane offsets
  // H: FP16 populations, g_i 2^k (raw: the moments are scaled back, the update is applied
  // at the stored scale)
  constexpr uint32_t es = H ? 2u : 4u;
  const float inv = d.store_inv, sc = d.store_scale;
  const uint32_t plane = (uint32_t)pitch * (uint32_t)ny * (uint32_t)nz;
  const uint32_t pb = plane * es;
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void *)d.pop[p], (short)0, (int)(L * pb), kBufferFlags);
  const uint32_t vx0 = (uint32_t)xc * es;  // the node's own column (stores)
  // the column whose populations the lane pulls: its own, or a boundary node's neighbour
  const int xl = OPEN && bnd ? (x == 0 ? 1 : nx - 2) : xc;
  const uint32_t vxl = (uint32_t)xl * es;
  const uint32_t vxm = (uint32_t)(xl == 0 ? nx - 1 : xl - 1) * es;  // source x - 1
  const uint32_t vxp = (uint32_t)(xl + 1 == nx ? 0 : xl + 1) * es;  // source x + 1
  uint32_t row[3][3];  // row[dz + 1][dy + 1]: byte offset of row (y + dy, z + dz)
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
      row[dz + 1][dy + 1] = __builtin_amdgcn_readfirstlane(
          ((uint32_t)wrapi(z + dz, nz) * (uint32_t)ny + (uint32_t)wrapi(yc + dy, ny)) *
          (uint32_t)pitch * es);
  float g[L];
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const uint32_t v = C3X[i] == 0 ? vxl : (C3X[i] > 0 ? vxm : vxp);
    const uint32_t s = (uint32_t)i * pb + row[1 - C3Z[i]][1 - C3Y[i]];
    if (H)
      g[i] = (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(rs, v, s, 0));
    else
      g[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, v, s, 0));
  }

  // the tile's head (sphere count and first list entry, one scalar load) and that
  // sphere's snapshot, in flight with the populations; the first entry is clamped into
  // range for the snapshot load and used only when the count lists it
  const int ls = *(const DILBM_CONST int32_t *)(d.lsel + p);  // the list set of this step
  const uint64_t hv = *(const DILBM_CONST uint64_t *)(d.tile_head[ls] + 2 * lt);
  const int32_t raw0 = (int32_t)(hv >> 32);
  const int nb = min((int32_t)(uint32_t)hv, d.list_cap);
  const int nbs = d.nbodies;
  const DILBM_CONST int32_t *list =
      (const DILBM_CONST int32_t *)(d.tile_list[ls] + lt * d.list_cap);
  const DILBM_CONST SphereSnap *snap = (const DILBM_CONST SphereSnap *)d.bsnap[p];
  SphereSnap s0{};
  if (nbs > 0) s0 = load_snap3(snap + min(raw0 & kListIndexMask, nbs - 1));
  if (MODE == kStep3) {
    // the sphere step after this one rebins into the other set: it starts empty
    if (tid == 0 && *(const DILBM_CONST int32_t *)(d.rb_flag + p) != 0)
      d.tile_head[ls ^ 1][2 * lt] = 0;
    if (lt == 0) {
      double *a = d.acc[p ^ 1];
      const int na = (int)acc_words(nbs, 6);
      for (int i = tid; i < na; i += 256) a[i] = 0.0;
      if (tid == 0) d.rb_flag[p ^ 1] = 0;  // read by the last sphere step, raised by the next
    }
  }

  // ---- storage frame: step t's populations are stored relative to V_t; the step moves
  // them to the frame of step t + 1 first (exact constants, one rounding per population),
  // so that the rounding of each output sees an offset that changes from step to step.
  // The step count passes through an empty asm: the frame constants are then computed
  // here, next to their use, not hoisted out of the tile loop into vector registers held
  // across the whole tile.
  int64_t tc = t;
  asm volatile("" : "+s"(tc));
  float3 Vf = H ? make_float3(0.0f, 0.0f, 0.0f) : ref_velocity3<L>(tc);  // FP16: no frame
  if (MODE == kStep3 && !H) {
    const float3 Vt = Vf;
    Vf = ref_velocity3<L>(tc + 1);
    const float dvx = Vf.x - Vt.x, dvy = Vf.y - Vt.y, dvz = Vf.z - Vt.z;
#pragma unroll
    for (int i = 1; i < L; ++i)
      g[i] -= (3.0f * kw3<L>(i)) *
              ((float)C3X[i] * dvx + (float)C3Y[i] * dvy + (float)C3Z[i] * dvz);
  }
  constexpr float S = Lat3<L>::S, invS = 1.0f / S, halfS = 0.5f * S;
  const float V36x = S * Vf.x, V36y = S * Vf.y, V36z = S * Vf.z;  // S V, exact

  // ---- moments, Eqs. (5) and (16), in g units (D = S drho, J = S j - S V; the frame
  // carries no mass) ------------------------------------------------------------------
  float D = 0.f, Jx = 0.f, Jy = 0.f, Jz = 0.f;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    D += g[i];
    if (C3X[i]) Jx += C3X[i] > 0 ? g[i] : -g[i];
    if (C3Y[i]) Jy += C3Y[i] > 0 ? g[i] : -g[i];
    if (C3Z[i]) Jz += C3Z[i] > 0 ? g[i] : -g[i];
  }
  if (H) {  // back to g units (exact: a power of two)
    D *= inv;
    Jx *= inv;
    Jy *= inv;
    Jz *= inv;
  }
  const float R = S * d.rho0 + D;  // S rho
  const float rho = R * invS;
  const float drho = D * invS;
  float Rinv = __builtin_amdgcn_rcpf(R);
  Rinv = fmaf(fmaf(-R, Rinv, 1.0f), Rinv, Rinv);
  // S rho u* = S (j + G/2), back in the fixed frame
  const float Jgx = Jx + (V36x + halfS * d.Gx), Jgy = Jy + (V36y + halfS * d.Gy);
  const float Jgz = Jz + (V36z + halfS * d.Gz);
  const float usx = Jgx * Rinv, usy = Jgy * Rinv, usz = Jgz * Rinv;

  // ---- diffuse solid field, Eq. (14), and its sums over spheres and walls ---------------
  float Phi = 0.f, Ax = 0.f, Ay = 0.f, Az = 0.f;
  float Mxx = 0.f, Myy = 0.f, Mzz = 0.f, Mxy = 0.f, Mxz = 0.f, Myz = 0.f;
  const float lcut = d.lcut, phik = d.phi_k, kap = d.kappa;
  // walls: does this tile reach into the support of a slab? (axis order x, y, z)
  const bool wx = (d.wall_mask & 2u) && (x0 < d.wall_lo[0] || x0 + TX > d.wall_hi[0]);
  const bool wy = (d.wall_mask & 1u) && (y0 < d.wall_lo[1] || y0 + TY > d.wall_hi[1]);
  const bool wz = (d.wall_mask & 4u) && (z < d.wall_lo[2] || z + 1 > d.wall_hi[2]);
  const bool any_solid = nb > 0 || wx || wy || wz;
  if (any_solid) {
    // the populations wait in LDS while the spheres are summed, so that their registers
    // serve the sphere loop (each lane its own slots: no barrier); the empty asm with a
    // memory clobber keeps the compiler from forwarding the stored values past the loop
    if (MODE == kStep3) {
#pragma unroll
      for (int i = 0; i < kStash3<L>; ++i) stash[i * 256 + tid] = g[i];
      asm volatile("" ::: "memory");
    }
    float lw[3] = {-1e30f, -1e30f, -1e30f};
    if (wx) {
      float c = (float)xc + 0.5f;
      if (c >= 0.5f * (float)nx) c -= (float)nx;
      lw[0] = d.wall_h - fabsf(c);
    }
    if (wy) {
      float c = (float)yc + 0.5f;
      if (c >= 0.5f * (float)ny) c -= (float)ny;
      lw[1] = d.wall_h - fabsf(c);
    }
    if (wz) {
      float c = (float)z + 0.5f;
      if (c >= 0.5f * (float)nz) c -= (float)nz;
      lw[2] = d.wall_h - fabsf(c);
    }
    const double xn = (double)xc + 0.5, yn = (double)yc + 0.5, zn = (double)z + 0.5;
    const double dnx = nx, dny = ny, dnz = nz;
    // listed sphere j: its index (checked: a bad entry is flagged and skipped), whether its
    // support reaches this wave's nodes (the entry's wave mask), and its snapshot
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    auto body = [&](const int j, int &e, SphereSnap &sj) -> bool {
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
        sj = load_snap3(snap + e);
      return true;
    };
    // One pass over the listed spheres with unit weights.  The weights of several
    // overlapping supports are w_b = phi_b min(1, 1/S), S = sum of phi over the spheres
    // and walls; every sum below is linear in the weights, so the node-local sums are
    // scaled once afterwards, and the force sums, already added, are corrected by a
    // second pass only in waves where some node has S > 1.
    double *__restrict__ acc = d.acc[p];
    float S = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (own && lw[a] >= lcut) S += phi_of(lw[a], phik);
    // the wave's six sums of one sphere's force and torque, by a transpose through its own
    // LDS rows: each lane stores its six values, lanes 8k..8k+7 add the 64 values of
    // component k (eight each, in FP64), three DPP steps combine the eight, and one atomic
    // instruction with six active lanes adds the totals
    auto reduce6 = [&](const int e, const float fx, const float fy, const float fz,
                       const float rx, const float ry, const float rz) {
      float(*r)[64] = red[tid >> 6];
      r[0][lane] = fx;
      r[1][lane] = fy;
      r[2][lane] = fz;
      r[3][lane] = ry * fz - rz * fy;
      r[4][lane] = rz * fx - rx * fz;
      r[5][lane] = rx * fy - ry * fx;
      __builtin_amdgcn_wave_barrier();
      double part = 0.0;
      if (lane < 48) {
        const float *q = &r[lane >> 3][(lane & 7) * 8];
#pragma unroll
        for (int k = 0; k < 8; ++k) part += (double)q[k];
      }
      __builtin_amdgcn_wave_barrier();
      part += dpp_f64<0xB1>(part);   // quad_perm [1, 0, 3, 2]
      part += dpp_f64<0x4E>(part);   // quad_perm [2, 3, 0, 1]
      part += dpp_f64<0x141>(part);  // row_half_mirror: the eight lanes of a group
      if (lane < 48 && (lane & 7) == 0) unsafeAtomicAdd(acc + 6 * e + (lane >> 3), part);
    };
    for (int j = 0; j < nb; ++j) {
      int e;
      SphereSnap sj;
      if (!body(j, e, sj)) continue;
      const float rx = (float)min_image(xn - sj.x, dnx);
      const float ry = (float)min_image(yn - sj.y, dny);
      const float rz = (float)min_image(zn - sj.z, dnz);
      const float l = sj.r - __builtin_amdgcn_sqrtf(rx * rx + ry * ry + rz * rz);
      float fx = 0.f, fy = 0.f, fz = 0.f;
      if (own && l >= lcut) {
        const float w = phi_of(l, phik);
        S += w;
        // rigid-body velocity of the solid at the node: U + omega x r
        const float vx = sj.u + (sj.oy * rz - sj.oz * ry);
        const float vy = sj.v + (sj.oz * rx - sj.ox * rz);
        const float vz = sj.w + (sj.ox * ry - sj.oy * rx);
        Phi += w;
        Ax += w * vx;
        Ay += w * vy;
        Az += w * vz;
        Mxx += w * vx * vx;
        Myy += w * vy * vy;
        Mzz += w * vz * vz;
        Mxy += w * vx * vy;
        Mxz += w * vx * vz;
        Myz += w * vy * vz;
        // force on the sphere: -w rho (u_s - u*) (times the Eq. (18) scale)
        const float k = -kap * w * rho;
        fx = k * (vx - usx);
        fy = k * (vy - usy);
        fz = k * (vz - usz);
      }
      if (MODE == kStep3 && __ballot(fx != 0.f || fy != 0.f || fz != 0.f) != 0)
        reduce6(e, fx, fy, fz, rx, ry, rz);
    }
    const float scale = S > 1.0f ? 1.0f / S : 1.0f;
    Phi *= scale;
    Ax *= scale;
    Ay *= scale;
    Az *= scale;
    Mxx *= scale;
    Myy *= scale;
    Mzz *= scale;
    Mxy *= scale;
    Mxz *= scale;
    Myz *= scale;
    // where S > 1 the forces above took phi_b for w_b: add (scale - 1) times them
    if (MODE == kStep3 && __ballot(own && S > 1.0f) != 0) {
      const float c = scale - 1.0f;  // 0 where S <= 1
      for (int j = 0; j < nb; ++j) {
        int e;
        SphereSnap sj;
        if (!body(j, e, sj)) continue;
        const float rx = (float)min_image(xn - sj.x, dnx);
        const float ry = (float)min_image(yn - sj.y, dny);
        const float rz = (float)min_image(zn - sj.z, dnz);
        const float l = sj.r - __builtin_amdgcn_sqrtf(rx * rx + ry * ry + rz * rz);
        float fx = 0.f, fy = 0.f, fz = 0.f;
        if (own && c != 0.0f && l >= lcut) {
          const float w = phi_of(l, phik);
          const float vx = sj.u + (sj.oy * rz - sj.oz * ry);
          const float vy = sj.v + (sj.oz * rx - sj.ox * rz);
          const float vz = sj.w + (sj.ox * ry - sj.oy * rx);
          const float k = -kap * w * rho;
          fx = c * (k * (vx - usx));
          fy = c * (k * (vy - usy));
          fz = c * (k * (vz - usz));
        }
        if (__ballot(fx != 0.f || fy != 0.f || fz != 0.f) != 0) reduce6(e, fx, fy, fz, rx, ry, rz);
      }
    }
    // wall slabs: solid velocity 0; their force goes to the last accumulator slot
    if (wx || wy || wz) {
      float fx = 0.f, fy = 0.f, fz = 0.f;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (own && lw[a] >= lcut) {
          const float w = scale * phi_of(lw[a], phik);
          Phi += w;
          const float k = kap * w * rho;
          fx += k * usx;
          fy += k * usy;
          fz += k * usz;
        }
      }
      if (MODE == kStep3 && __ballot(fx != 0.f || fy != 0.f || fz != 0.f) != 0) {
        const double sx = wave_sum((double)fx), sy = wave_sum((double)fy);
        const double sz = wave_sum((double)fz);
        if (lane == 0) {
          double *a = acc + wall_base(6 * nbs) + (blockIdx.x % kWallSlots) * kWallSlotWords;
          unsafeAtomicAdd(a + 0, sx);
          unsafeAtomicAdd(a + 1, sy);
          unsafeAtomicAdd(a + 2, sz);
        }
      }
    }
    if (MODE == kStep3) {
      asm volatile("" ::: "memory");
#pragma unroll
      for (int i = 0; i < kStash3<L>; ++i) g[i] = stash[i * 256 + tid];
    }
  }

  // ---- corrected velocity, Eq. (17): S rho u = S rho u* + (S/2) P, P = rho (A - Phi u*) --
  const float Px = rho * (Ax - Phi * usx), Py = rho * (Ay - Phi * usy);
  const float Pz = rho * (Az - Phi * usz);
  const float Mx = fmaf(halfS, Px, Jgx), My = fmaf(halfS, Py, Jgy), Mz = fmaf(halfS, Pz, Jgz);
  const float ux = Mx * Rinv, uy = My * Rinv, uz = Mz * Rinv;

  // ---- open ends: the boundary state of an inlet or outlet node (the moments above are
  // its neighbour's): prescribed, or the neighbour's ----------------------------------
  float drho_b = drho, ubx = ux, uby = uy, ubz = uz;
  if (OPEN && bnd) {
    if (x == 0) {
      if (d.inlet_kind == 0) {  // velocity inlet, rho from the neighbour
        float sh = 1.0f;
        if (d.inlet_profile >= 1) {
          const float sy = ((float)yc + 0.5f - d.prof_y0) * d.prof_inv_hy;
          sh = (sy > 0.0f && sy < 1.0f) ? 4.0f * sy * (1.0f - sy) : 0.0f;
          if (d.inlet_profile == 2) {
            const float sz = ((float)z + 0.5f - d.prof_z0) * d.prof_inv_hz;
            sh *= (sz > 0.0f && sz < 1.0f) ? 4.0f * sz * (1.0f - sz) : 0.0f;
          }
        }
        ubx = sh * d.u_in[0];
        uby = sh * d.u_in[1];
        ubz = sh * d.u_in[2];
      } else {
        drho_b = d.drho_in;
      }
    } else if (d.outlet_kind == 0) {
      drho_b = d.drho_out;
    }
  }
  const float rho_b = d.rho0 + drho_b;

  if (MODE == kFields3) {
    if (valid) {
      const bool b = OPEN && bnd;
      const int64_t o = ((int64_t)z * ny + y) * nx + x;
      out_rho[o] = (double)(b ? rho_b : rho);
      out_ux[o] = (double)(b ? ubx : ux);
      out_uy[o] = (double)(b ? uby : uy);
      out_uz[o] = (double)(b ? ubz : uz);
    }
    return;
  }

  // ---- collision, Eq. (13), in g units ------------------------------------------------
  // g_i* = g_i + omega (geq_i - g_i) + khalf K_i S_i with
  //   geq_i = K_i [drho + 3 c.(rho u - V) + rho (4.5 (c.u)^2 - 1.5 u.u)]   (frame V),
  //   S_i   = 3 (c - u).G + 9 (c.u)(c.G)            (uniform body force)
  //         + 3 c.P + 4.5 c.Q.c - 1.5 tr Q           (spheres and walls, Eq. (15) summed)
  // taken per pair of opposite directions, which share the even part.
  // rho u - V, from S rho u - S V directly (exact frame constant)
  const float mx = divS<L>(Mx - V36x), my = divS<L>(My - V36y), mz = divS<L>(Mz - V36z);
  const float uu = ux * ux + uy * uy + uz * uz;
  const float Gx = d.Gx, Gy = d.Gy, Gz = d.Gz;
  const float uG = ux * Gx + uy * Gy + uz * Gz;
  float Qxx = 0.f, Qyy = 0.f, Qzz = 0.f, Qxy = 0.f, Qxz = 0.f, Qyz = 0.f, trQ = 0.f;
  if (any_solid) {
    Qxx = rho * (Mxx - Phi * usx * usx);
    Qyy = rho * (Myy - Phi * usy * usy);
    Qzz = rho * (Mzz - Phi * usz * usz);
    Qxy = rho * (Mxy - Phi * usx * usy);
    Qxz = rho * (Mxz - Phi * usx * usz);
    Qyz = rho * (Myz - Phi * usy * usz);
    trQ = Qxx + Qyy + Qzz;
  }
  const float om = d.omega, kh = d.khalf;
  // the forcing term's inputs: P, Q and the body force; for an inlet or outlet node (OPEN
  // above) they are set so that khalf K_i S_i is the bracket geq_i(boundary) -
  // geq_i(neighbour): P = (m_b - m) / khalf, Q = (rho_b u_b u_b - rho u u) / khalf, the
  // scalar (drho_b - drho) / khalf and no body force (m = rho u - V, m_b = rho_b u_b - V)
  float sPx = Px, sPy = Py, sPz = Pz, sg = -3.0f * uG, gk = 1.0f;
  if (OPEN && bnd) {
    const float ik = d.inv_khalf;
    sPx = (rho_b * ubx - Vf.x - mx) * ik;
    sPy = (rho_b * uby - Vf.y - my) * ik;
    sPz = (rho_b * ubz - Vf.z - mz) * ik;
    Qxx = (rho_b * ubx * ubx - rho * ux * ux) * ik;
    Qyy = (rho_b * uby * uby - rho * uy * uy) * ik;
    Qzz = (rho_b * ubz * ubz - rho * uz * uz) * ik;
    Qxy = (rho_b * ubx * uby - rho * ux * uy) * ik;
    Qxz = (rho_b * ubx * ubz - rho * ux * uz) * ik;
    Qyz = (rho_b * uby * ubz - rho * uy * uz) * ik;
    trQ = Qxx + Qyy + Qzz;
    sg = (drho_b - drho) * ik;
    gk = 0.0f;
  }
  const float base = drho - 1.5f * rho * uu;            // even part shared by all i
  const float sbase = sg - 1.5f * trQ;                  // even part of S shared by all i
  float out[L];
  // each output is g + (small update), applied once at the scale of g (FP16: g 2^k)
#pragma unroll
  for (int i = 1; i < L; i += 2) {
    const float cx = (float)C3X[i], cy = (float)C3Y[i], cz = (float)C3Z[i];
    const float cu = cx * ux + cy * uy + cz * uz;
    const float cm = cx * mx + cy * my + cz * mz;
    // c.G of the pair, from the descriptor (0 for an inlet or outlet node)
    const float cG = OPEN ? d.cg[i >> 1] * gk : d.cg[i >> 1];
    const float cP = cx * sPx + cy * sPy + cz * sPz;
    const float cQc = cx * cx * Qxx + cy * cy * Qyy + cz * cz * Qzz +
                      2.0f * (cx * cy * Qxy + cx * cz * Qxz + cy * cz * Qyz);
    const float K = kw3<L>(i);
    const float ev = K * (base + 4.5f * rho * cu * cu);     // even part of geq
    const float od = K * 3.0f * cm;                           // odd part of geq
    const float sev = K * (sbase + 9.0f * cu * cG + 4.5f * cQc);
    const float sod = K * 3.0f * (cG + cP);
    if (H) {
      out[i] = fmaf(sc, om * (ev + od - inv * g[i]) + kh * (sev + sod), g[i]);
      out[i + 1] = fmaf(sc, om * (ev - od - inv * g[i + 1]) + kh * (sev - sod), g[i + 1]);
    } else {
      out[i] = g[i] + om * (ev + od - g[i]) + kh * (sev + sod);
      out[i + 1] = g[i + 1] + om * (ev - od - g[i + 1]) + kh * (sev - sod);
    }
  }
  if (H)
    out[0] = fmaf(sc, om * (kw3<L>(0) * base - inv * g[0]) + kh * kw3<L>(0) * sbase, g[0]);
  else
    out[0] = g[0] + om * (kw3<L>(0) * base - g[0]) + kh * kw3<L>(0) * sbase;

  const bool b = OPEN && bnd;
  const float rc = b ? rho_b : rho;
  const float vv = b ? ubx * ubx + uby * uby + ubz * ubz : ux * ux + uy * uy + uz * uz;
  if (__ballot(valid && !(rc > 0.0f && vv <= 0.25f)) != 0 && lane == 0)
    atomicOr(d.err, (int32_t)kErrUnstable);
  uint16_t hb[L];  // FP16: the stochastically rounded halves
  if (H) {
    // 13 random bits per population, from one hash of (node, step) and xorshifts, each
    // 32-bit word serving two populations
    const uint32_t tk = lowbias32((uint32_t)t ^ lowbias32((uint32_t)((uint64_t)t >> 32)));
    uint32_t hw = lowbias32((((uint32_t)z * (uint32_t)ny + (uint32_t)yc) * (uint32_t)nx +
                            (uint32_t)xc) ^ tk);
#pragma unroll
    for (int i = 0; i < L; ++i) {
      if (i > 0 && (i & 1) == 0) hw = xorshift32(hw);
      hb[i] = sr_half(out[i], (i & 1) ? __builtin_amdgcn_alignbit(hw, hw, 13) : hw);
    }
  }
  if (valid) {
    const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(
        (void *)d.pop[p ^ 1], (short)0, (int)(L * pb), kBufferFlags);
    const uint32_t s0r = row[1][1];
    auto put_all = [&](auto nt) {
      constexpr int CP = decltype(nt)::value ? kStoreNT : 0;
#pragma unroll
      for (int i = 0; i < L; ++i) {
        if (H)
          __builtin_amdgcn_raw_buffer_store_b16(hb[i], rd, vx0, (uint32_t)i * pb + s0r, CP);
        else
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, out[i]), rd, vx0,
                                                (uint32_t)i * pb + s0r, CP);
      }
    };
    if (d.store_nt)
      put_all(std::true_type{});
    else
      put_all(std::false_type{});
  }
}

// Register budget of the collide kernels (waves per SIMD)
template <int L, bool H>
constexpr int collide3_waves() {
  return H ? DILBM3D_COLLIDE_WAVES_F16 : (L == 19 ? DILBM3D_COLLIDE_WAVES : DILBM3D27_COLLIDE_WAVES);
}

template <int TX, int L, bool H, bool OPEN>
__global__ __launch_bounds__(256, (collide3_waves<L, H>()))
void k3_collide(const Desc3 *__restrict__ desc, int p, int64_t step) {
  __shared__ float red[4][6][64];  // per wave: the force and torque of its lanes
  __shared__ float stash[kStash3<L> * 256];  // populations of the block's lanes
  const Desc3 &d = *desc;
  if (TX == 256) {
    // whole-row tiles: tile b to block b, so neighbouring row segments run on the eight
    // XCDs at once
    for (int64_t t = blockIdx.x; t < d.ntiles; t += gridDim.x)
      tile3<kStep3, TX, L, H, OPEN>(d, t, p, step, red, stash, nullptr, nullptr, nullptr,
                                    nullptr);
    return;
  }
  const WorkSplit ws = xcd_split(d.ntiles);
  // odd chunks are walked backwards, so neighbouring chunks reach their common edge
  // together (the x-shifted loads share cache lines across it)
  const bool rev = (blockIdx.x >> 3) & 1;
  for (int64_t i = ws.begin; i < ws.end; ++i) {
    const int64_t t = rev ? ws.end - 1 - (i - ws.begin) : i;
    tile3<kStep3, TX, L, H, OPEN>(d, t, p, step, red, stash, nullptr, nullptr, nullptr,
                                  nullptr);
  }
}

// The collide of a batch of solves in one launch: tile t of the concatenated tiles belongs
// to member tile_solve[t]; member s steps from its own state (parity (parity0 + k) & 1,
// step step0 + k), as in its own k3_collide.  Whole-row tiles go tile b to block b;
// 64-wide tiles sweep chunks of each XCD's eighth.
template <int TX, int L, bool H, bool OPEN>
__global__ __launch_bounds__(256, (collide3_waves<L, H>()))
void k3_collide_batch(const Desc3 *__restrict__ descs, const int32_t *__restrict__ tile_solve,
                      int64_t total_tiles, int k) {
  __shared__ float red[4][6][64];
  __shared__ float stash[kStash3<L> * 256];
  auto run = [&](const int64_t t) {
    const int s = __builtin_amdgcn_readfirstlane(tile_solve[t]);
    const Desc3 &d = descs[s];
    tile3<kStep3, TX, L, H, OPEN>(d, t - d.tile_base, (d.parity0 + k) & 1, d.step0 + k, red,
                                  stash, nullptr, nullptr, nullptr, nullptr);
  };
  if (TX == 256) {
    for (int64_t t = blockIdx.x; t < total_tiles; t += gridDim.x) run(t);
    return;
  }
  const WorkSplit ws = xcd_split(total_tiles);
  const bool rev = (blockIdx.x >> 3) & 1;
  for (int64_t i = ws.begin; i < ws.end; ++i) run(rev ? ws.end - 1 - (i - ws.begin) : i);
}

template <int TX, int L, bool H>
__global__ __launch_bounds__(256) void k3_fields(const Desc3 *__restrict__ desc, int p,
                                                 int64_t step, double *__restrict__ rho,
                                                 double *__restrict__ ux,
                                                 double *__restrict__ uy,
                                                 double *__restrict__ uz) {
  const Desc3 &d = *desc;
  for (int64_t t = blockIdx.x; t < d.ntiles; t += gridDim.x)
    tile3<kFields3, TX, L, H, true>(d, t, p, step, nullptr, nullptr, rho, ux, uy, uz);
}

// One block per sphere.  BIN_ONLY: bin the spheres of the current state into list set 0
// (after set_particles); otherwise do the sphere step of parity p and, when a rebuild is
// due, bin the moved spheres into the other list set.  Each of the four waves computes the
// same update (the same instructions on the same data: bitwise the same result), thread 0
// writes it, and the binning's candidate tiles are spread over all 256 threads: a sphere
// of R = 8 has about 1 100 candidate rows, whose slot claims are most of a binning's time.
template <bool BIN_ONLY, int TX>
__device__ __forceinline__ void bodies3(const Desc3 &d, const int b, const int p) {
  const int lane = threadIdx.x & 63;
  const int nb = d.nbodies;
  if (b >= nb) return;  // block-uniform
  const double *st = d.bstate[p];
  const double N[3] = {(double)d.nx, (double)d.ny, (double)d.nz};
  double X[3] = {st[b], st[nb + b], st[2 * nb + b]};
  double U[3] = {st[3 * nb + b], st[4 * nb + b], st[5 * nb + b]};
  double W[3] = {st[6 * nb + b], st[7 * nb + b], st[8 * nb + b]};
  const double R = d.bconst[b], rho_s = d.bconst[nb + b];
  const double m = d.bconst[2 * nb + b], I = d.bconst[3 * nb + b];
  const bool fixed = d.bconst[4 * nb + b] != 0.0;
  int q = p;
  // tile lists: the set this step read, and whether this sphere step rebuilds them (into
  // the other set; a fresh binning writes set 0 of a zeroed buffer)
  const int ls = d.lsel[p];
  const bool rebin = BIN_ONLY || d.rb_flag[p] != 0;
  const int lnew = BIN_ONLY ? 0 : (rebin ? ls ^ 1 : ls);
  if (!BIN_ONLY) {
    // hydrodynamic force and torque of the step (read now: in flight with the pair loads)
    const double *acc = d.acc[p] + 6 * b;
    double F[3] = {acc[0], acc[1], acc[2]};
    const double T[3] = {acc[3], acc[4], acc[5]};
    // Eq. (28): repulsion from every other sphere (minimum image); partners are read
    // kU rounds of 64 at a time so the loop pays one memory latency per batch
    double f[3] = {0.0, 0.0, 0.0};
    constexpr int kU = 8;
    for (int j0 = 0; j0 < nb; j0 += 64 * kU) {
      double px[kU], py[kU], pz[kU], pr[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int j = min(j0 + 64 * u + lane, nb - 1);  // clamped: a valid index
        px[u] = st[j];
        py[u] = st[nb + j];
        pz[u] = st[2 * nb + j];
        pr[u] = d.bconst[j];
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int j = j0 + 64 * u + lane;
        const double dx = min_image(X[0] - px[u], N[0]);
        const double dy = min_image(X[1] - py[u], N[1]);
        const double dz = min_image(X[2] - pz[u], N[2]);
        const double d2 = dx * dx + dy * dy + dz * dz;
        const double rr = R + pr[u];
        if (j >= nb || j == b || d2 > (rr + d.xi) * (rr + d.xi)) continue;
        const double dist = sqrt(d2);
        const double kk = dist <= rr ? (rr - dist) * d.inv_eps_p1
                                     : (rr + d.xi - dist) * (rr + d.xi - dist) * d.inv_eps_p;
        f[0] += kk * dx;
        f[1] += kk * dy;
        f[2] += kk * dz;
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) f[a] = wave_sum(f[a]);
    // Eq. (29): the image across the nearer surface of each wall slab
    const double hw = d.wall_h_d;
    const int axis_of_bit[3] = {1, 0, 2};
    for (int bit = 0; bit < 3; ++bit) {
      if (!(d.wall_mask & (1u << bit))) continue;
      const int a = axis_of_bit[bit];
      const double c = X[a], n = N[a];
      const double dd = (c - hw <= (n - hw) - c) ? 2.0 * (c - hw) : -2.0 * ((n - hw) - c);
      const double dist = fabs(dd);
      double kk = 0.0;
      if (dist <= 2.0 * R)
        kk = (2.0 * R - dist) * d.inv_eps_w1;
      else if (dist <= 2.0 * R + d.xi)
        kk = (2.0 * R + d.xi - dist) * (2.0 * R + d.xi - dist) * d.inv_eps_w;
      f[a] += kk * dd;
    }
    // Eq. (22): hydrodynamic force plus (rho_f / rho_s - 1) m g, rho_f = rho0
    const double gfac = (d.rho0_d / rho_s - 1.0) * m;
    F[0] += f[0] + gfac * d.gx;
    F[1] += f[1] + gfac * d.gy;
    F[2] += f[2] + gfac * d.gz;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (fixed) {
        X[a] += U[a];  // prescribed motion
      } else {
        // Eqs. (22)-(24), dt = 1: Euler velocity and spin, trapezoidal position
        const double Un = U[a] + F[a] / m;
        X[a] += 0.5 * (U[a] + Un);
        U[a] = Un;
        W[a] += T[a] / I;
      }
      X[a] = X[a] - N[a] * floor(X[a] / N[a]);
      if (X[a] >= N[a]) X[a] -= N[a];
    }
    // moved more than half the skin since the lists were built: rebuild them next step
    if (!rebin && threadIdx.x == 0) {
      double r2 = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double da = min_image(X[a] - d.bin_ref[3 * b + a], N[a]);
        r2 += da * da;
      }
      if (!(r2 <= 0.25 * kBinSkin3 * kBinSkin3)) d.rb_flag[p ^ 1] = 1;
    }
    if (b == 0 && threadIdx.x == 0) d.lsel[p ^ 1] = lnew;  // the set the next step reads
    q = p ^ 1;
    if (threadIdx.x == 0) {
      double *sn = d.bstate[q];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sn[a * nb + b] = X[a];
        sn[(3 + a) * nb + b] = U[a];
        sn[(6 + a) * nb + b] = W[a];
      }
    }
  }
  if (threadIdx.x == 0) {
    SphereSnap s;
    s.x = X[0];
    s.y = X[1];
    s.z = X[2];
    s.u = (float)U[0];
    s.v = (float)U[1];
    s.w = (float)U[2];
    s.ox = (float)W[0];
    s.oy = (float)W[1];
    s.oz = (float)W[2];
    s.r = (float)R;
    s.pad[0] = s.pad[1] = 0.0f;
    d.bsnap[q][b] = s;
  }
  // a blown-up sphere is flagged instead of binned (its tile indices would be garbage)
  if (!isfinite(X[0]) || !isfinite(X[1]) || !isfinite(X[2]) || !isfinite(R)) {
    if (lane == 0) atomicOr(d.err, (int32_t)kErrUnstable);
    return;
  }
  if (!rebin) return;  // the lists of the last rebuild still cover this sphere (uniform)
  if (threadIdx.x == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) d.bin_ref[3 * b + a] = X[a];
  }
  // bin into list set lnew: every tile holding a node within R + support + skin
  const double H = R + d.support + kBinSkin3 + 1e-3;
  const AxisTiles ax = axis_tiles(X[0], H, d.nx, d.tile_x, d.tiles_x);
  const AxisTiles ay = axis_tiles(X[1], H, d.ny, 256 / d.tile_x, d.tiles_y);
  const AxisTiles az = axis_tiles(X[2], H, d.nz, 1, d.nz);
  const int na1 = ax.a1 - ax.a0 + 1, nb1 = ay.a1 - ay.a0 + 1, nc1 = az.a1 - az.a0 + 1;
  const int na = na1 + max(0, ax.b1 - ax.b0 + 1);
  const int nbb = nb1 + max(0, ay.b1 - ay.b0 + 1);
  const int nc = nc1 + max(0, az.b1 - az.b0 + 1);
  int32_t *hd = d.tile_head[lnew];
  int32_t *lst = d.tile_list[lnew];
  // which of the tile's four waves (each 64 nodes of one row) hold a node within H of the
  // centre: per wave, each axis bounds the distance from below by the distance to the
  // middle of the wave's node range less half its extent (the periodic distance is
  // 1-Lipschitz), so no reached wave is left out; 0 when the support misses the tile
  // Candidates run x fastest over the box of na x nbb x nc tiles; the index is split with
  // FP64 reciprocals (the quotients are exact at these magnitudes), not integer division.
  const int ncand = na * nbb * nc;
  const double inv_na = 1.0 / (double)na, inv_nbb = 1.0 / (double)nbb;
  auto candidate = [&](const int e, int64_t &tile) -> uint32_t {
    if (e >= ncand) return 0u;
    const int r = (int)(((double)e + 0.5) * inv_na);
    const int ia = e - r * na;
    const int ic = (int)(((double)r + 0.5) * inv_nbb);
    const int ib = r - ic * nbb;
    const int tx = ia < na1 ? ax.a0 + ia : ax.b0 + (ia - na1);
    const int ty = ib < nb1 ? ay.a0 + ib : ay.b0 + (ib - nb1);
    const int tz = ic < nc1 ? az.a0 + ic : az.b0 + (ic - nc1);
    const double gz = fabs(min_image((double)tz + 0.5 - X[2], (double)d.nz));
    uint32_t mask = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int ya = ty * (256 / TX) + (64 * w) / TX;
      const int xa = tx * TX + (64 * w) % TX;
      const double gx = fmax(fabs(min_image((double)xa + 32.0 - X[0], (double)d.nx)) - 31.5, 0.0);
      const double gy = fabs(min_image((double)ya + 0.5 - X[1], (double)d.ny));
      if (gx * gx + gy * gy + gz * gz <= H * H) mask |= 1u << w;
    }
    tile = ((int64_t)tz * d.tiles_y + ty) * d.tiles_x + tx;
    return mask;
  };
  // kB candidates per lane at a time: their slot claims are in flight together
  constexpr int kB = 4;
  for (int e0 = threadIdx.x; e0 < ncand; e0 += 256 * kB) {
    int64_t tile[kB];
    uint32_t mask[kB];
    int slot[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) mask[u] = candidate(e0 + 256 * u, tile[u]);
#pragma unroll
    for (int u = 0; u < kB; ++u)
      if (mask[u])
        slot[u] = __hip_atomic_fetch_add((DILBM_GLOBAL int32_t *)(hd + 2 * tile[u]), 1,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      if (!mask[u]) continue;
      const int32_t entry = b | (int32_t)(mask[u] << kListIndexBits);
      if (slot[u] == 0)
        hd[2 * tile[u] + 1] = entry;  // the first entry sits in the tile's head
      else if (slot[u] < d.list_cap)
        lst[tile[u] * d.list_cap + slot[u]] = entry;
      else
        atomicOr(d.err, (int32_t)kErrCapacity);
    }
  }
}

// Populations in and out: fin / fout are [L][nz][ny][nx] FP64 deviations f_i - w_i rho0
// of the current state; node x keeps f_i at x - c_i (pull layout), as g = S (f - w rho0)
// in FP32 in the storage frame, or as g 2^k in FP16 (rounded to nearest; no frame).
template <bool BIN_ONLY, int TX>
__global__ __launch_bounds__(256) void k3_bodies(const Desc3 *__restrict__ desc, int p) {
  bodies3<BIN_ONLY, TX>(*desc, blockIdx.x, p);
}

// The sphere steps of a batch of solves in one launch: block g is sphere
// g - descs[s].body_base of member s = body_solve[g].
template <int TX>
__global__ __launch_bounds__(256) void k3_bodies_batch(const Desc3 *__restrict__ descs,
                                                       const int32_t *__restrict__ body_solve,
                                                       int k) {
  const int s = __builtin_amdgcn_readfirstlane(body_solve[blockIdx.x]);
  const Desc3 &d = descs[s];
  bodies3<false, TX>(d, (int)blockIdx.x - d.body_base, (d.parity0 + k) & 1);
}

template <int L, bool H>
__global__ void k3_set_pops(const Desc3 *__restrict__ desc, int p, int64_t step,
                            const double *__restrict__ fin) {
  const Desc3 &d = *desc;
  const int64_t plane = (int64_t)d.nx * d.ny * d.nz;      // the caller's dense planes
  const int64_t dplane = (int64_t)d.pitch * d.ny * d.nz;  // the stored planes
  const float3 V = H ? make_float3(0.0f, 0.0f, 0.0f) : ref_velocity3<L>(step);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < L * plane;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / plane);
    const int64_t n = e - i * plane;
    const int x = (int)(n % d.nx);
    const int64_t r = n / d.nx;
    const int y = (int)(r % d.ny), z = (int)(r / d.ny);
    const int xs = wrapi(x - C3X[i], d.nx), ys = wrapi(y - C3Y[i], d.ny);
    const int zs = wrapi(z - C3Z[i], d.nz);
    const int64_t o = i * dplane + ((int64_t)zs * d.ny + ys) * d.pitch + xs;
    const double g = (double)Lat3<L>::S * fin[e] - frame_offset3<L>(i, V);
    if (H)
      ((_Float16 *)d.pop[p])[o] = (_Float16)(float)(g * (double)d.store_scale);
    else
      d.pop[p][o] = (float)g;
  }
}

template <int L, bool H>
__global__ void k3_get_pops(const Desc3 *__restrict__ desc, int p, int64_t step,
                            double *__restrict__ fout) {
  const Desc3 &d = *desc;
  const int64_t plane = (int64_t)d.nx * d.ny * d.nz;      // the caller's dense planes
  const int64_t dplane = (int64_t)d.pitch * d.ny * d.nz;  // the stored planes
  const float3 V = H ? make_float3(0.0f, 0.0f, 0.0f) : ref_velocity3<L>(step);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < L * plane;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / plane);
    const int64_t n = e - i * plane;
    const int x = (int)(n % d.nx);
    const int64_t r = n / d.nx;
    const int y = (int)(r % d.ny), z = (int)(r / d.ny);
    const int xs = wrapi(x - C3X[i], d.nx), ys = wrapi(y - C3Y[i], d.ny);
    const int zs = wrapi(z - C3Z[i], d.nz);
    const int64_t o = i * dplane + ((int64_t)zs * d.ny + ys) * d.pitch + xs;
    const double g = H ? (double)((const _Float16 *)d.pop[p])[o] * (double)d.store_inv
                       : (double)d.pop[p][o];
    fout[e] = (g + frame_offset3<L>(i, V)) / (double)Lat3<L>::S;
  }
}

// The fluid at rest (every deviation zero) in the frame of step `step`, in both buffers.
template <int L, bool H>
__global__ void k3_rest_pops(const Desc3 *__restrict__ desc, int64_t step) {
  const Desc3 &d = *desc;
  const int64_t plane = (int64_t)d.pitch * d.ny * d.nz;  // padding columns included
  const float3 V = H ? make_float3(0.0f, 0.0f, 0.0f) : ref_velocity3<L>(step);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < L * plane;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float v = (float)(-frame_offset3<L>((int)(e / plane), V));  // exact
    if (H) {
      ((_Float16 *)d.pop[0])[e] = (_Float16)v;
      ((_Float16 *)d.pop[1])[e] = (_Float16)v;
    } else {
      d.pop[0][e] = v;
      d.pop[1][e] = v;
    }
  }
}

int grid_for(int64_t n, int64_t cap) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap)); }

}  // namespace

using Collide3 = void (*)(const Desc3 *, int, int64_t);
template <bool H, bool O>
static Collide3 collide3_kernel_of(int q, int tile_x) {
  if (q == 27) return tile_x == 256 ? &k3_collide<256, 27, H, O> : &k3_collide<64, 27, H, O>;
  return tile_x == 256 ? &k3_collide<256, 19, H, O> : &k3_collide<64, 19, H, O>;
}
static Collide3 collide3_kernel(int q, bool h, int tile_x, bool open) {
  if (open)
    return h ? collide3_kernel_of<true, true>(q, tile_x) : collide3_kernel_of<false, true>(q, tile_x);
  return h ? collide3_kernel_of<true, false>(q, tile_x) : collide3_kernel_of<false, false>(q, tile_x);
}

hipError_t launch3_collide(int q, bool h, bool open, int tile_x, int grid, hipStream_t stream,
                           const Desc3 *desc, int p, int64_t step) {
  hipLaunchKernelGGL(collide3_kernel(q, h, tile_x, open), dim3(grid), dim3(256), 0, stream,
                     desc, p, step);
  return hipGetLastError();
}

int collide3_blocks_per_cu(int q, bool h, bool open, int tile_x) {
  int n = 0;
  const void *f = reinterpret_cast<const void *>(collide3_kernel(q, h, tile_x, open));
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 256, 0) != hipSuccess) return 0;
  return n;
}

using Collide3B = void (*)(const Desc3 *, const int32_t *, int64_t, int);
using Fields3 = void (*)(const Desc3 *, int, int64_t, double *, double *, double *, double *);
template <bool H>
static Fields3 fields3_kernel_of(int q, int tile_x) {
  if (q == 27) return tile_x == 256 ? &k3_fields<256, 27, H> : &k3_fields<64, 27, H>;
  return tile_x == 256 ? &k3_fields<256, 19, H> : &k3_fields<64, 19, H>;
}

hipError_t launch3_fields(int q, bool h, int tile_x, int64_t ntiles, hipStream_t stream,
                          const Desc3 *desc, int p, int64_t step, double *rho, double *ux,
                          double *uy, double *uz) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ntiles, 1 << 20));
  auto k = h ? fields3_kernel_of<true>(q, tile_x) : fields3_kernel_of<false>(q, tile_x);
  hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, stream, desc, p, step, rho, ux, uy, uz);
  return hipGetLastError();
}

template <bool H, bool O>
static Collide3B collide3_batch_of(int q, int tile_x) {
  if (q == 27)
    return tile_x == 256 ? &k3_collide_batch<256, 27, H, O> : &k3_collide_batch<64, 27, H, O>;
  return tile_x == 256 ? &k3_collide_batch<256, 19, H, O> : &k3_collide_batch<64, 19, H, O>;
}
static Collide3B collide3_batch(int q, bool h, int tile_x, bool open) {
  if (open)
    return h ? collide3_batch_of<true, true>(q, tile_x) : collide3_batch_of<false, true>(q, tile_x);
  return h ? collide3_batch_of<true, false>(q, tile_x) : collide3_batch_of<false, false>(q, tile_x);
}

hipError_t launch3_collide_batch(int q, bool h, bool open, int tile_x, int grid,
                                 hipStream_t stream, const Desc3 *descs,
                                 const int32_t *tile_solve, int64_t total_tiles, int k) {
  hipLaunchKernelGGL(collide3_batch(q, h, tile_x, open), dim3(grid), dim3(256), 0, stream,
                     descs, tile_solve, total_tiles, k);
  return hipGetLastError();
}

int collide3_batch_blocks_per_cu(int q, bool h, bool open, int tile_x) {
  int n = 0;
  const void *f = reinterpret_cast<const void *>(collide3_batch(q, h, tile_x, open));
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 256, 0) != hipSuccess) return 0;
  return n;
}

hipError_t launch3_bodies_batch(int total_bodies, int tile_x, hipStream_t stream,
                                const Desc3 *descs, const int32_t *body_solve, int k) {
  if (total_bodies <= 0) return hipSuccess;
  auto kf = tile_x == 256 ? k3_bodies_batch<256> : k3_bodies_batch<64>;
  hipLaunchKernelGGL(kf, dim3(total_bodies), dim3(256), 0, stream, descs, body_solve, k);
  return hipGetLastError();
}

hipError_t launch3_bodies(bool bin_only, int nbodies, int tile_x, hipStream_t stream,
                          const Desc3 *desc, int p) {
  if (nbodies <= 0) return hipSuccess;
  const int grid = nbodies;
  auto k = bin_only ? (tile_x == 256 ? k3_bodies<true, 256> : k3_bodies<true, 64>)
                    : (tile_x == 256 ? k3_bodies<false, 256> : k3_bodies<false, 64>);
  hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, stream, desc, p);
  return hipGetLastError();
}

hipError_t launch3_set_pops(int q, bool h, int64_t count, hipStream_t stream,
                            const Desc3 *desc, int p, int64_t step, const double *fin) {
  auto k = q == 27 ? (h ? &k3_set_pops<27, true> : &k3_set_pops<27, false>)
                   : (h ? &k3_set_pops<19, true> : &k3_set_pops<19, false>);
  hipLaunchKernelGGL(k, dim3(grid_for(count, 1 << 16)), dim3(256), 0, stream, desc, p, step,
                     fin);
  return hipGetLastError();
}

hipError_t launch3_get_pops(int q, bool h, int64_t count, hipStream_t stream,
                            const Desc3 *desc, int p, int64_t step, double *fout) {
  auto k = q == 27 ? (h ? &k3_get_pops<27, true> : &k3_get_pops<27, false>)
                   : (h ? &k3_get_pops<19, true> : &k3_get_pops<19, false>);
  hipLaunchKernelGGL(k, dim3(grid_for(count, 1 << 16)), dim3(256), 0, stream, desc, p, step,
                     fout);
  return hipGetLastError();
}

hipError_t launch3_rest_pops(int q, bool h, int64_t count, hipStream_t stream,
                             const Desc3 *desc, int64_t step) {
  auto k = q == 27 ? (h ? &k3_rest_pops<27, true> : &k3_rest_pops<27, false>)
                   : (h ? &k3_rest_pops<19, true> : &k3_rest_pops<19, false>);
  hipLaunchKernelGGL(k, dim3(grid_for(count, 1 << 16)), dim3(256), 0, stream, desc, step);
  return hipGetLastError();
}

}  // namespace dilbm
