// device_common.h -- device helpers shared by the two- and three-dimensional kernels of
// libdilbm (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dilbm {
namespace {

// Global-address-space access.  Pointers read from a descriptor are generic, and generic
// accesses compile to flat instructions with a 64-bit address per lane; casting the
// (uniform) plane base to the global address space and adding a 32-bit byte offset lets
// each access be one global_load/global_store with a scalar base.
#define DILBM_GLOBAL __attribute__((address_space(1)))
// Constant address space: wave-uniform reads of data no kernel writes while it is read
// compile to scalar loads.
#define DILBM_CONST __attribute__((address_space(4)))

// Buffer resource word 3 for raw 32-bit buffer access on gfx9-family parts.
constexpr int kBufferFlags = 0x00020000;
// Cache-policy operand of the population stores: the gfx940-family non-temporal bit.  When
// the populations of a step exceed the last-level cache, a written population is next read
// one step later, after the whole lattice has streamed through the caches, so keeping it
// there only displaces the lines that neighbouring tiles still share for their shifted
// reads.  Measured on the 4096^2 D2Q9 suspension (FP32) 4% less time per collide launch,
// on the 256^3 D3Q19 and D3Q27 suspensions 5-6%.  It costs where rows do not start on
// 128-byte lines (partial lines then go to memory unmerged: 4090 x 4096 FP32 17% slower,
// FP16 38%) and where the populations would stay cached from step to step (1024^2 FP32
// 10% slower); the engines set it per solve (`store_nt`).  The same bit on the loads costs
// 6-8% (the shared lines then miss).
constexpr int kStoreNT = 2;
// A store through a pointer, with that hint or without.
template <bool NT, class V, class P>
__device__ __forceinline__ void put(V v, P *p) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// FP64 sum over a wave (every lane must be active).  DPP moves combine lanes at distance
// 1 and 2 (quad permutes), then mirrored half-rows and rows, without going through LDS;
// the four row totals are read out and added, so every lane gets the total.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo =
      (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xf, 0xf, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// (1 + tanh(2 l / eps)) / 2 written as the logistic 1 / (1 + e^(-4 l / eps)); phi_k holds
// 4 / eps * log2(e) so one hardware exp2 and one reciprocal do it.  (The hardware
// exp2 flushes results below 2^-126 to zero, where phi is 1 to FP32 precision anyway.)
__device__ __forceinline__ float phi_of(float l, float phi_k) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-l * phi_k));
}

// SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA 2014): the pseudo-random frame
// velocity of a step is drawn from it, keyed by the solve's own step count.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Counter-based 32-bit hash (Wellons' "lowbias32" integer finaliser) and one xorshift32
// step (Marsaglia, 2003): random bits for stochastic rounding, keyed by node and step.
__device__ __forceinline__ uint32_t lowbias32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
__device__ __forceinline__ uint32_t xorshift32(uint32_t x) {
  x ^= x << 13;
  x ^= x >> 17;
  x ^= x << 5;
  return x;
}

typedef _Float16 F16x2 __attribute__((ext_vector_type(2)));

// x rounded stochastically to FP16 with the gfx950 conversion v_cvt_sr_f16_f32, which adds
// the top 13 bits of rnd to the 13 FP32 mantissa bits that FP16 drops and truncates
// (normal range): with 13 uniform random bits the result rounds up with exactly its
// distance from the lower neighbour.
__device__ __forceinline__ uint16_t sr_half(float x, uint32_t rnd) {
  // the conversion writes the low half of its destination; seeding that register with x
  // itself costs no move (its high half is never stored)
  F16x2 z = __builtin_bit_cast(F16x2, x);
  z = __builtin_amdgcn_cvt_sr_f16_f32(z, x, rnd, false);
  return __builtin_bit_cast(uint16_t, z.x);
}

__device__ __forceinline__ double min_image(double d, double n) {
  if (d >= 0.5 * n) return d - n;
  if (d < -0.5 * n) return d + n;
  return d;
}

// Tile range along one axis: the tiles holding nodes k with |k + 0.5 - X| <= H (wrapped
// onto [0, n)); up to two disjoint ranges [a0, a1] and [b0, b1].
struct AxisTiles {
  int a0, a1, b0, b1;
};

__device__ __forceinline__ AxisTiles axis_tiles(double X, double H, int n, int t, int ntiles) {
  const double lo = ceil(X - H - 0.5);
  const double hi = floor(X + H - 0.5);
  if (hi - lo + 1.0 >= (double)n) return {0, ntiles - 1, 0, -1};
  int lw = (int)(lo - (double)n * floor(lo / (double)n));
  int hw = (int)(hi - (double)n * floor(hi / (double)n));
  if (lw >= n) lw -= n;
  if (hw >= n) hw -= n;
  if (lw <= hw) return {lw / t, hw / t, 0, -1};
  const int a0 = lw / t, b1 = hw / t;
  if (b1 >= a0) return {0, ntiles - 1, 0, -1};
  return {a0, ntiles - 1, 0, b1};
}

// Static split of [0, T) into contiguous chunks: workgroup b runs on XCD b % 8 and sweeps
// chunk b / 8 of that XCD's contiguous eighth.  Chunks are a few tiles long and the grid
// holds many more blocks than are resident: those resident at any moment cover a compact
// band of tiles (tiles share L2 lines at their edges, so a band re-reads little), and
// blocks that finish early make room for the next ones, which evens out slow tiles.
struct WorkSplit {
  int64_t begin, end;
};

__device__ __forceinline__ WorkSplit xcd_split(int64_t T) {
  const int64_t nblk = gridDim.x >> 3;  // blocks per XCD group (the grid is a multiple of 8)
  const int xcd = blockIdx.x & 7;
  const int64_t per = T >> 3, r = T & 7;
  const int64_t lo = xcd * per + (xcd < r ? xcd : r);
  const int64_t count = per + (xcd < r ? 1 : 0);
  const int64_t l = blockIdx.x >> 3;
  WorkSplit w;
  const int64_t chunk = (count + nblk - 1) / nblk;
  w.begin = lo + min(count, l * chunk);
  w.end = lo + min(count, (l + 1) * chunk);
  return w;
}

}  // namespace
}  // namespace dilbm
