// engine3d.hip -- host runtime and C ABI of the three-dimensional DI-LBM path of libdilbm.
//
// A dilbm3d_solver owns the device state of one 3-D problem: two population buffers (FP32
// or FP16), the per-tile sphere lists, the FP64 sphere state, snapshots and force
// accumulators, and a small device descriptor.  A step is one k3_collide launch over
// every tile (the open-ends instance when x_boundary asks for it) and one k3_bodies launch
// over the spheres; dilbm3d_step reads the sticky error word every kPollSteps3 steps while
// later steps run, and once more after the last.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "dilbm3d.h"
#include "dilbm3d_internal.h"
#include "dilbm_internal.h"
#include "fp16_scale.h"
#include "kernels.h"
#include "kernels3d.h"

namespace dilbm {
namespace {

struct Fail3 {
  dilbm_status st;
  std::string msg;
};

[[noreturn]] void fail3(dilbm_status st, const std::string &msg) { throw Fail3{st, msg}; }

#define HIPCHK3(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      dilbm_status st_ = (e_ == hipErrorOutOfMemory) ? DILBM_ENOMEM : DILBM_EDEVICE;    \
      fail3(st_, std::string(#expr) + ": " + hipGetErrorString(e_));                   \
    }                                                                                   \
  } while (0)

thread_local std::string g_thread_error3;

constexpr uint64_t kAlign3 = 256;
inline uint64_t up3(uint64_t v) { return (v + kAlign3 - 1) / kAlign3 * kAlign3; }

template <class F>
dilbm_status guard3(std::string *err, F &&f) {
  try {
    f();
    return DILBM_OK;
  } catch (const Fail3 &e) {
    if (err) *err = e.msg;
    g_thread_error3 = e.msg;
    return e.st;
  } catch (const std::bad_alloc &) {
    if (err) *err = "host allocation failed";
    g_thread_error3 = "host allocation failed";
    return DILBM_ENOMEM;
  } catch (...) {
    if (err) *err = "unexpected exception";
    g_thread_error3 = "unexpected exception";
    return DILBM_EDEVICE;
  }
}

// directions of the lattice: 19 (D3Q19, also for 0) or 27 (D3Q27)
int q_of(const dilbm3d_params &p) { return p.lattice == 27 ? 27 : 19; }
bool fp16_of(const dilbm3d_params &p) { return p.storage == DILBM_STORE_FP16; }
bool open_of(const dilbm3d_params &p) { return p.x_boundary == DILBM_XBC_INLET_OUTLET; }
// bytes of one population buffer: q planes of nz * ny rows of row_pitch3 values
uint64_t pop_half_bytes3(const dilbm3d_params &p) {
  return (uint64_t)q_of(p) * row_pitch3(p.nx, p.storage) * p.ny * p.nz * (fp16_of(p) ? 2 : 4);
}

void validate3(const dilbm3d_params *p) {
  if (!p) fail3(DILBM_EINVAL, "params is NULL");
  if (p->abi_version != DILBM3D_ABI_VERSION) fail3(DILBM_EABI, "abi_version mismatch");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) fail3(DILBM_EINVAL, "nx, ny, nz must be >= 1");
  if (p->lattice != 0 && p->lattice != 19 && p->lattice != 27)
    fail3(DILBM_EINVAL, "lattice must be 19 (D3Q19) or 27 (D3Q27)");
  if (p->storage != DILBM_STORE_FP32 && p->storage != DILBM_STORE_FP16)
    fail3(DILBM_EINVAL, "storage must be DILBM_STORE_FP32 or DILBM_STORE_FP16");
  if (p->fp16_scale_log2 != DILBM_FP16_SCALE_AUTO &&
      (p->fp16_scale_log2 < 0 || p->fp16_scale_log2 > 24))
    fail3(DILBM_EINVAL, "fp16_scale_log2 must be in [0, 24] or DILBM_FP16_SCALE_AUTO");
  if (pop_half_bytes3(*p) >= (1ull << 32) - 256)
    fail3(DILBM_EINVAL, "one population buffer (q planes, rows rounded up to 128 bytes) must "
                        "stay under 4 GB");
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) fail3(DILBM_EINVAL, "tau must be > 0.5");
  if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) fail3(DILBM_EINVAL, "rho0 must be > 0");
  if (!(p->interface_width > 0.0) || !std::isfinite(p->interface_width))
    fail3(DILBM_EINVAL, "interface_width must be > 0");
  if (!(p->phi_cutoff > 0.0) || !std::isfinite(p->phi_cutoff))
    fail3(DILBM_EINVAL, "phi_cutoff must be > 0");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->body_force[a]) || !std::isfinite(p->gravity[a]))
      fail3(DILBM_EINVAL, "body_force and gravity must be finite");
  if (p->wall_mask & ~7u) fail3(DILBM_EINVAL, "wall_mask has unknown bits");
  if (p->wall_mask && !(p->wall_half_thickness > 0.0))
    fail3(DILBM_EINVAL, "wall_half_thickness must be > 0 with walls");
  if (p->force_mode != DILBM_FORCE_MOMENTUM_EXCHANGE && p->force_mode != DILBM_FORCE_PAPER_LITERAL)
    fail3(DILBM_EINVAL, "unknown force_mode");
  if (!(p->coll_eps_p > 0.0) || !(p->coll_eps_p_overlap > 0.0) || !(p->coll_eps_w > 0.0) ||
      !(p->coll_eps_w_overlap > 0.0) || !(p->coll_xi >= 0.0))
    fail3(DILBM_EINVAL, "collision constants must be > 0 (xi >= 0)");
  if (p->list_capacity < 0 || p->list_capacity > kMaxListCap3)
    fail3(DILBM_EINVAL, "list_capacity must be in [0, 1024]");
  if (p->x_boundary != DILBM_XBC_PERIODIC && p->x_boundary != DILBM_XBC_INLET_OUTLET)
    fail3(DILBM_EINVAL, "unknown x_boundary");
  if (p->x_boundary == DILBM_XBC_INLET_OUTLET) {
    if (p->nx < 3) fail3(DILBM_EINVAL, "an inlet and an outlet need nx >= 3");
    if (p->wall_mask & DILBM3D_WALL_X) fail3(DILBM_EINVAL, "x_boundary excludes DILBM3D_WALL_X");
    if (p->inlet_kind != DILBM_INLET_VELOCITY && p->inlet_kind != DILBM_INLET_PRESSURE)
      fail3(DILBM_EINVAL, "unknown inlet_kind");
    if (p->outlet_kind != DILBM_OUTLET_PRESSURE && p->outlet_kind != DILBM_OUTLET_ZERO_GRADIENT)
      fail3(DILBM_EINVAL, "unknown outlet_kind");
    if (p->inlet_profile < 0 || p->inlet_profile > 2) fail3(DILBM_EINVAL, "unknown inlet_profile");
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(p->inlet_velocity[a]))
        fail3(DILBM_EINVAL, "inlet_velocity must be finite");
    if (p->inlet_kind == DILBM_INLET_PRESSURE &&
        !(p->inlet_density > 0.0 && std::isfinite(p->inlet_density)))
      fail3(DILBM_EINVAL, "inlet_density must be > 0");
    if (p->outlet_kind == DILBM_OUTLET_PRESSURE &&
        !(p->outlet_density > 0.0 && std::isfinite(p->outlet_density)))
      fail3(DILBM_EINVAL, "outlet_density must be > 0");
  }
}

struct Mem3 {
  void *ptr = nullptr;
  uint64_t bytes = 0;
};

Mem3 alloc3(uint64_t bytes) {
  Mem3 m;
  m.bytes = up3(std::max<uint64_t>(bytes, 1));
  HIPCHK3(hipMalloc(&m.ptr, m.bytes));
  return m;
}

void free3(Mem3 &m) {
  if (m.ptr) (void)hipFree(m.ptr);
  m.ptr = nullptr;
  m.bytes = 0;
}

}  // namespace
}  // namespace dilbm

using namespace dilbm;

struct dilbm3d_solver {
  dilbm3d_params prm{};
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int nb = 0;
  int cap = 1;
  int parity = 0;
  int64_t steps = 0;
  int grid = 8;
  int tile_x = 64;  // tile width of the current layout (64 or 256)
  Mem3 pops, body;
  uint64_t off_heads = 0, off_lists = 0, off_bstate = 0, off_bconst = 0, off_snap = 0,
           off_acc = 0, off_lsel = 0, off_bref = 0;
  Desc3 h{};
  Desc3 *d_desc = nullptr;
  int32_t *d_err = nullptr;
  int32_t *h_flag = nullptr;      // pinned copy of the error word, taken after a chunk
  hipEvent_t flag_ev = nullptr;   // marks that copy
  dilbm_status poison = DILBM_OK;
  std::string last_error;
  // kernel timing
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  double timed_ms = 0.0;
  int64_t timed_launches = 0;
  std::vector<float> launch_ms;  // every timed collide launch, in launch order
};

namespace dilbm {
namespace {

// Tile width: with long rows, a whole row of up to 256 nodes per block in natural order
// (tile b to block b); on the 256^3 suspension this takes 467 us per collide launch
// without spheres and 521 us with its 400 spheres, against 519 and 530 us for 64 x 4 x 1
// tiles in XCD-contiguous chunks, which short rows keep.  The per-wave masks of the tile
// lists let a wave skip the listed spheres whose support misses its 64 nodes.
int tile_x_for(const dilbm3d_params &p) { return p.nx >= DILBM3D_WIDE_MIN ? 256 : 64; }

int64_t tiles_of(const dilbm3d_params &p, int tile_x) {
  const int ty = 256 / tile_x;
  return (int64_t)((p.nx + tile_x - 1) / tile_x) * ((p.ny + ty - 1) / ty) * p.nz;
}

// the collide grid: one block per tile for whole-row tiles (natural order); otherwise a
// persistent grid of chunks of DILBM3D_CHUNK tiles, at least one resident wave
void size_grid3(dilbm3d_solver &s) {
  if (s.tile_x == 256) {
    s.grid = (int)std::max<int64_t>(1, std::min<int64_t>(tiles_of(s.prm, 256), (int64_t)1 << 30));
    return;
  }
  const int bpc = std::max(1, collide3_blocks_per_cu(q_of(s.prm), fp16_of(s.prm), open_of(s.prm), s.tile_x));
  int cus = 0;
  HIPCHK3(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s.device));
  const int64_t T = tiles_of(s.prm, s.tile_x), resident = (int64_t)cus * bpc;
  int64_t g = std::max(std::min(T, resident), (T + DILBM3D_CHUNK - 1) / DILBM3D_CHUNK);
  g = std::min<int64_t>(g, (int64_t)1 << 30);
  s.grid = (int)std::max<int64_t>(8, (g + 7) / 8 * 8);
}

// lay out and allocate the sphere buffer for n spheres; the solver's layout changes only
// once the allocation has succeeded
void body_layout3(dilbm3d_solver &s, int n) {
  const uint64_t T = (uint64_t)tiles_of(s.prm, s.tile_x);
  const int cap = s.prm.list_capacity > 0 ? s.prm.list_capacity : std::max(1, std::min(n, 128));
  const uint64_t nn = (uint64_t)std::max(n, 1);
  uint64_t off[8], o = 0;
  const uint64_t sizes[8] = {2 * T * 8, 2 * T * (uint64_t)cap * 4, 2 * 9 * nn * 8, 5 * nn * 8,
                             2 * nn * sizeof(SphereSnap), 2 * (uint64_t)acc_words(n, 6) * 8,
                             4 * 4, 3 * nn * 8};
  for (int k = 0; k < 8; ++k) {
    off[k] = o;
    o += up3(sizes[k]);
  }
  Mem3 fresh = alloc3(o);
  free3(s.body);
  s.body = fresh;
  s.cap = cap;
  s.off_heads = off[0];
  s.off_lists = off[1];
  s.off_bstate = off[2];
  s.off_bconst = off[3];
  s.off_snap = off[4];
  s.off_acc = off[5];
  s.off_lsel = off[6];  // lsel[2], then rb_flag[2]
  s.off_bref = off[7];
}

void fill_desc3(dilbm3d_solver &s) {
  const dilbm3d_params &p = s.prm;
  Desc3 &d = s.h;
  d = Desc3{};
  d.nx = p.nx;
  d.ny = p.ny;
  d.nz = p.nz;
  d.pitch = row_pitch3(p.nx, p.storage);
  d.storage = fp16_of(p) ? 1 : 0;
  // S w_i by |c_i|^2: D3Q19 (S = 36) 12, 2, 1; D3Q27 (S = 216) 64, 16, 4, 1
  static const double kSw19[3] = {12.0, 2.0, 1.0}, kSw27[4] = {64.0, 16.0, 4.0, 1.0};
  const int k = p.fp16_scale_log2 == DILBM_FP16_SCALE_AUTO
                    ? (q_of(p) == 27 ? auto_fp16_scale_log2(kSw27, 3, p.rho0)
                                     : auto_fp16_scale_log2(kSw19, 2, p.rho0))
                    : p.fp16_scale_log2;
  const double sc = fp16_of(p) ? std::ldexp(1.0, k) : 1.0;
  d.store_scale = (float)sc;
  d.store_inv = (float)(1.0 / sc);
  d.tile_x = s.tile_x;
  d.tiles_x = (p.nx + d.tile_x - 1) / d.tile_x;
  d.tiles_y = (p.ny + 256 / d.tile_x - 1) / (256 / d.tile_x);
  d.ntiles = tiles_of(p, s.tile_x);
  d.nbodies = s.nb;
  d.list_cap = s.cap;
  d.omega = (float)(1.0 / p.tau);
  d.khalf = (float)(1.0 - 0.5 / p.tau);
  d.inv_khalf = (float)(1.0 / (1.0 - 0.5 / p.tau));
  d.rho0 = (float)p.rho0;
  d.Gx = (float)p.body_force[0];
  d.Gy = (float)p.body_force[1];
  d.Gz = (float)p.body_force[2];
  for (int k = 0; k < kQ3Max / 2; ++k) {
    const int i = 2 * k + 1;
    d.cg[k] = (float)C3X[i] * d.Gx + (float)C3Y[i] * d.Gy + (float)C3Z[i] * d.Gz;
  }
  d.kappa = p.force_mode == DILBM_FORCE_PAPER_LITERAL ? (float)(1.0 - 0.5 / p.tau) : 1.0f;
  d.lcut = (float)(-p.phi_cutoff * p.interface_width);
  d.phi_k = (float)(4.0 / p.interface_width * 1.4426950408889634);
  d.wall_h = (float)p.wall_half_thickness;
  d.wall_mask = p.wall_mask;
  // non-temporal population stores once the populations exceed the last-level cache
  const uint64_t pops = 2ull * pop_half_bytes3(p);
  d.store_nt = pops > kStoreNtMinBytes3 ? 1 : 0;
  const int n3[3] = {p.nx, p.ny, p.nz};
  const double reach = p.wall_half_thickness + p.phi_cutoff * p.interface_width;
  for (int a = 0; a < 3; ++a) {
    // nodes k with k + 0.5 within reach of the seam: [0, lo) and [hi, n)
    int lo = (int)std::min<double>(n3[a], std::ceil(reach - 0.5) + 1.0);
    int hi = (int)std::max<double>(0.0, (double)n3[a] - (std::ceil(reach - 0.5) + 1.0));
    d.wall_lo[a] = std::max(0, lo);
    d.wall_hi[a] = std::min(n3[a], hi);
  }
  d.xbc = p.x_boundary == DILBM_XBC_INLET_OUTLET ? 1 : 0;
  d.inlet_kind = p.inlet_kind;
  d.inlet_profile = p.inlet_profile;
  d.outlet_kind = p.outlet_kind;
  for (int a = 0; a < 3; ++a) d.u_in[a] = (float)p.inlet_velocity[a];
  d.drho_in = (float)(p.inlet_density - p.rho0);
  d.drho_out = (float)(p.outlet_density - p.rho0);
  {
    // parabolic inlet: across the fluid between the wall slabs of an axis, else all of it
    const bool wy = p.wall_mask & DILBM3D_WALL_Y, wz = p.wall_mask & DILBM3D_WALL_Z;
    const double h = p.wall_half_thickness;
    const double y0 = wy ? h : 0.0, y1 = wy ? p.ny - h : (double)p.ny;
    const double z0 = wz ? h : 0.0, z1 = wz ? p.nz - h : (double)p.nz;
    d.prof_y0 = (float)y0;
    d.prof_inv_hy = (float)(1.0 / (y1 - y0));
    d.prof_z0 = (float)z0;
    d.prof_inv_hz = (float)(1.0 / (z1 - z0));
  }
  d.rho0_d = p.rho0;
  d.gx = p.gravity[0];
  d.gy = p.gravity[1];
  d.gz = p.gravity[2];
  d.inv_eps_p = 1.0 / p.coll_eps_p;
  d.inv_eps_p1 = 1.0 / p.coll_eps_p_overlap;
  d.inv_eps_w = 1.0 / p.coll_eps_w;
  d.inv_eps_w1 = 1.0 / p.coll_eps_w_overlap;
  d.xi = p.coll_xi;
  d.wall_h_d = p.wall_half_thickness;
  d.support = p.phi_cutoff * p.interface_width;
  const uint64_t half = pop_half_bytes3(p);
  d.pop[0] = (float *)s.pops.ptr;
  d.pop[1] = (float *)((char *)s.pops.ptr + half);
  char *bb = (char *)s.body.ptr;
  const uint64_t T = (uint64_t)d.ntiles, nn = (uint64_t)std::max(s.nb, 1);
  d.tile_head[0] = (int32_t *)(bb + s.off_heads);
  d.tile_head[1] = d.tile_head[0] + 2 * T;
  d.tile_list[0] = (int32_t *)(bb + s.off_lists);
  d.tile_list[1] = d.tile_list[0] + T * s.cap;
  d.bstate[0] = (double *)(bb + s.off_bstate);
  d.bstate[1] = d.bstate[0] + 9 * nn;
  d.bconst = (const double *)(bb + s.off_bconst);
  d.bsnap[0] = (SphereSnap *)(bb + s.off_snap);
  d.bsnap[1] = d.bsnap[0] + nn;
  d.acc[0] = (double *)(bb + s.off_acc);
  d.lsel = (int32_t *)(bb + s.off_lsel);
  d.rb_flag = d.lsel + 2;
  d.bin_ref = (double *)(bb + s.off_bref);
  d.acc[1] = d.acc[0] + acc_words(s.nb, 6);
  d.err = s.d_err;
}

void upload_desc3(dilbm3d_solver &s) {
  HIPCHK3(hipMemcpyAsync(s.d_desc, &s.h, sizeof(Desc3), hipMemcpyHostToDevice, s.stream));
  HIPCHK3(hipStreamSynchronize(s.stream));  // the host copy may change before the next call
}

void check_usable3(dilbm3d_solver *s) {
  if (s->poison != DILBM_OK) fail3(DILBM_ESTATE, "handle poisoned: " + s->last_error);
}

void raise_errors3(dilbm3d_solver &s, int32_t e) {
  if (e & kErrInternal) {
    s.poison = DILBM_EDEVICE;
    fail3(DILBM_EDEVICE, "internal error: a kernel met an out-of-range sphere index");
  }
  if (e & kErrCapacity) {
    s.poison = DILBM_ECAPACITY;
    fail3(DILBM_ECAPACITY, "a tile sphere list overflowed; raise list_capacity");
  }
  if (e & kErrUnstable) {
    s.poison = DILBM_EUNSTABLE;
    fail3(DILBM_EUNSTABLE, "unstable: rho <= 0, |u| > 0.5 or a non-finite value");
  }
}

void poll_errors3(dilbm3d_solver &s) {
  int32_t e = 0;
  HIPCHK3(hipMemcpyAsync(&e, s.d_err, sizeof(int32_t), hipMemcpyDeviceToHost, s.stream));
  HIPCHK3(hipStreamSynchronize(s.stream));
  raise_errors3(s, e);
}

// The error word after the work enqueued so far, copied to pinned memory (asynchronous).
void flag_copy_async3(dilbm3d_solver &s) {
  if (!s.flag_ev) HIPCHK3(hipEventCreateWithFlags(&s.flag_ev, hipEventDisableTiming));
  if (!s.h_flag) HIPCHK3(hipHostMalloc(&s.h_flag, sizeof(int32_t)));
  HIPCHK3(hipMemcpyAsync(s.h_flag, s.d_err, sizeof(int32_t), hipMemcpyDeviceToHost, s.stream));
  HIPCHK3(hipEventRecord(s.flag_ev, s.stream));
}

void collect_timing3(dilbm3d_solver &s) {
  for (auto &ev : s.events) {
    HIPCHK3(hipEventSynchronize(ev.second));
    float ms = 0.f;
    HIPCHK3(hipEventElapsedTime(&ms, ev.first, ev.second));
    s.timed_ms += ms;
    ++s.timed_launches;
    s.launch_ms.push_back(ms);
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  s.events.clear();
}

// copy a host array into a fresh device buffer on the solver's stream
struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace
}  // namespace dilbm

extern "C" {

dilbm_status dilbm3d_params_init(dilbm3d_params *p) {
  if (!p) return DILBM_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->abi_version = DILBM3D_ABI_VERSION;
  p->rho0 = 1.0;
  p->interface_width = 2.0;
  p->phi_cutoff = 4.0;
  p->wall_half_thickness = 4.0;
  p->force_mode = DILBM_FORCE_MOMENTUM_EXCHANGE;
  p->coll_eps_p = 1.0e4;
  p->coll_eps_p_overlap = 1.0e4;
  p->coll_eps_w = 0.5e4;
  p->coll_eps_w_overlap = 0.5e4;
  p->coll_xi = 1.0;
  p->fp16_scale_log2 = DILBM_FP16_SCALE_AUTO;
  p->x_boundary = DILBM_XBC_PERIODIC;
  p->inlet_density = 1.0;
  p->outlet_density = 1.0;
  return DILBM_OK;
}

dilbm_status dilbm3d_create(const dilbm3d_params *p, dilbm3d_solver **out) {
  if (!out) return DILBM_EINVAL;
  *out = nullptr;
  std::unique_ptr<dilbm3d_solver> h(new (std::nothrow) dilbm3d_solver);
  if (!h) return DILBM_ENOMEM;
  dilbm_status st = guard3(nullptr, [&] {
    validate3(p);
    int ndev = 0;
    HIPCHK3(hipGetDeviceCount(&ndev));
    if (p->device < 0 || p->device >= ndev) fail3(DILBM_EINVAL, "no such device");
    dilbm3d_solver &s = *h;
    s.prm = *p;
    s.device = p->device;
    HIPCHK3(hipSetDevice(s.device));
    if (p->stream) {
      s.stream = (hipStream_t)p->stream;
    } else {
      HIPCHK3(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
      s.own_stream = true;
    }
    const uint64_t half = pop_half_bytes3(*p);
    s.pops = alloc3(2 * half);
    HIPCHK3(hipMalloc(&s.d_desc, sizeof(Desc3)));
    HIPCHK3(hipMalloc(&s.d_err, sizeof(int32_t)));
    s.tile_x = tile_x_for(*p);
    body_layout3(s, 0);
    fill_desc3(s);
    // empty lists; then the fluid at rest (every deviation zero, in the frame of step 0)
    // in both buffers
    HIPCHK3(launch_zero_bytes(s.body.ptr, (int64_t)s.body.bytes, s.stream));
    HIPCHK3(launch_zero_bytes(s.d_err, sizeof(int32_t), s.stream));
    upload_desc3(s);
    HIPCHK3(launch3_rest_pops(q_of(*p), fp16_of(*p), (int64_t)q_of(*p) * p->nx * p->ny * p->nz, s.stream,
                              s.d_desc, 0));
    size_grid3(s);
  });
  if (st != DILBM_OK) {
    dilbm3d_destroy(h.release());
    return st;
  }
  *out = h.release();
  return DILBM_OK;
}

dilbm_status dilbm3d_set_particles(dilbm3d_solver *s, int32_t n, const double *pos,
                                   const double *vel, const double *omega, const double *radius,
                                   const double *density, const uint8_t *fixed) {
  if (!s) return DILBM_EINVAL;
  return guard3(&s->last_error, [&] {
    check_usable3(s);
    if (n < 0) fail3(DILBM_EINVAL, "n must be >= 0");
    if (n > kListIndexMask) fail3(DILBM_EINVAL, "at most 134217727 spheres per solve");
    if (n > 0 && (!pos || !radius || !density))
      fail3(DILBM_EINVAL, "pos, radius and density are required");
    for (int32_t b = 0; b < n; ++b) {
      for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(pos[3 * b + a])) fail3(DILBM_EINVAL, "sphere position not finite");
        if (vel && !std::isfinite(vel[3 * b + a])) fail3(DILBM_EINVAL, "sphere velocity not finite");
        if (omega && !std::isfinite(omega[3 * b + a])) fail3(DILBM_EINVAL, "sphere spin not finite");
      }
      if (!(radius[b] > 0.0) || !std::isfinite(radius[b])) fail3(DILBM_EINVAL, "radius must be > 0");
      if (!(density[b] > 0.0) || !std::isfinite(density[b]))
        fail3(DILBM_EINVAL, "density must be > 0");
    }
    HIPCHK3(hipSetDevice(s->device));
    HIPCHK3(hipStreamSynchronize(s->stream));
    const int nn = std::max(n, 1);
    std::vector<double> state(9 * (size_t)nn, 0.0), cst(5 * (size_t)nn, 0.0);
    const double N[3] = {(double)s->prm.nx, (double)s->prm.ny, (double)s->prm.nz};
    for (int32_t b = 0; b < n; ++b) {
      for (int a = 0; a < 3; ++a) {
        double c = std::fmod(pos[3 * b + a], N[a]);
        if (c < 0) c += N[a];
        if (c >= N[a]) c -= N[a];
        state[(size_t)a * n + b] = c;
        state[(size_t)(3 + a) * n + b] = vel ? vel[3 * b + a] : 0.0;
        state[(size_t)(6 + a) * n + b] = omega ? omega[3 * b + a] : 0.0;
      }
      const double R = radius[b], m = density[b] * 4.0 / 3.0 * M_PI * R * R * R;
      cst[b] = R;
      cst[(size_t)n + b] = density[b];
      cst[2 * (size_t)n + b] = m;
      cst[3 * (size_t)n + b] = 0.4 * m * R * R;
      cst[4 * (size_t)n + b] = (fixed && fixed[b]) ? 1.0 : 0.0;
    }
    body_layout3(*s, n);
    s->nb = n;
    fill_desc3(*s);
    size_grid3(*s);
    HIPCHK3(launch_zero_bytes(s->body.ptr, (int64_t)s->body.bytes, s->stream));
    const int p = s->parity;
    if (n > 0) {
      HIPCHK3(hipMemcpyAsync(s->h.bstate[p], state.data(), sizeof(double) * 9 * n,
                             hipMemcpyHostToDevice, s->stream));
      HIPCHK3(hipMemcpyAsync((void *)s->h.bconst, cst.data(), sizeof(double) * 5 * n,
                             hipMemcpyHostToDevice, s->stream));
    }
    upload_desc3(*s);
    HIPCHK3(launch3_bodies(true, n, s->tile_x, s->stream, s->d_desc, p));
    HIPCHK3(hipStreamSynchronize(s->stream));
    poll_errors3(*s);
  });
}

dilbm_status dilbm3d_set_populations(dilbm3d_solver *s, const double *f_dev) {
  if (!s || !f_dev) return DILBM_EINVAL;
  return guard3(&s->last_error, [&] {
    check_usable3(s);
    HIPCHK3(hipSetDevice(s->device));
    const int64_t count = (int64_t)q_of(s->prm) * s->prm.nx * s->prm.ny * s->prm.nz;
    DevBuf tmp;
    HIPCHK3(hipMalloc(&tmp.p, sizeof(double) * count));
    HIPCHK3(hipMemcpyAsync(tmp.p, f_dev, sizeof(double) * count, hipMemcpyHostToDevice,
                           s->stream));
    HIPCHK3(launch3_set_pops(q_of(s->prm), fp16_of(s->prm), count, s->stream, s->d_desc, s->parity, s->steps,
                             (const double *)tmp.p));
    HIPCHK3(hipStreamSynchronize(s->stream));
  });
}

dilbm_status dilbm3d_get_populations(dilbm3d_solver *s, double *f_dev) {
  if (!s || !f_dev) return DILBM_EINVAL;
  return guard3(&s->last_error, [&] {
    HIPCHK3(hipSetDevice(s->device));
    const int64_t count = (int64_t)q_of(s->prm) * s->prm.nx * s->prm.ny * s->prm.nz;
    DevBuf tmp;
    HIPCHK3(hipMalloc(&tmp.p, sizeof(double) * count));
    HIPCHK3(launch3_get_pops(q_of(s->prm), fp16_of(s->prm), count, s->stream, s->d_desc, s->parity, s->steps, (double *)tmp.p));
    HIPCHK3(hipMemcpyAsync(f_dev, tmp.p, sizeof(double) * count, hipMemcpyDeviceToHost,
                           s->stream));
    HIPCHK3(hipStreamSynchronize(s->stream));
  });
}

dilbm_status dilbm3d_step(dilbm3d_solver *s, int64_t nsteps) {
  if (!s) return DILBM_EINVAL;
  return guard3(&s->last_error, [&] {
    check_usable3(s);
    if (nsteps < 0) fail3(DILBM_EINVAL, "nsteps must be >= 0");
    HIPCHK3(hipSetDevice(s->device));
    bool pending = false;
    for (int64_t k = 0; k < nsteps; ++k) {
      // every kPollSteps3 steps: the flags as of the previous chunk's end (waiting for them
      // leaves this chunk queued), then a copy of the current ones; a failure stops the
      // call one chunk later
      if (k > 0 && k % kPollSteps3 == 0) {
        if (pending) {
          HIPCHK3(hipEventSynchronize(s->flag_ev));
          raise_errors3(*s, *s->h_flag);
        }
        flag_copy_async3(*s);
        pending = true;
      }
      const int p = s->parity;
      if (s->timing) {
        std::pair<hipEvent_t, hipEvent_t> ev;
        HIPCHK3(hipEventCreate(&ev.first));
        HIPCHK3(hipEventCreate(&ev.second));
        HIPCHK3(hipEventRecord(ev.first, s->stream));
        HIPCHK3(launch3_collide(q_of(s->prm), fp16_of(s->prm), open_of(s->prm), s->h.tile_x, s->grid, s->stream, s->d_desc, p,
                                s->steps));
        HIPCHK3(hipEventRecord(ev.second, s->stream));
        s->events.push_back(ev);
        if (s->events.size() >= 4096) collect_timing3(*s);
      } else {
        HIPCHK3(launch3_collide(q_of(s->prm), fp16_of(s->prm), open_of(s->prm), s->h.tile_x, s->grid, s->stream, s->d_desc, p,
                                s->steps));
      }
      HIPCHK3(launch3_bodies(false, s->nb, s->tile_x, s->stream, s->d_desc, p));
      s->parity ^= 1;
      ++s->steps;
    }
    HIPCHK3(hipStreamSynchronize(s->stream));
    poll_errors3(*s);
  });
}

dilbm_status dilbm3d_get_fields(dilbm3d_solver *s, double *rho, double *ux, double *uy,
                                double *uz) {
  if (!s) return DILBM_EINVAL;
  return guard3(&s->last_error, [&] {
    HIPCHK3(hipSetDevice(s->device));
    const int64_t n = (int64_t)s->prm.nx * s->prm.ny * s->prm.nz;
    DevBuf tmp;
    HIPCHK3(hipMalloc(&tmp.p, sizeof(double) * 4 * n));
    double *t = (double *)tmp.p;
    HIPCHK3(launch3_fields(q_of(s->prm), fp16_of(s->prm), s->h.tile_x, s->h.ntiles, s->stream, s->d_desc, s->parity, s->steps,
                           t, t + n, t + 2 * n, t + 3 * n));
    double *outs[4] = {rho, ux, uy, uz};
    for (int k = 0; k < 4; ++k)
      if (outs[k])
        HIPCHK3(hipMemcpyAsync(outs[k], t + k * n, sizeof(double) * n, hipMemcpyDeviceToHost,
                               s->stream));
    HIPCHK3(hipStreamSynchronize(s->stream));
  });
}

dilbm_status dilbm3d_get_particle_forces(dilbm3d_solver *s, double *force, double *torque) {
  if (!s) return DILBM_EINVAL;
  return guard3(&s->last_error, [&] {
    HIPCHK3(hipSetDevice(s->device));
    const int n = s->nb;
    if (n == 0) return;
    // the last step (parity ^ 1) accumulated into acc[parity ^ 1]
    std::vector<double> a(6 * (size_t)n);
    HIPCHK3(hipMemcpyAsync(a.data(), s->h.acc[s->parity ^ 1], sizeof(double) * 6 * n,
                           hipMemcpyDeviceToHost, s->stream));
    HIPCHK3(hipStreamSynchronize(s->stream));
    for (int b = 0; b < n; ++b)
      for (int c = 0; c < 3; ++c) {
        if (force) force[3 * b + c] = s->steps ? a[6 * b + c] : 0.0;
        if (torque) torque[3 * b + c] = s->steps ? a[6 * b + 3 + c] : 0.0;
      }
  });
}

dilbm_status dilbm3d_get_particles(dilbm3d_solver *s, double *pos, double *vel, double *omega) {
  if (!s) return DILBM_EINVAL;
  return guard3(&s->last_error, [&] {
    HIPCHK3(hipSetDevice(s->device));
    const int n = s->nb;
    if (n == 0) return;
    std::vector<double> st(9 * (size_t)n);
    HIPCHK3(hipMemcpyAsync(st.data(), s->h.bstate[s->parity], sizeof(double) * 9 * n,
                           hipMemcpyDeviceToHost, s->stream));
    HIPCHK3(hipStreamSynchronize(s->stream));
    for (int b = 0; b < n; ++b)
      for (int a = 0; a < 3; ++a) {
        if (pos) pos[3 * b + a] = st[(size_t)a * n + b];
        if (vel) vel[3 * b + a] = st[(size_t)(3 + a) * n + b];
        if (omega) omega[3 * b + a] = st[(size_t)(6 + a) * n + b];
      }
  });
}

dilbm_status dilbm3d_get_step_count(dilbm3d_solver *s, int64_t *steps) {
  if (!s || !steps) return DILBM_EINVAL;
  *steps = s->steps;
  return DILBM_OK;
}

dilbm_status dilbm3d_get_wall_force(dilbm3d_solver *s, double *force) {
  if (!s || !force) return DILBM_EINVAL;
  return guard3(&s->last_error, [&] {
    HIPCHK3(hipSetDevice(s->device));
    double a[3] = {0.0, 0.0, 0.0};
    if (s->steps) {  // the sum of the wall slots
      std::vector<double> w((size_t)kWallSlots * kWallSlotWords);
      HIPCHK3(hipMemcpyAsync(w.data(), s->h.acc[s->parity ^ 1] + wall_base(6 * s->nb),
                             sizeof(double) * w.size(), hipMemcpyDeviceToHost, s->stream));
      HIPCHK3(hipStreamSynchronize(s->stream));
      for (int k = 0; k < kWallSlots; ++k)
        for (int c = 0; c < 3; ++c) a[c] += w[(size_t)k * kWallSlotWords + c];
    }
    for (int c = 0; c < 3; ++c) force[c] = a[c];
  });
}

dilbm_status dilbm3d_set_kernel_timing(dilbm3d_solver *s, int32_t enable) {
  if (!s) return DILBM_EINVAL;
  return guard3(&s->last_error, [&] {
    collect_timing3(*s);
    s->timing = enable != 0;
    s->timed_ms = 0.0;
    s->timed_launches = 0;
    s->launch_ms.clear();
  });
}

dilbm_status dilbm3d_get_kernel_launch_times(dilbm3d_solver *s, double *ms, int64_t cap,
                                             int64_t *count) {
  if (!s || cap < 0 || (cap > 0 && !ms)) return DILBM_EINVAL;
  return guard3(&s->last_error, [&] {
    collect_timing3(*s);
    const int64_t n = std::min<int64_t>(cap, (int64_t)s->launch_ms.size());
    for (int64_t i = 0; i < n; ++i) ms[i] = s->launch_ms[i];
    if (count) *count = (int64_t)s->launch_ms.size();
  });
}

dilbm_status dilbm3d_get_kernel_timing(dilbm3d_solver *s, double *collide_ms,
                                       int64_t *launches) {
  if (!s) return DILBM_EINVAL;
  return guard3(&s->last_error, [&] {
    collect_timing3(*s);
    if (collide_ms) *collide_ms = s->timed_ms;
    if (launches) *launches = s->timed_launches;
  });
}

void dilbm3d_destroy(dilbm3d_solver *s) {
  if (!s) return;
  try {
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (auto &ev : s->events) {
      (void)hipEventDestroy(ev.first);
      (void)hipEventDestroy(ev.second);
    }
    free3(s->pops);
    free3(s->body);
    if (s->d_desc) (void)hipFree(s->d_desc);
    if (s->d_err) (void)hipFree(s->d_err);
    if (s->h_flag) (void)hipHostFree(s->h_flag);
    if (s->flag_ev) (void)hipEventDestroy(s->flag_ev);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
  } catch (...) {
  }
  delete s;
}

const char *dilbm3d_last_error(const dilbm3d_solver *s) {
  if (!s) return g_thread_error3.c_str();
  return s->last_error.c_str();
}

}  // extern "C"

// ---- batches: several solves advanced in one collide and one sphere launch per step ----

struct dilbm3d_batch {
  std::vector<dilbm3d_solver *> m;
  int device = 0;
  hipStream_t stream = nullptr;   // the first member's stream
  int q = 19, tile_x = 64;
  bool h = false, open = false;
  Desc3 *d_descs = nullptr;       // the members' descriptors, refreshed at every call
  int32_t *d_tile_solve = nullptr, *d_body_solve = nullptr;
  int64_t tile_cap = 0, body_cap = 0;
  int32_t *h_flags = nullptr;     // pinned copies of the members' error words
  hipEvent_t flag_ev = nullptr;
  std::string last_error;
};

dilbm_status dilbm3d_batch_create(dilbm3d_solver *const *members, int32_t n,
                                  dilbm3d_batch **out) {
  if (!out) return DILBM_EINVAL;
  *out = nullptr;
  std::unique_ptr<dilbm3d_batch> b(new (std::nothrow) dilbm3d_batch);
  if (!b) return DILBM_ENOMEM;
  dilbm_status st = guard3(nullptr, [&] {
    if (!members || n < 1) fail3(DILBM_EINVAL, "a batch needs n >= 1 members");
    for (int32_t i = 0; i < n; ++i) {
      dilbm3d_solver *s = members[i];
      if (!s) fail3(DILBM_EINVAL, "NULL member");
      for (int32_t j = 0; j < i; ++j)
        if (members[j] == s) fail3(DILBM_EINVAL, "a solver appears twice in the batch");
      check_usable3(s);
      const dilbm3d_solver *f = members[0];
      if (s->device != f->device || q_of(s->prm) != q_of(f->prm) ||
          fp16_of(s->prm) != fp16_of(f->prm) || s->tile_x != f->tile_x)
        fail3(DILBM_EINVAL,
              "batch members must share the device, the lattice, the population storage and "
              "the tile width (rows of 256 nodes or more, or all shorter)");
      b->open = b->open || open_of(s->prm);
      b->m.push_back(s);
    }
    b->device = members[0]->device;
    b->stream = members[0]->stream;
    b->q = q_of(members[0]->prm);
    b->h = fp16_of(members[0]->prm);
    b->tile_x = members[0]->tile_x;
    HIPCHK3(hipSetDevice(b->device));
    HIPCHK3(hipMalloc(&b->d_descs, sizeof(Desc3) * (size_t)n));
    HIPCHK3(hipHostMalloc(&b->h_flags, sizeof(int32_t) * (size_t)n));
    HIPCHK3(hipEventCreateWithFlags(&b->flag_ev, hipEventDisableTiming));
  });
  if (st != DILBM_OK) {
    dilbm3d_batch_destroy(b.release());
    return st;
  }
  *out = b.release();
  return DILBM_OK;
}

namespace dilbm {
namespace {

// The members' descriptors with their places in the concatenation and their current state,
// and the tile and sphere tables (rebuilt at every call: members may have new spheres).
int64_t batch_tables3(dilbm3d_batch &b, int64_t *total_bodies) {
  std::vector<Desc3> descs(b.m.size());
  int64_t T = 0, B = 0;
  for (size_t i = 0; i < b.m.size(); ++i) {
    dilbm3d_solver &s = *b.m[i];
    descs[i] = s.h;
    descs[i].tile_base = T;
    descs[i].body_base = (int32_t)B;
    descs[i].parity0 = s.parity;
    descs[i].step0 = s.steps;
    T += s.h.ntiles;
    B += s.nb;
  }
  if (T >= (int64_t)1 << 31 || B >= (int64_t)1 << 31)
    fail3(DILBM_EINVAL, "a batch holds at most 2^31 - 1 tiles and spheres");
  if (T > b.tile_cap) {
    if (b.d_tile_solve) (void)hipFree(b.d_tile_solve);
    b.d_tile_solve = nullptr;
    HIPCHK3(hipMalloc(&b.d_tile_solve, sizeof(int32_t) * (size_t)T));
    b.tile_cap = T;
  }
  if (B > b.body_cap) {
    if (b.d_body_solve) (void)hipFree(b.d_body_solve);
    b.d_body_solve = nullptr;
    HIPCHK3(hipMalloc(&b.d_body_solve, sizeof(int32_t) * (size_t)B));
    b.body_cap = B;
  }
  std::vector<int32_t> ts((size_t)T), bs((size_t)std::max<int64_t>(B, 1));
  for (size_t i = 0; i < b.m.size(); ++i) {
    std::fill(ts.begin() + descs[i].tile_base, ts.begin() + descs[i].tile_base + b.m[i]->h.ntiles,
              (int32_t)i);
    std::fill(bs.begin() + descs[i].body_base, bs.begin() + descs[i].body_base + b.m[i]->nb,
              (int32_t)i);
  }
  HIPCHK3(hipMemcpyAsync(b.d_descs, descs.data(), sizeof(Desc3) * descs.size(),
                         hipMemcpyHostToDevice, b.stream));
  HIPCHK3(hipMemcpyAsync(b.d_tile_solve, ts.data(), sizeof(int32_t) * (size_t)T,
                         hipMemcpyHostToDevice, b.stream));
  if (B > 0)
    HIPCHK3(hipMemcpyAsync(b.d_body_solve, bs.data(), sizeof(int32_t) * (size_t)B,
                           hipMemcpyHostToDevice, b.stream));
  HIPCHK3(hipStreamSynchronize(b.stream));  // the host tables go out of scope
  *total_bodies = B;
  return T;
}

void batch_flags_async3(dilbm3d_batch &b) {
  for (size_t i = 0; i < b.m.size(); ++i)
    HIPCHK3(hipMemcpyAsync(b.h_flags + i, b.m[i]->d_err, sizeof(int32_t),
                           hipMemcpyDeviceToHost, b.stream));
  HIPCHK3(hipEventRecord(b.flag_ev, b.stream));
}

}  // namespace
}  // namespace dilbm

dilbm_status dilbm3d_batch_step(dilbm3d_batch *b, int64_t nsteps) {
  if (!b) return DILBM_EINVAL;
  return guard3(&b->last_error, [&] {
    if (nsteps < 0) fail3(DILBM_EINVAL, "nsteps must be >= 0");
    if (nsteps >= ((int64_t)1 << 31)) fail3(DILBM_EINVAL, "nsteps must be < 2^31 per call");
    for (dilbm3d_solver *s : b->m) check_usable3(s);
    HIPCHK3(hipSetDevice(b->device));
    // the call returns with none of its work in flight, also when it fails part way: the
    // batch then never needs its first member's stream again (dilbm3d_batch_destroy may
    // come after that member is gone)
    struct DrainOnExit {
      hipStream_t st;
      ~DrainOnExit() { (void)hipStreamSynchronize(st); }
    } drain{b->stream};
    // members' own work on other streams finishes first
    for (dilbm3d_solver *s : b->m)
      if (s->stream != b->stream) HIPCHK3(hipStreamSynchronize(s->stream));
    int64_t nbodies = 0;
    const int64_t T = batch_tables3(*b, &nbodies);
    int grid;
    if (b->tile_x == 256) {
      grid = (int)std::max<int64_t>(1, std::min<int64_t>(T, (int64_t)1 << 30));
    } else {
      const int bpc = std::max(1, collide3_batch_blocks_per_cu(b->q, b->h, b->open, b->tile_x));
      int cus = 0;
      HIPCHK3(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
      int64_t g = std::max(std::min(T, (int64_t)cus * bpc), (T + DILBM3D_CHUNK - 1) / DILBM3D_CHUNK);
      g = std::min<int64_t>(g, (int64_t)1 << 30);
      grid = (int)std::max<int64_t>(8, (g + 7) / 8 * 8);
    }
    bool pending = false;
    int64_t k = 0;
    for (; k < nsteps; ++k) {
      // every kPollSteps3 steps: the flags as of the previous poll (a failed member stops
      // the call one chunk later), then a copy of the current ones
      if (k > 0 && k % kPollSteps3 == 0) {
        if (pending) {
          HIPCHK3(hipEventSynchronize(b->flag_ev));
          bool bad = false;
          for (size_t i = 0; i < b->m.size(); ++i) bad = bad || b->h_flags[i] != 0;
          if (bad) break;
        }
        batch_flags_async3(*b);
        pending = true;
      }
      HIPCHK3(launch3_collide_batch(b->q, b->h, b->open, b->tile_x, grid, b->stream,
                                    b->d_descs, b->d_tile_solve, T, (int)k));
      HIPCHK3(launch3_bodies_batch((int)nbodies, b->tile_x, b->stream, b->d_descs,
                                   b->d_body_solve, (int)k));
    }
    HIPCHK3(hipStreamSynchronize(b->stream));
    for (dilbm3d_solver *s : b->m) {
      s->parity ^= (int)(k & 1);
      s->steps += k;
    }
    // every member's error word: each failing member is poisoned, the first one named
    dilbm_status first = DILBM_OK;
    std::string msg;
    for (size_t i = 0; i < b->m.size(); ++i) {
      dilbm3d_solver *s = b->m[i];
      int32_t e = 0;
      HIPCHK3(hipMemcpy(&e, s->d_err, sizeof(int32_t), hipMemcpyDeviceToHost));
      if (e) {
        try {
          raise_errors3(*s, e);
        } catch (const Fail3 &f) {
          s->last_error = f.msg;
          if (first == DILBM_OK) {
            first = f.st;
            msg = "member " + std::to_string(i) + ": " + f.msg;
          }
        }
      }
    }
    if (first != DILBM_OK) fail3(first, msg);
  });
}

void dilbm3d_batch_destroy(dilbm3d_batch *b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  // no work of the batch is in flight (dilbm3d_batch_step drains its stream)
  if (b->d_descs) (void)hipFree(b->d_descs);
  if (b->d_tile_solve) (void)hipFree(b->d_tile_solve);
  if (b->d_body_solve) (void)hipFree(b->d_body_solve);
  if (b->h_flags) (void)hipHostFree(b->h_flags);
  if (b->flag_ev) (void)hipEventDestroy(b->flag_ev);
  delete b;
}

const char *dilbm3d_batch_last_error(const dilbm3d_batch *b) {
  return b ? b->last_error.c_str() : g_thread_error3.c_str();
}
