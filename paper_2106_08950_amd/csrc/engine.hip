// engine.hip -- host runtime and C ABI of libdilbm.
//
// A Solve owns the device state of one DI-LBM problem (populations, tile lists, bodies,
// force accumulators).  An Engine advances a set of member solves together: every step
// is one k_collide launch over the tiles of all members and one k_bodies launch over
// their bodies; K-step chunks are captured once into a HIP graph and replayed, while the
// per-solve step counts and parities live in a small descriptor table that is uploaded
// before every chunk.  dilbm_solver is an Engine with one member and its own device
// memory; dilbm_pool is an Engine whose members are carved out of one device arena and
// may join and leave between chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "dilbm.h"
#include "dilbm_internal.h"
#include "fp16_scale.h"
#include "kernels.h"

namespace dilbm {

// ---------------------------------------------------------------------------------------
// errors

struct Fail {
  dilbm_status st;
  std::string msg;
};

[[noreturn]] void fail(dilbm_status st, const std::string &msg) { throw Fail{st, msg}; }

#define HIPCHK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      dilbm_status st_ = (e_ == hipErrorOutOfMemory) ? DILBM_ENOMEM : DILBM_EDEVICE;    \
      fail(st_, std::string(#expr) + ": " + hipGetErrorString(e_));                    \
    }                                                                                   \
  } while (0)

thread_local std::string g_thread_error;

constexpr uint64_t kAlign = 256;
inline uint64_t align_up(uint64_t v, uint64_t a = kAlign) { return (v + a - 1) / a * a; }

// ---------------------------------------------------------------------------------------
// first-fit arena over caller- or pool-owned device memory

class Arena {
 public:
  Arena(char *base, uint64_t bytes) : base_(base), size_(bytes) {
    if (bytes) free_[0] = bytes;
  }
  char *base() const { return base_; }
  uint64_t size() const { return size_; }
  bool alloc(uint64_t bytes, uint64_t *off) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const uint64_t rest = it->second - bytes;
        const uint64_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    bytes = align_up(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  uint64_t free_bytes() const { return size_ - used_; }

 private:
  char *base_;
  uint64_t size_;
  uint64_t used_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

struct Mem {
  void *ptr = nullptr;
  uint64_t bytes = 0;
  Arena *arena = nullptr;
  uint64_t off = 0;
};

Mem mem_alloc(Arena *arena, uint64_t bytes) {
  Mem m;
  m.bytes = align_up(std::max<uint64_t>(bytes, kAlign));
  if (arena) {
    if (!arena->alloc(m.bytes, &m.off)) fail(DILBM_EAGAIN, "arena has no free block large enough");
    m.arena = arena;
    m.ptr = arena->base() + m.off;
  } else {
    HIPCHK(hipMalloc(&m.ptr, m.bytes));
  }
  return m;
}

void mem_free(Mem &m) {
  if (!m.ptr) return;
  if (m.arena)
    m.arena->release(m.off, m.bytes);
  else
    (void)hipFree(m.ptr);
  m = Mem{};
}

// ---------------------------------------------------------------------------------------
// parameters and per-solve layout

int max_tiles_for(int nx, int ny) {
  int m = 0;
  for (int s = 0; s < kNumTileShapes; ++s)
    m = std::max(m, ((nx + kTileTX[s] - 1) / kTileTX[s]) * ((ny + kTileTY[s] - 1) / kTileTY[s]));
  return m;
}

// Tile shape 5 holds two neighbouring nodes per lane: FP16 populations on an even nx.
bool shape_fits(int shape, const dilbm_params &p) {
  if (shape != kPairShape) return true;
  return p.storage == DILBM_STORE_FP16 && (p.nx % 2) == 0;
}

void validate(const dilbm_params *p) {
  if (!p) fail(DILBM_EINVAL, "params is NULL");
  if (p->abi_version != DILBM_ABI_VERSION) fail(DILBM_EABI, "abi_version mismatch");
  if (p->nx < 1 || p->ny < 1 || p->nx > 65536 || p->ny > 65536 ||
      (int64_t)row_pitch(p->nx, p->storage) * p->ny >= (int64_t)1 << 31)
    fail(DILBM_EINVAL,
         "nx, ny must be in [1, 65536] with nx*ny < 2^31 (nx rounded up to a multiple of 32, "
         "64 for FP16)");
  auto fin = [](double v) { return std::isfinite(v); };
  if (!(p->tau > 0.5) || !fin(p->tau)) fail(DILBM_EINVAL, "tau must be > 0.5");
  if (!(p->rho0 > 0.0) || !fin(p->rho0)) fail(DILBM_EINVAL, "rho0 must be > 0");
  if (!(p->interface_width > 0.0) || !fin(p->interface_width))
    fail(DILBM_EINVAL, "interface_width must be > 0");
  if (!(p->phi_cutoff > 0.0) || !fin(p->phi_cutoff)) fail(DILBM_EINVAL, "phi_cutoff must be > 0");
  for (int i = 0; i < 2; ++i)
    if (!fin(p->body_force[i]) || !fin(p->gravity[i]))
      fail(DILBM_EINVAL, "body_force and gravity must be finite");
  if (p->wall_mask & ~3u) fail(DILBM_EINVAL, "wall_mask has unknown bits");
  if (p->wall_mask && (!(p->wall_half_thickness > 0.0) || !fin(p->wall_half_thickness)))
    fail(DILBM_EINVAL, "wall_half_thickness must be > 0");
  if (p->force_mode != 0 && p->force_mode != 1) fail(DILBM_EINVAL, "unknown force_mode");
  if (!(p->coll_eps_p > 0) || !(p->coll_eps_p_overlap > 0) || !(p->coll_eps_w > 0) ||
      !(p->coll_eps_w_overlap > 0) || !(p->coll_xi >= 0) || !fin(p->coll_xi))
    fail(DILBM_EINVAL, "collision stiffnesses must be > 0 and xi >= 0");
  if (p->storage != DILBM_STORE_FP32 && p->storage != DILBM_STORE_FP16)
    fail(DILBM_EINVAL, "unknown storage");
  if (p->fp16_scale_log2 != DILBM_FP16_SCALE_AUTO &&
      (p->fp16_scale_log2 < 0 || p->fp16_scale_log2 > 24))
    fail(DILBM_EINVAL, "fp16_scale_log2 must be in [0, 24] or DILBM_FP16_SCALE_AUTO");
  if (p->list_capacity < 0 || p->list_capacity > kMaxListCap)
    fail(DILBM_EINVAL, "list_capacity must be in [0, 1024]");
  if (p->tile < -1 || p->tile >= kNumTileShapes) fail(DILBM_EINVAL, "unknown tile shape");
  if (p->tile >= 0 && !shape_fits(p->tile, *p))
    fail(DILBM_EINVAL, "tile shape 5 (512 x 1, two nodes per lane) needs FP16 storage and an "
                       "even nx");
  if (p->x_boundary != DILBM_XBC_PERIODIC && p->x_boundary != DILBM_XBC_INLET_OUTLET)
    fail(DILBM_EINVAL, "unknown x_boundary");
  if (p->x_boundary == DILBM_XBC_INLET_OUTLET) {
    if (p->nx < 3) fail(DILBM_EINVAL, "an inlet and an outlet need nx >= 3");
    if (p->wall_mask & DILBM_WALL_X) fail(DILBM_EINVAL, "x_boundary excludes DILBM_WALL_X");
    if (p->inlet_kind != DILBM_INLET_VELOCITY && p->inlet_kind != DILBM_INLET_PRESSURE)
      fail(DILBM_EINVAL, "unknown inlet_kind");
    if (p->outlet_kind != DILBM_OUTLET_PRESSURE && p->outlet_kind != DILBM_OUTLET_ZERO_GRADIENT)
      fail(DILBM_EINVAL, "unknown outlet_kind");
    if (p->inlet_profile != 0 && p->inlet_profile != 1) fail(DILBM_EINVAL, "unknown inlet_profile");
    if (!fin(p->inlet_velocity[0]) || !fin(p->inlet_velocity[1]))
      fail(DILBM_EINVAL, "inlet_velocity must be finite");
    if (p->inlet_kind == DILBM_INLET_PRESSURE && !(p->inlet_density > 0.0 && fin(p->inlet_density)))
      fail(DILBM_EINVAL, "inlet_density must be > 0");
    if (p->outlet_kind == DILBM_OUTLET_PRESSURE &&
        !(p->outlet_density > 0.0 && fin(p->outlet_density)))
      fail(DILBM_EINVAL, "outlet_density must be > 0");
  }
}

void validate_bodies(int32_t n, const double *pos, const double *vel, const double *omega,
                     const double *radius, const double *density) {
  if (n < 0) fail(DILBM_EINVAL, "negative body count");
  if (n > kListIndexMask) fail(DILBM_EINVAL, "at most 134217727 bodies per solve");
  if (n > 0 && (!pos || !radius || !density))
    fail(DILBM_EINVAL, "pos, radius and density are required");
  for (int32_t b = 0; b < n; ++b) {
    if (!std::isfinite(pos[2 * b]) || !std::isfinite(pos[2 * b + 1]))
      fail(DILBM_EINVAL, "body position not finite");
    if (!(radius[b] > 0.0) || !std::isfinite(radius[b])) fail(DILBM_EINVAL, "radius must be > 0");
    if (!(density[b] > 0.0) || !std::isfinite(density[b]))
      fail(DILBM_EINVAL, "density must be > 0");
    if (vel && (!std::isfinite(vel[2 * b]) || !std::isfinite(vel[2 * b + 1])))
      fail(DILBM_EINVAL, "body velocity not finite");
    if (omega && !std::isfinite(omega[b])) fail(DILBM_EINVAL, "body spin not finite");
  }
}

struct BodyLayout {
  int cap = 1;
  uint64_t heads = 0, lists = 0, bstate = 0, bconst = 0, bsnap = 0, bxy = 0, acc = 0;
  uint64_t nbr_cnt = 0, nbr_list = 0, nbr_ref = 0, nl_flag = 0, lsel = 0, rb_flag = 0,
           bin_ref = 0, total = 0;
};

BodyLayout body_layout(const dilbm_params &p, int nb) {
  BodyLayout L;
  L.cap = p.list_capacity > 0 ? p.list_capacity : std::max(1, std::min(nb, 128));
  const uint64_t mt = (uint64_t)max_tiles_for(p.nx, p.ny);
  uint64_t o = 0;
  L.heads = o;
  o += align_up(2 * mt * 8);
  L.lists = o;
  o += align_up(2 * mt * (uint64_t)L.cap * 4);
  L.bstate = o;
  o += align_up(2 * 5 * (uint64_t)std::max(nb, 1) * 8);
  L.bconst = o;
  o += align_up(5 * (uint64_t)std::max(nb, 1) * 8);
  L.bsnap = o;
  o += align_up(2 * (uint64_t)std::max(nb, 1) * sizeof(BodySnap));
  L.bxy = o;
  o += align_up(2 * 2 * (uint64_t)std::max(nb, 1) * 4);
  L.acc = o;
  o += align_up(2 * (uint64_t)acc_words(nb, 3) * 8);
  L.nbr_cnt = o;
  o += align_up(4 * (uint64_t)std::max(nb, 1));
  L.nbr_list = o;
  o += align_up(4 * (uint64_t)kNbrCap * std::max(nb, 1));
  L.nbr_ref = o;
  o += align_up(2 * 8 * (uint64_t)std::max(nb, 1));
  L.nl_flag = o;
  o += align_up(2 * 4);
  L.lsel = o;
  o += align_up(2 * 4);
  L.rb_flag = o;
  o += align_up(2 * 4);
  L.bin_ref = o;
  o += align_up(2 * 8 * (uint64_t)std::max(nb, 1));
  L.total = o;
  return L;
}

// Default tile shape of a plain solve: whole-row 256 x 1 tiles (natural collide order)
// for FP32 populations on rows of 1024 nodes or more, else 64 x 4.  (FP16 in 512 x 1
// tiles with two nodes per lane measured slower than 64 x 4 on the 4096^2 suspension:
// 168 against about 150 us per collide launch.)
int default_shape(const dilbm_params &p) {
  return (p.storage == DILBM_STORE_FP32 && p.nx >= 1024) ? 2 : 0;
}

// one population buffer: nine planes of ny rows of row_pitch values
uint64_t pop_half_bytes(const dilbm_params &p) {
  return (uint64_t)kQ * row_pitch(p.nx, p.storage) * p.ny *
         (p.storage == DILBM_STORE_FP16 ? 2 : 4);
}

uint64_t pop_bytes(const dilbm_params &p) { return align_up(2ull * pop_half_bytes(p)); }

// ---------------------------------------------------------------------------------------

struct Solve {
  dilbm_params prm{};
  int nb = 0;
  int shape = 0;
  Mem pops, body;
  BodyLayout L;
  SolveDesc desc{};
  int64_t steps_done = 0;  // steps enqueued
  int64_t target = -1;     // pool: steps requested
  int slot = -1;
  int64_t ticket = -1;
  bool forces_valid = false;
  bool finished = false;   // pool: all steps enqueued, left the member set
  hipEvent_t done_ev = nullptr;
  dilbm_status poison = DILBM_OK;
  std::string err;

  int64_t remaining() const { return target < 0 ? INT64_MAX : target - steps_done; }
  int parity() const { return (int)(steps_done & 1); }
  int tiles() const { return desc.tiles_x * desc.tiles_y; }
};

void fill_desc(Solve &s) {
  const dilbm_params &p = s.prm;
  SolveDesc &d = s.desc;
  d.nx = p.nx;
  d.ny = p.ny;
  d.pitch = row_pitch(p.nx, p.storage);
  d.tx = kTileTX[s.shape];
  d.ty = kTileTY[s.shape];
  d.tiles_x = (p.nx + d.tx - 1) / d.tx;
  d.tiles_y = (p.ny + d.ty - 1) / d.ty;
  d.nbodies = s.nb;
  d.list_cap = s.L.cap;
  d.wall_mask = p.wall_mask;
  d.omega = (float)(1.0 / p.tau);
  d.khalf = (float)(1.0 - 0.5 / p.tau);
  d.rho0 = (float)p.rho0;
  d.rho36 = (float)(36.0 * p.rho0);
  d.Gx = (float)p.body_force[0];
  d.Gy = (float)p.body_force[1];
  {
    // in FP32 arithmetic: the values the kernels' own expressions in d.Gx, d.Gy would take
    const float cg[4] = {d.Gx, d.Gy, d.Gx + d.Gy, d.Gy - d.Gx};
    for (int k = 0; k < 4; ++k) {
      d.g9[k] = 9.0f * cg[k];
      d.g3[k] = 3.0f * cg[k];
    }
    d.khk4 = d.khalf * 4.0f;
    d.khk16 = d.khalf * 16.0f;
  }
  d.phi_k = (float)(4.0 / p.interface_width * 1.4426950408889634);
  d.lcut = (float)(-p.phi_cutoff * p.interface_width);
  d.wall_h = (float)p.wall_half_thickness;
  {
    // node j (centre j + 1/2) is within reach of the seam at 0 when j + 1/2 <= h + cut,
    // and of the seam at n when n - (j + 1/2) <= h + cut; one node of slack each side
    const double reach = p.wall_half_thickness + p.phi_cutoff * p.interface_width;
    const int lo = (int)std::floor(reach - 0.5) + 2;
    d.wall_y_lo = std::min(lo, p.ny);
    d.wall_y_hi = std::max(p.ny - lo, 0);
    d.wall_x_lo = std::min(lo, p.nx);
    d.wall_x_hi = std::max(p.nx - lo, 0);
  }
  d.kappa = p.force_mode == DILBM_FORCE_PAPER_LITERAL ? (float)(1.0 - 0.5 / p.tau) : 1.0f;
  d.xbc = p.x_boundary;
  d.inlet_kind = p.inlet_kind;
  d.inlet_profile = p.inlet_profile;
  d.outlet_kind = p.outlet_kind;
  d.u_in_x = (float)p.inlet_velocity[0];
  d.u_in_y = (float)p.inlet_velocity[1];
  d.rho36_in = (float)(36.0 * p.inlet_density);
  d.rho36_out = (float)(36.0 * p.outlet_density);
  {
    // parabolic inlet: s = (y + 1/2 - y0) / (y1 - y0) across the fluid between the y wall
    // slabs (or the full height)
    const double y0 = (p.wall_mask & DILBM_WALL_Y) ? p.wall_half_thickness : 0.0;
    const double y1 = (p.wall_mask & DILBM_WALL_Y) ? p.ny - p.wall_half_thickness : (double)p.ny;
    d.prof_y0 = (float)y0;
    d.prof_inv_h = (float)(1.0 / (y1 - y0));
  }
  d.storage = p.storage;
  // D2Q9: S w_i = 16, 4, 1 for |c_i|^2 = 0, 1, 2 (S = 36)
  static const double kSw[3] = {16.0, 4.0, 1.0};
  const int k = p.fp16_scale_log2 == DILBM_FP16_SCALE_AUTO
                    ? auto_fp16_scale_log2(kSw, 2, p.rho0)
                    : p.fp16_scale_log2;
  const double sc = p.storage == DILBM_STORE_FP16 ? std::ldexp(1.0, k) : 1.0;
  d.store_scale = (float)sc;
  d.store_inv = (float)(1.0 / sc);
  d.rho0_d = p.rho0;
  d.gx = p.gravity[0];
  d.gy = p.gravity[1];
  d.inv_eps_p = 1.0 / p.coll_eps_p;
  d.inv_eps_p1 = 1.0 / p.coll_eps_p_overlap;
  d.inv_eps_w = 1.0 / p.coll_eps_w;
  d.inv_eps_w1 = 1.0 / p.coll_eps_w_overlap;
  d.xi = p.coll_xi;
  d.wall_h_d = p.wall_half_thickness;
  d.support = p.phi_cutoff * p.interface_width;
  const uint64_t half = pop_half_bytes(p);
  char *pp = (char *)s.pops.ptr;
  d.pop[0] = pp;
  d.pop[1] = pp + half;
  char *bb = (char *)s.body.ptr;
  const uint64_t mt = (uint64_t)max_tiles_for(p.nx, p.ny);
  d.tile_head[0] = (int32_t *)(bb + s.L.heads);
  d.tile_head[1] = d.tile_head[0] + 2 * mt;
  d.tile_list[0] = (int32_t *)(bb + s.L.lists);
  d.tile_list[1] = d.tile_list[0] + mt * s.L.cap;
  const uint64_t nbs = (uint64_t)std::max(s.nb, 1);
  d.bstate[0] = (double *)(bb + s.L.bstate);
  d.bstate[1] = d.bstate[0] + 5 * nbs;
  d.bconst = (const double *)(bb + s.L.bconst);
  d.bsnap[0] = (BodySnap *)(bb + s.L.bsnap);
  d.bsnap[1] = d.bsnap[0] + nbs;
  d.bxy[0] = (float *)(bb + s.L.bxy);
  d.bxy[1] = d.bxy[0] + 2 * nbs;
  d.acc[0] = (double *)(bb + s.L.acc);
  d.acc[1] = d.acc[0] + acc_words(s.nb, 3);
  d.nbr_cnt = (int32_t *)(bb + s.L.nbr_cnt);
  d.nbr_list = (int32_t *)(bb + s.L.nbr_list);
  d.nbr_ref = (double *)(bb + s.L.nbr_ref);
  d.nl_flag = (int32_t *)(bb + s.L.nl_flag);
  d.lsel = (int32_t *)(bb + s.L.lsel);
  d.rb_flag = (int32_t *)(bb + s.L.rb_flag);
  d.bin_ref = (double *)(bb + s.L.bin_ref);
}

// ---------------------------------------------------------------------------------------
// Engine

class Engine {
 public:
  Engine(int device, void *stream) : device_(device) {
    HIPCHK(hipSetDevice(device));
    if (stream) {
      stream_ = (hipStream_t)stream;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking));
      own_stream_ = true;
    }
    HIPCHK(hipStreamCreateWithFlags(&aux_, hipStreamNonBlocking));
    HIPCHK(hipMalloc(&d_hdr_, sizeof(BatchHeader)));
    HIPCHK(hipMalloc(&d_one_desc_, sizeof(SolveDesc) * 2));
    HIPCHK(hipMalloc(&d_one_hdr_, sizeof(BatchHeader) * 2));
    HIPCHK(hipHostMalloc(&h_one_, sizeof(SolveDesc) * 2 + sizeof(BatchHeader) * 2));
    for (int i = 0; i < 2; ++i) HIPCHK(hipEventCreateWithFlags(&one_ev_[i], hipEventDisableTiming));
    for (int i = 0; i < kRing; ++i)
      HIPCHK(hipEventCreateWithFlags(&ring_ev_[i], hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&table_ev_, hipEventDisableTiming));
    HIPCHK(hipDeviceGetAttribute(&num_cu_, hipDeviceAttributeMultiprocessorCount, device));
  }

  ~Engine() {
    (void)hipSetDevice(device_);
    (void)hipStreamSynchronize(stream_);
    (void)hipStreamSynchronize(aux_);
    clear_graphs();
    for (auto &e : timing_ev_) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    (void)hipFree(d_descs_);
    (void)hipFree(d_tile_solve_);
    (void)hipFree(d_body_solve_);
    (void)hipFree(d_err_);
    (void)hipFree(d_hdr_);
    (void)hipFree(d_one_desc_);
    (void)hipFree(d_one_hdr_);
    (void)hipFree(d_one_bodies_);
    (void)hipHostFree(h_one_);
    for (int i = 0; i < kRing; ++i) {
      (void)hipHostFree(h_ring_[i]);
      (void)hipEventDestroy(ring_ev_[i]);
    }
    (void)hipHostFree(h_tile_solve_);
    (void)hipHostFree(h_body_solve_);
    (void)hipHostFree(h_err_);
    (void)hipHostFree(h_flag_);
    if (flag_ev_) (void)hipEventDestroy(flag_ev_);
    for (int i = 0; i < 2; ++i) (void)hipEventDestroy(one_ev_[i]);
    (void)hipEventDestroy(table_ev_);
    (void)hipStreamDestroy(aux_);
    if (own_stream_) (void)hipStreamDestroy(stream_);
  }

  hipStream_t stream() const { return stream_; }
  hipStream_t aux() const { return aux_; }
  int device() const { return device_; }
  int shape() const { return shape_; }
  int storage() const { return storage_; }
  void set_storage(int st) { storage_ = st; }
  int graph_steps() const { return graph_steps_; }
  void set_graph_steps(int k) {
    if (k != graph_steps_) clear_graphs();
    graph_steps_ = k;
  }
  const std::vector<Solve *> &members() const { return members_; }

  // ---- membership ---------------------------------------------------------------------
  void add(Solve *s) {
    ensure_err_capacity();
    int slot = -1;
    for (int i = 0; i < (int)slot_used_.size(); ++i)
      if (!slot_used_[i]) {
        slot = i;
        break;
      }
    if (slot < 0) {
      slot = (int)slot_used_.size();
      slot_used_.push_back(false);
      ensure_err_capacity();
    }
    slot_used_[slot] = true;
    s->slot = slot;
    s->desc.err = d_err_ + slot;
    HIPCHK(launch_fill_i32(d_err_ + slot, 1, 0, stream_));
    members_.push_back(s);
    dirty_ = true;
  }

  // Leave the member set; the slot (and its error bits) stays reserved until release().
  void leave(Solve *s) {
    auto it = std::find(members_.begin(), members_.end(), s);
    if (it != members_.end()) {
      members_.erase(it);
      dirty_ = true;
    }
  }

  void remove(Solve *s) {
    leave(s);
    if (s->slot >= 0 && s->slot < (int)slot_used_.size()) slot_used_[s->slot] = false;
    s->slot = -1;
  }

  void mark_dirty() { dirty_ = true; }

  // ---- one-solve helpers (scratch descriptor) ----------------------------------------
  // Upload s's descriptor (with parity0 = its current parity) into the scratch slot used by
  // single-solve kernels on `st`; waits for the previous use of the staging buffer.
  SolveDesc *one_desc(Solve &s, hipStream_t st, int which) {
    HIPCHK(hipEventSynchronize(one_ev_[which]));
    SolveDesc *h = (SolveDesc *)h_one_ + which;
    *h = s.desc;
    h->step0 = s.steps_done;
    h->parity0 = s.parity();
    h->active_steps = 1;
    // one-solve launches number tiles and bodies from 0, not from the solve's place in
    // the batch
    h->tile_base = 0;
    h->body_base = 0;
    // the error word of the solve's slot: the table may have moved since the solve's
    // descriptor was filled (a pool solve that has finished keeps its slot until release)
    if (s.slot >= 0) h->err = d_err_ + s.slot;
    HIPCHK(hipMemcpyAsync(d_one_desc_ + which, h, sizeof(SolveDesc), hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(one_ev_[which], st));
    return d_one_desc_ + which;
  }

  // Bin the bodies of s's current state into list set 0, which the next step reads (both
  // sets emptied, no rebin pending).
  void bin_current(Solve &s, hipStream_t st) {
    const int64_t mt = max_tiles_for(s.prm.nx, s.prm.ny);
    HIPCHK(launch_fill_i32(s.desc.tile_head[0], 2 * mt, 0, st));
    HIPCHK(launch_fill_i32(s.desc.tile_head[1], 2 * mt, 0, st));
    HIPCHK(launch_fill_i32(s.desc.lsel, 2, 0, st));
    HIPCHK(launch_fill_i32(s.desc.rb_flag, 2, 0, st));
    if (s.nb == 0) return;
    SolveDesc *dd = one_desc(s, st, 0);
    if (s.nb > one_bodies_cap_) {
      HIPCHK(hipStreamSynchronize(st));
      (void)hipFree(d_one_bodies_);
      d_one_bodies_ = nullptr;
      HIPCHK(hipMalloc(&d_one_bodies_, sizeof(int32_t) * s.nb));
      one_bodies_cap_ = s.nb;
    }
    HIPCHK(launch_fill_i32(d_one_bodies_, s.nb, 0, st));
    BatchHeader *hh = (BatchHeader *)((SolveDesc *)h_one_ + 2);
    HIPCHK(hipEventSynchronize(table_ev_));
    hh->total_tiles = 0;
    hh->total_bodies = s.nb;
    hh->nsolves = 1;
    hh->solo_slot = 0;
    hh->natural = 0;
    HIPCHK(hipMemcpyAsync(d_one_hdr_, hh, sizeof(BatchHeader), hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(table_ev_, st));
    HIPCHK(launch_bodies(true, std::max(1, (s.nb + 3) / 4), st, dd, d_one_bodies_, d_one_hdr_, 0));
  }

  void set_shape(int shape) {
    if (shape == shape_) return;
    shape_ = shape;
    clear_graphs();
    for (Solve *s : members_) {
      s->shape = shape;
      fill_desc(*s);
      s->desc.err = d_err_ + s->slot;
      bin_current(*s, stream_);
    }
    dirty_ = true;
  }

  // ---- chunks ---------------------------------------------------------------------------
  // Enqueue up to K steps of every member (fewer for members with fewer left).  Returns
  // the largest number of steps any member took.
  int run_chunk(int K, bool allow_graph) {
    if (members_.empty() || K <= 0) return 0;
    if (dirty_) rebuild_tables();
    int kmax = 0;
    // descriptor upload through a ring of pinned staging buffers
    const int r = ring_pos_;
    ring_pos_ = (ring_pos_ + 1) % kRing;
    HIPCHK(hipEventSynchronize(ring_ev_[r]));
    ensure_ring(r);
    SolveDesc *h = (SolveDesc *)h_ring_[r];
    for (int i = 0; i < (int)slot_used_.size(); ++i) {
      h[i] = SolveDesc{};
      h[i].active_steps = 0;
    }
    for (Solve *s : members_) {
      const int64_t a = std::min<int64_t>(K, s->remaining());
      s->desc.step0 = s->steps_done;
      s->desc.active_steps = (int32_t)a;
      s->desc.parity0 = s->parity();
      h[s->slot] = s->desc;
      h[s->slot].err = d_err_ + s->slot;
      kmax = std::max<int>(kmax, (int)a);
    }
    HIPCHK(hipMemcpyAsync(d_descs_, h, sizeof(SolveDesc) * slot_used_.size(),
                          hipMemcpyHostToDevice, stream_));
    HIPCHK(hipEventRecord(ring_ev_[r], stream_));
    if (kmax == 0) return 0;
    if (timing_) {
      launch_steps(kmax, true);
    } else if (allow_graph && kmax > 1) {
      hipGraphExec_t g = graph_for(kmax);
      HIPCHK(hipGraphLaunch(g, stream_));
    } else {
      launch_steps(kmax, false);
    }
    for (Solve *s : members_) {
      s->steps_done += s->desc.active_steps;
      if (s->desc.active_steps > 0) s->forces_valid = true;
    }
    return kmax;
  }

  // Error bits of every slot (synchronous).
  void read_errors() {
    if (slot_used_.empty()) return;
    HIPCHK(hipMemcpyAsync(h_err_, d_err_, sizeof(int32_t) * slot_used_.size(),
                          hipMemcpyDeviceToHost, stream_));
    HIPCHK(hipStreamSynchronize(stream_));
  }
  int32_t err_of(const Solve &s) const { return h_err_[s.slot]; }
  // One solve's error word, copied after the work enqueued so far into pinned memory
  // (asynchronous); flag_wait() waits for the last such copy and returns the word.
  void flag_copy_async(const Solve &s) {
    if (!flag_ev_) HIPCHK(hipEventCreateWithFlags(&flag_ev_, hipEventDisableTiming));
    if (!h_flag_) HIPCHK(hipHostMalloc(&h_flag_, sizeof(int32_t)));
    HIPCHK(hipMemcpyAsync(h_flag_, d_err_ + s.slot, sizeof(int32_t), hipMemcpyDeviceToHost,
                          stream_));
    HIPCHK(hipEventRecord(flag_ev_, stream_));
  }
  int32_t flag_wait() {
    HIPCHK(hipEventSynchronize(flag_ev_));
    return *h_flag_;
  }
  // The error table as it stands on the device: its address and the slots in use.
  const int32_t *err_table() const { return d_err_; }
  int err_slots() const { return (int)slot_used_.size(); }
  int32_t read_error_of(Solve &s, hipStream_t st) {
    int32_t v = 0;
    HIPCHK(hipMemcpyAsync(&h_err_[s.slot], d_err_ + s.slot, sizeof(int32_t),
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    v = h_err_[s.slot];
    return v;
  }

  // ---- timing -------------------------------------------------------------------------
  void set_timing(bool on) {
    collect_timing();
    timing_ = on;
    timing_used_ = 0;
    timed_ms_ = 0.0;
    timed_launches_ = 0;
    launch_ms_.clear();
  }
  void collect_timing() {
    if (!timing_used_) return;
    HIPCHK(hipStreamSynchronize(stream_));
    for (int i = 0; i < timing_used_; ++i) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, timing_ev_[i].first, timing_ev_[i].second));
      timed_ms_ += ms;
      launch_ms_.push_back(ms);
    }
    timed_launches_ += timing_used_;
    timing_used_ = 0;
  }
  double timed_ms() const { return timed_ms_; }
  const std::vector<float> &launch_ms() const { return launch_ms_; }
  int64_t timed_launches() const { return timed_launches_; }

  int64_t total_tiles() const { return total_tiles_; }
  int total_bodies() const { return total_bodies_; }

  void set_persistent(bool p) {
    if (p != persistent_) {
      persistent_ = p;
      clear_graphs();
    }
  }

 private:
  static constexpr int kRing = 4;

  void ensure_err_capacity() {
    const int need = std::max<int>(8, (int)slot_used_.size());
    if (need <= err_cap_) return;
    int cap = std::max(need, err_cap_ * 2);
    int32_t *d = nullptr;
    HIPCHK(hipMalloc(&d, sizeof(int32_t) * cap));
    HIPCHK(launch_fill_i32(d, cap, 0, stream_));
    if (d_err_) {
      HIPCHK(hipMemcpyAsync(d, d_err_, sizeof(int32_t) * err_cap_, hipMemcpyDeviceToDevice,
                            stream_));
      HIPCHK(hipStreamSynchronize(stream_));
      (void)hipFree(d_err_);
    }
    d_err_ = d;
    int32_t *h = nullptr;
    HIPCHK(hipHostMalloc(&h, sizeof(int32_t) * cap));
    std::memset(h, 0, sizeof(int32_t) * cap);
    (void)hipHostFree(h_err_);
    h_err_ = h;
    err_cap_ = cap;
    for (Solve *s : members_) s->desc.err = d_err_ + s->slot;
    clear_graphs();
  }

  void ensure_ring(int r) {
    const size_t need = sizeof(SolveDesc) * std::max<size_t>(1, slot_used_.size());
    if (need <= ring_bytes_[r]) return;
    (void)hipHostFree(h_ring_[r]);
    h_ring_[r] = nullptr;
    const size_t bytes = std::max(need, ring_bytes_[r] * 2);
    HIPCHK(hipHostMalloc(&h_ring_[r], bytes));
    ring_bytes_[r] = bytes;
  }

  void rebuild_tables() {
    // descriptor capacity follows the slot count
    const int nslots = (int)slot_used_.size();
    if (nslots > desc_cap_) {
      HIPCHK(hipStreamSynchronize(stream_));
      (void)hipFree(d_descs_);
      desc_cap_ = std::max(nslots, desc_cap_ * 2);
      HIPCHK(hipMalloc(&d_descs_, sizeof(SolveDesc) * desc_cap_));
      clear_graphs();
    }
    // global tile and body numbering; solves in member order
    int64_t T = 0;
    int64_t B = 0;
    for (Solve *s : members_) {
      s->desc.tile_base = T;
      s->desc.body_base = (int32_t)B;
      T += s->tiles();
      B += s->nb;
    }
    if (B >= ((int64_t)1 << 31)) fail(DILBM_EINVAL, "too many bodies in one pool");
    HIPCHK(hipEventSynchronize(table_ev_));
    if (T > tile_cap_) {
      HIPCHK(hipStreamSynchronize(stream_));
      (void)hipFree(d_tile_solve_);
      (void)hipHostFree(h_tile_solve_);
      tile_cap_ = std::max<int64_t>(T, tile_cap_ * 2);
      HIPCHK(hipMalloc(&d_tile_solve_, sizeof(int32_t) * tile_cap_));
      HIPCHK(hipHostMalloc(&h_tile_solve_, sizeof(int32_t) * tile_cap_));
      clear_graphs();
    }
    if (B > body_cap_ || !d_body_solve_) {
      HIPCHK(hipStreamSynchronize(stream_));
      (void)hipFree(d_body_solve_);
      (void)hipHostFree(h_body_solve_);
      body_cap_ = std::max<int64_t>(std::max<int64_t>(B, 1), body_cap_ * 2);
      HIPCHK(hipMalloc(&d_body_solve_, sizeof(int32_t) * body_cap_));
      HIPCHK(hipHostMalloc(&h_body_solve_, sizeof(int32_t) * body_cap_));
      clear_graphs();
    }
    for (Solve *s : members_) {
      std::fill(h_tile_solve_ + s->desc.tile_base, h_tile_solve_ + s->desc.tile_base + s->tiles(),
                s->slot);
      std::fill(h_body_solve_ + s->desc.body_base, h_body_solve_ + s->desc.body_base + s->nb,
                s->slot);
    }
    BatchHeader &hh = *((BatchHeader *)((SolveDesc *)h_one_ + 2) + 1);
    hh.total_tiles = T;
    hh.total_bodies = (int32_t)B;
    hh.nsolves = (int32_t)members_.size();
    hh.solo_slot = members_.size() == 1 ? members_[0]->slot : -1;
    hh.natural = natural_order() ? 1 : 0;
    if (T) HIPCHK(hipMemcpyAsync(d_tile_solve_, h_tile_solve_, sizeof(int32_t) * T,
                                 hipMemcpyHostToDevice, stream_));
    if (B) HIPCHK(hipMemcpyAsync(d_body_solve_, h_body_solve_, sizeof(int32_t) * B,
                                 hipMemcpyHostToDevice, stream_));
    HIPCHK(hipMemcpyAsync(d_hdr_, &hh, sizeof(BatchHeader), hipMemcpyHostToDevice, stream_));
    HIPCHK(hipEventRecord(table_ev_, stream_));
    // population addressing: one buffer resource while a population buffer (9 planes)
    // stays under 2 GB, 32-bit plane offsets while a plane stays under 2 GB, else 64-bit
    int addr = 0;
    for (Solve *s : members_) {
      const uint64_t pb = pop_half_bytes(s->prm) / kQ;
      const int a = kQ * pb < (1ull << 31) ? 0 : (pb < (1ull << 31) ? 1 : 2);
      addr = std::max(addr, a);
    }
    if (addr != addr_) {
      addr_ = addr;
      clear_graphs();
    }
    // non-temporal population stores once the members' populations together exceed the
    // last-level cache (rows start on 128-byte lines: row_pitch)
    uint64_t total_pop = 0;
    for (Solve *s : members_) total_pop += pop_bytes(s->prm);
    for (Solve *s : members_) s->desc.store_nt = total_pop > kStoreNtMinBytes ? 1 : 0;
    bool open = false;
    for (Solve *s : members_) open = open || s->prm.x_boundary != DILBM_XBC_PERIODIC;
    if (open != open_) {
      open_ = open;
      clear_graphs();
    }
    const bool grid_change =
        collide_grid_for(T) != collide_grid_ || bodies_grid_for(B) != bodies_grid_;
    total_tiles_ = T;
    total_bodies_ = (int)B;
    if (grid_change) {
      collide_grid_ = collide_grid_for(T);
      bodies_grid_ = bodies_grid_for(B);
      clear_graphs();
    }
    dirty_ = false;
  }

  // Collide order: FP32 populations in whole-row 256 x 1 tiles go tile b -> block b, so
  // consecutive tiles (neighbouring row segments) run on the eight XCDs at once: 5.8 TB/s
  // against 5.4 for the best chunked order in a copy probe with the same access pattern,
  // 6% faster for the FP32 step.  Other shapes, and FP16 (whose natural-order step is 25%
  // slower), sweep XCD-contiguous chunks.
  bool natural_order() const {
    return (storage_ == DILBM_STORE_FP32 && kTileTX[shape_] == 256) || shape_ == kPairShape;
  }

  int collide_grid_for(int64_t T) {
    if (natural_order()) return (int)std::max<int64_t>(1, std::min<int64_t>(T, (int64_t)1 << 30));
    // a persistent grid: each block sweeps one contiguous chunk of tiles of a set length
    // (per-block set-up is paid once per chunk; shorter chunks keep the tiles in flight
    // closer together), and at least the blocks resident at once while tiles last
    int &bpc = blocks_per_cu_[shape_][storage_][addr_][open_ ? 1 : 0];
    if (bpc == 0) bpc = std::max(1, collide_blocks_per_cu(shape_, storage_, addr_, open_));
    const int64_t chunk = storage_ == DILBM_STORE_FP16 ? DILBM_CHUNK_FP16 : DILBM_CHUNK_FP32;
    const int64_t resident = (int64_t)num_cu_ * bpc;
    int64_t g = chunk > 0 ? std::max(std::min(T, resident), (T + chunk - 1) / chunk) : T;
    g = std::min<int64_t>(g, (int64_t)1 << 30);
    g = std::max<int64_t>(8, (g + 7) / 8 * 8);
    return (int)g;
  }
  int bodies_grid_for(int64_t B) const {
    int64_t g = (B + 3) / 4;  // one wave per body, four waves per block
    g = std::min<int64_t>(g, (int64_t)num_cu_ * 16);
    return (int)std::max<int64_t>(1, g);
  }

  void launch_steps(int K, bool timed) {
    for (int k = 0; k < K; ++k) {
      if (timed) {
        if (timing_used_ == (int)timing_ev_.size()) {
          hipEvent_t a, b;
          HIPCHK(hipEventCreate(&a));
          HIPCHK(hipEventCreate(&b));
          timing_ev_.push_back({a, b});
        }
        HIPCHK(hipEventRecord(timing_ev_[timing_used_].first, stream_));
      }
      HIPCHK(launch_collide(shape_, storage_, addr_, open_, collide_grid_, stream_, d_descs_,
                            d_tile_solve_, d_hdr_, k));
      if (timed) {
        HIPCHK(hipEventRecord(timing_ev_[timing_used_].second, stream_));
        ++timing_used_;
      }
      if (total_bodies_ > 0)
        HIPCHK(launch_bodies(false, bodies_grid_, stream_, d_descs_, d_body_solve_, d_hdr_, k));
    }
    if (timed && timing_used_ >= 1024) collect_timing();
  }

  hipGraphExec_t graph_for(int K) {
    const int key = K * 2 + (total_bodies_ > 0 ? 1 : 0);
    auto it = graphs_.find(key);
    if (it != graphs_.end()) return it->second;
    // one graph per chunk length in use (the full length and a remainder or two); a
    // caller that keeps changing lengths re-captures instead of piling up graphs
    if (graphs_.size() >= 8) clear_graphs();
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(stream_, hipStreamCaptureModeRelaxed));
    try {
      launch_steps(K, false);
    } catch (...) {
      (void)hipStreamEndCapture(stream_, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIPCHK(hipStreamEndCapture(stream_, &g));
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(e);
    graphs_[key] = ex;
    return ex;
  }

  void clear_graphs() {
    if (graphs_.empty()) return;
    (void)hipStreamSynchronize(stream_);
    for (auto &kv : graphs_) (void)hipGraphExecDestroy(kv.second);
    graphs_.clear();
  }

  int device_;
  hipStream_t stream_ = nullptr;
  hipStream_t aux_ = nullptr;
  bool own_stream_ = false;
  int num_cu_ = 256;
  int shape_ = 0;
  int storage_ = 0;
  int graph_steps_ = 32;
  bool persistent_ = false;
  int addr_ = 0;
  int blocks_per_cu_[kNumTileShapes][2][3][2] = {};
  bool open_ = false;  // some member has open ends in x
  std::vector<Solve *> members_;
  std::vector<bool> slot_used_;
  bool dirty_ = true;
  // device tables
  SolveDesc *d_descs_ = nullptr;
  int desc_cap_ = 0;
  int32_t *d_tile_solve_ = nullptr;
  int32_t *h_tile_solve_ = nullptr;
  int64_t tile_cap_ = 0;
  int32_t *d_body_solve_ = nullptr;
  int32_t *h_body_solve_ = nullptr;
  int64_t body_cap_ = 0;
  BatchHeader *d_hdr_ = nullptr;
  int32_t *d_err_ = nullptr;
  int32_t *h_err_ = nullptr;
  int32_t *h_flag_ = nullptr;
  hipEvent_t flag_ev_ = nullptr;
  int err_cap_ = 0;
  int64_t total_tiles_ = 0;
  int total_bodies_ = 0;
  int collide_grid_ = 8;
  int bodies_grid_ = 1;
  // staging
  void *h_ring_[kRing] = {};
  size_t ring_bytes_[kRing] = {};
  hipEvent_t ring_ev_[kRing] = {};
  int ring_pos_ = 0;
  hipEvent_t table_ev_ = nullptr;
  SolveDesc *d_one_desc_ = nullptr;
  BatchHeader *d_one_hdr_ = nullptr;
  int32_t *d_one_bodies_ = nullptr;
  int one_bodies_cap_ = 0;
  void *h_one_ = nullptr;
  hipEvent_t one_ev_[2] = {};
  // graphs
  std::map<int, hipGraphExec_t> graphs_;
  // timing
  bool timing_ = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> timing_ev_;
  int timing_used_ = 0;
  double timed_ms_ = 0.0;
  int64_t timed_launches_ = 0;
  std::vector<float> launch_ms_;  // every timed collide launch, in launch order
};

// ---------------------------------------------------------------------------------------
// solve setup shared by the solver and the pool

void upload_bodies(Solve &s, hipStream_t st, const double *pos, const double *vel,
                   const double *omega, const double *radius, const double *density,
                   const uint8_t *fixed) {
  const int nb = s.nb;
  const int p = s.parity();
  double rmax = 0.0;
  for (int b = 0; b < nb; ++b) rmax = std::max(rmax, radius[b]);
  s.desc.rmax = rmax;
  // host arrays in the device SoA order
  std::vector<double> state(5 * (size_t)std::max(nb, 1), 0.0);
  std::vector<double> cst(5 * (size_t)std::max(nb, 1), 0.0);
  const double nx = s.prm.nx, ny = s.prm.ny;
  for (int b = 0; b < nb; ++b) {
    double x = std::fmod(pos[2 * b], nx);
    if (x < 0) x += nx;
    if (x >= nx) x -= nx;
    double y = std::fmod(pos[2 * b + 1], ny);
    if (y < 0) y += ny;
    if (y >= ny) y -= ny;
    state[b] = x;
    state[nb + b] = y;
    state[2 * nb + b] = vel ? vel[2 * b] : 0.0;
    state[3 * nb + b] = vel ? vel[2 * b + 1] : 0.0;
    state[4 * nb + b] = omega ? omega[b] : 0.0;
    const double R = radius[b], m = density[b] * M_PI * R * R;
    cst[b] = R;
    cst[nb + b] = density[b];
    cst[2 * nb + b] = m;
    cst[3 * nb + b] = 0.5 * m * R * R;
    cst[4 * nb + b] = (fixed && fixed[b]) ? 1.0 : 0.0;
  }
  if (nb > 0) {
    HIPCHK(hipMemcpyAsync(s.desc.bstate[p], state.data(), sizeof(double) * 5 * nb,
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync((void *)s.desc.bconst, cst.data(), sizeof(double) * 5 * nb,
                          hipMemcpyHostToDevice, st));
  }
  HIPCHK(launch_fill_f64(s.desc.acc[0], 2 * acc_words(nb, 3), 0.0, st));
  HIPCHK(hipStreamSynchronize(st));  // the host vectors die here
}

// the fluid at rest (rho = rho0, u = 0) at the solve's current step
void init_populations(Engine &eng, Solve &s, hipStream_t st) {
  SolveDesc *dd = eng.one_desc(s, st, 0);
  HIPCHK(launch_rest_pops(s.prm.storage, (int64_t)kQ * s.prm.nx * s.prm.ny, st, dd));
}

// copy a body-buffer range to the host (synchronous on st)
void d2h(void *dst, const void *src, size_t bytes, hipStream_t st) {
  if (!bytes) return;
  HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
}

void get_particles_of(Solve &s, hipStream_t st, double *pos, double *vel, double *omega) {
  const int nb = s.nb;
  if (nb == 0) return;
  std::vector<double> h(5 * (size_t)nb);
  d2h(h.data(), s.desc.bstate[s.parity()], sizeof(double) * 5 * nb, st);
  for (int b = 0; b < nb; ++b) {
    if (pos) {
      pos[2 * b] = h[b];
      pos[2 * b + 1] = h[nb + b];
    }
    if (vel) {
      vel[2 * b] = h[2 * nb + b];
      vel[2 * b + 1] = h[3 * nb + b];
    }
    if (omega) omega[b] = h[4 * nb + b];
  }
}

void get_forces_of(Solve &s, hipStream_t st, double *force, double *torque, double *wall) {
  const int nb = s.nb;
  std::vector<double> h((size_t)acc_words(nb, 3), 0.0);
  if (s.forces_valid && s.steps_done > 0)
    d2h(h.data(), s.desc.acc[(s.steps_done - 1) & 1], sizeof(double) * h.size(), st);
  for (int b = 0; b < nb; ++b) {
    if (force) {
      force[2 * b] = h[3 * b];
      force[2 * b + 1] = h[3 * b + 1];
    }
    if (torque) torque[b] = h[3 * b + 2];
  }
  if (wall) {  // the sum of the wall slots
    wall[0] = wall[1] = 0.0;
    for (int k = 0; k < kWallSlots; ++k) {
      wall[0] += h[wall_base(3 * nb) + k * kWallSlotWords];
      wall[1] += h[wall_base(3 * nb) + k * kWallSlotWords + 1];
    }
  }
}

void check_region(const Solve &s, Region rg) {
  if (rg.w < 1 || rg.h < 1 || rg.x < 0 || rg.y < 0 || rg.x + rg.w > s.prm.nx ||
      rg.y + rg.h > s.prm.ny)
    fail(DILBM_EINVAL, "region outside the lattice");
}

// rho, u of the region through the device staging buffer b (3 w h doubles) into the host
// arrays (synchronous on st)
void fields_through(Engine &eng, Solve &s, hipStream_t st, double *b, Region rg, double *rho,
                    double *ux, double *uy) {
  const uint64_t n = (uint64_t)rg.w * rg.h;
  SolveDesc *dd = eng.one_desc(s, st, 1);
  const int64_t ntiles = (int64_t)((rg.x + rg.w - 1) / s.desc.tx - rg.x / s.desc.tx + 1) *
                         ((rg.y + rg.h - 1) / s.desc.ty - rg.y / s.desc.ty + 1);
  HIPCHK(launch_fields(s.shape, s.prm.storage, ntiles, st, dd, s.parity(), rg, b, b + n,
                       b + 2 * n));
  if (rho) HIPCHK(hipMemcpyAsync(rho, b, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  if (ux) HIPCHK(hipMemcpyAsync(ux, b + n, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  if (uy) HIPCHK(hipMemcpyAsync(uy, b + 2 * n, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
}

void get_fields_of(Engine &eng, Solve &s, hipStream_t st, double **scratch, uint64_t *scratch_n,
                   Region rg, double *rho, double *ux, double *uy) {
  check_region(s, rg);
  const uint64_t n = (uint64_t)rg.w * rg.h;
  if (*scratch_n < n) {
    HIPCHK(hipStreamSynchronize(st));
    (void)hipFree(*scratch);
    *scratch = nullptr;
    *scratch_n = 0;
    HIPCHK(hipMalloc(scratch, sizeof(double) * 3 * n));
    *scratch_n = n;
  }
  fields_through(eng, s, st, *scratch, rg, rho, ux, uy);
}

// ---------------------------------------------------------------------------------------
// Staging for dilbm_get_fields_region_noalloc: a fixed device array, so that the call
// allocates nothing.  Each GPU holds its own copy until the process ends; every call on a
// GPU shares it (calls that overlap on one GPU race).  Host code never uses the array's
// name as an address: the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device with that device current.

constexpr int64_t kNoAllocMaxNodes = (int64_t)1 << 20;  // 3 x 8 MiB of FP64
static __device__ __align__(256) double scratch[3 * kNoAllocMaxNodes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

double *scratch_on(int device) {
  if (device < 0 || device >= kMaxDevices) fail(DILBM_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    HIPCHK(hipSetDevice(device));
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(DILBM_EDEVICE, "no device address for the staging array");
    g_scratch_ptr[device] = (double *)p;
  }
  return g_scratch_ptr[device];
}

}  // namespace dilbm

// =======================================================================================
// C ABI

using namespace dilbm;

struct dilbm_solver {
  std::unique_ptr<Engine> eng;
  Solve s;
  std::string last_error;
  double *scratch = nullptr;
  uint64_t scratch_n = 0;
};

struct dilbm_pool {
  std::unique_ptr<Engine> eng;
  std::unique_ptr<Arena> arena;
  void *own_arena = nullptr;
  std::map<int64_t, std::unique_ptr<Solve>> solves;
  std::vector<std::pair<hipEvent_t, Mem>> deferred;  // memory freed once the event is done
  int64_t next_ticket = 1;
  int pending_shape = -1;
  std::string last_error;
  double *scratch = nullptr;
  uint64_t scratch_n = 0;
  // error words of the members after the last enqueued chunk, copied asynchronously into
  // pinned memory; `poll_who` names the (ticket, slot) pairs the copy covers
  int32_t *h_poll = nullptr;
  int poll_cap = 0;
  hipEvent_t poll_ev = nullptr;
  bool poll_pending = false;
  std::vector<std::pair<int64_t, int>> poll_who;
};

namespace {

template <class F>
dilbm_status guard(std::string *err, F &&f) {
  try {
    f();
    return DILBM_OK;
  } catch (const Fail &e) {
    if (err) *err = e.msg;
    g_thread_error = e.msg;
    return e.st;
  } catch (const std::bad_alloc &) {
    if (err) *err = "host allocation failed";
    g_thread_error = "host allocation failed";
    return DILBM_ENOMEM;
  } catch (...) {
    if (err) *err = "unexpected exception";
    g_thread_error = "unexpected exception";
    return DILBM_EDEVICE;
  }
}

void check_usable(dilbm_solver *s) {
  if (s->s.poison != DILBM_OK) fail(DILBM_ESTATE, "handle poisoned: " + s->s.err);
}

void raise_errors(Solve &s, int32_t e) {
  if (e & kErrInternal) {
    s.poison = DILBM_EDEVICE;
    s.err = "internal error: a kernel met an out-of-range body index";
    fail(DILBM_EDEVICE, s.err);
  }
  if (e & kErrCapacity) {
    s.poison = DILBM_ECAPACITY;
    s.err = "a tile body list overflowed; raise list_capacity";
    fail(DILBM_ECAPACITY, s.err);
  }
  if (e & kErrUnstable) {
    s.poison = DILBM_EUNSTABLE;
    s.err = "unstable: rho <= 0, |u| > 0.5 or a non-finite value";
    fail(DILBM_EUNSTABLE, s.err);
  }
}

void poll_errors(Engine &eng, Solve &s) { raise_errors(s, eng.read_error_of(s, eng.stream())); }

void process_deferred(dilbm_pool *p) {
  auto &v = p->deferred;
  for (size_t i = 0; i < v.size();) {
    if (hipEventQuery(v[i].first) == hipSuccess) {
      (void)hipEventDestroy(v[i].first);
      mem_free(v[i].second);
      v[i] = v.back();
      v.pop_back();
    } else {
      ++i;
    }
  }
}

}  // namespace

extern "C" {

void dilbm_params_init(dilbm_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->abi_version = DILBM_ABI_VERSION;
  p->tau = 0.8;
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
  p->storage = DILBM_STORE_FP32;
  p->fp16_scale_log2 = DILBM_FP16_SCALE_AUTO;
  p->list_capacity = 0;
  p->tile = -1;
  p->x_boundary = DILBM_XBC_PERIODIC;
  p->inlet_kind = DILBM_INLET_VELOCITY;
  p->inlet_profile = 0;
  p->outlet_kind = DILBM_OUTLET_PRESSURE;
  p->inlet_density = 1.0;
  p->outlet_density = 1.0;
  p->device = 0;
  p->stream = nullptr;
}

int32_t dilbm_num_tile_shapes(void) { return kNumTileShapes; }

dilbm_status dilbm_tile_shape(int32_t id, int32_t *tx, int32_t *ty) {
  if (id < 0 || id >= kNumTileShapes) return DILBM_EINVAL;
  if (tx) *tx = kTileTX[id];
  if (ty) *ty = kTileTY[id];
  return DILBM_OK;
}

dilbm_status dilbm_footprint(const dilbm_params *p, int32_t n_bodies, uint64_t *bytes) {
  return guard(nullptr, [&] {
    validate(p);
    if (n_bodies < 0 || !bytes) fail(DILBM_EINVAL, "bad footprint query");
    *bytes = pop_bytes(*p) + body_layout(*p, n_bodies).total;
  });
}

dilbm_status dilbm_create(const dilbm_params *p, dilbm_solver **out) {
  if (!out) return DILBM_EINVAL;
  *out = nullptr;
  std::unique_ptr<dilbm_solver> h(new (std::nothrow) dilbm_solver);
  if (!h) return DILBM_ENOMEM;
  dilbm_status st = guard(nullptr, [&] {
    validate(p);
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (p->device < 0 || p->device >= ndev) fail(DILBM_EINVAL, "no such device");
    h->eng.reset(new Engine(p->device, p->stream));
    Solve &s = h->s;
    s.prm = *p;
    s.nb = 0;
    s.shape = p->tile >= 0 ? p->tile : default_shape(*p);
    h->eng->set_storage(p->storage);
    h->eng->set_shape(s.shape);
    s.L = body_layout(*p, 0);
    s.pops = mem_alloc(nullptr, pop_bytes(*p));
    s.body = mem_alloc(nullptr, s.L.total);
    fill_desc(s);
    h->eng->add(&s);
    init_populations(*h->eng, s, h->eng->stream());
    HIPCHK(launch_zero_bytes(s.body.ptr, (int64_t)s.body.bytes, h->eng->stream()));
    HIPCHK(hipStreamSynchronize(h->eng->stream()));
  });
  if (st != DILBM_OK) {
    if (h->eng) {
      mem_free(h->s.pops);
      mem_free(h->s.body);
    }
    return st;
  }
  *out = h.release();
  return DILBM_OK;
}

dilbm_status dilbm_set_particles(dilbm_solver *h, int32_t n, const double *pos, const double *vel,
                                 const double *omega, const double *radius, const double *density,
                                 const uint8_t *fixed) {
  if (!h) return DILBM_EINVAL;
  return guard(&h->last_error, [&] {
    check_usable(h);
    validate_bodies(n, pos, vel, omega, radius, density);
    HIPCHK(hipSetDevice(h->eng->device()));
    Solve &s = h->s;
    hipStream_t st = h->eng->stream();
    BodyLayout L = body_layout(s.prm, n);
    HIPCHK(hipStreamSynchronize(st));
    Mem nm = mem_alloc(nullptr, L.total);  // strong guarantee: allocate before freeing
    mem_free(s.body);
    s.body = nm;
    s.L = L;
    s.nb = n;
    const int32_t *err = s.desc.err;
    fill_desc(s);
    s.desc.err = const_cast<int32_t *>(err);
    HIPCHK(launch_zero_bytes(s.body.ptr, (int64_t)s.body.bytes, st));
    upload_bodies(s, st, pos, vel, omega, radius, density, fixed);
    h->eng->bin_current(s, st);
    s.forces_valid = false;
    h->eng->mark_dirty();
    HIPCHK(hipStreamSynchronize(st));
    poll_errors(*h->eng, s);
  });
}

dilbm_status dilbm_set_populations(dilbm_solver *h, const double *f_dev) {
  if (!h || !f_dev) return DILBM_EINVAL;
  return guard(&h->last_error, [&] {
    check_usable(h);
    HIPCHK(hipSetDevice(h->eng->device()));
    Solve &s = h->s;
    hipStream_t st = h->eng->stream();
    const int64_t count = (int64_t)kQ * s.prm.nx * s.prm.ny;
    double *tmp = nullptr;
    HIPCHK(hipMalloc(&tmp, sizeof(double) * count));
    hipError_t e = hipMemcpyAsync(tmp, f_dev, sizeof(double) * count, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
      SolveDesc *dd = h->eng->one_desc(s, st, 0);
      e = launch_set_pops(s.prm.storage, count, st, dd, s.parity(), tmp);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(tmp);
    HIPCHK(e);
  });
}

dilbm_status dilbm_get_populations(dilbm_solver *h, double *f_dev) {
  if (!h || !f_dev) return DILBM_EINVAL;
  return guard(&h->last_error, [&] {
    HIPCHK(hipSetDevice(h->eng->device()));
    Solve &s = h->s;
    hipStream_t st = h->eng->stream();
    const int64_t count = (int64_t)kQ * s.prm.nx * s.prm.ny;
    double *tmp = nullptr;
    HIPCHK(hipMalloc(&tmp, sizeof(double) * count));
    SolveDesc *dd = h->eng->one_desc(s, st, 0);
    hipError_t e = launch_get_pops(s.prm.storage, count, st, dd, s.parity(), tmp);
    if (e == hipSuccess)
      e = hipMemcpyAsync(f_dev, tmp, sizeof(double) * count, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(tmp);
    HIPCHK(e);
  });
}

dilbm_status dilbm_step(dilbm_solver *h, int64_t nsteps) {
  if (!h) return DILBM_EINVAL;
  return guard(&h->last_error, [&] {
    check_usable(h);
    if (nsteps < 0) fail(DILBM_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return;
    HIPCHK(hipSetDevice(h->eng->device()));
    Engine &eng = *h->eng;
    const int K = eng.graph_steps();
    int64_t left = nsteps;
    bool pending = false;
    while (left > 0) {
      const int k = (int)std::min<int64_t>(left, K);
      eng.run_chunk(k, true);
      left -= k;
      // the flags as of the previous chunk's end: waiting for them leaves this chunk
      // queued, so the device does not idle; a failure stops the call one chunk later
      if (pending) raise_errors(h->s, eng.flag_wait());
      eng.flag_copy_async(h->s);
      pending = true;
    }
    eng.collect_timing();
    HIPCHK(hipStreamSynchronize(eng.stream()));
    // the copy queued after the last chunk has completed with the stream
    raise_errors(h->s, eng.flag_wait());
  });
}

dilbm_status dilbm_get_fields(dilbm_solver *h, double *rho, double *ux, double *uy) {
  if (!h) return DILBM_EINVAL;
  return guard(&h->last_error, [&] {
    HIPCHK(hipSetDevice(h->eng->device()));
    get_fields_of(*h->eng, h->s, h->eng->stream(), &h->scratch, &h->scratch_n,
                  Region{0, 0, h->s.prm.nx, h->s.prm.ny}, rho, ux, uy);
  });
}

dilbm_status dilbm_get_fields_region(dilbm_solver *h, int32_t x0, int32_t y0, int32_t w,
                                     int32_t hgt, double *rho, double *ux, double *uy) {
  if (!h) return DILBM_EINVAL;
  return guard(&h->last_error, [&] {
    HIPCHK(hipSetDevice(h->eng->device()));
    get_fields_of(*h->eng, h->s, h->eng->stream(), &h->scratch, &h->scratch_n,
                  Region{x0, y0, w, hgt}, rho, ux, uy);
  });
}

dilbm_status dilbm_get_fields_region_noalloc(dilbm_solver *h, int32_t x0, int32_t y0, int32_t w,
                                             int32_t hgt, double *rho, double *ux, double *uy) {
  if (!h) return DILBM_EINVAL;
  return guard(&h->last_error, [&] {
    const Region rg{x0, y0, w, hgt};
    check_region(h->s, rg);
    if ((int64_t)w * hgt > kNoAllocMaxNodes)
      fail(DILBM_EINVAL, "region larger than the fixed staging array (2^20 nodes)");
    double *b = scratch_on(h->eng->device());
    HIPCHK(hipSetDevice(h->eng->device()));
    fields_through(*h->eng, h->s, h->eng->stream(), b, rg, rho, ux, uy);
  });
}

dilbm_status dilbm_get_particle_forces(dilbm_solver *h, double *force, double *torque) {
  if (!h) return DILBM_EINVAL;
  return guard(&h->last_error, [&] {
    HIPCHK(hipSetDevice(h->eng->device()));
    get_forces_of(h->s, h->eng->stream(), force, torque, nullptr);
  });
}

dilbm_status dilbm_get_particles(dilbm_solver *h, double *pos, double *vel, double *omega) {
  if (!h) return DILBM_EINVAL;
  return guard(&h->last_error, [&] {
    HIPCHK(hipSetDevice(h->eng->device()));
    get_particles_of(h->s, h->eng->stream(), pos, vel, omega);
  });
}

dilbm_status dilbm_get_wall_force(dilbm_solver *h, double *force) {
  if (!h || !force) return DILBM_EINVAL;
  return guard(&h->last_error, [&] {
    HIPCHK(hipSetDevice(h->eng->device()));
    get_forces_of(h->s, h->eng->stream(), nullptr, nullptr, force);
  });
}

dilbm_status dilbm_get_step_count(dilbm_solver *h, int64_t *steps) {
  if (!h || !steps) return DILBM_EINVAL;
  *steps = h->s.steps_done;
  return DILBM_OK;
}

dilbm_status dilbm_get_body_count(dilbm_solver *h, int32_t *n) {
  if (!h || !n) return DILBM_EINVAL;
  *n = h->s.nb;
  return DILBM_OK;
}

dilbm_status dilbm_set_kernel_timing(dilbm_solver *h, int32_t enable) {
  if (!h) return DILBM_EINVAL;
  return guard(&h->last_error, [&] { h->eng->set_timing(enable != 0); });
}

dilbm_status dilbm_get_kernel_timing(dilbm_solver *h, double *collide_ms, int64_t *launches) {
  if (!h) return DILBM_EINVAL;
  return guard(&h->last_error, [&] {
    h->eng->collect_timing();
    if (collide_ms) *collide_ms = h->eng->timed_ms();
    if (launches) *launches = h->eng->timed_launches();
  });
}

dilbm_status dilbm_get_kernel_launch_times(dilbm_solver *h, double *ms, int64_t cap,
                                           int64_t *count) {
  if (!h || cap < 0 || (cap > 0 && !ms)) return DILBM_EINVAL;
  return guard(&h->last_error, [&] {
    h->eng->collect_timing();
    const std::vector<float> &v = h->eng->launch_ms();
    const int64_t n = std::min<int64_t>(cap, (int64_t)v.size());
    for (int64_t i = 0; i < n; ++i) ms[i] = v[i];
    if (count) *count = (int64_t)v.size();
  });
}

void dilbm_destroy(dilbm_solver *h) {
  if (!h) return;
  try {
    if (h->eng) {
      (void)hipSetDevice(h->eng->device());
      (void)hipStreamSynchronize(h->eng->stream());
      h->eng->remove(&h->s);
    }
    mem_free(h->s.pops);
    mem_free(h->s.body);
    (void)hipFree(h->scratch);
    h->eng.reset();
  } catch (...) {
  }
  delete h;
}

const char *dilbm_last_error(const dilbm_solver *h) {
  if (!h) return g_thread_error.c_str();
  return h->last_error.c_str();
}

// ---- pool ---------------------------------------------------------------------------

dilbm_status dilbm_pool_create(int32_t device, void *stream, void *arena, uint64_t arena_bytes,
                               dilbm_pool **out) {
  if (!out) return DILBM_EINVAL;
  *out = nullptr;
  std::unique_ptr<dilbm_pool> p(new (std::nothrow) dilbm_pool);
  if (!p) return DILBM_ENOMEM;
  dilbm_status st = guard(nullptr, [&] {
    if (arena_bytes < (1u << 20)) fail(DILBM_EINVAL, "arena_bytes must be at least 1 MiB");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) fail(DILBM_EINVAL, "no such device");
    p->eng.reset(new Engine(device, stream));
    p->eng->set_persistent(true);
    char *base = (char *)arena;
    if (!base) {
      HIPCHK(hipMalloc(&p->own_arena, arena_bytes));
      base = (char *)p->own_arena;
    }
    p->arena.reset(new Arena(base, arena_bytes));
  });
  if (st != DILBM_OK) {
    if (p->own_arena) (void)hipFree(p->own_arena);
    return st;
  }
  *out = p.release();
  return DILBM_OK;
}

dilbm_status dilbm_pool_submit(dilbm_pool *pool, const dilbm_params *prm, int32_t n,
                               const double *pos, const double *vel, const double *omega,
                               const double *radius, const double *density,
                               const uint8_t *fixed, int64_t nsteps, int64_t *ticket) {
  if (!pool || !ticket) return DILBM_EINVAL;
  return guard(&pool->last_error, [&] {
    validate(prm);
    validate_bodies(n, pos, vel, omega, radius, density);
    if (nsteps < 0) fail(DILBM_EINVAL, "nsteps must be >= 0");
    Engine &eng = *pool->eng;
    HIPCHK(hipSetDevice(eng.device()));
    if (!eng.members().empty() && prm->storage != eng.storage())
      fail(DILBM_EINVAL, "all members of a pool share one storage type");
    const int want = pool->solves.empty() && eng.members().empty() && pool->pending_shape >= 0
                         ? pool->pending_shape
                         : eng.shape();
    if (!shape_fits(want, *prm))
      fail(DILBM_EINVAL, "the pool's tile shape 5 needs FP16 storage and an even nx");
    process_deferred(pool);
    const BodyLayout L = body_layout(*prm, n);
    const uint64_t need = pop_bytes(*prm) + L.total;
    if (need > pool->arena->size()) fail(DILBM_ENOMEM, "solve larger than the whole arena");
    std::unique_ptr<Solve> s(new Solve);
    s->prm = *prm;
    s->nb = n;
    s->L = L;
    s->shape = eng.shape();
    if (pool->solves.empty() && eng.members().empty()) {
      eng.set_storage(prm->storage);
      if (pool->pending_shape >= 0) eng.set_shape(pool->pending_shape);
      s->shape = eng.shape();
    }
    s->pops = mem_alloc(pool->arena.get(), pop_bytes(*prm));
    try {
      s->body = mem_alloc(pool->arena.get(), L.total);
    } catch (...) {
      mem_free(s->pops);
      throw;
    }
    s->target = nsteps;
    fill_desc(*s);
    hipStream_t st = eng.stream();
    eng.add(s.get());
    try {
      init_populations(eng, *s, st);
      HIPCHK(launch_zero_bytes(s->body.ptr, (int64_t)s->body.bytes, st));
      upload_bodies(*s, st, pos, vel, omega, radius, density, fixed);
      eng.bin_current(*s, st);
      HIPCHK(hipEventCreateWithFlags(&s->done_ev, hipEventDisableTiming));
      HIPCHK(hipEventRecord(s->done_ev, st));
    } catch (...) {
      (void)hipStreamSynchronize(st);
      eng.remove(s.get());
      mem_free(s->pops);
      mem_free(s->body);
      if (s->done_ev) (void)hipEventDestroy(s->done_ev);
      throw;
    }
    s->ticket = pool->next_ticket++;
    *ticket = s->ticket;
    if (nsteps == 0) {
      s->finished = true;
      eng.leave(s.get());
    }
    pool->solves[s->ticket] = std::move(s);
  });
}

// A member leaves the pool: its completion is marked by an event after the work enqueued
// so far.
static void finish_member(Engine &eng, Solve *s) {
  HIPCHK(hipEventRecord(s->done_ev, eng.stream()));
  s->finished = true;
  eng.leave(s);
}

// The sticky error bits of a pool solve, as its status and message.
static void poison_from_flags(Solve *s, int32_t e) {
  if (s->poison != DILBM_OK) return;
  if (e & kErrInternal) {
    s->poison = DILBM_EDEVICE;
    s->err = "internal error: a kernel met an out-of-range body index";
  } else if (e & kErrCapacity) {
    s->poison = DILBM_ECAPACITY;
    s->err = "a tile body list overflowed";
  } else if (e & kErrUnstable) {
    s->poison = DILBM_EUNSTABLE;
    s->err = "unstable";
  }
}

// Wait for the members' error words copied after the previous chunk and stop every
// member whose solve has failed (it runs at most the one chunk enqueued since).
static void poll_wait(dilbm_pool *pool) {
  if (!pool->poll_pending) return;
  Engine &eng = *pool->eng;
  HIPCHK(hipEventSynchronize(pool->poll_ev));
  pool->poll_pending = false;
  for (const auto &w : pool->poll_who) {
    auto it = pool->solves.find(w.first);
    if (it == pool->solves.end()) continue;  // released since
    Solve *s = it->second.get();
    const int32_t e = pool->h_poll[w.second];
    if (e == 0 || s->slot != w.second) continue;
    poison_from_flags(s, e);
    if (!s->finished) finish_member(eng, s);
  }
}

// Copy the members' error words after the work enqueued so far (asynchronous).
static void poll_copy_async(dilbm_pool *pool) {
  Engine &eng = *pool->eng;
  const int n = eng.err_slots();
  if (n == 0 || eng.members().empty()) return;
  if (!pool->poll_ev) HIPCHK(hipEventCreateWithFlags(&pool->poll_ev, hipEventDisableTiming));
  if (n > pool->poll_cap) {
    (void)hipHostFree(pool->h_poll);
    pool->h_poll = nullptr;
    pool->poll_cap = 0;
    HIPCHK(hipHostMalloc(&pool->h_poll, sizeof(int32_t) * n));
    pool->poll_cap = n;
  }
  HIPCHK(hipMemcpyAsync(pool->h_poll, eng.err_table(), sizeof(int32_t) * n,
                        hipMemcpyDeviceToHost, eng.stream()));
  HIPCHK(hipEventRecord(pool->poll_ev, eng.stream()));
  pool->poll_who.clear();
  for (Solve *s : eng.members()) pool->poll_who.push_back({s->ticket, s->slot});
  pool->poll_pending = true;
}

dilbm_status dilbm_pool_run(dilbm_pool *pool, int32_t steps) {
  if (!pool || steps < 0) return DILBM_EINVAL;
  return guard(&pool->last_error, [&] {
    Engine &eng = *pool->eng;
    HIPCHK(hipSetDevice(eng.device()));
    process_deferred(pool);
    int left = steps;
    const int K = eng.graph_steps();
    while (left > 0 && !eng.members().empty()) {
      const int k = std::min(left, K);
      eng.run_chunk(k, true);
      left -= k;
      // members whose last step is enqueued leave the member set
      std::vector<Solve *> done;
      for (Solve *s : eng.members())
        if (s->remaining() <= 0) done.push_back(s);
      for (Solve *s : done) finish_member(eng, s);
      // the flags as of the previous chunk's end: waiting for them leaves this chunk
      // queued, so the device does not idle; a failed member stops one chunk later
      poll_wait(pool);
      poll_copy_async(pool);
    }
  });
}

dilbm_status dilbm_pool_sync(dilbm_pool *pool) {
  if (!pool) return DILBM_EINVAL;
  return guard(&pool->last_error, [&] {
    HIPCHK(hipSetDevice(pool->eng->device()));
    HIPCHK(hipStreamSynchronize(pool->eng->stream()));
    poll_wait(pool);
    process_deferred(pool);
  });
}

static Solve *find_ticket(dilbm_pool *pool, int64_t t) {
  auto it = pool->solves.find(t);
  if (it == pool->solves.end()) fail(DILBM_EINVAL, "unknown ticket");
  return it->second.get();
}

dilbm_status dilbm_pool_query(dilbm_pool *pool, int64_t ticket, int64_t *steps_enqueued,
                              int32_t *done) {
  if (!pool) return DILBM_EINVAL;
  return guard(&pool->last_error, [&] {
    Solve *s = find_ticket(pool, ticket);
    if (steps_enqueued) *steps_enqueued = s->steps_done;
    if (done) *done = (s->finished && hipEventQuery(s->done_ev) == hipSuccess) ? 1 : 0;
  });
}

// wait (on the auxiliary stream) for the ticket's enqueued work, then check its flags
static void ready_for_results(dilbm_pool *pool, Solve *s) {
  Engine &eng = *pool->eng;
  HIPCHK(hipSetDevice(eng.device()));
  HIPCHK(hipEventSynchronize(s->done_ev));
  if (s->poison == DILBM_OK) poison_from_flags(s, eng.read_error_of(*s, eng.aux()));
}

dilbm_status dilbm_pool_get_fields(dilbm_pool *pool, int64_t ticket, double *rho, double *ux,
                                   double *uy) {
  if (!pool) return DILBM_EINVAL;
  return guard(&pool->last_error, [&] {
    Solve *s = find_ticket(pool, ticket);
    if (!s->finished) fail(DILBM_ESTATE, "ticket still running; results need all its steps");
    ready_for_results(pool, s);
    get_fields_of(*pool->eng, *s, pool->eng->aux(), &pool->scratch, &pool->scratch_n,
                  Region{0, 0, s->prm.nx, s->prm.ny}, rho, ux, uy);
    if (s->poison != DILBM_OK) fail(s->poison, s->err);
  });
}

dilbm_status dilbm_pool_get_particles(dilbm_pool *pool, int64_t ticket, double *pos, double *vel,
                                      double *omega) {
  if (!pool) return DILBM_EINVAL;
  return guard(&pool->last_error, [&] {
    Solve *s = find_ticket(pool, ticket);
    if (!s->finished) fail(DILBM_ESTATE, "ticket still running; results need all its steps");
    ready_for_results(pool, s);
    get_particles_of(*s, pool->eng->aux(), pos, vel, omega);
    if (s->poison != DILBM_OK) fail(s->poison, s->err);
  });
}

dilbm_status dilbm_pool_get_particle_forces(dilbm_pool *pool, int64_t ticket, double *force,
                                            double *torque) {
  if (!pool) return DILBM_EINVAL;
  return guard(&pool->last_error, [&] {
    Solve *s = find_ticket(pool, ticket);
    if (!s->finished) fail(DILBM_ESTATE, "ticket still running; results need all its steps");
    ready_for_results(pool, s);
    get_forces_of(*s, pool->eng->aux(), force, torque, nullptr);
    if (s->poison != DILBM_OK) fail(s->poison, s->err);
  });
}

dilbm_status dilbm_pool_release(dilbm_pool *pool, int64_t ticket) {
  if (!pool) return DILBM_EINVAL;
  return guard(&pool->last_error, [&] {
    Engine &eng = *pool->eng;
    HIPCHK(hipSetDevice(eng.device()));
    auto it = pool->solves.find(ticket);
    if (it == pool->solves.end()) fail(DILBM_EINVAL, "unknown ticket");
    Solve *s = it->second.get();
    eng.remove(s);
    // the memory goes back once everything enqueued so far (which may still touch it)
    // has completed
    hipEvent_t ev;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ev, eng.stream()));
    hipEvent_t ev2;
    HIPCHK(hipEventCreateWithFlags(&ev2, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ev2, eng.stream()));
    pool->deferred.push_back({ev, s->pops});
    pool->deferred.push_back({ev2, s->body});
    s->pops = Mem{};
    s->body = Mem{};
    if (s->done_ev) (void)hipEventDestroy(s->done_ev);
    pool->solves.erase(it);
    process_deferred(pool);
  });
}

dilbm_status dilbm_pool_set_launch(dilbm_pool *pool, int32_t graph_steps, int32_t tile) {
  if (!pool) return DILBM_EINVAL;
  return guard(&pool->last_error, [&] {
    if (graph_steps < 1 || graph_steps > 256) fail(DILBM_EINVAL, "graph_steps in [1, 256]");
    if (tile < -1 || tile >= kNumTileShapes) fail(DILBM_EINVAL, "unknown tile shape");
    if (tile >= 0)
      for (Solve *m : pool->eng->members())
        if (!shape_fits(tile, m->prm)) fail(DILBM_EINVAL, "tile shape does not fit a member");
    HIPCHK(hipSetDevice(pool->eng->device()));
    pool->eng->set_graph_steps(graph_steps);
    if (tile >= 0) {
      pool->pending_shape = tile;
      pool->eng->set_shape(tile);
    }
  });
}

dilbm_status dilbm_pool_autotune(dilbm_pool *pool, int32_t steps_per_trial,
                                 int32_t *best_graph_steps, int32_t *best_tile) {
  if (!pool || steps_per_trial < 1) return DILBM_EINVAL;
  return guard(&pool->last_error, [&] {
    Engine &eng = *pool->eng;
    HIPCHK(hipSetDevice(eng.device()));
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    // Time one candidate: the first graph launch of K steps captures the graph (untimed),
    // then whole K-step graph launches covering at least steps_per_trial steps are timed.
    // Every trial step is a real step of the members.  Returns ms per node update, or a
    // negative value when the members ran out of steps.
    auto trial = [&](int tile, int K) -> double {
      if (eng.members().empty()) return -1.0;
      eng.set_shape(tile);
      eng.set_graph_steps(K);
      eng.run_chunk(K, true);
      const int launches = (steps_per_trial + K - 1) / K;
      double nodes = 0;
      for (Solve *s : eng.members())
        nodes += (double)s->prm.nx * s->prm.ny *
                 (double)std::min<int64_t>((int64_t)launches * K, s->remaining());
      if (nodes == 0) return -1.0;
      HIPCHK(hipEventRecord(a, eng.stream()));
      for (int l = 0; l < launches && !eng.members().empty(); ++l) eng.run_chunk(K, true);
      HIPCHK(hipEventRecord(b, eng.stream()));
      HIPCHK(hipEventSynchronize(b));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, a, b));
      return ms / nodes;
    };
    // tile shapes at a short graph, then the graph length at the best shape
    const int k_short = 16, k_long = 128;
    double best = 1e300;
    int bk = eng.graph_steps(), bt = eng.shape();
    for (int tile = 0; tile < kNumTileShapes; ++tile) {
      bool fits = true;
      for (Solve *m : eng.members()) fits = fits && shape_fits(tile, m->prm);
      if (!fits) continue;
      const double t = trial(tile, k_short);
      if (t >= 0 && t < best) {
        best = t;
        bk = k_short;
        bt = tile;
      }
    }
    if (best < 1e300) {
      const double t = trial(bt, k_long);
      if (t >= 0 && t < best) {
        best = t;
        bk = k_long;
      }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    eng.set_shape(bt);
    eng.set_graph_steps(bk);
    pool->pending_shape = bt;
    // members that ran out of steps during the trials leave the member set
    std::vector<Solve *> done;
    for (Solve *s : eng.members())
      if (s->remaining() <= 0) done.push_back(s);
    for (Solve *s : done) {
      HIPCHK(hipEventRecord(s->done_ev, eng.stream()));
      s->finished = true;
      eng.leave(s);
    }
    if (best_graph_steps) *best_graph_steps = bk;
    if (best_tile) *best_tile = bt;
  });
}

dilbm_status dilbm_pool_stats(dilbm_pool *pool, uint64_t *free_bytes, int32_t *members) {
  if (!pool) return DILBM_EINVAL;
  return guard(&pool->last_error, [&] {
    process_deferred(pool);
    if (free_bytes) *free_bytes = pool->arena->free_bytes();
    if (members) *members = (int32_t)pool->eng->members().size();
  });
}

const char *dilbm_pool_last_error(const dilbm_pool *pool) {
  if (!pool) return g_thread_error.c_str();
  return pool->last_error.c_str();
}

void dilbm_pool_destroy(dilbm_pool *pool) {
  if (!pool) return;
  try {
    if (pool->eng) {
      (void)hipSetDevice(pool->eng->device());
      (void)hipStreamSynchronize(pool->eng->stream());
      (void)hipStreamSynchronize(pool->eng->aux());
      for (auto &kv : pool->solves) {
        pool->eng->remove(kv.second.get());
        mem_free(kv.second->pops);
        mem_free(kv.second->body);
        if (kv.second->done_ev) (void)hipEventDestroy(kv.second->done_ev);
      }
      pool->solves.clear();
      for (auto &d : pool->deferred) {
        (void)hipEventSynchronize(d.first);
        (void)hipEventDestroy(d.first);
        mem_free(d.second);
      }
      pool->deferred.clear();
      (void)hipFree(pool->scratch);
      (void)hipHostFree(pool->h_poll);
      if (pool->poll_ev) (void)hipEventDestroy(pool->poll_ev);
      pool->eng.reset();
    }
    pool->arena.reset();
    if (pool->own_arena) (void)hipFree(pool->own_arena);
  } catch (...) {
  }
  delete pool;
}

}  // extern "C"
