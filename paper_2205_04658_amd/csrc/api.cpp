// librlb C ABI: argument validation, workspace layout, launch sequencing and
// error state.  Every device action is enqueued on the lattice's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dirset.hpp"
#include "internal.hpp"

using namespace rlb;

namespace {

thread_local std::string g_err;

rlb_status fail(rlb_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

rlb_status hip_fail(hipError_t e, const char* what) {
  return fail(RLB_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                      \
  do {                                           \
    hipError_t _e = (expr);                      \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

constexpr uint64_t kMagic = 0x4554415453424C52ull;   // "RLBSTATE"
constexpr size_t kHeaderBytes = 256;

struct StateHeader {
  uint64_t magic;
  int32_t version, nx, ny, q;
  int64_t pitch, step;
  double eps_ref, n_ref, tau, cfl;
  uint32_t flags;
};

int planes_of(const rlb_params* p) {
  return (p->flags & RLB_PLANAR) ? 12 : ((p->flags & RLB_FULL26) ? 26 : 17);
}

rlb_status check_params(const rlb_params* p) {
  if (!p) return fail(RLB_EINVAL, "params is null");
  if (p->nx < 4 || p->ny < 4) return fail(RLB_EINVAL, "nx, ny must be >= 4 (got %d x %d)", p->nx, p->ny);
  if ((int64_t)p->ny * (((int64_t)p->nx + 63) / 64 * 64) >= (int64_t)1 << 30)
    return fail(RLB_EINVAL, "ny * (nx rounded up to 64) must be < 2^30");
  if (!std::isfinite(p->tau) || !(p->tau > 0.5)) return fail(RLB_EINVAL, "tau must be finite and > 1/2");
  if (!std::isfinite(p->cfl) || !(p->cfl > 0.0) || p->cfl > 2.0)
    return fail(p->cfl > 2.0 && std::isfinite(p->cfl) ? RLB_EUNSUPPORTED : RLB_EINVAL,
                "cfl must be in (0, 2] (bilinear pull over at most a two-node neighbourhood)");
  if (p->cfl > 1.0 && (p->flags & (RLB_WALLS_Y | RLB_OPEN_X)))
    return fail(RLB_EUNSUPPORTED, "cfl > 1 is supported on periodic lattices (no walls, no open borders)");
  if (p->flags & ~(RLB_WALLS_Y | RLB_FULL26 | RLB_OPEN_X | RLB_PLANAR))
    return fail(RLB_EINVAL, "unknown flags 0x%x", p->flags);
  if ((p->flags & RLB_PLANAR) && (p->flags & RLB_FULL26))
    return fail(RLB_EINVAL, "RLB_PLANAR and RLB_FULL26 select different momentum sets");
  if ((p->flags & RLB_PLANAR) && (p->flags & RLB_OPEN_X))
    return fail(RLB_EUNSUPPORTED, "open x borders are implemented for the 3D momentum set");
  if (!std::isfinite(p->eps_ref) || !std::isfinite(p->n_ref))
    return fail(RLB_EINVAL, "eps_ref and n_ref must be finite");
  // column offsets inside a state row are 32-bit byte offsets
  const int64_t row_bytes = ((int64_t)p->nx + 63) / 64 * 64 * 2 * planes_of(p) * (int64_t)sizeof(float);
  if (row_bytes >= (int64_t)1 << 32)
    return fail(RLB_EINVAL, "a state row of nx = %d nodes takes %lld bytes, must be < 2^32", p->nx,
                (long long)row_bytes);
  return RLB_OK;
}

Workspace layout(const rlb_params* p, int Q, int64_t pitch) {
  Workspace w;
  size_t off = 0;
  const size_t state = align_up((size_t)2 * Q * pitch * sizeof(float));
  w.state_off[0] = off; off += state;
  w.state_off[1] = off; off += state;
  w.mask_off = off; off += align_up((size_t)p->nx * p->ny);
  w.coef_off = off; off += align_up((size_t)kMaxModes * 4 * sizeof(double));
  w.modes_off = off; off += align_up((size_t)kMaxModes * sizeof(int4));
  w.bins_off = off; off += align_up((size_t)(kMaxK + 2) * sizeof(int32_t));
  // series coefficients: (kMaxK + 1) / 8 chunks x 2 halves x 2 components
  // x hi | lo x ny rows, 16 bytes each
  w.table_off = off; off += align_up((size_t)(kMaxK + 1) / 8 * 2 * p->ny * 4 * sizeof(uint4));
  w.phase_off = off; off += align_up((size_t)p->ny * sizeof(double2));
  w.force_off = off; off += align_up((size_t)2 * pitch * sizeof(float));
  // twiddles: (kMaxK + 1) / 8 chunks x 2 halves x hi | lo x nx columns
  w.twiddle_off = off; off += align_up((size_t)(kMaxK + 1) / 8 * 2 * p->nx * 2 * sizeof(uint4));
  w.partial_off = off; off += align_up((size_t)kRedBlocks * 4 * sizeof(double));
  w.desc_off = off; off += align_up(sizeof(LatDesc));
  w.misc_off = off; off += align_up(256);
  w.total = off;
  return w;
}


// Bilinear tap weights per plane, quantised to multiples of 2^-24 with the
// last weight taking the exact remainder, so the four float32 weights sum to
// exactly 1 and streaming does not scale a plane's total.
template <class DS>
void fill_taps(rlb_lattice* lat) {
  const double q = 16777216.0;   // 2^24
  const bool wide = lat->p.cfl > 1.0;
  for (int k = 0; k < DS::Q; ++k) {
    double ax = lat->p.cfl * std::fabs(DS::vx[k]);
    double ay = lat->p.cfl * std::fabs(DS::vy[k]);
    // 1 < cfl <= 2: a displacement of one cell or more starts one cell
    // upstream (taps one and two cells away, fraction in [0, 1])
    lat->shift[k][0] = (uint8_t)(wide && ax >= 1.0);
    lat->shift[k][1] = (uint8_t)(wide && ay >= 1.0);
    if (lat->shift[k][0]) ax -= 1.0;
    if (lat->shift[k][1]) ay -= 1.0;
    const double w00 = std::nearbyint((1 - ax) * (1 - ay) * q) / q;
    const double w10 = std::nearbyint(ax * (1 - ay) * q) / q;
    const double w01 = std::nearbyint((1 - ax) * ay * q) / q;
    const double w11 = 1.0 - w00 - w10 - w01;     // exact: multiples of 2^-24
    lat->tap[k][0] = (float)w00;
    lat->tap[k][1] = (float)w10;
    lat->tap[k][2] = (float)w01;
    lat->tap[k][3] = (float)w11;
  }
}

rlb_status check_lat(const rlb_lattice* lat) {
  if (!lat) return fail(RLB_EINVAL, "lattice is null");
  return RLB_OK;
}

StirArgs stir_args(const rlb_lattice* lat) {
  StirArgs a;
  a.modes = lat->modes;
  a.bins = lat->bins;
  a.coef = lat->coef;
  a.table = lat->table;
  a.phase = lat->phase;
  a.twiddle = lat->twiddle;
  a.scale = lat->stir_scale > 0.0f ? lat->stir_scale : 1.0f;   // 0 before rlb_set_stirring
  a.inv_scale = 1.0f / a.scale;
  a.force = lat->force;
  a.force_pitch = lat->pitch;
  a.row = lat->row;
  a.dstep = lat->dstep;
  a.nmodes = lat->nmodes;
  a.K = lat->K;
  a.nx = lat->p.nx;
  a.ny = lat->p.ny;
  a.amplitude = lat->amp;
  a.seed = lat->seed;
  a.stream = 0;
  return a;
}

rlb_status read_err(rlb_lattice* lat) {
  uint32_t h = 0;
  HIP_TRY(hipMemcpyAsync(&h, lat->err, sizeof h, hipMemcpyDeviceToHost, lat->stream), "read error flag");
  HIP_TRY(hipStreamSynchronize(lat->stream), "stream synchronize");
  if (h & ERR_LANDAU) return fail(RLB_ELANDAU, "a fluid node had no timelike Landau frame (step %lld)", (long long)lat->step);
  if (h & ERR_NONFINITE) return fail(RLB_ENONFINITE, "a population became non-finite (step %lld)", (long long)lat->step);
  return RLB_OK;
}

constexpr int kEvRing = 16;

// Fold the elapsed time of pending event pair i into the totals.
rlb_status drain_event(rlb_lattice* lat, int i) {
  if (!(lat->ev_pending & (1u << i))) return RLB_OK;
  HIP_TRY(hipEventSynchronize(lat->ev[i][1]), "event synchronize");
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, lat->ev[i][0], lat->ev[i][1]), "event elapsed");
  lat->timed_ms += ms;
  lat->timed_launches += 1;
  lat->ev_pending &= ~(1u << i);
  return RLB_OK;
}

rlb_status accumulate_timing(rlb_lattice* lat) {
  for (int i = 0; i < kEvRing; ++i)
    if (rlb_status s = drain_event(lat, i)) return s;
  return RLB_OK;
}

}  // namespace

void rlb::set_error_message(const char* msg) { g_err = msg; }

rlb_status rlb::set_open(rlb_lattice* lat, double bx, double by, double n_in, double eps_out) {
  if (!(lat->p.flags & RLB_OPEN_X)) return fail(RLB_EINVAL, "the lattice was created without RLB_OPEN_X");
  if (!std::isfinite(bx) || !std::isfinite(by) || !(bx * bx + by * by < 1.0))
    return fail(RLB_EINVAL, "inlet velocity must be finite with |beta| < 1");
  if (!std::isfinite(n_in)) return fail(RLB_EINVAL, "inlet charge density must be finite");
  if (!std::isfinite(eps_out) || !(eps_out > 0.0)) return fail(RLB_EINVAL, "outlet energy density must be > 0");
  lat->open.bx = bx;
  lat->open.by = by;
  lat->open.n_in = n_in;
  lat->open.eps_out = eps_out;
  return RLB_OK;
}

extern "C" {

const char* rlb_last_error(void) { return g_err.c_str(); }

const char* rlb_version(void) { return "librlb 0.1 (gfx950)"; }

rlb_status rlb_workspace_bytes(const rlb_params* p, size_t* bytes) {
  rlb_status s = check_params(p);
  if (s) return s;
  if (!bytes) return fail(RLB_EINVAL, "bytes is null");
  const int Q = planes_of(p);
  const int64_t pitch = (int64_t)align_up((size_t)p->ny * align_up((size_t)p->nx, 64), 64);
  *bytes = layout(p, Q, pitch).total;
  return RLB_OK;
}

rlb_status rlb_create(const rlb_params* p, void* d_workspace, size_t bytes,
                      void* hip_stream, rlb_lattice** out) {
  rlb_status s = check_params(p);
  if (s) return s;
  if (!out) return fail(RLB_EINVAL, "out is null");
  *out = nullptr;
  if (!d_workspace || !aligned(d_workspace, kAlign))
    return fail(RLB_EINVAL, "workspace must be a non-null 256-byte aligned device pointer");
  const int Q = planes_of(p);
  const int row = (int)align_up((size_t)p->nx, 64);
  const int64_t pitch = (int64_t)align_up((size_t)p->ny * row, 64);
  const Workspace w = layout(p, Q, pitch);
  if (bytes < w.total) return fail(RLB_ENOMEM, "workspace has %zu bytes, needs %zu", bytes, w.total);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "no HIP device");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "device properties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(RLB_EDEVICE, "device %d is %s; librlb is built for gfx950", dev, prop.gcnArchName);
  hipPointerAttribute_t attr;
  e = hipPointerGetAttributes(&attr, d_workspace);
  if (e != hipSuccess || attr.type != hipMemoryTypeDevice)
    return fail(RLB_EINVAL, "workspace is not device memory");

  rlb_lattice* lat = new (std::nothrow) rlb_lattice();
  if (!lat) return fail(RLB_ENOMEM, "host allocation failed");
  lat->p = *p;
  lat->device = dev;
  lat->stream = (hipStream_t)hip_stream;
  lat->Q = Q;
  lat->row = row;
  lat->pitch = pitch;
  lat->ws = (char*)d_workspace;
  lat->ws_bytes = bytes;
  lat->lay = w;
  lat->state[0] = (float*)(lat->ws + w.state_off[0]);
  lat->state[1] = (float*)(lat->ws + w.state_off[1]);
  lat->cur = 0;
  lat->mask = (uint8_t*)(lat->ws + w.mask_off);
  lat->coef = (double*)(lat->ws + w.coef_off);
  lat->modes = (int4*)(lat->ws + w.modes_off);
  lat->bins = (int32_t*)(lat->ws + w.bins_off);
  lat->table = (uint4*)(lat->ws + w.table_off);
  lat->phase = (double2*)(lat->ws + w.phase_off);
  lat->force = (float*)(lat->ws + w.force_off);
  lat->twiddle = (uint4*)(lat->ws + w.twiddle_off);
  lat->partials = (double*)(lat->ws + w.partial_off);
  lat->err = (uint32_t*)(lat->ws + w.misc_off);
  lat->dstep = (int64_t*)(lat->ws + w.misc_off + 64);
  lat->d_desc = (LatDesc*)(lat->ws + w.desc_off);
  lat->num_cu = prop.multiProcessorCount;
  lat->shape = LaunchShape{4, 0, 16};
  lat->open = OpenArgs{0.0, 0.0, p->n_ref, p->eps_ref, 0.0, 0.0, nullptr};
  lat->desc.state[0] = lat->state[0];
  lat->desc.state[1] = lat->state[1];
  lat->desc.mask = lat->mask;
  lat->desc.force = (const float*)(lat->ws + w.force_off);
  lat->desc.pitch = pitch;
  lat->desc.nx = p->nx;
  lat->desc.ny = p->ny;
  lat->desc.tiles_x = (p->nx + 63) / 64;
  lat->desc.tile_begin = 0;
  lat->desc.row = row;
  lat->desc.rec_row = 0;
  lat->result = (double*)(lat->ws + w.misc_off + 128);
  if (Q == 17) fill_taps<Dir17>(lat);
  else if (Q == 12) fill_taps<DirP12>(lat);
  else fill_taps<Dir26>(lat);

  rlb_status st = RLB_OK;
  // zero both state copies and the force planes: the row padding is never
  // written by the kernels, so saved states are then byte-deterministic
  e = launch_fill_u8((uint8_t*)lat->state[0], 2 * (w.state_off[1] - w.state_off[0]), 0, lat->stream);
  if (e == hipSuccess)
    e = launch_fill_u8((uint8_t*)(lat->ws + w.force_off), (size_t)2 * pitch * sizeof(float), 0, lat->stream);
  if (e == hipSuccess) e = launch_fill_u8(lat->mask, (size_t)p->nx * p->ny, 0, lat->stream);
  if (e == hipSuccess) e = launch_fill_u8((uint8_t*)lat->err, 64, 0, lat->stream);
  if (e == hipSuccess) e = launch_set_i64(lat->dstep, 0, lat->stream);
  if (e == hipSuccess) e = launch_phase(lat);
  if (e == hipSuccess)
    e = hipMemcpyAsync(lat->d_desc, &lat->desc, sizeof(LatDesc), hipMemcpyHostToDevice, lat->stream);
  if (e == hipSuccess && (p->flags & RLB_WALLS_Y)) {
    e = launch_walls(lat);
    lat->any_solid = true;
  }
  if (e != hipSuccess) st = hip_fail(e, "workspace initialisation");
  if (st) {
    delete lat;
    return st;
  }
  *out = lat;
  return RLB_OK;
}

static void drop_lattice_graph(rlb_lattice* lat) {
  if (lat->exec) (void)hipGraphExecDestroy(lat->exec);
  if (lat->graph) (void)hipGraphDestroy(lat->graph);
  lat->exec = nullptr;
  lat->graph = nullptr;
  lat->graph_valid = false;
}

rlb_status rlb_destroy(rlb_lattice* lat) {
  if (!lat) return RLB_OK;
  drop_lattice_graph(lat);
  if (lat->aux) {
    (void)hipStreamSynchronize(lat->aux);
    (void)hipStreamDestroy(lat->aux);
    for (auto& e : lat->aux_ev)
      if (e) (void)hipEventDestroy(e);
  }
  if (lat->ev[0][0]) {
    for (int i = 0; i < kEvRing; ++i)
      for (int j = 0; j < 2; ++j)
        if (lat->ev[i][j]) (void)hipEventDestroy(lat->ev[i][j]);
  }
  delete lat;
  return RLB_OK;
}

rlb_status rlb_init_fields(rlb_lattice* lat, const float* d_eps, const float* d_bx,
                           const float* d_by, const float* d_n) {
  if (rlb_status s = check_lat(lat)) return s;
  if (!d_eps || !d_bx || !d_by || !d_n) return fail(RLB_EINVAL, "field pointers must be non-null");
  if (!aligned(d_eps, 4) || !aligned(d_bx, 4) || !aligned(d_by, 4) || !aligned(d_n, 4))
    return fail(RLB_EINVAL, "field pointers must be 4-byte aligned");
  HIP_TRY(launch_fill_u8((uint8_t*)lat->err, 64, 0, lat->stream), "clear error flag");
  lat->cur = 0;
  HIP_TRY(launch_init(lat, d_eps, d_bx, d_by, d_n, lat->state[0]), "init kernel");
  lat->step = 0;
  HIP_TRY(launch_set_i64(lat->dstep, 0, lat->stream), "step counter");
  return RLB_OK;
}

rlb_status rlb_set_obstacles(rlb_lattice* lat, const uint8_t* d_mask) {
  if (rlb_status s = check_lat(lat)) return s;
  if (!d_mask) return fail(RLB_EINVAL, "mask is null");
  HIP_TRY(launch_mask_or(lat, d_mask), "mask kernel");
  lat->any_solid = true;
  return RLB_OK;
}

rlb_status rlb_add_disks(rlb_lattice* lat, int32_t count, const double* h) {
  if (rlb_status s = check_lat(lat)) return s;
  if (count < 0) return fail(RLB_EINVAL, "count must be >= 0");
  if (count > 0 && !h) return fail(RLB_EINVAL, "disc array is null");
  for (int i = 0; i < count; ++i) {
    if (!std::isfinite(h[3 * i]) || !std::isfinite(h[3 * i + 1]) || !std::isfinite(h[3 * i + 2]) ||
        !(h[3 * i + 2] > 0.0))
      return fail(RLB_EINVAL, "disc %d: centre must be finite and radius > 0", i);
  }
  // stage through the coefficient area of the workspace, in chunks
  const int chunk = (int)(kMaxModes * 4 / 3);
  for (int b = 0; b < count; b += chunk) {
    const int n = std::min(chunk, count - b);
    HIP_TRY(hipMemcpyAsync(lat->coef, h + 3 * (size_t)b, sizeof(double) * 3 * n,
                           hipMemcpyHostToDevice, lat->stream), "upload discs");
    HIP_TRY(launch_disks(lat, lat->coef, n), "disc kernel");
    HIP_TRY(hipStreamSynchronize(lat->stream), "stream synchronize");
  }
  if (count > 0) lat->any_solid = true;
  return RLB_OK;
}

rlb_status rlb_clear_obstacles(rlb_lattice* lat) {
  if (rlb_status s = check_lat(lat)) return s;
  HIP_TRY(launch_fill_u8(lat->mask, (size_t)lat->p.nx * lat->p.ny, 0, lat->stream), "clear mask");
  lat->any_solid = false;
  if (lat->p.flags & RLB_WALLS_Y) {
    HIP_TRY(launch_walls(lat), "walls");
    lat->any_solid = true;
  }
  return RLB_OK;
}

rlb_status rlb_set_body_force(rlb_lattice* lat, double fx, double fy) {
  if (rlb_status s = check_lat(lat)) return s;
  if (lat->owner) return fail(RLB_EINVAL, "lattice is a batch member: use the batch's body force (rlb_batch_set_body_force)");
  if (lat->p.flags & RLB_PLANAR)
    return fail(RLB_EUNSUPPORTED, "the planar momentum set has no driving term");
  if (!std::isfinite(fx) || !std::isfinite(fy)) return fail(RLB_EINVAL, "force must be finite");
  lat->fx = fx;
  lat->fy = fy;
  return RLB_OK;
}

rlb_status rlb_set_stirring(rlb_lattice* lat, double kmin, double kmax, double amplitude,
                            uint64_t seed) {
  if (rlb_status s = check_lat(lat)) return s;
  if (lat->owner) return fail(RLB_EINVAL, "lattice is a batch member: batches have no stirring");
  if (lat->p.flags & RLB_PLANAR)
    return fail(RLB_EUNSUPPORTED, "the planar momentum set has no driving term");
  // the twiddle table's items, (kMaxK + 1) * nx, are indexed with 32-bit
  // integers (the row limit of check_params keeps the 3D sets below this)
  if ((int64_t)(kMaxK + 1) * lat->p.nx >= ((int64_t)1 << 31))
    return fail(RLB_EUNSUPPORTED, "stirring supports nx < %d", (int)(((int64_t)1 << 31) / (kMaxK + 1)));
  if (!std::isfinite(amplitude) || amplitude < 0.0) return fail(RLB_EINVAL, "amplitude must be finite and >= 0");
  if (amplitude == 0.0) {
    lat->stir = false;
    lat->amp = 0.0;
    return RLB_OK;
  }
  if (!std::isfinite(kmin) || !std::isfinite(kmax) || kmin < 0.0 || kmin > kmax)
    return fail(RLB_EINVAL, "need 0 <= kmin <= kmax");
  if (kmax > (double)kMaxK) return fail(RLB_EUNSUPPORTED, "kmax must be <= %d", kMaxK);
  if (kmax >= 0.5 * std::min(lat->p.nx, lat->p.ny))
    return fail(RLB_EINVAL, "kmax must be below min(nx, ny) / 2");
  // canonical half-shell order: ky ascending, then kx ascending
  std::vector<int4> modes;
  const int K = (int)std::floor(kmax);
  for (int ky = 0; ky <= K; ++ky)
    for (int kx = -K; kx <= K; ++kx) {
      if (ky == 0 && kx <= 0) continue;
      const double k2 = (double)kx * kx + (double)ky * ky;
      if (k2 >= kmin * kmin && k2 <= kmax * kmax)
        modes.push_back(make_int4((int)modes.size(), kx, ky, 0));
    }
  if (modes.empty()) return fail(RLB_EINVAL, "the shell [%g, %g] holds no integer mode", kmin, kmax);
  if ((int)modes.size() > kMaxModes) return fail(RLB_EUNSUPPORTED, "too many modes");
  int kmaxx = 0;
  for (auto& m : modes) kmaxx = std::max(kmaxx, std::abs(m.y));
  // bins by |kx|, modes in canonical order inside a bin
  std::vector<int4> binned;
  std::vector<int32_t> bins(kMaxK + 2, 0);
  for (int k = 0; k <= kmaxx; ++k) {
    bins[k] = (int32_t)binned.size();
    for (auto& m : modes)
      if (std::abs(m.y) == k) binned.push_back(m);
  }
  for (int k = kmaxx + 1; k <= kMaxK + 1; ++k) bins[k] = (int32_t)binned.size();
  HIP_TRY(hipMemcpyAsync(lat->modes, binned.data(), sizeof(int4) * binned.size(),
                         hipMemcpyHostToDevice, lat->stream), "upload modes");
  HIP_TRY(hipMemcpyAsync(lat->bins, bins.data(), sizeof(int32_t) * bins.size(),
                         hipMemcpyHostToDevice, lat->stream), "upload bins");
  HIP_TRY(hipStreamSynchronize(lat->stream), "stream synchronize");
  lat->stir = true;
  lat->kmin = kmin;
  lat->kmax = kmax;
  lat->amp = amplitude;
  lat->seed = seed;
  lat->nmodes = (int)modes.size();
  lat->K = kmaxx;
  // the series coefficients are about 2 amplitude sqrt(modes of a bin) or
  // less: a power of two brings that to ~2^8, well inside float16's normal
  // range, before the hi + lo split
  {
    const double typ = 2.0 * amplitude * std::sqrt((double)modes.size());
    const int e = std::max(-60, std::min(60, 8 - (int)std::ceil(std::log2(typ))));
    lat->stir_scale = std::ldexp(1.0f, e);
  }
  HIP_TRY(launch_twiddle(lat->twiddle, kmaxx, lat->p.nx, lat->stream), "twiddle table");
  HIP_TRY(launch_set_i64(lat->dstep, lat->step, lat->stream), "step counter");
  return RLB_OK;
}

// Everything the kernels of one step capture by value: a graph is valid for
// the configuration it was captured with.
static void graph_key(const rlb_lattice* lat, double* k) {
  int i = 0;
  const int force = lat->stir ? FORCE_STIR : ((lat->fx != 0.0 || lat->fy != 0.0) ? FORCE_BODY : FORCE_NONE);
  k[i++] = force; k[i++] = lat->fx; k[i++] = lat->fy; k[i++] = lat->stir;
  k[i++] = lat->kmin; k[i++] = lat->kmax; k[i++] = lat->amp; k[i++] = (double)lat->seed;
  k[i++] = lat->nmodes; k[i++] = lat->K; k[i++] = lat->p.tau; k[i++] = lat->tau_k;
  k[i++] = lat->open.bx; k[i++] = lat->open.by; k[i++] = lat->open.n_in; k[i++] = lat->open.eps_out;
  k[i++] = lat->shape.tile_rows; k[i++] = lat->shape.grid_per_cu; k[i++] = lat->shape.strip;
  k[i++] = lat->any_solid; k[i++] = (double)(uintptr_t)lat->stream;
  while (i < 24) k[i++] = 0.0;
}

// The kernels of one step from state copy `parity` (stirring draw, row
// series and synthesis; the step; the open borders of the new state).
static hipError_t launch_one_step(rlb_lattice* lat, const StirArgs& sa, int force, int parity,
                                  int slot, double* rec = nullptr, int rec_x = 0) {
  hipError_t e = hipSuccess;
  if (lat->stir) {
    if ((e = launch_stir_table(sa, -1, lat->stream)) != hipSuccess) return e;
    if ((e = launch_stir_synth(sa, true, lat->stream)) != hipSuccess) return e;
  }
  if (slot >= 0 && (e = hipEventRecord(lat->ev[slot][0], lat->stream)) != hipSuccess) return e;
  const int mode = step_mode(lat);
  if ((e = launch_step(lat, mode, force, parity, nullptr, 0, rec, rec_x)) != hipSuccess) return e;
  if (slot >= 0 && (e = hipEventRecord(lat->ev[slot][1], lat->stream)) != hipSuccess) return e;
  if ((lat->p.flags & RLB_OPEN_X) && mode == MODE_STEP)   // borders not set by the step
    e = launch_open_borders(lat, lat->state[parity ^ 1]);
  return e;
}

// One step launched kernel by kernel (timed when timing is on).
static rlb_status step_direct(rlb_lattice* lat, const StirArgs& sa, int force,
                              double* rec = nullptr, int rec_x = 0) {
  int slot = -1;
  if (lat->timing && lat->step % lat->timing_every == 0) {
    slot = (int)((lat->step / lat->timing_every) % kEvRing);
    if (rlb_status s = drain_event(lat, slot)) return s;
  }
  HIP_TRY(launch_one_step(lat, sa, force, lat->cur, slot, rec, rec_x), "step");
  if (slot >= 0) lat->ev_pending |= 1u << slot;
  lat->cur ^= 1;
  lat->step += 1;
  return RLB_OK;
}

static int force_mode(const rlb_lattice* lat) {
  return lat->stir ? FORCE_STIR : ((lat->fx != 0.0 || lat->fy != 0.0) ? FORCE_BODY : FORCE_NONE);
}

rlb_status rlb_step(rlb_lattice* lat, int64_t nsteps) {
  if (rlb_status s = check_lat(lat)) return s;
  if (nsteps < 0) return fail(RLB_EINVAL, "nsteps must be >= 0");
  if (lat->owner) return fail(RLB_EINVAL, "lattice is a batch member: step it with rlb_batch_step");
  const int force = force_mode(lat);
  const StirArgs sa = stir_args(lat);
  auto direct = [&]() { return step_direct(lat, sa, force); };
  int64_t left = nsteps;
  const int K = lat->graph_steps;
  if (K > 0 && !lat->timing && lat->stream != nullptr && left >= K + lat->cur) {
    if (lat->cur == 1) {   // replays start from the first copy
      if (rlb_status s = direct()) return s;
      --left;
    }
    double key[24];
    graph_key(lat, key);
    if (lat->graph_valid && std::memcmp(key, lat->graph_key, sizeof key) != 0) drop_lattice_graph(lat);
    if (!lat->graph_valid) {
      drop_lattice_graph(lat);   // a graph whose instantiation failed
      HIP_TRY(hipStreamBeginCapture(lat->stream, hipStreamCaptureModeThreadLocal), "begin capture");
      hipError_t e = hipSuccess;
      for (int k = 0; k < K && e == hipSuccess; ++k) e = launch_one_step(lat, sa, force, k & 1, -1);
      hipGraph_t g = nullptr;
      const hipError_t e2 = hipStreamEndCapture(lat->stream, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(e != hipSuccess ? e : e2, "graph capture");
      }
      lat->graph = g;
      HIP_TRY(hipGraphInstantiate(&lat->exec, lat->graph, nullptr, nullptr, 0), "graph instantiate");
      lat->graph_valid = true;
      std::memcpy(lat->graph_key, key, sizeof key);
    }
    while (left >= K) {
      HIP_TRY(hipGraphLaunch(lat->exec, lat->stream), "graph launch");
      lat->step += K;   // K is even: the current copy is again the first
      left -= K;
    }
  }
  while (left > 0) {
    if (rlb_status s = direct()) return s;
    --left;
  }
  return RLB_OK;
}

rlb_status rlb_use_graph(rlb_lattice* lat, int32_t steps_per_graph) {
  if (rlb_status s = check_lat(lat)) return s;
  if (lat->owner) return fail(RLB_EINVAL, "lattice is a batch member: use the batch's graphs (rlb_batch_use_graph)");
  if (steps_per_graph < 0 || (steps_per_graph & 1) || steps_per_graph > 4096)
    return fail(RLB_EINVAL, "steps_per_graph must be 0 or even in [2, 4096]");
  if (steps_per_graph != lat->graph_steps) drop_lattice_graph(lat);
  lat->graph_steps = steps_per_graph;
  return RLB_OK;
}

static bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

static rlb_status check_spectrum(const rlb_lattice* lat, int32_t kmax) {
  if (!pow2_in(lat->p.nx, 4, 4096) || !pow2_in(lat->p.ny, 4, 4096))
    return fail(RLB_EUNSUPPORTED, "spectral analysis needs nx and ny powers of two in [4, 4096]");
  if (kmax < 0 || kmax > 65535) return fail(RLB_EINVAL, "kmax must be in [0, 65535]");
  return RLB_OK;
}

rlb_status rlb_spectrum_workspace_bytes(const rlb_lattice* lat, int32_t kmax, size_t* bytes) {
  if (rlb_status s = check_lat(lat)) return s;
  if (rlb_status s = check_spectrum(lat, kmax)) return s;
  if (!bytes) return fail(RLB_EINVAL, "bytes is null");
  *bytes = spectral_layout(lat->p.nx, lat->p.ny, kmax).total;
  return RLB_OK;
}

rlb_status rlb_energy_spectrum(rlb_lattice* lat, int32_t kmax, double k_cut, double* d_out,
                               double* d_acc, void* d_work, size_t bytes) {
  if (rlb_status s = check_lat(lat)) return s;
  if (rlb_status s = check_spectrum(lat, kmax)) return s;
  if (!std::isfinite(k_cut) || k_cut < 0.0) return fail(RLB_EINVAL, "k_cut must be finite and >= 0");
  if (!d_out || !aligned(d_out, 8) || (d_acc && !aligned(d_acc, 8)))
    return fail(RLB_EINVAL, "d_out (and d_acc) must be 8-byte aligned device pointers");
  if (!d_work || !aligned(d_work, 256)) return fail(RLB_EINVAL, "workspace must be a 256-byte aligned device pointer");
  const size_t need = spectral_layout(lat->p.nx, lat->p.ny, kmax).total;
  if (bytes < need) return fail(RLB_ENOMEM, "spectral workspace has %zu bytes, needs %zu", bytes, need);
  HIP_TRY(launch_spectrum(lat, kmax, k_cut, d_out, d_acc, (char*)d_work), "energy spectrum");
  return RLB_OK;
}

rlb_status rlb_spectrum_average(const double* h_acc, int32_t kmax, int64_t count, double* h_mean,
                                double* h_err) {
  if (!h_acc || !h_mean || !h_err) return fail(RLB_EINVAL, "null pointer");
  if (kmax < 0 || count < 1) return fail(RLB_EINVAL, "kmax must be >= 0 and count >= 1");
  const double m = (double)count;
  for (int s = 0; s <= kmax; ++s) {
    const double mean = h_acc[s] / m;
    const double ss = h_acc[kmax + 1 + s] - m * mean * mean;   // sum (E - mean)^2
    h_mean[s] = mean;
    h_err[s] = count > 1 ? std::sqrt(std::max(ss, 0.0) / (m * (m - 1.0))) : 0.0;
  }
  return RLB_OK;
}

rlb_status rlb_power_law_fit(const double* h_k, const double* h_y, int32_t n, double* h_slope,
                             double* h_intercept) {
  if (!h_k || !h_y || !h_slope || !h_intercept) return fail(RLB_EINVAL, "null pointer");
  if (n < 2) return fail(RLB_EINVAL, "need at least two points");
  double sx = 0, sy = 0, sxx = 0, sxy = 0;
  for (int i = 0; i < n; ++i) {
    if (!(h_k[i] > 0.0) || !(h_y[i] > 0.0)) return fail(RLB_EINVAL, "k and y must be positive");
    const double x = std::log(h_k[i]), y = std::log(h_y[i]);
    sx += x; sy += y; sxx += x * x; sxy += x * y;
  }
  const double d = n * sxx - sx * sx;
  if (!(d > 0.0)) return fail(RLB_EINVAL, "the k values must not all be equal");
  *h_slope = (n * sxy - sx * sy) / d;
  *h_intercept = (sy - *h_slope * sx) / n;
  return RLB_OK;
}


rlb_status rlb_set_open_borders(rlb_lattice* lat, double bx, double by, double n_in, double eps_out) {
  if (rlb_status s = check_lat(lat)) return s;
  if (lat->owner)
    return fail(RLB_EINVAL, "lattice is a batch member: members share the batch's borders");
  return set_open(lat, bx, by, n_in, eps_out);
}

rlb_status rlb_column_current(rlb_lattice* lat, int32_t x, double* d_out) {
  if (rlb_status s = check_lat(lat)) return s;
  if (x < 0 || x >= lat->p.nx) return fail(RLB_EINVAL, "column %d outside [0, %d)", x, lat->p.nx);
  if (lat->p.cfl > 1.0) return fail(RLB_EUNSUPPORTED, "the column current supports cfl <= 1");
  if (!d_out || !aligned(d_out, 8)) return fail(RLB_EINVAL, "d_out must be an 8-byte aligned device pointer");
  HIP_TRY(launch_column_current(lat, x, d_out), "column current");
  return RLB_OK;
}

rlb_status rlb_record_workspace_bytes(const rlb_lattice* lat, int32_t chunk, size_t* bytes) {
  if (rlb_status s = check_lat(lat)) return s;
  if (chunk < 1 || chunk > 65536) return fail(RLB_EINVAL, "chunk must be in [1, 65536]");
  if (!bytes) return fail(RLB_EINVAL, "bytes is null");
  *bytes = align_up((size_t)chunk * (size_t)lat->p.ny * sizeof(double));
  return RLB_OK;
}

namespace {

// Checks shared by rlb_record_current and rlb_record_current_noalloc
// (everything but the workspace).  *done is set when there is nothing to do.
rlb_status check_record(const rlb_lattice* lat, int64_t nsteps, int32_t x, const double* d_series,
                        bool* done) {
  if (rlb_status s = check_lat(lat)) return s;
  if (nsteps < 0) return fail(RLB_EINVAL, "nsteps must be >= 0");
  if (lat->owner) return fail(RLB_EINVAL, "lattice is a batch member: step it with rlb_batch_step");
  if (x < 0 || x >= lat->p.nx) return fail(RLB_EINVAL, "column %d outside [0, %d)", x, lat->p.nx);
  if (lat->p.cfl > 1.0) return fail(RLB_EUNSUPPORTED, "the column current supports cfl <= 1");
  *done = nsteps == 0;
  if (*done) return RLB_OK;
  if (!d_series || !aligned(d_series, 8))
    return fail(RLB_EINVAL, "d_series must be an 8-byte aligned device pointer");
  return RLB_OK;
}

// The recording steps, with `rows` (chunk * ny float64) holding the per-row
// currents of up to `chunk` steps.  Every row of a recorded step is written
// by the step kernel before the row means read it, so `rows` needs no
// clearing.
rlb_status record_steps(rlb_lattice* lat, int64_t nsteps, int32_t x, double* d_series, double* rows,
                        int64_t chunk) {
  const int force = force_mode(lat);
  const StirArgs sa = stir_args(lat);
  if (!records_current(lat)) {   // record with the column kernel before each step
    for (int64_t t = 0; t < nsteps; ++t) {
      HIP_TRY(launch_column_current(lat, x, d_series + t), "column current");
      if (rlb_status s = step_direct(lat, sa, force)) return s;
    }
    return RLB_OK;
  }
  for (int64_t t0 = 0; t0 < nsteps; t0 += chunk) {
    const int64_t cnt = std::min(chunk, nsteps - t0);
    for (int64_t i = 0; i < cnt; ++i)
      if (rlb_status s = step_direct(lat, sa, force, rows + i * lat->p.ny, x)) return s;
    HIP_TRY(launch_row_means(rows, lat->p.ny, (int)cnt, d_series + t0, lat->stream), "row means");
  }
  return RLB_OK;
}

}  // namespace

rlb_status rlb_record_current(rlb_lattice* lat, int64_t nsteps, int32_t x, double* d_series,
                              void* d_work, size_t bytes) {
  bool done = false;
  if (rlb_status s = check_record(lat, nsteps, x, d_series, &done)) return s;
  if (done) return RLB_OK;
  if (!d_work || !aligned(d_work, 256)) return fail(RLB_EINVAL, "workspace must be a 256-byte aligned device pointer");
  const size_t row_bytes = (size_t)lat->p.ny * sizeof(double);
  const int64_t chunk = (int64_t)std::min<size_t>(bytes / row_bytes, 65536);
  if (chunk < 1) return fail(RLB_ENOMEM, "record workspace has %zu bytes, needs at least %zu", bytes, row_bytes);
  return record_steps(lat, nsteps, x, d_series, (double*)d_work, chunk);
}

rlb_status rlb_record_current_noalloc(rlb_lattice* lat, int64_t nsteps, int32_t x, double* d_series) {
  bool done = false;
  if (rlb_status s = check_record(lat, nsteps, x, d_series, &done)) return s;
  if (done) return RLB_OK;
  const size_t row_bytes = (size_t)lat->p.ny * sizeof(double);
  if (row_bytes > kStaticScratchBytes)
    return fail(RLB_ENOMEM, "ny = %d rows need %zu bytes per step; the fixed scratch holds %zu "
                "(ny <= %zu)", lat->p.ny, row_bytes, kStaticScratchBytes,
                kStaticScratchBytes / sizeof(double));
  double* rows = nullptr;
  HIP_TRY(static_scratch(lat->device, &rows), "fixed scratch address");
  const int64_t chunk = (int64_t)std::min<size_t>(kStaticScratchBytes / row_bytes, 65536);
  return record_steps(lat, nsteps, x, d_series, rows, chunk);
}

rlb_status rlb_power_spectrum(const double* d_series, int64_t n, double* d_out, void* hip_stream) {
  if (!d_series || !d_out || !aligned(d_series, 8) || !aligned(d_out, 8))
    return fail(RLB_EINVAL, "series and output must be 8-byte aligned device pointers");
  if (n < 2 || n > ((int64_t)1 << 26)) return fail(RLB_EINVAL, "series length must be in [2, 2^26]");
  HIP_TRY(launch_power_spectrum(d_series, n, d_out, (hipStream_t)hip_stream), "power spectrum");
  return RLB_OK;
}

rlb_status rlb_read_fields(rlb_lattice* lat, uint32_t field_mask, float* d_out) {
  if (rlb_status s = check_lat(lat)) return s;
  if (field_mask == 0 || field_mask >= (1u << RLB_FIELD_COUNT))
    return fail(RLB_EINVAL, "field_mask must select fields 0..%d", RLB_FIELD_COUNT - 1);
  if (!d_out || !aligned(d_out, 4)) return fail(RLB_EINVAL, "output must be a 4-byte aligned device pointer");
  HIP_TRY(launch_step(lat, MODE_FIELDS, FORCE_NONE, lat->cur, d_out, field_mask), "fields kernel");
  return RLB_OK;
}

rlb_status rlb_conserved(rlb_lattice* lat, double h_out[4]) {
  if (rlb_status s = check_lat(lat)) return s;
  if (!h_out) return fail(RLB_EINVAL, "output is null");
  HIP_TRY(launch_totals(lat, lat->state[lat->cur], lat->result), "totals kernel");
  double tmp[4];
  HIP_TRY(hipMemcpyAsync(tmp, lat->result, sizeof tmp, hipMemcpyDeviceToHost, lat->stream), "read totals");
  if (rlb_status s = read_err(lat)) return s;
  std::memcpy(h_out, tmp, sizeof tmp);
  return RLB_OK;
}

rlb_status rlb_force_injection(rlb_lattice* lat, double h_out[3]) {
  if (rlb_status s = check_lat(lat)) return s;
  if (!h_out) return fail(RLB_EINVAL, "output is null");
  if (lat->owner) return fail(RLB_EINVAL, "lattice is a batch member: the batch holds its force");
  if (lat->Q == 12) return fail(RLB_EUNSUPPORTED, "the planar set has no driving term");
  if (lat->stir) {   // the next step's stirring field into the force planes
    const StirArgs a = stir_args(lat);
    HIP_TRY(launch_stir_table(a, lat->step, lat->stream), "stirring table");
    HIP_TRY(launch_stir_synth(a, false, lat->stream), "stirring synthesis");
  }
  HIP_TRY(launch_injection(lat, lat->stir, lat->result), "injection kernel");
  double tmp[4];
  HIP_TRY(hipMemcpyAsync(tmp, lat->result, sizeof tmp, hipMemcpyDeviceToHost, lat->stream), "read injection");
  if (rlb_status s = read_err(lat)) return s;
  std::memcpy(h_out, tmp, 3 * sizeof(double));
  return RLB_OK;
}

rlb_status rlb_sync(rlb_lattice* lat) {
  if (rlb_status s = check_lat(lat)) return s;
  return read_err(lat);
}

rlb_status rlb_get_step(const rlb_lattice* lat, int64_t* step) {
  if (rlb_status s = check_lat(lat)) return s;
  if (!step) return fail(RLB_EINVAL, "step is null");
  *step = lat->step;
  return RLB_OK;
}

rlb_status rlb_state_bytes(const rlb_lattice* lat, size_t* bytes) {
  if (rlb_status s = check_lat(lat)) return s;
  if (!bytes) return fail(RLB_EINVAL, "bytes is null");
  *bytes = kHeaderBytes + (size_t)2 * lat->Q * lat->pitch * sizeof(float);
  return RLB_OK;
}

rlb_status rlb_layout(const rlb_lattice* lat, int32_t* planes, int32_t* row_pitch,
                      int64_t* row_stride, size_t* header_bytes) {
  if (rlb_status s = check_lat(lat)) return s;
  if (planes) *planes = lat->Q;
  if (row_pitch) *row_pitch = lat->row;
  if (row_stride) *row_stride = (int64_t)2 * lat->Q * lat->row;
  if (header_bytes) *header_bytes = kHeaderBytes;
  return RLB_OK;
}

rlb_status rlb_save_state(rlb_lattice* lat, void* d_buf, size_t bytes) {
  if (rlb_status s = check_lat(lat)) return s;
  size_t need = 0;
  rlb_state_bytes(lat, &need);
  if (!d_buf || !aligned(d_buf, kAlign)) return fail(RLB_EINVAL, "buffer must be a 256-byte aligned device pointer");
  if (bytes < need) return fail(RLB_ENOMEM, "state buffer has %zu bytes, needs %zu", bytes, need);
  // the header staging area lives in the handle, so it outlives the copy
  HIP_TRY(hipStreamSynchronize(lat->stream), "stream synchronize");
  StateHeader h{};
  h.magic = kMagic;
  h.version = 1;
  h.nx = lat->p.nx;
  h.ny = lat->p.ny;
  h.q = lat->Q;
  h.pitch = lat->pitch;
  h.step = lat->step;
  h.eps_ref = lat->p.eps_ref;
  h.n_ref = lat->p.n_ref;
  h.tau = lat->p.tau;
  h.cfl = lat->p.cfl;
  h.flags = lat->p.flags;
  std::memset(lat->header, 0, sizeof lat->header);
  std::memcpy(lat->header, &h, sizeof h);
  HIP_TRY(hipMemcpyAsync(d_buf, lat->header, kHeaderBytes, hipMemcpyHostToDevice, lat->stream), "write header");
  HIP_TRY(hipMemcpyAsync((char*)d_buf + kHeaderBytes, lat->state[lat->cur],
                         (size_t)2 * lat->Q * lat->pitch * sizeof(float),
                         hipMemcpyDeviceToDevice, lat->stream), "copy state");
  HIP_TRY(hipStreamSynchronize(lat->stream), "stream synchronize");
  return RLB_OK;
}

rlb_status rlb_load_state(rlb_lattice* lat, const void* d_buf, size_t bytes) {
  if (rlb_status s = check_lat(lat)) return s;
  size_t need = 0;
  rlb_state_bytes(lat, &need);
  if (!d_buf || !aligned(d_buf, kAlign)) return fail(RLB_EINVAL, "buffer must be a 256-byte aligned device pointer");
  if (bytes < need) return fail(RLB_ENOMEM, "state buffer has %zu bytes, needs %zu", bytes, need);
  StateHeader h{};
  HIP_TRY(hipMemcpyAsync(&h, d_buf, sizeof h, hipMemcpyDeviceToHost, lat->stream), "read header");
  HIP_TRY(hipStreamSynchronize(lat->stream), "stream synchronize");
  if (h.magic != kMagic || h.version != 1) return fail(RLB_ESTATE, "not an RLB state buffer");
  if (h.nx != lat->p.nx || h.ny != lat->p.ny || h.q != lat->Q || h.pitch != lat->pitch ||
      h.eps_ref != lat->p.eps_ref || h.n_ref != lat->p.n_ref)
    return fail(RLB_ESTATE, "state shape or references differ from this lattice");
  HIP_TRY(hipMemcpyAsync(lat->state[lat->cur], (const char*)d_buf + kHeaderBytes,
                         (size_t)2 * lat->Q * lat->pitch * sizeof(float),
                         hipMemcpyDeviceToDevice, lat->stream), "copy state");
  HIP_TRY(launch_fill_u8((uint8_t*)lat->err, 64, 0, lat->stream), "clear error flag");
  lat->step = h.step;
  HIP_TRY(launch_set_i64(lat->dstep, lat->step, lat->stream), "step counter");
  return RLB_OK;
}

rlb_status rlb_stirring_coefficients(rlb_lattice* lat, int64_t step, double* d_out, int32_t* count) {
  if (rlb_status s = check_lat(lat)) return s;
  if (!lat->stir) return fail(RLB_EINVAL, "stirring is not set");
  if (step < 0) return fail(RLB_EINVAL, "step must be >= 0");
  if (!d_out || !aligned(d_out, 8)) return fail(RLB_EINVAL, "output must be an 8-byte aligned device pointer");
  StirArgs a = stir_args(lat);
  a.coef = d_out;
  HIP_TRY(launch_stir_draw(a, step, lat->stream), "stirring draw");
  if (count) *count = lat->nmodes;
  return RLB_OK;
}

rlb_status rlb_stirring_field(rlb_lattice* lat, int64_t step, float* d_out) {
  if (rlb_status s = check_lat(lat)) return s;
  if (!lat->stir) return fail(RLB_EINVAL, "stirring is not set");
  if (step < 0) return fail(RLB_EINVAL, "step must be >= 0");
  if (!d_out || !aligned(d_out, 4)) return fail(RLB_EINVAL, "output must be a 4-byte aligned device pointer");
  const StirArgs a = stir_args(lat);
  HIP_TRY(launch_stir_table(a, step, lat->stream), "stirring table");
  HIP_TRY(launch_stir_synth(a, false, lat->stream), "stirring synthesis");
  const size_t plane = (size_t)lat->p.nx * lat->p.ny;
  for (int c = 0; c < 2; ++c)
    HIP_TRY(hipMemcpy2DAsync(d_out + c * plane, sizeof(float) * lat->p.nx, lat->force + c * lat->pitch,
                             sizeof(float) * lat->row, sizeof(float) * lat->p.nx, lat->p.ny,
                             hipMemcpyDeviceToDevice, lat->stream), "copy force");
  return RLB_OK;
}

rlb_status rlb_philox(uint64_t k0, uint64_t k1, uint64_t c1, int64_t count, uint64_t* d_out,
                      void* hip_stream) {
  if (count < 0) return fail(RLB_EINVAL, "count must be >= 0");
  if (count > 0 && (!d_out || !aligned(d_out, 8))) return fail(RLB_EINVAL, "output must be an 8-byte aligned device pointer");
  HIP_TRY(launch_philox(k0, k1, c1, count, d_out, (hipStream_t)hip_stream), "philox kernel");
  return RLB_OK;
}

rlb_status rlb_timing(rlb_lattice* lat, int32_t enable) {
  if (rlb_status s = check_lat(lat)) return s;
  if (lat->owner) return fail(RLB_EINVAL, "lattice is a batch member: use the batch's timing (rlb_batch_timing)");
  if (enable < 0) return fail(RLB_EINVAL, "enable must be >= 0");
  if (enable) {
    lat->timing_every = enable;
    if (!lat->ev[0][0]) {
      for (int i = 0; i < kEvRing; ++i)
        for (int j = 0; j < 2; ++j) HIP_TRY(hipEventCreate(&lat->ev[i][j]), "event create");
    }
    if (rlb_status s = accumulate_timing(lat)) return s;
    lat->timed_ms = 0.0;
    lat->timed_launches = 0;
    lat->timing = true;
  } else {
    if (rlb_status s = accumulate_timing(lat)) return s;
    lat->timing = false;
  }
  return RLB_OK;
}

rlb_status rlb_timing_read(rlb_lattice* lat, double* total_ms, int64_t* launches) {
  if (rlb_status s = check_lat(lat)) return s;
  if (rlb_status s = accumulate_timing(lat)) return s;
  if (total_ms) *total_ms = lat->timed_ms;
  if (launches) *launches = lat->timed_launches;
  return RLB_OK;
}

rlb_status rlb_set_launch_shape(rlb_lattice* lat, int32_t tile_rows, int32_t grid_per_cu,
                                int32_t strip) {
  if (rlb_status s = check_lat(lat)) return s;
  if (lat->owner) return fail(RLB_EINVAL, "lattice is a batch member: use the batch's launch shape (rlb_batch_set_launch_shape)");
  if (!(tile_rows == 1 || tile_rows == 2 || tile_rows == 4 || tile_rows == 8))
    return fail(RLB_EINVAL, "tile_rows must be 1, 2, 4 or 8");
  if (lat->Q != 17 && tile_rows != 4 && !(lat->Q == 26 && tile_rows == 2))
    return fail(RLB_EUNSUPPORTED, "tile_rows 1 and 8 need the folded layout, 2 the folded or the full one");
  if (grid_per_cu < 0 || grid_per_cu > 64) return fail(RLB_EINVAL, "grid_per_cu must be in [0, 64]");
  if (strip < 1 || strip > 65536) return fail(RLB_EINVAL, "strip must be in [1, 65536]");
  lat->shape = LaunchShape{tile_rows, grid_per_cu, strip};
  return RLB_OK;
}

rlb_status rlb_get_launch_shape(const rlb_lattice* lat, int32_t* tile_rows, int32_t* grid_per_cu,
                                int32_t* strip) {
  if (rlb_status s = check_lat(lat)) return s;
  if (tile_rows) *tile_rows = lat->shape.tile_rows;
  if (grid_per_cu) *grid_per_cu = lat->shape.grid_per_cu;
  if (strip) *strip = lat->shape.strip;
  return RLB_OK;
}

rlb_status rlb_autotune(rlb_lattice* lat, int32_t trials, double* h_ms, int32_t max_results) {
  if (rlb_status s = check_lat(lat)) return s;
  if (lat->owner) return fail(RLB_EINVAL, "lattice is a batch member: use the batch's autotuner (rlb_batch_autotune)");
  if (trials < 1 || trials > 1000) return fail(RLB_EINVAL, "trials must be in [1, 1000]");
  const int force = force_mode(lat);
  const LaunchShape best = lat->shape;
  auto run = [&](int n) -> hipError_t {
    for (int i = 0; i < n; ++i) {   // reads the current copy, writes the other: state unchanged
      hipError_t e = launch_step(lat, step_mode(lat), force, lat->cur, nullptr, 0);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  const std::vector<LaunchShape> cand = launch_candidates(lat->Q, false);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0), "event");
  HIP_TRY(hipEventCreate(&e1), "event");
  double best_ms = 1e300;
  LaunchShape win = best;
  int k = 0;
  for (const LaunchShape& c : cand) {
    lat->shape = c;
    hipError_t e = run(2);
    if (e == hipSuccess) e = hipEventRecord(e0, lat->stream);
    if (e == hipSuccess) e = run(trials);
    if (e == hipSuccess) e = hipEventRecord(e1, lat->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      lat->shape = best;
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return hip_fail(e, "autotune");
    }
    const double per = ms / trials;
    if (h_ms && k < max_results) {
      h_ms[4 * k] = c.tile_rows;
      h_ms[4 * k + 1] = c.grid_per_cu;
      h_ms[4 * k + 2] = c.strip;
      h_ms[4 * k + 3] = per;
    }
    ++k;
    if (per < best_ms) { best_ms = per; win = c; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  lat->shape = win;
  return RLB_OK;
}

rlb_status rlb_copy_probe(const void* d_src, void* d_dst, size_t bytes, void* hip_stream) {
  if (!d_src || !d_dst || !aligned(d_src, 16) || !aligned(d_dst, 16))
    return fail(RLB_EINVAL, "copy probe needs 16-byte aligned device pointers");
  if (bytes % 16) return fail(RLB_EINVAL, "bytes must be a multiple of 16");
  HIP_TRY(launch_copy(d_src, d_dst, bytes, (hipStream_t)hip_stream), "copy kernel");
  return RLB_OK;
}

}  // extern "C"
