// Adjoint run: forward with checkpoints every K steps, then segments in
// reverse order -- restore the checkpoint, recompute and store the K states
// of the segment, sweep the adjoint kernel back through them -- and reduce
// the per-node parameter adjoints to dJ/d(F_b, tau, A_1..A_M).
//
// The recomputed states are double-buffered: segment s - 1 is recomputed on
// the lattice stream while the adjoint sweeps segment s on a second stream
// (both are latency-bound on channel-sized lattices).  Events order the
// buffer reuse; the adjoint kernels keep one stream and one order, so the
// gradient is the same bit for bit.  The forward pass steps the last
// segments (one per buffer) inside the buffers themselves, so the sweep
// starts at once and those segments are never recomputed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "internal.hpp"

using namespace rlb;

namespace {

constexpr int kObjBlocks = 512;
constexpr int kGradCols = 256;
constexpr int kMaxModesAdj = 64;
constexpr int kAdjStrip = 16;   // adjoint-kernel tile order: strips of 16 tiles (1024 nodes)

rlb_status afail(rlb_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  set_error_message(buf);
  return s;
}

#define AHIP(expr, what)                                                                \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess) return afail(RLB_EDEVICE, "%s: %s", what, hipGetErrorString(_e)); \
  } while (0)

struct AdjLayout {
  size_t state_bytes, ck_off, store_off, mu_off, accf_off, acct_off, obj_off, modes_off,
      partial_off, result_off, desc_off, total;
  int64_t nseg, nbuf;
};

// Lattice settings the adjoint differentiates (shared by rlb_adjoint_run
// and rlb_adjoint_apply).
rlb_status check_adjoint_lattice(const rlb_lattice* lat) {
  if (!lat) return afail(RLB_EINVAL, "lattice is null");
  if (lat->tau_k > 0.0)
    return afail(RLB_EUNSUPPORTED, "the adjoint needs a constant relaxation time (rlb_set_relaxation_time)");
  if (lat->p.flags & RLB_OPEN_X)
    return afail(RLB_EUNSUPPORTED, "the adjoint supports periodic x borders only");
  if (lat->p.cfl > 1.0) return afail(RLB_EUNSUPPORTED, "the adjoint supports cfl <= 1 only");
  if (lat->p.flags & RLB_PLANAR) return afail(RLB_EUNSUPPORTED, "the adjoint supports the 3D momentum set only");
  return RLB_OK;
}

rlb_status check_cfg(const rlb_lattice* lat, const rlb_adjoint_cfg* c) {
  if (rlb_status s = check_adjoint_lattice(lat)) return s;
  if (!c) return afail(RLB_EINVAL, "config is null");
  if (c->nsteps < 2 || (c->nsteps & 1)) return afail(RLB_EINVAL, "nsteps must be even and >= 2");
  if (c->checkpoint < 1) return afail(RLB_EINVAL, "checkpoint interval must be >= 1");
  if (c->resident < 0) return afail(RLB_EINVAL, "resident segments must be >= 0");
  if (c->objective != RLB_OBJ_CURRENT && c->objective != RLB_OBJ_DISSIPATION)
    return afail(RLB_EINVAL, "unknown objective %d", c->objective);
  if (c->nmodes < 0 || c->nmodes > kMaxModesAdj) return afail(RLB_EINVAL, "nmodes must be in [0, 64]");
  if (c->nmodes > 0 && (!c->h_modes || !c->h_amps)) return afail(RLB_EINVAL, "mode arrays are null");
  if (!std::isfinite(c->body_force)) return afail(RLB_EINVAL, "body force must be finite");
  for (int m = 0; m < c->nmodes; ++m) {
    for (int k = 0; k < 5; ++k)
      if (!std::isfinite(c->h_modes[5 * m + k])) return afail(RLB_EINVAL, "mode %d is not finite", m);
    if (!std::isfinite(c->h_amps[m])) return afail(RLB_EINVAL, "amplitude %d is not finite", m);
    if (c->h_modes[5 * m] != std::floor(c->h_modes[5 * m]) ||
        c->h_modes[5 * m + 1] != std::floor(c->h_modes[5 * m + 1]))
      return afail(RLB_EINVAL, "mode %d wave numbers must be integers", m);
  }
  return RLB_OK;
}

AdjLayout adj_layout(const rlb_lattice* lat, const rlb_adjoint_cfg* c) {
  AdjLayout L;
  const size_t ncell = (size_t)lat->p.nx * lat->p.ny;
  L.state_bytes = align_up((size_t)2 * lat->Q * lat->pitch * sizeof(float));
  L.nseg = (c->nsteps + c->checkpoint - 1) / c->checkpoint;
  const int64_t K = std::min<int64_t>(c->checkpoint, c->nsteps);
  // segment buffers: at least two when there is more than one segment (one
  // is recomputed while the adjoint sweeps the other); checkpoints only for
  // the segments that are not resident
  L.nbuf = L.nseg > 1 ? std::min<int64_t>(std::max<int64_t>(c->resident, 2), L.nseg) : 1;
  size_t off = 0;
  L.ck_off = off; off += L.state_bytes * (size_t)(L.nseg - L.nbuf);
  L.store_off = off; off += L.state_bytes * (size_t)K * (size_t)L.nbuf;
  L.mu_off = off; off += 2 * L.state_bytes;
  L.accf_off = off; off += align_up(ncell * sizeof(double2));
  L.acct_off = off; off += align_up(ncell * sizeof(double));
  // objective partials: kernel blocks (count, final state), then one slot
  // per row and 64-node column of the step kernel's wavefronts
  L.obj_off = off;
  off += align_up((2 * kObjBlocks + (size_t)lat->p.ny * ((lat->p.nx + 63) / 64)) * sizeof(double));
  L.modes_off = off; off += align_up(kMaxModesAdj * 6 * sizeof(double));
  L.partial_off = off; off += align_up((size_t)(2 + kMaxModesAdj) * kGradCols * sizeof(double));
  L.result_off = off; off += align_up(128 * sizeof(double));
  // recompute descriptors, then per buffer the two exits of a forward
  // segment stepped in the buffer (its last state -> lattice copy 0 | 1)
  L.desc_off = off; off += align_up(sizeof(LatDesc) * ((size_t)K + 2) * (size_t)L.nbuf);
  L.total = off;
  return L;
}

}  // namespace

extern "C" {

rlb_status rlb_set_relaxation_time(rlb_lattice* lat, double tau) {
  if (!lat) return afail(RLB_EINVAL, "lattice is null");
  if (lat->owner) return afail(RLB_EINVAL, "lattice is a batch member: members share the batch's tau");
  if (!std::isfinite(tau) || !(tau > 0.5)) return afail(RLB_EINVAL, "tau must be finite and > 1/2");
  lat->p.tau = tau;
  lat->tau_k = 0.0;
  return RLB_OK;
}

rlb_status rlb_set_relaxation_eta_s(rlb_lattice* lat, double eta_over_s, double dt) {
  if (!lat) return afail(RLB_EINVAL, "lattice is null");
  if (lat->owner) return afail(RLB_EINVAL, "lattice is a batch member: members share the batch's tau");
  if (!std::isfinite(eta_over_s) || !(eta_over_s > 0.0) || !std::isfinite(dt) || !(dt > 0.0))
    return afail(RLB_EINVAL, "eta/s and dt must be finite and > 0");
  // 1/tau = dt T / (5 eta/s), T = (pi^2 eps / 3)^(1/4)
  const double pi = 3.14159265358979323846;
  lat->tau_k = dt * std::pow(pi * pi / 3.0, 0.25) / (5.0 * eta_over_s);
  return RLB_OK;
}

rlb_status rlb_adjoint_workspace_bytes(const rlb_lattice* lat, const rlb_adjoint_cfg* cfg,
                                       size_t* bytes) {
  if (rlb_status s = check_cfg(lat, cfg)) return s;
  if (!bytes) return afail(RLB_EINVAL, "bytes is null");
  *bytes = adj_layout(lat, cfg).total;
  return RLB_OK;
}

rlb_status rlb_adjoint_run(rlb_lattice* lat, const rlb_adjoint_cfg* cfg, void* d_ws, size_t bytes,
                           double* h_objective, double* h_grad) {
  if (rlb_status s = check_cfg(lat, cfg)) return s;
  if (lat->owner) return afail(RLB_EINVAL, "lattice is a batch member");
  const AdjLayout L = adj_layout(lat, cfg);
  if (!d_ws || ((uintptr_t)d_ws % kAlign)) return afail(RLB_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < L.total) return afail(RLB_ENOMEM, "adjoint workspace has %zu bytes, needs %zu", bytes, L.total);
  if (!h_objective) return afail(RLB_EINVAL, "objective output is null");
  char* ws = (char*)d_ws;
  hipStream_t st = lat->stream;
  const int nx = lat->p.nx, ny = lat->p.ny, M = cfg->nmodes;
  const int64_t N = cfg->nsteps, K = std::min<int64_t>(cfg->checkpoint, N);
  const size_t SB = L.state_bytes;
  const size_t state_copy = (size_t)2 * lat->Q * lat->pitch * sizeof(float);
  auto ck = [&](int64_t k) { return (float*)(ws + L.ck_off + SB * k); };
  auto store = [&](int64_t b, int64_t j) { return (float*)(ws + L.store_off + SB * (b * K + j)); };
  float* mu[2] = {(float*)(ws + L.mu_off), (float*)(ws + L.mu_off + SB)};
  double2* acc_f = (double2*)(ws + L.accf_off);
  double* acc_t = (double*)(ws + L.acct_off);
  double* obj = (double*)(ws + L.obj_off);
  const size_t nslots = (size_t)ny * ((nx + 63) / 64);
  double* obj_slots = obj + 2 * kObjBlocks;   // step-kernel wavefront slots
  double* d_modes = (double*)(ws + L.modes_off);
  double* partial = (double*)(ws + L.partial_off);
  double* result = (double*)(ws + L.result_off);
  LatDesc* d_desc = (LatDesc*)(ws + L.desc_off);

  // static force: F_b along x (uniform) + sum_m A_m phi_m (force planes)
  std::vector<double> host(6 * kMaxModesAdj, 0.0);
  for (int m = 0; m < M; ++m) {
    for (int k = 0; k < 5; ++k) host[5 * m + k] = cfg->h_modes[5 * m + k];
    host[5 * kMaxModesAdj + m] = cfg->h_amps[m];
  }
  AHIP(hipMemcpyAsync(d_modes, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice, st),
       "upload modes");
  AHIP(hipStreamSynchronize(st), "stream synchronize");
  AHIP(launch_basis_force(d_modes, d_modes + 5 * kMaxModesAdj, M, nx, ny, lat->row, lat->pitch,
                          (float*)lat->desc.force, st), "basis force");
  const double saved_fx = lat->fx, saved_fy = lat->fy;
  lat->fx = cfg->body_force;
  lat->fy = 0.0;
  StepShared sh = shared_of(lat);
  const bool unit = lat->p.cfl == 1.0, mask = lat->any_solid;

  // recompute descriptors of buffer b: store(b, j) -> store(b, j + 1); then
  // the exits of the segments the forward pass steps in the buffers (the
  // last nbuf, one per buffer, when a gradient is asked for): exit(b, c) is
  // store(b, len - 1) -> lattice copy c
  const int64_t kept_from = h_grad ? L.nseg - L.nbuf : L.nseg;
  std::vector<LatDesc> hd((size_t)((K + 2) * L.nbuf));
  for (int64_t b = 0; b < L.nbuf; ++b)
    for (int64_t j = 0; j < K; ++j) {
      LatDesc d = lat->desc;
      d.state[0] = store(b, j);
      d.state[1] = store(b, std::min<int64_t>(j + 1, K - 1));
      hd[(size_t)(b * K + j)] = d;
    }
  for (int64_t seg = kept_from; seg < L.nseg; ++seg) {
    const int64_t b = seg % L.nbuf, len = std::min<int64_t>(K, N - seg * K);
    for (int c = 0; c < 2; ++c) {
      LatDesc d = lat->desc;
      d.state[0] = store(b, len - 1);
      d.state[1] = lat->state[c];
      hd[(size_t)(K * L.nbuf + 2 * b + c)] = d;
    }
  }
  AHIP(hipMemcpyAsync(d_desc, hd.data(), sizeof(LatDesc) * hd.size(), hipMemcpyHostToDevice, st),
       "descriptors");
  AHIP(hipStreamSynchronize(st), "stream synchronize");

  ObjArgs oa;
  oa.sh = sh;
  oa.mask = mask ? lat->mask : nullptr;
  oa.pitch = lat->pitch;
  oa.nx = nx;
  oa.ny = ny;
  oa.row = lat->row;
  AHIP(launch_zero_f64(obj, 2 * kObjBlocks + nslots, st), "zero objective");
  // fluid node count
  oa.state = lat->state[lat->cur];
  oa.acc = obj + kObjBlocks;
  oa.kind = 2;
  AHIP(launch_objective(lat->Q, unit, mask, oa, kObjBlocks, st), "count fluid");
  AHIP(launch_sum_rows(obj + kObjBlocks, kObjBlocks, 1, 1.0, result + 64, st), "sum");
  double nfluid = 0.0;
  AHIP(hipMemcpyAsync(&nfluid, result + 64, sizeof(double), hipMemcpyDeviceToHost, st), "read count");
  AHIP(hipStreamSynchronize(st), "stream synchronize");
  if (!(nfluid > 0.0)) {
    lat->fx = saved_fx;
    lat->fy = saved_fy;
    return afail(RLB_EINVAL, "the lattice has no fluid node");
  }
  const double cw = 1.0 / ((double)(N - N / 2) * nfluid);
  oa.kind = cfg->objective;
  oa.acc = obj;

  // ---- forward with checkpoints ----
  // J_t of the states s_t, N/2 < t < N, is summed by the step kernel that
  // streams s_t (MODE_OBJ, per-wavefront slots); s_N by the objective kernel.
  // Segments from kept_from on run in their recompute buffers: s_t0 copied
  // in, s_t0+j -> s_t0+j+1 inside the buffer, the last state out to the
  // lattice's other copy.
  TileArgs tf;
  tf.sh = sh;
  tf.sh.obj = obj_slots;
  tf.sh.obj_kind = cfg->objective;
  tf.tile_lat = nullptr;
  tf.parity = 0;
  tf.tile_first = 0;
  tf.fields = nullptr;
  for (int64_t t = 0; t < N; ++t) {
    const int64_t seg = t / K, j = t - seg * K;
    if (seg < kept_from) {
      if (j == 0 && h_grad)   // seg < nseg - nbuf: the backward pass recomputes it
        AHIP(hipMemcpyAsync(ck(seg), lat->state[lat->cur], state_copy, hipMemcpyDeviceToDevice, st),
             "checkpoint");
      if (t > N / 2)
        AHIP(launch_step(lat, MODE_OBJ, FORCE_STIR, lat->cur, nullptr, 0, nullptr, 0, obj_slots,
                         cfg->objective), "step");
      else
        AHIP(launch_step(lat, MODE_STEP, FORCE_STIR, lat->cur, nullptr, 0), "step");
      lat->cur ^= 1;
    } else {
      const int64_t b = seg % L.nbuf, len = std::min<int64_t>(K, N - seg * K);
      if (j == 0)
        AHIP(hipMemcpyAsync(store(b, 0), lat->state[lat->cur], state_copy, hipMemcpyDeviceToDevice, st),
             "segment start");
      const bool last = j + 1 == len;
      const int md = t > N / 2 ? MODE_OBJ : MODE_STEP;
      tf.lats = last ? d_desc + K * L.nbuf + 2 * b + (lat->cur ^ 1) : d_desc + b * K + j;
      tf.ntiles = tiles_of(nx, ny, kernel_tile_rows(lat->Q, md, lat->shape.tile_rows));
      AHIP(launch_tiles(lat->Q, stream_mode(lat->p.cfl), mask, md, FORCE_STIR, tf, lat->shape,
                        lat->num_cu, st), "step");
      if (last) lat->cur ^= 1;
    }
    lat->step += 1;
  }
  oa.state = lat->state[lat->cur];
  AHIP(launch_objective(lat->Q, unit, mask, oa, kObjBlocks, st), "objective");
  AHIP(launch_sum_rows(obj, kObjBlocks, 1, 1.0, result, st), "objective sum");
  AHIP(launch_sum_rows(obj_slots, (int)nslots, 1, 1.0, result + 100, st), "objective sum");
  double Jp[2] = {0.0, 0.0};
  AHIP(hipMemcpyAsync(&Jp[0], result, sizeof(double), hipMemcpyDeviceToHost, st), "read objective");
  AHIP(hipMemcpyAsync(&Jp[1], result + 100, sizeof(double), hipMemcpyDeviceToHost, st), "read objective");
  AHIP(hipStreamSynchronize(st), "stream synchronize");
  *h_objective = cw * (Jp[1] + Jp[0]);

  if (h_grad) {
    // ---- backward ----
    if (!lat->aux) {
      AHIP(hipStreamCreateWithFlags(&lat->aux, hipStreamNonBlocking), "second stream");
      for (auto& e : lat->aux_ev) AHIP(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
    }
    hipStream_t sa = lat->aux;   // the adjoint sweep
    hipEvent_t ev_fwd = lat->aux_ev[0], ev_rec = lat->aux_ev[1], ev_join = lat->aux_ev[2];
    hipEvent_t ev_adj[2] = {lat->aux_ev[3], lat->aux_ev[4]};
    const size_t ncell = (size_t)nx * ny;
    AHIP(launch_zero_f64((double*)acc_f, 2 * ncell, st), "zero");
    AHIP(launch_zero_f64(acc_t, ncell, st), "zero");
    AHIP(hipEventRecord(ev_fwd, st), "event record");
    AHIP(hipStreamWaitEvent(sa, ev_fwd, 0), "stream wait");
    AdjArgs aa;
    aa.sh = sh;
    aa.mask = mask ? lat->mask : nullptr;
    aa.force = lat->desc.force;
    aa.acc_f = acc_f;
    aa.acc_itau = acc_t;
    aa.pitch = lat->pitch;
    aa.nx = nx;
    aa.ny = ny;
    aa.row = lat->row;
    aa.tiles_x = (nx + 63) / 64;
    aa.ntiles = aa.tiles_x * ((ny + 3) / 4);
    aa.tiles_per_xcd = (aa.ntiles + 7) / 8;
    aa.strip = kAdjStrip;
    aa.kind = cfg->objective;
    int cm = 0;
    // t = N: mu_N = dJ_N / dF~ only
    aa.state = lat->state[lat->cur];
    aa.mu_in = nullptr;
    aa.mu_out = mu[cm];
    aa.obj_c = (float)cw;
    AHIP(launch_adjoint(lat->Q, unit, mask, aa, sa), "adjoint");
    TileArgs ta;
    ta.sh = sh;
    ta.tile_lat = nullptr;
    ta.parity = 0;
    ta.tile_first = 0;
    ta.ntiles = tiles_of(nx, ny, kernel_tile_rows(lat->Q, MODE_STEP, lat->shape.tile_rows));
    ta.fields = nullptr;
    // restore segment seg's checkpoint into buffer seg % nbuf and recompute
    // its states on the lattice stream
    auto recompute = [&](int64_t seg) -> rlb_status {
      const int64_t b = seg % L.nbuf, len = std::min<int64_t>(K, N - seg * K);
      AHIP(hipMemcpyAsync(store(b, 0), ck(seg), state_copy, hipMemcpyDeviceToDevice, st), "restore");
      for (int64_t j = 0; j + 1 < len; ++j) {
        ta.lats = d_desc + b * K + j;
        AHIP(launch_tiles(lat->Q, stream_mode(lat->p.cfl), mask, MODE_STEP, FORCE_STIR, ta, lat->shape,
                          lat->num_cu, st), "recompute");
      }
      AHIP(hipEventRecord(ev_rec, st), "event record");
      return RLB_OK;
    };
    // segments from kept_from on are in their buffers already
    if (kept_from > L.nseg - 1) {
      if (rlb_status s = recompute(L.nseg - 1)) return s;
    } else {
      AHIP(hipEventRecord(ev_rec, st), "event record");
    }
    for (int64_t seg = L.nseg - 1; seg >= 0; --seg) {
      const int64_t t0 = seg * K, len = std::min<int64_t>(K, N - t0), b = seg % L.nbuf;
      AHIP(hipStreamWaitEvent(sa, ev_rec, 0), "stream wait");   // segment seg recomputed
      for (int64_t t = t0 + len - 1; t >= t0; --t) {
        aa.state = store(b, t - t0);
        aa.mu_in = mu[cm];
        aa.mu_out = mu[cm ^ 1];
        aa.obj_c = t > N / 2 ? (float)cw : 0.0f;
        AHIP(launch_adjoint(lat->Q, unit, mask, aa, sa), "adjoint");
        cm ^= 1;
      }
      AHIP(hipEventRecord(ev_adj[seg & 1], sa), "event record");
      if (seg > 0) {
        // the buffer of segment seg - 1 last held segment seg - 1 + nbuf,
        // swept no later than seg + 1 (nbuf >= 2 whenever there is more
        // than one segment; the sweep stream runs in order)
        if (seg + 1 < L.nseg) AHIP(hipStreamWaitEvent(st, ev_adj[(seg + 1) & 1], 0), "stream wait");
        if (seg - 1 < kept_from) {
          if (rlb_status s = recompute(seg - 1)) return s;
        }
      }
    }
    AHIP(hipEventRecord(ev_join, sa), "event record");
    AHIP(hipStreamWaitEvent(st, ev_join, 0), "stream wait");
    AHIP(launch_grad_reduce(acc_f, acc_t, d_modes, M, nx, ny, lat->p.tau, partial, kGradCols,
                            result + 1, st), "gradient reduce");
    std::vector<double> g((size_t)(2 + M));
    AHIP(hipMemcpyAsync(g.data(), result + 1, sizeof(double) * (2 + M), hipMemcpyDeviceToHost, st),
         "read gradient");
    AHIP(hipStreamSynchronize(st), "stream synchronize");
    std::memcpy(h_grad, g.data(), sizeof(double) * (2 + M));
  }
  lat->fx = saved_fx;
  lat->fy = saved_fy;
  uint32_t h = 0;
  AHIP(hipMemcpyAsync(&h, lat->err, sizeof h, hipMemcpyDeviceToHost, st), "read error flag");
  AHIP(hipStreamSynchronize(st), "stream synchronize");
  if (h & ERR_LANDAU) return afail(RLB_ELANDAU, "a fluid node had no timelike Landau frame");
  return RLB_OK;
}

rlb_status rlb_adjoint_apply(rlb_lattice* lat, int32_t op, const float* d_state, const float* d_mu,
                             float* d_out, double* d_acc) {
  if (rlb_status s = check_adjoint_lattice(lat)) return s;
  if (op != RLB_ADJ_STEP && op != RLB_ADJ_PULL_T) return afail(RLB_EINVAL, "unknown operation %d", op);
  auto ok = [](const void* p) { return p && ((uintptr_t)p % kAlign) == 0; };
  if (!ok(d_mu) || !ok(d_out)) return afail(RLB_EINVAL, "d_mu and d_out must be 256-byte aligned device pointers");
  if ((const void*)d_out == (const void*)d_mu || (const void*)d_out == (const void*)d_state)
    return afail(RLB_EINVAL, "d_out must not alias the inputs");
  const bool unit = lat->p.cfl == 1.0;
  if (op == RLB_ADJ_PULL_T) {
    AHIP(launch_transpose_pull(lat->Q, unit, d_mu, d_out, lat->p.nx, lat->p.ny, lat->row,
                               shared_of(lat), lat->stream), "transposed pull");
    return RLB_OK;
  }
  if (!ok(d_state) || !ok(d_acc))
    return afail(RLB_EINVAL, "d_state and d_acc must be 256-byte aligned device pointers");
  const size_t ncell = (size_t)lat->p.nx * lat->p.ny;
  // no stirring: the force planes the adjoint kernel adds to the body force are zero
  AHIP(launch_zero_f64((double*)lat->desc.force, (size_t)lat->pitch, lat->stream), "zero force");
  AHIP(launch_zero_f64(d_acc, 3 * ncell, lat->stream), "zero accumulators");
  AdjArgs aa;
  aa.sh = shared_of(lat);
  aa.state = d_state;
  aa.mu_in = d_mu;
  aa.mu_out = d_out;
  aa.mask = lat->any_solid ? lat->mask : nullptr;
  aa.force = lat->desc.force;
  aa.acc_f = (double2*)d_acc;
  aa.acc_itau = d_acc + 2 * ncell;
  aa.pitch = lat->pitch;
  aa.nx = lat->p.nx;
  aa.ny = lat->p.ny;
  aa.row = lat->row;
  aa.tiles_x = (lat->p.nx + 63) / 64;
  aa.ntiles = aa.tiles_x * ((lat->p.ny + 3) / 4);
  aa.tiles_per_xcd = (aa.ntiles + 7) / 8;
  aa.strip = kAdjStrip;
  aa.obj_c = 0.0f;
  aa.kind = 0;
  AHIP(launch_adjoint(lat->Q, unit, lat->any_solid, aa, lat->stream), "adjoint");
  return RLB_OK;
}

}  // extern "C"
