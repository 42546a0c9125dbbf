// Batched stepping of many lattices of uneven sizes in one launch.
//
// A batch owns one workspace carved into member lattices (ordinary
// rlb_lattice handles over sub-workspaces, so initialisation, obstacles,
// read-out and save/load are the single-lattice calls) plus a tile table:
// every member's 64 x tile_rows tiles are listed back to back and each
// tile records its member.  One step is one launch of the tile kernel over
// the whole list with a persistent or one-workgroup-per-tile grid; the
// per-node arithmetic is the single-lattice step's, so each member evolves
// bitwise as it would alone.  Runs of steps are captured once into a
// hipGraph (alternating ping-pong copies) and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace rlb;

struct rlb_batch {
  rlb_params p;
  int count;
  std::vector<rlb_lattice*> mem;
  std::vector<size_t> mem_off;
  char* ws;
  size_t ws_bytes;
  hipStream_t stream;
  int Q;
  int num_cu;
  LatDesc* d_desc;
  int32_t* d_tile_lat;
  uint32_t* d_err;
  std::vector<LatDesc> h_desc;
  std::vector<int32_t> h_tile_lat;
  LaunchShape shape;
  int ntiles;
  int table_rows;          // tile_rows the table was built for (0 = none)
  // (first tile, tiles) of consecutive members whose state fits the
  // last-level cache; a captured graph, and a run of direct steps, steps
  // each group through all its steps before the next
  std::vector<std::pair<int32_t, int32_t>> groups;
  int64_t rec_rows;        // rows of all members (recorded current density)
  double fx, fy;
  int64_t step;
  // graph
  int graph_steps;         // steps per captured graph (even), 0 = off
  hipGraph_t graph;
  hipGraphExec_t exec;
  bool graph_valid;
  bool graph_mask;
  int graph_force;
  // timing
  bool timing;
  hipEvent_t ev[2];
  double timed_ms;
  int64_t timed_steps;
};

namespace {

thread_local std::string g_berr;

constexpr int kBatchRecChunk = 32768;   // steps per row-means launch (grid y)

rlb_status bfail(rlb_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_berr = buf;
  set_error_message(buf);
  return s;
}

#define BHIP(expr, what)                                                        \
  do {                                                                          \
    hipError_t _e = (expr);                                                     \
    if (_e != hipSuccess) return bfail(RLB_EDEVICE, "%s: %s", what, hipGetErrorString(_e)); \
  } while (0)

struct BatchLayout {
  std::vector<size_t> mem_off, mem_bytes;
  size_t desc_off, tile_off, err_off, total;
};

rlb_status batch_layout(const rlb_params* p, int count, const int32_t* nx, const int32_t* ny,
                        BatchLayout& L) {
  if (!p) return bfail(RLB_EINVAL, "params is null");
  if (count < 1 || count > 65536) return bfail(RLB_EINVAL, "count must be in [1, 65536]");
  if (!nx || !ny) return bfail(RLB_EINVAL, "size arrays are null");
  size_t off = 0;
  int64_t tiles = 0, rows = 0;
  for (int b = 0; b < count; ++b) {
    // open borders in a batch are set inside the step kernel, which needs the
    // outlet column and the one before it in one 64-node tile
    if ((p->flags & RLB_OPEN_X) && nx[b] % 64 == 1)
      return bfail(RLB_EUNSUPPORTED, "member %d: open borders in batches need nx %% 64 != 1 (nx = %d)", b,
                   nx[b]);
    rlb_params q = *p;
    q.nx = nx[b];
    q.ny = ny[b];
    size_t n = 0;
    if (rlb_status s = rlb_workspace_bytes(&q, &n)) return s;
    L.mem_off.push_back(off);
    L.mem_bytes.push_back(n);
    off += align_up(n);
    tiles += (int64_t)((nx[b] + 63) / 64) * ny[b];   // tile_rows = 1 is the largest table
    rows += ny[b];
  }
  if (tiles >= (int64_t)1 << 31) return bfail(RLB_EINVAL, "too many tiles");
  if (rows >= (int64_t)1 << 31) return bfail(RLB_EINVAL, "too many rows");
  L.desc_off = off; off += align_up(sizeof(LatDesc) * (size_t)count);
  L.tile_off = off; off += align_up(sizeof(int32_t) * (size_t)tiles);
  L.err_off = off; off += align_up(64);
  L.total = off;
  return RLB_OK;
}

rlb_status build_tables(rlb_batch* B, int tile_rows) {
  if (B->table_rows == tile_rows) return RLB_OK;
  B->h_desc.resize(B->count);
  B->h_tile_lat.clear();
  int begin = 0, rec_row = 0;
  for (int b = 0; b < B->count; ++b) {
    LatDesc d = B->mem[b]->desc;
    d.tile_begin = begin;
    d.rec_row = rec_row;
    rec_row += d.ny;
    B->h_desc[b] = d;
    const int n = tiles_of(d.nx, d.ny, tile_rows);
    B->h_tile_lat.insert(B->h_tile_lat.end(), (size_t)n, b);
    begin += n;
  }
  B->ntiles = begin;
  B->groups.clear();
  {
    const double per_tile = 2.0 * 64 * tile_rows * 2 * B->Q * sizeof(float);
    int first = 0, count = 0;
    for (int b = 0; b < B->count; ++b) {
      const int n = tiles_of(B->h_desc[b].nx, B->h_desc[b].ny, tile_rows);
      if (count > 0 && (double)(count + n) * per_tile > kCachedStateBytes) {
        B->groups.emplace_back(first, count);
        first += count;
        count = 0;
      }
      count += n;
    }
    if (count > 0) B->groups.emplace_back(first, count);
  }
  BHIP(hipMemcpyAsync(B->d_desc, B->h_desc.data(), sizeof(LatDesc) * B->count,
                      hipMemcpyHostToDevice, B->stream), "upload descriptors");
  BHIP(hipMemcpyAsync(B->d_tile_lat, B->h_tile_lat.data(), sizeof(int32_t) * B->ntiles,
                      hipMemcpyHostToDevice, B->stream), "upload tile table");
  BHIP(hipStreamSynchronize(B->stream), "stream synchronize");
  B->table_rows = tile_rows;
  return RLB_OK;
}

void drop_graph(rlb_batch* B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
  B->graph_valid = false;
}

int force_mode(const rlb_batch* B) {
  return (B->fx != 0.0 || B->fy != 0.0) ? FORCE_BODY : FORCE_NONE;
}

bool any_solid(const rlb_batch* B) {
  for (auto* m : B->mem)
    if (m->any_solid) return true;
  return false;
}

TileArgs tile_args(const rlb_batch* B, int parity) {
  TileArgs a;
  a.sh = shared_of(B->mem[0]);
  a.sh.fx = (float)B->fx;
  a.sh.fy = (float)B->fy;
  a.sh.err = B->d_err;
  a.lats = B->d_desc;
  a.tile_lat = B->d_tile_lat;
  a.parity = parity;
  a.tile_first = 0;
  a.ntiles = B->ntiles;
  a.fields = nullptr;
  return a;
}

// rec: J^x of column rec_x of every member, written row by row (see
// records_current) into rec[rec_row + y]
hipError_t launch_batch_step(const rlb_batch* B, int parity, bool mask, int force,
                             double* rec = nullptr, int rec_x = 0, int tile_first = 0,
                             int tiles = -1) {
  const int mode = (B->p.flags & RLB_OPEN_X) ? MODE_OPEN : MODE_STEP;
  TileArgs a = tile_args(B, parity);
  if (tiles >= 0) {   // one group of members
    a.tile_first = tile_first;
    a.ntiles = tiles;
  }
  a.sh.rec = rec;
  a.sh.rec_x = rec_x;
  return launch_tiles(B->Q, stream_mode(B->p.cfl), mask, mode, force, a, B->shape, B->num_cu,
                      B->stream);
}

// the open-channel step kernels write the recorded column themselves
// (every member has nx % 64 != 1)
bool records_current(const rlb_batch* B) { return (B->p.flags & RLB_OPEN_X) != 0; }

rlb_status check_batch(const rlb_batch* B) {
  if (!B) return bfail(RLB_EINVAL, "batch is null");
  return RLB_OK;
}

rlb_status member_parity(const rlb_batch* B, int* parity) {
  const int c = B->mem[0]->cur;
  for (auto* m : B->mem)
    if (m->cur != c)
      return bfail(RLB_ESTATE, "batch members are at different ping-pong phases");
  *parity = c;
  return RLB_OK;
}

void advance(rlb_batch* B, int64_t n) {
  for (auto* m : B->mem) {
    m->cur ^= (int)(n & 1);
    m->step += n;
  }
  B->step += n;
}

}  // namespace

extern "C" {

rlb_status rlb_batch_workspace_bytes(const rlb_params* p, int32_t count, const int32_t* h_nx,
                                     const int32_t* h_ny, size_t* bytes) {
  if (!bytes) return bfail(RLB_EINVAL, "bytes is null");
  BatchLayout L;
  if (rlb_status s = batch_layout(p, count, h_nx, h_ny, L)) return s;
  *bytes = L.total;
  return RLB_OK;
}

rlb_status rlb_batch_create(const rlb_params* p, int32_t count, const int32_t* h_nx,
                            const int32_t* h_ny, void* d_workspace, size_t bytes,
                            void* hip_stream, rlb_batch** out) {
  if (!out) return bfail(RLB_EINVAL, "out is null");
  *out = nullptr;
  BatchLayout L;
  if (rlb_status s = batch_layout(p, count, h_nx, h_ny, L)) return s;
  if (!d_workspace || ((uintptr_t)d_workspace % kAlign))
    return bfail(RLB_EINVAL, "workspace must be a non-null 256-byte aligned device pointer");
  if (bytes < L.total) return bfail(RLB_ENOMEM, "workspace has %zu bytes, needs %zu", bytes, L.total);
  rlb_batch* B = new (std::nothrow) rlb_batch();
  if (!B) return bfail(RLB_ENOMEM, "host allocation failed");
  B->p = *p;
  B->count = count;
  B->ws = (char*)d_workspace;
  B->ws_bytes = bytes;
  B->stream = (hipStream_t)hip_stream;
  B->shape = LaunchShape{4, 0, 16};
  B->graph_steps = 64;
  for (int b = 0; b < count; ++b) B->rec_rows += h_ny[b];
  for (int b = 0; b < count; ++b) {
    rlb_params q = *p;
    q.nx = h_nx[b];
    q.ny = h_ny[b];
    rlb_lattice* m = nullptr;
    rlb_status s = rlb_create(&q, B->ws + L.mem_off[b], L.mem_bytes[b], hip_stream, &m);
    if (s) {
      for (auto* x : B->mem) rlb_destroy(x);
      delete B;
      return s;
    }
    m->owner = B;
    B->mem.push_back(m);
  }
  B->Q = B->mem[0]->Q;
  B->num_cu = B->mem[0]->num_cu;
  B->d_desc = (LatDesc*)(B->ws + L.desc_off);
  B->d_tile_lat = (int32_t*)(B->ws + L.tile_off);
  B->d_err = (uint32_t*)(B->ws + L.err_off);
  hipError_t e = launch_fill_u8((uint8_t*)B->d_err, 64, 0, B->stream);
  rlb_status s = e == hipSuccess ? build_tables(B, B->shape.tile_rows)
                                 : bfail(RLB_EDEVICE, "clear error word: %s", hipGetErrorString(e));
  if (s) {
    for (auto* x : B->mem) rlb_destroy(x);
    delete B;
    return s;
  }
  *out = B;
  return RLB_OK;
}

rlb_status rlb_batch_destroy(rlb_batch* B) {
  if (!B) return RLB_OK;
  drop_graph(B);
  if (B->ev[0]) {
    (void)hipEventDestroy(B->ev[0]);
    (void)hipEventDestroy(B->ev[1]);
  }
  for (auto* m : B->mem) {
    m->owner = nullptr;
    rlb_destroy(m);
  }
  delete B;
  return RLB_OK;
}

rlb_status rlb_batch_member(rlb_batch* B, int32_t b, rlb_lattice** out) {
  if (rlb_status s = check_batch(B)) return s;
  if (!out) return bfail(RLB_EINVAL, "out is null");
  if (b < 0 || b >= B->count) return bfail(RLB_EINVAL, "member %d out of range [0, %d)", b, B->count);
  *out = B->mem[b];
  return RLB_OK;
}

rlb_status rlb_batch_set_body_force(rlb_batch* B, double fx, double fy) {
  if (rlb_status s = check_batch(B)) return s;
  if (!std::isfinite(fx) || !std::isfinite(fy)) return bfail(RLB_EINVAL, "force must be finite");
  if (fx != B->fx || fy != B->fy) drop_graph(B);
  B->fx = fx;
  B->fy = fy;
  for (auto* m : B->mem) {
    m->fx = fx;
    m->fy = fy;
  }
  return RLB_OK;
}

rlb_status rlb_batch_set_open_borders(rlb_batch* B, double bx, double by, double n_in,
                                      double eps_out) {
  if (rlb_status s = check_batch(B)) return s;
  if (!(B->p.flags & RLB_OPEN_X)) return bfail(RLB_EINVAL, "the batch was created without RLB_OPEN_X");
  for (auto* m : B->mem)
    if (rlb_status s = set_open(m, bx, by, n_in, eps_out)) return s;
  drop_graph(B);
  return RLB_OK;
}

rlb_status rlb_batch_set_launch_shape(rlb_batch* B, int32_t tile_rows, int32_t grid_per_cu,
                                      int32_t strip) {
  if (rlb_status s = check_batch(B)) return s;
  if (!(tile_rows == 1 || tile_rows == 2 || tile_rows == 4 || tile_rows == 8))
    return bfail(RLB_EINVAL, "tile_rows must be 1, 2, 4 or 8");
  if (B->Q != 17 && tile_rows != 4) return bfail(RLB_EUNSUPPORTED, "tile_rows != 4 needs the folded layout");
  if (grid_per_cu < 0 || grid_per_cu > 64) return bfail(RLB_EINVAL, "grid_per_cu must be in [0, 64]");
  if (strip < 1 || strip > 65536) return bfail(RLB_EINVAL, "strip must be in [1, 65536]");
  drop_graph(B);
  B->shape = LaunchShape{tile_rows, grid_per_cu, strip};
  return build_tables(B, tile_rows);
}

rlb_status rlb_batch_get_launch_shape(const rlb_batch* B, int32_t* tile_rows, int32_t* grid_per_cu,
                                      int32_t* strip) {
  if (rlb_status s = check_batch(B)) return s;
  if (tile_rows) *tile_rows = B->shape.tile_rows;
  if (grid_per_cu) *grid_per_cu = B->shape.grid_per_cu;
  if (strip) *strip = B->shape.strip;
  return RLB_OK;
}

rlb_status rlb_batch_use_graph(rlb_batch* B, int32_t steps_per_graph) {
  if (rlb_status s = check_batch(B)) return s;
  if (steps_per_graph < 0 || steps_per_graph > 1024 || (steps_per_graph & 1))
    return bfail(RLB_EINVAL, "steps_per_graph must be even and in [0, 1024]");
  drop_graph(B);
  B->graph_steps = steps_per_graph;
  return RLB_OK;
}

rlb_status rlb_batch_step(rlb_batch* B, int64_t nsteps) {
  if (rlb_status s = check_batch(B)) return s;
  if (nsteps < 0) return bfail(RLB_EINVAL, "nsteps must be >= 0");
  int parity = 0;
  if (rlb_status s = member_parity(B, &parity)) return s;
  const bool mask = any_solid(B);
  const int force = force_mode(B);
  if (B->graph_valid && (B->graph_mask != mask || B->graph_force != force)) drop_graph(B);
  if (B->timing) BHIP(hipEventRecord(B->ev[0], B->stream), "event record");
  int64_t left = nsteps;
  const bool graphs = B->graph_steps > 0 && B->stream != nullptr;
  // align to parity 0 so that a replay starts from the first copy
  if (graphs && parity == 1 && left > 0) {
    BHIP(launch_batch_step(B, 1, mask, force), "batch step");
    advance(B, 1);
    --left;
    parity = 0;
  }
  if (graphs && left >= B->graph_steps) {
    if (!B->graph_valid) {
      drop_graph(B);   // a graph whose instantiation failed
      BHIP(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal), "begin capture");
      hipError_t e = hipSuccess;
      if (B->groups.size() > 1) {
        // group by group: each group's state stays in the last-level cache
        // through its graph_steps steps (the members are independent)
        for (const auto& g : B->groups)
          for (int k = 0; k < B->graph_steps && e == hipSuccess; ++k)
            e = launch_batch_step(B, k & 1, mask, force, nullptr, 0, g.first, g.second);
      } else {
        for (int k = 0; k < B->graph_steps && e == hipSuccess; ++k)
          e = launch_batch_step(B, k & 1, mask, force);
      }
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(B->stream, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return bfail(RLB_EDEVICE, "graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
      }
      B->graph = g;
      BHIP(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0), "graph instantiate");
      B->graph_valid = true;
      B->graph_mask = mask;
      B->graph_force = force;
    }
    while (left >= B->graph_steps) {
      BHIP(hipGraphLaunch(B->exec, B->stream), "graph launch");
      advance(B, B->graph_steps);
      left -= B->graph_steps;
    }
  }
  if (left > 1 && B->groups.size() > 1) {
    // direct launches, group by group as in the graph
    for (const auto& g : B->groups)
      for (int64_t k = 0; k < left; ++k)
        BHIP(launch_batch_step(B, (int)((parity + k) & 1), mask, force, nullptr, 0, g.first,
                               g.second), "batch step");
    advance(B, left);
    left = 0;
  }
  while (left > 0) {
    BHIP(launch_batch_step(B, parity, mask, force), "batch step");
    advance(B, 1);
    parity ^= 1;
    --left;
  }
  if (B->timing) {
    BHIP(hipEventRecord(B->ev[1], B->stream), "event record");
    BHIP(hipEventSynchronize(B->ev[1]), "event synchronize");
    float ms = 0.f;
    BHIP(hipEventElapsedTime(&ms, B->ev[0], B->ev[1]), "event elapsed");
    B->timed_ms += ms;
    B->timed_steps += nsteps;
  }
  return RLB_OK;
}

rlb_status rlb_batch_record_workspace_bytes(const rlb_batch* B, int32_t chunk, size_t* bytes) {
  if (rlb_status s = check_batch(B)) return s;
  if (!bytes) return bfail(RLB_EINVAL, "bytes is null");
  if (chunk < 1 || chunk > kBatchRecChunk) return bfail(RLB_EINVAL, "chunk must be in [1, %d]", kBatchRecChunk);
  *bytes = align_up((size_t)chunk * (size_t)B->rec_rows * sizeof(double));
  return RLB_OK;
}

rlb_status rlb_batch_record_current(rlb_batch* B, int64_t nsteps, int32_t x, double* d_series,
                                    int64_t stride, void* d_work, size_t bytes) {
  if (rlb_status s = check_batch(B)) return s;
  if (nsteps < 0) return bfail(RLB_EINVAL, "nsteps must be >= 0");
  for (int b = 0; b < B->count; ++b) {
    const int nx = B->mem[b]->p.nx;
    if (x >= nx || x < -nx)
      return bfail(RLB_EINVAL, "column %d outside member %d (nx = %d)", x, b, nx);
  }
  if (B->p.cfl > 1.0) return bfail(RLB_EUNSUPPORTED, "the column current supports cfl <= 1");
  if (nsteps == 0) return RLB_OK;
  if (stride < nsteps) return bfail(RLB_EINVAL, "stride %lld is below nsteps %lld", (long long)stride,
                                    (long long)nsteps);
  if (!d_series || (uintptr_t)d_series % 8)
    return bfail(RLB_EINVAL, "d_series must be an 8-byte aligned device pointer");
  if (!d_work || (uintptr_t)d_work % kAlign)
    return bfail(RLB_EINVAL, "workspace must be a 256-byte aligned device pointer");
  const size_t step_bytes = (size_t)B->rec_rows * sizeof(double);
  const int64_t chunk = (int64_t)std::min<size_t>(bytes / step_bytes, kBatchRecChunk);
  if (chunk < 1)
    return bfail(RLB_ENOMEM, "record workspace has %zu bytes, needs at least %zu", bytes, step_bytes);
  int parity = 0;
  if (rlb_status s = member_parity(B, &parity)) return s;
  const bool mask = any_solid(B);
  const int force = force_mode(B);
  if (B->timing) BHIP(hipEventRecord(B->ev[0], B->stream), "event record");
  if (records_current(B)) {
    double* rows = (double*)d_work;
    for (int64_t t0 = 0; t0 < nsteps; t0 += chunk) {
      const int64_t cnt = std::min(chunk, nsteps - t0);
      for (int64_t i = 0; i < cnt; ++i) {
        BHIP(launch_batch_step(B, parity, mask, force, rows + i * B->rec_rows, x), "batch step");
        advance(B, 1);
        parity ^= 1;
      }
      BHIP(launch_batch_row_means(B->d_desc, B->count, rows, B->rec_rows, (int)cnt, d_series + t0,
                                  stride, B->stream), "row means");
    }
  } else {   // the column kernel before each step
    const StepShared sh = shared_of(B->mem[0]);
    for (int64_t t = 0; t < nsteps; ++t) {
      BHIP(launch_batch_column_current(sh, B->Q, B->d_desc, B->count, parity, B->p.cfl == 1.0, mask,
                                       x, stride, d_series + t, B->stream), "column current");
      BHIP(launch_batch_step(B, parity, mask, force), "batch step");
      advance(B, 1);
      parity ^= 1;
    }
  }
  if (B->timing) {
    BHIP(hipEventRecord(B->ev[1], B->stream), "event record");
    BHIP(hipEventSynchronize(B->ev[1]), "event synchronize");
    float ms = 0.f;
    BHIP(hipEventElapsedTime(&ms, B->ev[0], B->ev[1]), "event elapsed");
    B->timed_ms += ms;
    B->timed_steps += nsteps;
  }
  return RLB_OK;
}

rlb_status rlb_batch_sync(rlb_batch* B) {
  if (rlb_status s = check_batch(B)) return s;
  uint32_t h = 0;
  BHIP(hipMemcpyAsync(&h, B->d_err, sizeof h, hipMemcpyDeviceToHost, B->stream), "read error flag");
  BHIP(hipStreamSynchronize(B->stream), "stream synchronize");
  if (h & ERR_LANDAU) return bfail(RLB_ELANDAU, "a fluid node had no timelike Landau frame");
  if (h & ERR_NONFINITE) return bfail(RLB_ENONFINITE, "a population became non-finite");
  return RLB_OK;
}

rlb_status rlb_batch_info(const rlb_batch* B, int32_t* count, int64_t* cells, int32_t* planes,
                          int64_t* step) {
  if (rlb_status s = check_batch(B)) return s;
  int64_t c = 0;
  for (auto* m : B->mem) c += (int64_t)m->p.nx * m->p.ny;
  if (count) *count = B->count;
  if (cells) *cells = c;
  if (planes) *planes = B->Q;
  if (step) *step = B->step;
  return RLB_OK;
}

rlb_status rlb_batch_autotune(rlb_batch* B, int32_t trials, double* h_ms, int32_t max_results) {
  if (rlb_status s = check_batch(B)) return s;
  if (trials < 1 || trials > 1000) return bfail(RLB_EINVAL, "trials must be in [1, 1000]");
  int parity = 0;
  if (rlb_status s = member_parity(B, &parity)) return s;
  const bool mask = any_solid(B);
  const int force = force_mode(B);
  drop_graph(B);
  const std::vector<LaunchShape> cand = launch_candidates(B->Q, true);
  hipEvent_t e0, e1;
  BHIP(hipEventCreate(&e0), "event");
  BHIP(hipEventCreate(&e1), "event");
  double best = 1e300;
  LaunchShape win = B->shape;
  int k = 0;
  rlb_status st = RLB_OK;
  for (const LaunchShape& c : cand) {
    B->shape = c;
    if ((st = build_tables(B, c.tile_rows))) break;
    hipError_t e = hipSuccess;
    // reads the current copies and overwrites the others: no member advances
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = launch_batch_step(B, parity, mask, force);
    if (e == hipSuccess) e = hipEventRecord(e0, B->stream);
    for (int i = 0; i < trials && e == hipSuccess; ++i) e = launch_batch_step(B, parity, mask, force);
    if (e == hipSuccess) e = hipEventRecord(e1, B->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      st = bfail(RLB_EDEVICE, "autotune: %s", hipGetErrorString(e));
      break;
    }
    const double per = ms / trials;
    if (h_ms && k < max_results) {
      h_ms[4 * k] = c.tile_rows;
      h_ms[4 * k + 1] = c.grid_per_cu;
      h_ms[4 * k + 2] = c.strip;
      h_ms[4 * k + 3] = per;
    }
    ++k;
    if (per < best) {
      best = per;
      win = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  B->shape = win;
  if (rlb_status s2 = build_tables(B, win.tile_rows)) return s2;
  return st;
}

rlb_status rlb_batch_timing(rlb_batch* B, int32_t enable) {
  if (rlb_status s = check_batch(B)) return s;
  if (enable && !B->ev[0]) {
    BHIP(hipEventCreate(&B->ev[0]), "event create");
    BHIP(hipEventCreate(&B->ev[1]), "event create");
  }
  B->timing = enable != 0;
  B->timed_ms = 0.0;
  B->timed_steps = 0;
  return RLB_OK;
}

rlb_status rlb_batch_timing_read(rlb_batch* B, double* total_ms, int64_t* steps) {
  if (rlb_status s = check_batch(B)) return s;
  if (total_ms) *total_ms = B->timed_ms;
  if (steps) *steps = B->timed_steps;
  return RLB_OK;
}

}  // extern "C"
