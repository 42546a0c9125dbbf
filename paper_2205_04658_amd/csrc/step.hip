// The fused RLB step for gfx950: pull-stream -> moments -> Landau matching
// -> equilibrium -> Anderson-Witting relaxation + driving term, with
// bounce-back at solid nodes (the kernel templates: step_kernels.hpp; this
// file holds their non-temporal-store instantiations, the launch logic and
// the initialisation kernels).  Modes of the tile kernel: a step; the
// field read-out; a step that also sets the open x borders (and may record
// a column's current); a step that also sums the adjoint's objective.
//
// Layout: node bricks (brick.hpp): each lattice row is a run of 64-node
// bricks holding the 2Q planes of their nodes (F planes 0..Q-1, then G
// planes Q..2Q-1).  The stirring force keeps two plain [ny][row] planes.
// One thread per node; a tile is 64 x TY nodes, one wavefront per row, so
// row-uniform quantities are scalar.  A launch walks a list of tiles that
// may span many lattices (the batched path): each tile names its lattice,
// whose descriptor is read with scalar loads.  A lattice's tiles are
// ordered in vertical strips a few tiles wide and the eight XCDs each take
// a contiguous band of that order, so tiles that share halo rows and
// columns run on the same XCD close together and meet in its L2.  The grid
// is either one workgroup per tile or a persistent set of workgroups per
// CU.

#include <algorithm>

#include "step_kernels.hpp"

namespace rlb {

// Initial state: F = F_eq(eps, u), G = G_eq(n, u) in shifted form.
template <class DS>
__global__ __launch_bounds__(256) void init_kernel(
    const float* __restrict__ eps, const float* __restrict__ bx,
    const float* __restrict__ by, const float* __restrict__ nn, float* dst,
    int32_t nx, int32_t ny, int32_t row, double eps_ref, double n_ref,
    uint32_t* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nx * ny) return;
  const int yy = i / nx, xx = i - yy * nx;
  Frame fr;
  if (!frame_from_beta((double)eps[i], (double)bx[i], (double)by[i], fr)) {
    atomicOr(err, ERR_LANDAU);
    fr.eps = eps_ref; fr.u0 = 1.0; fr.ux = 0.0; fr.uy = 0.0;
  }
  const EqCoef ec = eq_coef<DS::planar>(fr, (double)nn[i], eps_ref, n_ref, DS::kappa);
  const float ux = (float)fr.ux, uy = (float)fr.uy;
  static_for<0, DS::Q>([&](auto P) {
    constexpr int p = decltype(P)::value;
    constexpr float vx = (float)DS::vx[p], vy = (float)DS::vy[p];
    constexpr float w = DS::w32[p];
    const float s = ux * vx + uy * vy;
    dst[state_elem<DS::Q>(p, xx, yy, row)] = w * (ec.A + s * (ec.B + s * ec.C));
    dst[state_elem<DS::Q>(DS::Q + p, xx, yy, row)] = w * (ec.Ag + s * ec.Bg);
  });
}

// Disc rasterisation: solid when dx^2 + dy^2 <= r^2 (periodic minimum
// image).  Contraction is off so the test matches an unfused evaluation.
__global__ __launch_bounds__(256) void disks_kernel(uint8_t* mask, int nx,
                                                    int ny,
                                                    const double* __restrict__ d,
                                                    int count) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nx * ny) return;
  const int y = i / nx, x = i - y * nx;
  uint8_t s = 0;
  for (int k = 0; k < count; ++k) {
    double dx = (double)x - d[3 * k];
    dx = dx - (double)nx * rint(dx / (double)nx);
    double dy = (double)y - d[3 * k + 1];
    dy = dy - (double)ny * rint(dy / (double)ny);
    const double r = d[3 * k + 2];
    const double lhs = dx * dx + dy * dy;
    if (lhs <= r * r) s = 1;
  }
  if (s) mask[i] = 1;
}

__global__ __launch_bounds__(256) void mask_or_kernel(uint8_t* mask,
                                                      const uint8_t* __restrict__ m,
                                                      int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && m[i]) mask[i] = 1;
}

__global__ __launch_bounds__(256) void walls_kernel(uint8_t* mask, int nx,
                                                    int ny) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nx) {
    mask[i] = 1;
    mask[(size_t)(ny - 1) * nx + i] = 1;
  }
}

__global__ __launch_bounds__(256) void fill_u8_kernel(uint8_t* p, size_t n,
                                                      uint8_t v) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
StepShared shared_of(const rlb_lattice* lat) {
  StepShared a;
  for (int p = 0; p < kMaxQ; ++p) {
    for (int c = 0; c < 4; ++c) a.tap[p][c] = lat->tap[p][c];
    a.shift[p][0] = lat->shift[p][0];
    a.shift[p][1] = lat->shift[p][1];
  }
  a.inv_tau = (float)(1.0 / lat->p.tau);
  a.tau_k = lat->tau_k;
  a.eps_ref = lat->p.eps_ref;
  a.n_ref = lat->p.n_ref;
  a.fx = (float)lat->fx;
  a.fy = (float)lat->fy;
  a.o_bx = lat->open.bx;
  a.o_by = lat->open.by;
  a.o_n = lat->open.n_in;
  a.o_eps = lat->open.eps_out;
  a.err = lat->err;
  a.field_mask = 0;
  a.rec = nullptr;
  a.rec_x = 0;
  a.obj = nullptr;
  a.obj_kind = 0;
  return a;
}

int tiles_of(int nx, int ny, int tile_rows) {
  return ((nx + 63) / 64) * ((ny + tile_rows - 1) / tile_rows);
}

int kernel_tile_rows(int Q, int mode, int tile_rows) {
  if (mode == MODE_FIELDS) return 4;
  if (Q == 17) return tile_rows;
  if (Q == 26 && mode == MODE_STEP && tile_rows == 2) return 2;
  return 4;
}

std::vector<LaunchShape> launch_candidates(int Q, bool batch) {
  std::vector<LaunchShape> c;
  for (int ty : {1, 2, 4, 8})
    for (int g : {0, 4})
      for (int sw : {4, 8, 16, 32})
        if (Q == 17 || ty == 4 || (Q == 26 && ty == 2 && !batch)) c.push_back(LaunchShape{ty, g, sw});
  return c;
}

int step_mode(const rlb_lattice* lat) {
  return ((lat->p.flags & RLB_OPEN_X) && lat->p.nx % 64 != 1) ? MODE_OPEN : MODE_STEP;
}

bool records_current(const rlb_lattice* lat) {
  return step_mode(lat) == MODE_OPEN || lat->Q == 26;
}

int stream_mode(double cfl) { return cfl == 1.0 ? SM_UNIT : (cfl > 1.0 ? SM_WIDE : SM_GENERAL); }

hipError_t launch_tiles(int Q, int sm, bool mask, int mode, int force_mode,
                        const TileArgs& a0, LaunchShape shape, int num_cu, hipStream_t s) {
  if (a0.ntiles <= 0) return hipSuccess;
  TileArgs a = a0;
  const int ty = kernel_tile_rows(Q, mode, shape.tile_rows);
  a.tiles_per_xcd = (a.ntiles + 7) / 8;
  a.strip = std::max(1, shape.strip);
  int grid;
  if (shape.grid_per_cu <= 0) {
    grid = 8 * a.tiles_per_xcd;
  } else {
    // resident workgroups, rounded to a multiple of the 8 XCDs
    grid = std::max(8, (num_cu * shape.grid_per_cu * 4 / ty) / 8 * 8);
    grid = std::min(grid, 8 * a.tiles_per_xcd);
  }
  // both state copies of the launch (padding columns included)
  const double state_bytes = 2.0 * a.ntiles * 64 * ty * (2 * Q) * sizeof(float);
  if (mode != MODE_FIELDS && state_bytes <= kCachedStateBytes)
    return launch_tiles_cached(Q, sm, mask, mode, force_mode, a, ty, grid, s);
  if (Q == 17) by_flags<Dir17, true>(sm, mask, mode, force_mode, ty, a, grid, s);
  else if (Q == 12) by_flags<DirP12, true>(sm, mask, mode, force_mode, ty, a, grid, s);
  else by_flags<Dir26, true>(sm, mask, mode, force_mode, ty, a, grid, s);
  return hipGetLastError();
}

hipError_t launch_step(const rlb_lattice* lat, int mode, int force_mode, int parity,
                       float* fields, uint32_t field_mask, double* rec, int rec_x, double* obj,
                       int obj_kind) {
  TileArgs a;
  a.sh = shared_of(lat);
  a.sh.field_mask = field_mask;
  a.sh.rec = rec;
  a.sh.rec_x = rec_x;
  a.sh.obj = obj;
  a.sh.obj_kind = obj_kind;
  a.lats = lat->d_desc;
  a.tile_lat = nullptr;
  a.parity = parity;
  a.tile_first = 0;
  const int ty = kernel_tile_rows(lat->Q, mode, lat->shape.tile_rows);
  a.ntiles = tiles_of(lat->p.nx, lat->p.ny, ty);
  a.fields = fields;
  LaunchShape sh = lat->shape;
  if (mode == MODE_FIELDS) sh.grid_per_cu = 0;
  return launch_tiles(lat->Q, stream_mode(lat->p.cfl), lat->any_solid, mode, force_mode, a, sh,
                      lat->num_cu, lat->stream);
}

hipError_t launch_init(const rlb_lattice* lat, const float* eps,
                       const float* bx, const float* by, const float* n,
                       float* dst) {
  const int ncell = lat->p.nx * lat->p.ny;
  const dim3 grid((ncell + 255) / 256);
  if (lat->Q == 17)
    hipLaunchKernelGGL(init_kernel<Dir17>, grid, dim3(256), 0, lat->stream, eps,
                       bx, by, n, dst, lat->p.nx, lat->p.ny, lat->row,
                       lat->p.eps_ref, lat->p.n_ref, lat->err);
  else if (lat->Q == 12)
    hipLaunchKernelGGL(init_kernel<DirP12>, grid, dim3(256), 0, lat->stream, eps,
                       bx, by, n, dst, lat->p.nx, lat->p.ny, lat->row,
                       lat->p.eps_ref, lat->p.n_ref, lat->err);
  else
    hipLaunchKernelGGL(init_kernel<Dir26>, grid, dim3(256), 0, lat->stream, eps,
                       bx, by, n, dst, lat->p.nx, lat->p.ny, lat->row,
                       lat->p.eps_ref, lat->p.n_ref, lat->err);
  return hipGetLastError();
}

hipError_t launch_disks(const rlb_lattice* lat, const double* d_discs,
                        int count) {
  const int ncell = lat->p.nx * lat->p.ny;
  hipLaunchKernelGGL(disks_kernel, dim3((ncell + 255) / 256), dim3(256), 0,
                     lat->stream, lat->mask, lat->p.nx, lat->p.ny, d_discs, count);
  return hipGetLastError();
}

hipError_t launch_mask_or(const rlb_lattice* lat, const uint8_t* d_mask) {
  const int ncell = lat->p.nx * lat->p.ny;
  hipLaunchKernelGGL(mask_or_kernel, dim3((ncell + 255) / 256), dim3(256), 0,
                     lat->stream, lat->mask, d_mask, ncell);
  return hipGetLastError();
}

hipError_t launch_walls(const rlb_lattice* lat) {
  hipLaunchKernelGGL(walls_kernel, dim3((lat->p.nx + 255) / 256), dim3(256), 0,
                     lat->stream, lat->mask, lat->p.nx, lat->p.ny);
  return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, size_t n, uint8_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(fill_u8_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace rlb
