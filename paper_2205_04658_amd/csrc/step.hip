// The fused RLB step for gfx950: pull-stream -> moments -> Landau matching
// -> equilibrium -> Anderson-Witting relaxation + driving term, with
// bounce-back at solid nodes; plus the field read-out and initialisation
// kernels that reuse its pieces.
//
// Layout: 2Q float32 planes [plane][ny][nx] (F planes 0..Q-1, G planes
// Q..2Q-1), x fastest, plane pitch a multiple of 64 elements.  One thread
// per node; a 256-thread workgroup covers 64 x 4 nodes and each wavefront
// one row, so row-uniform quantities (y, the stirring table row) are scalar.
// Workgroups are mapped to tiles so that each of the eight XCDs walks a
// contiguous band of tiles: vertically adjacent tiles, which share halo
// rows, then run on the same XCD and meet in its L2.
#include "internal.hpp"
#include "device_common.hpp"
#include "dirset.hpp"

namespace rlb {

template <class DS, int P>
struct Taps {
  static constexpr double vx = DS::vx[P], vy = DS::vy[P];
  static constexpr int sx = vx > 0 ? 1 : (vx < 0 ? -1 : 0);
  static constexpr int sy = vy > 0 ? 1 : (vy < 0 ? -1 : 0);
  static constexpr bool unit_x = vx == 1.0 || vx == -1.0;
  static constexpr bool unit_y = vy == 1.0 || vy == -1.0;
};

// Pull value of plane P at node (x, y): bilinear interpolation of the
// pre-stream plane at the departure point (x, y) - cfl (vx, vy).
template <class DS, bool UNIT, int P>
__device__ __forceinline__ float pull(const float* __restrict__ pl,
                                      const StepArgs& a, int r0, int rm,
                                      int rp, int x, int xm, int xp) {
  using T = Taps<DS, P>;
  const int xs = T::sx > 0 ? xm : xp;      // column x - sx
  const int rs = T::sy > 0 ? rm : rp;      // row y - sy
  if constexpr (T::sx == 0 && T::sy == 0) {
    return pl[r0 + x];
  } else if constexpr (UNIT && T::unit_x) {
    return pl[r0 + xs];                    // full step along x
  } else if constexpr (UNIT && T::unit_y) {
    return pl[rs + x];                     // full step along y
  } else if constexpr (T::sy == 0) {
    return a.tap[P][0] * pl[r0 + x] + a.tap[P][1] * pl[r0 + xs];
  } else if constexpr (T::sx == 0) {
    return a.tap[P][0] * pl[r0 + x] + a.tap[P][2] * pl[rs + x];
  } else {
    return a.tap[P][0] * pl[r0 + x] + a.tap[P][1] * pl[r0 + xs] +
           a.tap[P][2] * pl[rs + x] + a.tap[P][3] * pl[rs + xs];
  }
}

template <class DS, bool UNIT, bool MASK, int FORCE, int MODE>
__global__ __launch_bounds__(kBlock) void step_kernel(const StepArgs a) {
  constexpr int Q = DS::Q;
  const int hw = blockIdx.x;
  const int tile = (hw & 7) * a.tiles_per_xcd + (hw >> 3);
  if (tile >= a.ntiles) return;
  const int ty = tile / a.tiles_x;
  const int tx = tile - ty * a.tiles_x;
  const int x = tx * kTileX + (threadIdx.x & (kTileX - 1));
  const int y = __builtin_amdgcn_readfirstlane(ty * kTileY + (threadIdx.x >> 6));
  if (x >= a.nx || y >= a.ny) return;

  const int nx = a.nx, ny = a.ny;
  const int xm = x == 0 ? nx - 1 : x - 1;
  const int xp = x == nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1;
  const int yp = y == ny - 1 ? 0 : y + 1;
  const int r0 = y * nx, rm = ym * nx, rp = yp * nx;
  const int node = r0 + x;

  // 1. pull-stream every plane
  float f[Q], g[Q];
  static_for<0, Q>([&](auto P) {
    constexpr int p = decltype(P)::value;
    f[p] = pull<DS, UNIT, p>(a.src + p * a.pitch, a, r0, rm, rp, x, xm, xp);
    g[p] = pull<DS, UNIT, p>(a.src + (Q + p) * a.pitch, a, r0, rm, rp, x, xm, xp);
  });

  bool solid = false;
  if constexpr (MASK) solid = a.mask[node] != 0;

  if constexpr (MODE == MODE_STEP) {
    if (solid) {   // bounce-back: F'_i = F~_opp(i)
      static_for<0, Q>([&](auto P) {
        constexpr int p = decltype(P)::value;
        __builtin_nontemporal_store(f[DS::opp[p]], a.dst + p * a.pitch + node);
        __builtin_nontemporal_store(g[DS::opp[p]], a.dst + (Q + p) * a.pitch + node);
      });
      return;
    }
  }

  // 2. moments of the deviations from the reference (float32 sums of small
  //    numbers), then the reference added in float64
  float m00 = 0, m0x = 0, m0y = 0, mxx = 0, mxy = 0, myy = 0;
  float j0 = 0, jx = 0, jy = 0;
  static_for<0, Q>([&](auto P) {
    constexpr int p = decltype(P)::value;
    constexpr float vx = (float)DS::vx[p], vy = (float)DS::vy[p];
    m00 += f[p];
    j0 += g[p];
    constexpr float vxx = (float)(DS::vx[p] * DS::vx[p]);
    constexpr float vyy = (float)(DS::vy[p] * DS::vy[p]);
    constexpr float vxy = (float)(DS::vx[p] * DS::vy[p]);
    if constexpr (DS::vx[p] != 0.0) { m0x += vx * f[p]; jx += vx * g[p]; mxx += vxx * f[p]; }
    if constexpr (DS::vy[p] != 0.0) { m0y += vy * f[p]; jy += vy * g[p]; myy += vyy * f[p]; }
    if constexpr (DS::vx[p] != 0.0 && DS::vy[p] != 0.0) mxy += vxy * f[p];
  });
  const double T00 = a.eps_ref + (double)m00;
  const double T0x = (double)m0x, T0y = (double)m0y;
  const double Txx = a.eps_ref * (1.0 / 3.0) + (double)mxx;
  const double Tyy = a.eps_ref * (1.0 / 3.0) + (double)myy;
  const double Txy = (double)mxy;
  const double J0 = a.n_ref + (double)j0, Jx = (double)jx, Jy = (double)jy;

  // 3. Landau frame and charge density
  Frame fr{0.0, 1.0, 0.0, 0.0};
  bool ok = landau3(T00, T0x, T0y, Txx, Txy, Tyy, fr);
  const double n = fr.u0 * J0 - fr.ux * Jx - fr.uy * Jy;
  ok = ok && (n == n);

  if constexpr (MODE == MODE_FIELDS) {
    const double vals[RLB_FIELD_COUNT] = {
        fr.eps, fr.ux / fr.u0, fr.uy / fr.u0, n, T00, T0x, T0y,
        Txx, Txy, Tyy, J0, Jx, Jy};
    if (!ok && !solid) atomicOr(a.err, ERR_LANDAU);
    int k = 0;
    const size_t plane = (size_t)nx * ny;
#pragma unroll
    for (int fld = 0; fld < RLB_FIELD_COUNT; ++fld) {
      if (a.field_mask & (1u << fld)) {
        a.fields[k * plane + node] = (solid || !ok) ? 0.0f : (float)vals[fld];
        ++k;
      }
    }
    return;
  } else {
    if (!ok) {   // no rest frame: flag it and leave the node uncollided
      atomicOr(a.err, ERR_LANDAU);
      static_for<0, Q>([&](auto P) {
        constexpr int p = decltype(P)::value;
        a.dst[p * a.pitch + node] = f[p];
        a.dst[(Q + p) * a.pitch + node] = g[p];
      });
      return;
    }

    // 4. equilibrium and collision-rate coefficients
    const EqCoef ec = eq_coef(fr, n, a.eps_ref, a.n_ref);
    const float ux = (float)fr.ux, uy = (float)fr.uy;
    const float w0 = (float)fr.u0 * a.inv_tau;
    const float wx = ux * a.inv_tau, wy = uy * a.inv_tau;

    // 5. driving term coefficients: Phi(v) = p0 + px vx + py vy + pxx vx^2
    //    + pxy vx vy + pyy vy^2 (vz^2 = 1 - vx^2 - vy^2 folded in)
    float p0 = 0, px = 0, py = 0, pxx = 0, pxy = 0, pyy = 0;
    if constexpr (FORCE != FORCE_NONE) {
      float Fx = a.fx, Fy = a.fy;
      if constexpr (FORCE == FORCE_STIR) stir_series(a.table, a.K, a.theta_scale, nx, x, y, Fx, Fy);
      float q3xxx = 0, q3xxy = 0, q3xyy = 0, q3yyy = 0, q3xzz = 0, q3yzz = 0;
      static_for<0, Q>([&](auto P) {
        constexpr int p = decltype(P)::value;
        constexpr double vx = DS::vx[p], vy = DS::vy[p], vz2 = DS::vz2[p];
        if constexpr (vx != 0.0) {
          q3xxx += (float)(vx * vx * vx) * f[p];
          if constexpr (vz2 != 0.0) q3xzz += (float)(vx * vz2) * f[p];
        }
        if constexpr (vy != 0.0) {
          q3yyy += (float)(vy * vy * vy) * f[p];
          if constexpr (vz2 != 0.0) q3yzz += (float)(vy * vz2) * f[p];
        }
        if constexpr (vx != 0.0 && vy != 0.0) {
          q3xxy += (float)(vx * vx * vy) * f[p];
          q3xyy += (float)(vx * vy * vy) * f[p];
        }
      });
      const float M0 = (float)T00, M1x = (float)T0x, M1y = (float)T0y;
      const float Qxx = Fx * q3xxx + Fy * q3xxy;
      const float Qxy = Fx * q3xxy + Fy * q3xyy;
      const float Qyy = Fx * q3xyy + Fy * q3yyy;
      const float Qzz = Fx * q3xzz + Fy * q3yzz;
      const float FM1 = Fx * M1x + Fy * M1y;
      const float pzz = 1.25f * Qzz;
      p0 = 0.25f * FM1 + pzz;
      px = -0.5f * Fx * M0;
      py = -0.5f * Fy * M0;
      pxx = 1.25f * Qxx - 2.5f * Fx * M1x - pzz;
      pxy = 2.5f * Qxy - 2.5f * (Fx * M1y + Fy * M1x);
      pyy = 1.25f * Qyy - 2.5f * Fy * M1y - pzz;
    }

    // 6. relax and drive, store
    static_for<0, Q>([&](auto P) {
      constexpr int p = decltype(P)::value;
      constexpr float vx = (float)DS::vx[p], vy = (float)DS::vy[p];
      constexpr float w = (float)DS::w[p];
      const float s = ux * vx + uy * vy;
      const float om = w0 - (wx * vx + wy * vy);
      const float feq = w * (ec.A + s * (ec.B + s * ec.C));
      const float geq = w * (ec.Ag + s * ec.Bg);
      float fn = f[p] - om * (f[p] - feq);
      if constexpr (FORCE != FORCE_NONE) {
        const float phi = p0 + vx * (px + vx * pxx + vy * pxy) + vy * (py + vy * pyy);
        fn -= w * phi;
      }
      const float gn = g[p] - om * (g[p] - geq);
      __builtin_nontemporal_store(fn, a.dst + p * a.pitch + node);
      __builtin_nontemporal_store(gn, a.dst + (Q + p) * a.pitch + node);
    });
  }
}

// Initial state: F = F_eq(eps, u), G = G_eq(n, u) in shifted form.
template <class DS>
__global__ __launch_bounds__(256) void init_kernel(
    const float* __restrict__ eps, const float* __restrict__ bx,
    const float* __restrict__ by, const float* __restrict__ nn, float* dst,
    int64_t pitch, int32_t ncell, double eps_ref, double n_ref, uint32_t* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncell) return;
  Frame fr;
  if (!frame_from_beta((double)eps[i], (double)bx[i], (double)by[i], fr)) {
    atomicOr(err, ERR_LANDAU);
    fr.eps = eps_ref; fr.u0 = 1.0; fr.ux = 0.0; fr.uy = 0.0;
  }
  const EqCoef ec = eq_coef(fr, (double)nn[i], eps_ref, n_ref);
  const float ux = (float)fr.ux, uy = (float)fr.uy;
  static_for<0, DS::Q>([&](auto P) {
    constexpr int p = decltype(P)::value;
    constexpr float vx = (float)DS::vx[p], vy = (float)DS::vy[p];
    constexpr float w = (float)DS::w[p];
    const float s = ux * vx + uy * vy;
    dst[p * pitch + i] = w * (ec.A + s * (ec.B + s * ec.C));
    dst[(DS::Q + p) * pitch + i] = w * (ec.Ag + s * ec.Bg);
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
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static void fill_args(const rlb_lattice* lat, StepArgs& a) {
  const int nx = lat->p.nx, ny = lat->p.ny;
  a.pitch = lat->pitch;
  a.nx = nx;
  a.ny = ny;
  a.tiles_x = (nx + kTileX - 1) / kTileX;
  a.ntiles = a.tiles_x * ((ny + kTileY - 1) / kTileY);
  a.tiles_per_xcd = (a.ntiles + 7) / 8;
  a.mask = lat->any_solid ? lat->mask : nullptr;
  for (int p = 0; p < kMaxQ; ++p)
    for (int c = 0; c < 4; ++c) a.tap[p][c] = lat->tap[p][c];
  a.inv_tau = (float)(1.0 / lat->p.tau);
  a.eps_ref = lat->p.eps_ref;
  a.n_ref = lat->p.n_ref;
  a.fx = (float)lat->fx;
  a.fy = (float)lat->fy;
  a.table = lat->table;
  a.K = lat->K;
  a.theta_scale = 2.0f / (float)nx;
  a.err = lat->err;
}

template <class DS, bool UNIT, bool MASK, int MODE>
static hipError_t dispatch_force(int force, const StepArgs& a, dim3 grid,
                                 hipStream_t s) {
  if constexpr (MODE == MODE_FIELDS) {
    hipLaunchKernelGGL((step_kernel<DS, UNIT, MASK, FORCE_NONE, MODE>), grid,
                       dim3(kBlock), 0, s, a);
  } else {
    switch (force) {
      case FORCE_NONE:
        hipLaunchKernelGGL((step_kernel<DS, UNIT, MASK, FORCE_NONE, MODE>),
                           grid, dim3(kBlock), 0, s, a);
        break;
      case FORCE_BODY:
        hipLaunchKernelGGL((step_kernel<DS, UNIT, MASK, FORCE_BODY, MODE>),
                           grid, dim3(kBlock), 0, s, a);
        break;
      default:
        hipLaunchKernelGGL((step_kernel<DS, UNIT, MASK, FORCE_STIR, MODE>),
                           grid, dim3(kBlock), 0, s, a);
        break;
    }
  }
  return hipGetLastError();
}

template <class DS>
static hipError_t dispatch(bool unit, bool mask, int mode, int force,
                           const StepArgs& a, dim3 grid, hipStream_t s) {
  if (mode == MODE_FIELDS) {
    if (unit) return mask ? dispatch_force<DS, true, true, MODE_FIELDS>(force, a, grid, s)
                          : dispatch_force<DS, true, false, MODE_FIELDS>(force, a, grid, s);
    return mask ? dispatch_force<DS, false, true, MODE_FIELDS>(force, a, grid, s)
                : dispatch_force<DS, false, false, MODE_FIELDS>(force, a, grid, s);
  }
  if (unit) return mask ? dispatch_force<DS, true, true, MODE_STEP>(force, a, grid, s)
                        : dispatch_force<DS, true, false, MODE_STEP>(force, a, grid, s);
  return mask ? dispatch_force<DS, false, true, MODE_STEP>(force, a, grid, s)
              : dispatch_force<DS, false, false, MODE_STEP>(force, a, grid, s);
}

hipError_t launch_step(const rlb_lattice* lat, int mode, int force_mode,
                       const float* src, float* dst, float* fields,
                       uint32_t field_mask) {
  StepArgs a;
  fill_args(lat, a);
  a.src = src;
  a.dst = dst;
  a.fields = fields;
  a.field_mask = field_mask;
  const dim3 grid(8 * a.tiles_per_xcd);
  const bool unit = lat->p.cfl == 1.0;
  const bool mask = a.mask != nullptr;
  if (lat->Q == 17) return dispatch<Dir17>(unit, mask, mode, force_mode, a, grid, lat->stream);
  return dispatch<Dir26>(unit, mask, mode, force_mode, a, grid, lat->stream);
}

hipError_t launch_init(const rlb_lattice* lat, const float* eps,
                       const float* bx, const float* by, const float* n,
                       float* dst) {
  const int ncell = lat->p.nx * lat->p.ny;
  const dim3 grid((ncell + 255) / 256);
  if (lat->Q == 17)
    hipLaunchKernelGGL(init_kernel<Dir17>, grid, dim3(256), 0, lat->stream, eps,
                       bx, by, n, dst, lat->pitch, ncell, lat->p.eps_ref,
                       lat->p.n_ref, lat->err);
  else
    hipLaunchKernelGGL(init_kernel<Dir26>, grid, dim3(256), 0, lat->stream, eps,
                       bx, by, n, dst, lat->pitch, ncell, lat->p.eps_ref,
                       lat->p.n_ref, lat->err);
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
  hipLaunchKernelGGL(fill_u8_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256),
                     0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace rlb
