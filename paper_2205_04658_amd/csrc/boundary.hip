// Open x borders and the current-density diagnostics of the channel-flow
// workload (Ch. 5, "Model and Methods": a fixed velocity enters along the
// inflow border, lateral borders are periodic; the current density is
// recorded at the outflow border over time and along the channel, and its
// fluctuations are examined in frequency and wave-number space).
//
// Borders of the new state after every step:
//   * velocity inlet, column 0: equilibrium at the prescribed 3-velocity
//     and charge density, with the energy density of column 1;
//   * pressure outlet, column nx-1: equilibrium at the prescribed energy
//     density, with the velocity and charge density of column nx-2.
// The adjacent columns' frames come from Landau matching of their stored
// (post-collision) moments.  Streaming stays periodic: the wrapped values
// reach only the two border columns, which are overwritten.  The step
// kernel sets the borders itself (open_borders in step_kernels.hpp, same
// arithmetic); the kernel here serves widths with nx % 64 == 1, where the
// outlet column and column nx-2 fall in different 64-node tiles.
#include <algorithm>

#include "internal.hpp"
#include "device_common.hpp"
#include "dirset.hpp"
#include "brick.hpp"

namespace rlb {

template <class DS>
__global__ __launch_bounds__(256) void open_borders_kernel(float* __restrict__ st, int nx, int ny,
                                                           int row, const OpenArgs o) {
  constexpr int Q = DS::Q;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * ny) return;
  const int side = i / ny, y = i - side * ny;   // 0 inlet, 1 outlet
  const int xs = side == 0 ? 1 : nx - 2;        // adjacent column
  const int xd = side == 0 ? 0 : nx - 1;        // border column
  // moments of the adjacent node (deviations summed in float32, the
  // references added in float64, as in the step)
  float m00 = 0, m0x = 0, m0y = 0, mxx = 0, mxy = 0, myy = 0, j0 = 0, jx = 0, jy = 0;
  static_for<0, Q>([&](auto P) {
    constexpr int p = decltype(P)::value;
    constexpr double vx = DS::vx[p], vy = DS::vy[p];
    const float f = st[state_elem<Q>(p, xs, y, row)];
    const float g = st[state_elem<Q>(Q + p, xs, y, row)];
    m00 += f;
    j0 += g;
    if constexpr (vx != 0.0) { m0x += (float)vx * f; jx += (float)vx * g; mxx += (float)(vx * vx) * f; }
    if constexpr (vy != 0.0) { m0y += (float)vy * f; jy += (float)vy * g; myy += (float)(vy * vy) * f; }
    if constexpr (vx != 0.0 && vy != 0.0) mxy += (float)(vx * vy) * f;
  });
  const double T00 = o.eps_ref + (double)m00;
  const double Txx = o.eps_ref * (1.0 / 3.0) + (double)mxx;
  const double Tyy = o.eps_ref * (1.0 / 3.0) + (double)myy;
  Frame fr{o.eps_ref, 1.0, 0.0, 0.0};
  if (!landau3(T00, (double)m0x, (double)m0y, Txx, (double)mxy, Tyy, fr)) {
    atomicOr(o.err, ERR_LANDAU);
    fr = Frame{o.eps_ref, 1.0, 0.0, 0.0};
  }
  Frame b;
  double n;
  if (side == 0) {
    frame_from_beta(fr.eps, o.bx, o.by, b);   // |beta| < 1 checked on the host
    n = o.n_in;
  } else {
    b = Frame{o.eps_out, fr.u0, fr.ux, fr.uy};
    n = fr.u0 * (o.n_ref + (double)j0) - fr.ux * (double)jx - fr.uy * (double)jy;
  }
  const EqCoef ec = eq_coef(b, n, o.eps_ref, o.n_ref, DS::kappa);
  const float ux = (float)b.ux, uy = (float)b.uy;
  static_for<0, Q>([&](auto P) {
    constexpr int p = decltype(P)::value;
    constexpr float vx = (float)DS::vx[p], vy = (float)DS::vy[p];
    constexpr float w = DS::w32[p];
    const float s = ux * vx + uy * vy;
    st[state_elem<Q>(p, xd, y, row)] = w * (ec.A + s * (ec.B + s * ec.C));
    st[state_elem<Q>(Q + p, xd, y, row)] = w * (ec.Ag + s * ec.Bg);
  });
}

// j at column x: the mean over the column's nodes of the charge current
// J^x of the streamed populations (solid nodes count as zero), one
// workgroup of 256, fixed summation order; the result is valid in thread 0.
template <class DS, bool UNIT, bool MASK>
__device__ double column_mean(const float* __restrict__ st, const uint8_t* __restrict__ mask,
                              const StepShared& sh, int nx, int ny, int row, int x) {
  constexpr int Q = DS::Q;
  double acc = 0.0;
  for (int y = threadIdx.x; y < ny; y += blockDim.x) {
    if (MASK && mask[(size_t)y * nx + x]) continue;
    const Nbr nb = neighbourhood<Q>(x, y, nx, ny, row);
    float jx = 0.0f;
    static_for<0, Q>([&](auto P) {
      constexpr int p = decltype(P)::value;
      if constexpr (DS::vx[p] != 0.0)
        jx += (float)DS::vx[p] * pull<DS, UNIT, p, Q + p, false>(st, nb, sh.tap[p]);
    });
    acc += (double)jx;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  return ((red[0] + red[1]) + (red[2] + red[3])) / (double)ny;
}

template <class DS, bool UNIT, bool MASK>
__global__ __launch_bounds__(256) void column_current_kernel(const float* __restrict__ st,
                                                             const uint8_t* __restrict__ mask,
                                                             const StepShared sh, int nx, int ny,
                                                             int row, int x, double* out) {
  const double j = column_mean<DS, UNIT, MASK>(st, mask, sh, nx, ny, row, x);
  if (threadIdx.x == 0) *out = j;
}

// The same column mean for every lattice of a batch, one workgroup per
// lattice: out[b * stride] for lattice b at column x (x < 0 counts from
// that lattice's last column, x + nx), state copy `parity`.
template <class DS, bool UNIT, bool MASK>
__global__ __launch_bounds__(256) void batch_column_current_kernel(const LatDesc* __restrict__ lats,
                                                                   const StepShared sh, int parity,
                                                                   int x, int64_t stride,
                                                                   double* out) {
  const LatDesc d = lats[blockIdx.x];
  const int xc = x < 0 ? x + d.nx : x;   // in range: checked on the host
  const double j = column_mean<DS, UNIT, MASK>(d.state[parity], d.mask, sh, d.nx, d.ny, d.row, xc);
  if (threadIdx.x == 0) out[(int64_t)blockIdx.x * stride] = j;
}

// ---------------------------------------------------------------------------
// One-sided power spectrum of a series' fluctuations, as the plain sum
//   P(k) = |sum_t (s_t - mean) e^{-2 pi i k t / n}|^2 / n^2,  k = 0 .. n/2,
// float64, angles reduced exactly ((k t) mod n).  Three launches: the mean
// (kept in out[0]), the bins k >= 1 (one workgroup each), then P(0).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void series_mean_kernel(const double* __restrict__ s, int64_t n,
                                                          double* out) {
  __shared__ double red[4];
  double a = 0.0;
  for (int64_t t = threadIdx.x; t < n; t += blockDim.x) a += s[t];
  a = block_sum(a, red);
  if (threadIdx.x == 0) out[0] = a / (double)n;
}

__global__ __launch_bounds__(256) void dft_power_kernel(const double* __restrict__ s, int64_t n,
                                                        double* out) {
  __shared__ double red[4];
  const int64_t k = (int64_t)blockIdx.x + 1;
  if (k > n / 2) return;   // workgroup-uniform
  const double mean = out[0];
  double re = 0.0, im = 0.0;
  for (int64_t t = threadIdx.x; t < n; t += blockDim.x) {
    const double d = s[t] - mean;
    double sn, cs;
    sincospi(2.0 * (double)((k * t) % n) / (double)n, &sn, &cs);
    re += d * cs;
    im -= d * sn;
  }
  re = block_sum(re, red);
  im = block_sum(im, red);
  if (threadIdx.x == 0) out[k] = (re * re + im * im) / ((double)n * (double)n);
}

__global__ __launch_bounds__(256) void dft_power0_kernel(const double* __restrict__ s, int64_t n,
                                                         double* out) {
  __shared__ double red[4];
  const double mean = out[0];
  double a = 0.0;
  for (int64_t t = threadIdx.x; t < n; t += blockDim.x) a += s[t] - mean;
  a = block_sum(a, red);
  if (threadIdx.x == 0) out[0] = a * a / ((double)n * (double)n);
}

// ---------------------------------------------------------------------------
hipError_t launch_open_borders(const rlb_lattice* lat, float* state) {
  OpenArgs o = lat->open;
  o.eps_ref = lat->p.eps_ref;
  o.n_ref = lat->p.n_ref;
  o.err = lat->err;
  const dim3 grid((2 * lat->p.ny + 255) / 256);
  if (lat->Q == 17)
    hipLaunchKernelGGL(open_borders_kernel<Dir17>, grid, dim3(256), 0, lat->stream, state,
                       lat->p.nx, lat->p.ny, lat->row, o);
  else
    hipLaunchKernelGGL(open_borders_kernel<Dir26>, grid, dim3(256), 0, lat->stream, state,
                       lat->p.nx, lat->p.ny, lat->row, o);
  return hipGetLastError();
}

template <class DS>
static void column_go(const rlb_lattice* lat, const StepShared& sh, int x, double* out) {
  const float* st = lat->state[lat->cur];
  const bool unit = lat->p.cfl == 1.0, mask = lat->any_solid;
#define RLB_COL(U, M)                                                                          \
  hipLaunchKernelGGL((column_current_kernel<DS, U, M>), dim3(1), dim3(256), 0, lat->stream, st, \
                     lat->mask, sh, lat->p.nx, lat->p.ny, lat->row, x, out)
  if (unit) { if (mask) RLB_COL(true, true); else RLB_COL(true, false); }
  else { if (mask) RLB_COL(false, true); else RLB_COL(false, false); }
#undef RLB_COL
}

template <class DS>
static void batch_column_go(const StepShared& sh, const LatDesc* lats, int count, int parity,
                            bool unit, bool mask, int x, int64_t stride, double* out,
                            hipStream_t stream) {
#define RLB_BCOL(U, M)                                                                    \
  hipLaunchKernelGGL((batch_column_current_kernel<DS, U, M>), dim3(count), dim3(256), 0, \
                     stream, lats, sh, parity, x, stride, out)
  if (unit) { if (mask) RLB_BCOL(true, true); else RLB_BCOL(true, false); }
  else { if (mask) RLB_BCOL(false, true); else RLB_BCOL(false, false); }
#undef RLB_BCOL
}

hipError_t launch_batch_column_current(const StepShared& sh, int Q, const LatDesc* lats, int count,
                                       int parity, bool unit, bool mask, int x, int64_t stride,
                                       double* out, hipStream_t stream) {
  if (Q == 17) batch_column_go<Dir17>(sh, lats, count, parity, unit, mask, x, stride, out, stream);
  else if (Q == 12) batch_column_go<DirP12>(sh, lats, count, parity, unit, mask, x, stride, out, stream);
  else batch_column_go<Dir26>(sh, lats, count, parity, unit, mask, x, stride, out, stream);
  return hipGetLastError();
}

hipError_t launch_column_current(const rlb_lattice* lat, int x, double* out) {
  const StepShared sh = shared_of(lat);
  if (lat->Q == 17) column_go<Dir17>(lat, sh, x, out);
  else if (lat->Q == 12) column_go<DirP12>(lat, sh, x, out);
  else column_go<Dir26>(lat, sh, x, out);
  return hipGetLastError();
}

// Mean of r[0 .. ny) by one workgroup of 256 in a fixed order; valid in
// thread 0.
__device__ double row_mean(const double* __restrict__ r, int ny) {
  double acc = 0.0;
  for (int y = threadIdx.x; y < ny; y += blockDim.x) acc += r[y];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  return ((red[0] + red[1]) + (red[2] + red[3])) / (double)ny;
}

// One workgroup per row of `rows`: out[t] = (sum_y rows[t][y]) / ny.
__global__ __launch_bounds__(256) void row_means_kernel(const double* __restrict__ rows, int ny,
                                                        double* __restrict__ out) {
  const double m = row_mean(rows + (size_t)blockIdx.x * ny, ny);
  if (threadIdx.x == 0) out[blockIdx.x] = m;
}

// Workgroup (b, t): lattice b's rows of step t.
__global__ __launch_bounds__(256) void batch_row_means_kernel(const LatDesc* __restrict__ lats,
                                                              const double* __restrict__ rows,
                                                              int64_t total, int64_t stride,
                                                              double* __restrict__ out) {
  const LatDesc& d = lats[blockIdx.x];
  const double m = row_mean(rows + (int64_t)blockIdx.y * total + d.rec_row, d.ny);
  if (threadIdx.x == 0) out[(int64_t)blockIdx.x * stride + blockIdx.y] = m;
}

hipError_t launch_row_means(const double* rows, int ny, int count, double* out, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(row_means_kernel, dim3(count), dim3(256), 0, st, rows, ny, out);
  return hipGetLastError();
}

hipError_t launch_batch_row_means(const LatDesc* lats, int members, const double* rows, int64_t total,
                                  int count, double* out, int64_t stride, hipStream_t st) {
  if (count <= 0 || members <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_row_means_kernel, dim3(members, count), dim3(256), 0, st, lats, rows,
                     total, stride, out);
  return hipGetLastError();
}

hipError_t launch_power_spectrum(const double* s, int64_t n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(series_mean_kernel, dim3(1), dim3(256), 0, st, s, n, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (n / 2 >= 1) {
    hipLaunchKernelGGL(dft_power_kernel, dim3((unsigned)(n / 2)), dim3(256), 0, st, s, n, out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(dft_power0_kernel, dim3(1), dim3(256), 0, st, s, n, out);
  return hipGetLastError();
}

}  // namespace rlb
