// Spectral analysis of the velocity field (Ch. 2 "Turbulence": E(k) with the
// spectral energy density 1/2 <|v~(k)|^2> over integer shells; Ch. 4: the
// velocities are filtered to remove the driven range, E(k) is averaged over
// decorrelated samples and compared with the k^-5/3 law).
//
// One complex transform serves both components: with z = beta_x + i beta_y,
// Z = FFT2(z) satisfies |X(k)|^2 + |Y(k)|^2 = (|Z(k)|^2 + |Z(-k)|^2) / 2, and
// every shell (and the low-pass disc) is symmetric under k -> -k, so
//     E(s) = 1/2 sum_{k in shell s} |Z(k)|^2 / (Nx Ny)^2,
//     rms of the filtered speed^2 = sum_{|k| < k_cut} |Z(k)|^2 / (Nx Ny)^2,
// and the inverse transform of the masked Z is beta_x,f + i beta_y,f.
//
// Transforms: float64 radix-2 decimation in time over one line per
// workgroup, the line held in LDS (lengths 4 .. 4096, powers of two),
// rows then columns.  Shell sums are per row in a fixed order (each shell's
// kx range found with exact integer bounds), then over rows in a fixed
// order: the result does not depend on scheduling.
#include <algorithm>

#include "internal.hpp"
#include "device_common.hpp"

namespace rlb {

__global__ __launch_bounds__(256) void pack_kernel(const float* __restrict__ bx,
                                                   const float* __restrict__ by, double2* z,
                                                   int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = make_double2((double)bx[i], (double)by[i]);
}

// tw[j] = exp(-2 pi i j / n), j < n / 2, angle reduced exactly
__global__ __launch_bounds__(256) void twiddle64_kernel(double2* tw, int n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n / 2) return;
  double s, c;
  sincospi(2.0 * (double)j / (double)n, &s, &c);
  tw[j] = make_double2(c, -s);
}

// In-place transform of nlines lines of length n = 2^log2n: element j of
// line l at data[l * line_stride + j * elem_stride].  INV uses the
// conjugate twiddles (unnormalised inverse).
template <bool INV>
__global__ __launch_bounds__(256) void fft_lines_kernel(double2* data, const double2* __restrict__ tw,
                                                        int n, int log2n, int64_t elem_stride,
                                                        int64_t line_stride) {
  extern __shared__ double2 buf[];
  double2* base = data + (int64_t)blockIdx.x * line_stride;
  for (int j = threadIdx.x; j < n; j += blockDim.x)
    buf[__brev((unsigned)j) >> (32 - log2n)] = base[(int64_t)j * elem_stride];
  __syncthreads();
  for (int s = 1; s <= log2n; ++s) {
    const int half = 1 << (s - 1);
    for (int b = threadIdx.x; b < n / 2; b += blockDim.x) {
      const int pos = b & (half - 1);
      const int i0 = ((b >> (s - 1)) << s) + pos, i1 = i0 + half;
      double2 w = tw[pos << (log2n - s)];
      if (INV) w.y = -w.y;
      const double2 u = buf[i0], v = buf[i1];
      const double tr = w.x * v.x - w.y * v.y, ti = w.x * v.y + w.y * v.x;
      buf[i0] = make_double2(u.x + tr, u.y + ti);
      buf[i1] = make_double2(u.x - tr, u.y - ti);
    }
    __syncthreads();
  }
  for (int j = threadIdx.x; j < n; j += blockDim.x) base[(int64_t)j * elem_stride] = buf[j];
}

__device__ __forceinline__ double block_sum256(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

__device__ __forceinline__ double abs2(double2 z) { return z.x * z.x + z.y * z.y; }

// Row r (wave number ky): part[r][s] = sum over the row's |Z|^2 in shell s
// (s - 1/2 <= |k| < s + 1/2, i.e. (2s-1)^2 <= 4|k|^2 < (2s+1)^2), s <= kmax;
// part[r][kmax+1] = sum over |k|^2 < k_cut^2.
__global__ __launch_bounds__(256) void shell_rows_kernel(const double2* __restrict__ Z, int nx, int ny,
                                                         int kmax, double kcut2, double* part) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  const int64_t ky = r < ny / 2 ? r : r - ny;
  const double2* row = Z + (int64_t)r * nx;
  double* out = part + (int64_t)r * (kmax + 2);
  const int64_t ky4 = 4 * ky * ky;
  for (int s = threadIdx.x; s <= kmax; s += blockDim.x) {
    const int64_t lo2 = s == 0 ? 0 : (int64_t)(2 * s - 1) * (2 * s - 1);   // 4|k|^2 >= lo2
    const int64_t hi2 = (int64_t)(2 * s + 1) * (2 * s + 1);                // 4|k|^2 < hi2
    // smallest kx >= 0 with 4 kx^2 + ky4 >= lo2, largest with 4 kx^2 + ky4 < hi2
    int64_t lo = lo2 > ky4 ? (int64_t)floor(sqrt((double)(lo2 - ky4) / 4.0)) : 0;
    while (lo > 0 && 4 * (lo - 1) * (lo - 1) + ky4 >= lo2) --lo;
    while (4 * lo * lo + ky4 < lo2) ++lo;
    double acc = 0.0;
    if (ky4 < hi2) {
      int64_t hi = (int64_t)floor(sqrt((double)(hi2 - ky4) / 4.0)) + 1;
      while (4 * hi * hi + ky4 >= hi2) --hi;
      hi = std::min<int64_t>(hi, nx / 2);
      for (int64_t kx = lo; kx <= hi; ++kx) {
        if (kx <= nx / 2 - 1) acc += abs2(row[kx]);                  // +kx
        if (kx >= 1) acc += abs2(row[nx - kx]);                       // -kx (includes -nx/2)
      }
    }
    out[s] = acc;
  }
  // low-pass disc
  double lp = 0.0;
  for (int c = threadIdx.x; c < nx; c += blockDim.x) {
    const double kx = c < nx / 2 ? c : c - nx;
    if (kx * kx + (double)(ky * ky) < kcut2) lp += abs2(row[c]);
  }
  lp = block_sum256(lp, red);
  if (threadIdx.x == 0) out[kmax + 1] = lp;
}

// bin b: sum over rows in order; E(s) for b <= kmax, filtered rms for
// b = kmax + 1; optional accumulation of E and E^2.
__global__ __launch_bounds__(256) void shell_sum_kernel(const double* __restrict__ part, int ny, int kmax,
                                                        double norm, double* out, double* acc) {
  __shared__ double red[4];
  const int b = blockIdx.x;
  double a = 0.0;
  for (int r = threadIdx.x; r < ny; r += blockDim.x) a += part[(int64_t)r * (kmax + 2) + b];
  a = block_sum256(a, red);
  if (threadIdx.x != 0) return;
  if (b <= kmax) {
    const double E = 0.5 * a * norm;
    out[b] = E;
    if (acc) {
      acc[b] += E;
      acc[kmax + 1 + b] += E * E;
    }
  } else {
    out[kmax + 1] = sqrt(a * norm);
  }
}

__global__ __launch_bounds__(256) void lowpass_kernel(double2* Z, int nx, int ny, double kcut2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nx * ny) return;
  const int r = (int)(i / nx), c = (int)(i - (int64_t)r * nx);
  const double kx = c < nx / 2 ? c : c - nx, ky = r < ny / 2 ? r : r - ny;
  if (!(kx * kx + ky * ky < kcut2)) Z[i] = make_double2(0.0, 0.0);
}

// mean |z| / (nx ny) over nodes: per-block partials in a fixed grid
__global__ __launch_bounds__(256) void speed_kernel(const double2* __restrict__ z, int64_t n,
                                                    double scale, double* part) {
  __shared__ double red[4];
  double a = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a += sqrt(abs2(z[i])) * scale;
  a = block_sum256(a, red);
  if (threadIdx.x == 0) part[blockIdx.x] = a;
}

__global__ __launch_bounds__(256) void speed_final_kernel(const double* __restrict__ part, int nb,
                                                          double inv_n, double* out) {
  __shared__ double red[4];
  double a = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) a += part[i];
  a = block_sum256(a, red);
  if (threadIdx.x == 0) *out = a * inv_n;
}

// Enstrophy Z = sum over nodes of omega^2, omega = d_x beta_y - d_y beta_x
// by periodic central differences of the read-out fields (Ch. 2
// "Turbulence"), float64, per-block partials in a fixed grid.
__global__ __launch_bounds__(256) void enstrophy_kernel(const float* __restrict__ bx,
                                                        const float* __restrict__ by, int nx,
                                                        int ny, double* part) {
  __shared__ double red[4];
  double a = 0.0;
  const int64_t n = (int64_t)nx * ny;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / nx), x = (int)(i - (int64_t)y * nx);
    const int xp = x + 1 < nx ? x + 1 : 0, xm = x > 0 ? x - 1 : nx - 1;
    const int yp = y + 1 < ny ? y + 1 : 0, ym = y > 0 ? y - 1 : ny - 1;
    const double w = 0.5 * ((double)by[(int64_t)y * nx + xp] - (double)by[(int64_t)y * nx + xm]) -
                     0.5 * ((double)bx[(int64_t)yp * nx + x] - (double)bx[(int64_t)ym * nx + x]);
    a += w * w;
  }
  a = block_sum256(a, red);
  if (threadIdx.x == 0) part[blockIdx.x] = a;
}

// ---------------------------------------------------------------------------
constexpr int kSpeedBlocks = 1024;

SpectralLayout spectral_layout(int nx, int ny, int kmax) {
  SpectralLayout L;
  size_t off = 0;
  const size_t nodes = (size_t)nx * ny;
  L.z_off = off; off += align_up(nodes * sizeof(double2));
  L.fields_off = off; off += align_up(2 * nodes * sizeof(float));
  L.twx_off = off; off += align_up((size_t)(nx / 2) * sizeof(double2));
  L.twy_off = off; off += align_up((size_t)(ny / 2) * sizeof(double2));
  L.part_off = off; off += align_up((size_t)ny * (kmax + 2) * sizeof(double));
  L.speed_off = off; off += align_up(kSpeedBlocks * sizeof(double));
  L.total = off;
  return L;
}

static int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

hipError_t launch_spectrum(rlb_lattice* lat, int kmax, double kcut, double* out, double* acc,
                           char* ws) {
  const int nx = lat->p.nx, ny = lat->p.ny;
  const SpectralLayout L = spectral_layout(nx, ny, kmax);
  double2* z = (double2*)(ws + L.z_off);
  float* f = (float*)(ws + L.fields_off);
  double2* twx = (double2*)(ws + L.twx_off);
  double2* twy = (double2*)(ws + L.twy_off);
  double* part = (double*)(ws + L.part_off);
  double* sp = (double*)(ws + L.speed_off);
  const int64_t nodes = (int64_t)nx * ny;
  const hipStream_t s = lat->stream;
  const uint32_t mask = (1u << RLB_FIELD_BETA_X) | (1u << RLB_FIELD_BETA_Y);
  hipError_t e = launch_step(lat, MODE_FIELDS, FORCE_NONE, lat->cur, f, mask);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(enstrophy_kernel, dim3(kSpeedBlocks), dim3(256), 0, s, f, f + nodes, nx, ny, sp);
  hipLaunchKernelGGL(speed_final_kernel, dim3(1), dim3(256), 0, s, sp, kSpeedBlocks, 1.0,
                     out + kmax + 3);
  const unsigned gn = (unsigned)((nodes + 255) / 256);
  hipLaunchKernelGGL(pack_kernel, dim3(gn), dim3(256), 0, s, f, f + nodes, z, nodes);
  hipLaunchKernelGGL(twiddle64_kernel, dim3((nx / 2 + 255) / 256), dim3(256), 0, s, twx, nx);
  hipLaunchKernelGGL(twiddle64_kernel, dim3((ny / 2 + 255) / 256), dim3(256), 0, s, twy, ny);
  const int lx = ilog2(nx), ly = ilog2(ny);
  hipLaunchKernelGGL(fft_lines_kernel<false>, dim3(ny), dim3(256), nx * sizeof(double2), s, z, twx,
                     nx, lx, (int64_t)1, (int64_t)nx);
  hipLaunchKernelGGL(fft_lines_kernel<false>, dim3(nx), dim3(256), ny * sizeof(double2), s, z, twy,
                     ny, ly, (int64_t)nx, (int64_t)1);
  const double kc2 = kcut * kcut;
  hipLaunchKernelGGL(shell_rows_kernel, dim3(ny), dim3(256), 0, s, z, nx, ny, kmax, kc2, part);
  const double norm = 1.0 / ((double)nodes * (double)nodes);
  hipLaunchKernelGGL(shell_sum_kernel, dim3(kmax + 2), dim3(256), 0, s, part, ny, kmax, norm, out, acc);
  // filtered field: mask, inverse transform (columns, rows), mean speed
  hipLaunchKernelGGL(lowpass_kernel, dim3(gn), dim3(256), 0, s, z, nx, ny, kc2);
  hipLaunchKernelGGL(fft_lines_kernel<true>, dim3(nx), dim3(256), ny * sizeof(double2), s, z, twy,
                     ny, ly, (int64_t)nx, (int64_t)1);
  hipLaunchKernelGGL(fft_lines_kernel<true>, dim3(ny), dim3(256), nx * sizeof(double2), s, z, twx,
                     nx, lx, (int64_t)1, (int64_t)nx);
  hipLaunchKernelGGL(speed_kernel, dim3(kSpeedBlocks), dim3(256), 0, s, z, nodes, 1.0 / (double)nodes, sp);
  hipLaunchKernelGGL(speed_final_kernel, dim3(1), dim3(256), 0, s, sp, kSpeedBlocks,
                     1.0 / (double)nodes, out + kmax + 2);
  return hipGetLastError();
}

}  // namespace rlb
