// Random k-shell stirring (Ch. 4 "Model and Methods": a random driving term
// on the spectral lattice inside the driving band, transformed to
// configuration space every step).
//
// Per step: (1) one workgroup draws the complex coefficients of every
// half-shell mode from Philox4x64-10 + Box-Muller in float64 (counter
// (m, step, 0, 0), key (seed, stream)); (2) one wavefront per row folds the
// shell sum along ky into the row's real trigonometric series in x,
// a_k cos(k th) + b_k sin(k th), th = 2 pi x / nx, summing modes in a fixed
// order; (3) the synthesis kernel evaluates the series at every node and
// writes the two force planes the step kernel reads.  Each synthesis thread
// owns one column, loads its cos/sin(k th) once from a static twiddle table
// and sweeps 32 rows, so the per-node cost is 4 FMAs per k.
#include "internal.hpp"
#include "device_common.hpp"

namespace rlb {

__global__ __launch_bounds__(256) void stir_draw_kernel(const StirArgs a,
                                                        int64_t fixed_step) {
  __shared__ int64_t s_step;
  if (threadIdx.x == 0) s_step = fixed_step >= 0 ? fixed_step : *a.dstep;
  __syncthreads();
  const int64_t t = s_step;
  for (int m = threadIdx.x; m < a.nmodes; m += blockDim.x) {
    const U64x4 r = philox4x64_10((uint64_t)m, (uint64_t)t, 0, 0, a.seed, a.stream);
    double z0, z1, z2, z3;
    box_muller(r.v[0], r.v[1], z0, z1);
    box_muller(r.v[2], r.v[3], z2, z3);
    double* c = a.coef + 4 * (size_t)m;
    c[0] = a.amplitude * z0;
    c[1] = a.amplitude * z1;
    c[2] = a.amplitude * z2;
    c[3] = a.amplitude * z3;
  }
  __syncthreads();
  if (fixed_step < 0 && threadIdx.x == 0) *a.dstep = t + 1;
}

// One wavefront per row y; lane k builds the series coefficients of |kx| = k
// from the modes of its bin:  mode (kx, ky) with coefficient c contributes
// prod = 2 c e^{2 pi i ky y / ny} to cos(|kx| th) with Re(prod) and to
// sin(|kx| th) with -sign(kx) Im(prod).
__global__ __launch_bounds__(64) void stir_table_kernel(const StirArgs a) {
  const int y = blockIdx.x;
  const int k = threadIdx.x;
  if (y >= a.ny) return;
  float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
  if (k <= a.K) {
    double ax = 0.0, bx = 0.0, ay = 0.0, by = 0.0;
    const int j1 = a.bins[k + 1];
    for (int j = a.bins[k]; j < j1; ++j) {
      const int4 md = a.modes[j];
      // e^{2 pi i ky y / ny} from the phase table, index reduced exactly
      const double2 e = a.phase[((long long)md.z * y) % a.ny];
      const double cs = e.x, sn = e.y;
      const double* c = a.coef + 4 * (size_t)md.x;
      const double pxr = 2.0 * (c[0] * cs - c[1] * sn);
      const double pxi = 2.0 * (c[0] * sn + c[1] * cs);
      const double pyr = 2.0 * (c[2] * cs - c[3] * sn);
      const double pyi = 2.0 * (c[2] * sn + c[3] * cs);
      const double sg = md.y > 0 ? -1.0 : 1.0;   // kx = 0 has no sine part
      ax += pxr;
      bx += sg * pxi;
      ay += pyr;
      by += sg * pyi;
    }
    out = make_float4((float)ax, (float)(k ? bx : 0.0), (float)ay, (float)(k ? by : 0.0));
  }
  a.table[(size_t)y * kTableStride + k] = out;
}

constexpr int kSynthRows = 32;

// Column twiddles (cos, sin)(2 pi k x / nx), k = 1..K, table [K][nx],
// exactly reduced; static per lattice and shell.
__global__ __launch_bounds__(256) void twiddle_kernel(float2* tw, int K, int nx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K * nx) return;
  const int k = i / nx + 1, x = i - (k - 1) * nx;
  double sn, cs;
  sincospi(2.0 * (double)(((long long)k * x) % nx) / (double)nx, &sn, &cs);
  tw[i] = make_float2((float)cs, (float)sn);
}

template <int KB>
__global__ __launch_bounds__(64) void stir_synth_kernel(const float4* __restrict__ table,
                                                        const float2* __restrict__ tw,
                                                        float* __restrict__ force,
                                                        int64_t force_pitch, int K,
                                                        int nx, int ny, int row_pitch) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y0 = blockIdx.y * kSynthRows;
  if (x >= nx) return;
  float c[KB], s[KB];
#pragma unroll
  for (int k = 1; k <= KB; ++k) {
    float2 t = make_float2(0.0f, 0.0f);
    if (k <= K) t = tw[(size_t)(k - 1) * nx + x];
    c[k - 1] = t.x;
    s[k - 1] = t.y;
  }
  const int y1 = min(y0 + kSynthRows, ny);
  for (int y = y0; y < y1; ++y) {
    // the row's coefficients are wave-uniform: scalar loads
    const float4* __restrict__ row = table + (size_t)y * kTableStride;
    float4 t = row[0];
    float fx = t.x, fy = t.z;
#pragma unroll
    for (int k = 1; k <= KB; ++k) {
      t = row[k];   // zero beyond K
      fx += t.x * c[k - 1] + t.y * s[k - 1];
      fy += t.z * c[k - 1] + t.w * s[k - 1];
    }
    force[(size_t)y * row_pitch + x] = fx;
    force[force_pitch + (size_t)y * row_pitch + x] = fy;
  }
}

__global__ __launch_bounds__(256) void phase_kernel(double2* phase, int ny) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= ny) return;
  double sn, cs;
  sincospi(2.0 * (double)m / (double)ny, &sn, &cs);
  phase[m] = make_double2(cs, sn);
}

__global__ __launch_bounds__(256) void philox_kernel(uint64_t k0, uint64_t k1,
                                                     uint64_t c1, int64_t count,
                                                     uint64_t* out) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= count) return;
  const U64x4 r = philox4x64_10((uint64_t)m, c1, 0, 0, k0, k1);
  out[4 * m + 0] = r.v[0];
  out[4 * m + 1] = r.v[1];
  out[4 * m + 2] = r.v[2];
  out[4 * m + 3] = r.v[3];
}

__global__ void set_i64_kernel(int64_t* p, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

hipError_t launch_stir_draw(const StirArgs& a, int64_t fixed_step,
                            hipStream_t s) {
  hipLaunchKernelGGL(stir_draw_kernel, dim3(1), dim3(256), 0, s, a, fixed_step);
  return hipGetLastError();
}

hipError_t launch_stir_table(const StirArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(stir_table_kernel, dim3(a.ny), dim3(kTableStride), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_stir_synth(const StirArgs& a, hipStream_t s) {
  const dim3 grid((a.nx + 63) / 64, (a.ny + kSynthRows - 1) / kSynthRows);
  const float4* t = a.table;
#define RLB_SYNTH(KB)                                                                  \
  hipLaunchKernelGGL(stir_synth_kernel<KB>, grid, dim3(64), 0, s, t, a.twiddle, a.force,     \
                     a.force_pitch, a.K, a.nx, a.ny, a.row)
  if (a.K <= 8) RLB_SYNTH(8);
  else if (a.K <= 16) RLB_SYNTH(16);
  else if (a.K <= 24) RLB_SYNTH(24);
  else if (a.K <= 34) RLB_SYNTH(34);
  else if (a.K <= 48) RLB_SYNTH(48);
  else RLB_SYNTH(63);
#undef RLB_SYNTH
  return hipGetLastError();
}

hipError_t launch_twiddle(float2* tw, int K, int nx, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  hipLaunchKernelGGL(twiddle_kernel, dim3((K * nx + 255) / 256), dim3(256), 0, s, tw, K, nx);
  return hipGetLastError();
}

hipError_t launch_phase(const rlb_lattice* lat) {
  hipLaunchKernelGGL(phase_kernel, dim3((lat->p.ny + 255) / 256), dim3(256), 0,
                     lat->stream, lat->phase, lat->p.ny);
  return hipGetLastError();
}

hipError_t launch_philox(uint64_t k0, uint64_t k1, uint64_t c1, int64_t count,
                         uint64_t* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(philox_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256),
                     0, s, k0, k1, c1, count, out);
  return hipGetLastError();
}

hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s) {
  hipLaunchKernelGGL(set_i64_kernel, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

}  // namespace rlb
