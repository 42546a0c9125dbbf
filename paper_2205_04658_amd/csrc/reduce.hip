// Conservation diagnostics: global E = sum F, P^x = sum F v_x,
// P^y = sum F v_y, Q = sum G over all nodes (Ch. 2: d_mu T^{mu nu} = 0 and
// charge conservation), in float64 with a fixed summation order: every
// thread walks a fixed node set, wavefronts reduce with lane exchanges, the
// workgroup through LDS, and one final workgroup sums the fixed number of
// partials.  Also the plain copy kernel used to calibrate byte counters.
#include "dirset.hpp"
#include "internal.hpp"
#include "device_common.hpp"
#include "brick.hpp"

namespace rlb {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <class DS>
__global__ __launch_bounds__(256) void totals_kernel(const float* __restrict__ st,
                                                     int nx, int ny, int row,
                                                     double* partial) {
  constexpr int Q = DS::Q;
  double e = 0.0, px = 0.0, py = 0.0, q = 0.0;
  const int stride = gridDim.x * blockDim.x;
  const int ncell = nx * ny;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < ncell; j += stride) {
    const int yy = j / nx;
    const float* b = st + state_elem<Q>(0, j - yy * nx, yy, row);   // plane 0 of node j
    static_for<0, Q>([&](auto P) {
      constexpr int p = decltype(P)::value;
      const double f = (double)b[p * 64];
      e += f;
      if constexpr (DS::vx[p] != 0.0) px += DS::vx[p] * f;
      if constexpr (DS::vy[p] != 0.0) py += DS::vy[p] * f;
      q += (double)b[(Q + p) * 64];
    });
  }
  __shared__ double red[4][4];
  e = wave_sum(e);
  px = wave_sum(px);
  py = wave_sum(py);
  q = wave_sum(q);
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  if (ln == 0) {
    red[wv][0] = e; red[wv][1] = px; red[wv][2] = py; red[wv][3] = q;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int c = threadIdx.x;
    partial[4 * blockIdx.x + c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
  }
}

__global__ __launch_bounds__(256) void totals_final_kernel(const double* __restrict__ partial,
                                                           int nblocks, double ncell,
                                                           double eps_ref, double n_ref,
                                                           double* out) {
  __shared__ double red[4][4];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
    for (int c = 0; c < 4; ++c) acc[c] += partial[4 * b + c];
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  for (int c = 0; c < 4; ++c) {
    acc[c] = wave_sum(acc[c]);
    if (ln == 0) red[wv][c] = acc[c];
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int c = threadIdx.x;
    double v = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
    if (c == 0) v += ncell * eps_ref;
    if (c == 3) v += ncell * n_ref;
    out[c] = v;
  }
}

// Energy and momentum the driving term adds in the next step (Ch. 4 eq.
// forceTerm with its discretisation in the appendix on the forcing term):
// per fluid node, with T^{0 mu} of the streamed current state (the pull the
// step applies) and F the next step's force (body force + stirring planes,
// added in float32 as the step adds them),
//   dE = F.T^{0k} / 6,   dP^k = F^k T^{00} / 6,
// summed in float64 in the totals' fixed order (component 3 left zero).
template <class DS, int SM>
__global__ __launch_bounds__(256) void injection_kernel(const float* __restrict__ st,
                                                        const uint8_t* __restrict__ mask,
                                                        const float* __restrict__ force,
                                                        int64_t pitch, int planes, float fx,
                                                        float fy, const StepShared sh, int nx,
                                                        int ny, int row, double* partial) {
  constexpr int Q = DS::Q;
  double e = 0.0, px = 0.0, py = 0.0;
  const int stride = gridDim.x * blockDim.x;
  const int ncell = nx * ny;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < ncell; j += stride) {
    if (mask && mask[j]) continue;
    const int y = j / nx, x = j - y * nx;
    // moments of the streamed deviations from the reference (whose T^{0k}
    // vanishes and whose weights sum to one)
    double m00 = 0.0, m0x = 0.0, m0y = 0.0;
    auto add = [&](auto P, float v) {
      constexpr int p = decltype(P)::value;
      const double f = (double)v;
      m00 += f;
      if constexpr (DS::vx[p] != 0.0) m0x += DS::vx[p] * f;
      if constexpr (DS::vy[p] != 0.0) m0y += DS::vy[p] * f;
    };
    if constexpr (SM == SM_WIDE) {
      const Nbr5 nb = neighbourhood5<Q>(x, y, nx, ny, row);
      static_for<0, Q>([&](auto P) {
        constexpr int p = decltype(P)::value;
        add(P, pull_wide<DS, p, p>(st, nb, sh.tap[p], sh.shift[p]));
      });
    } else {
      const Nbr nb = neighbourhood<Q>(x, y, nx, ny, row);
      static_for<0, Q>([&](auto P) {
        constexpr int p = decltype(P)::value;
        add(P, pull<DS, SM == SM_UNIT, p, p, false>(st, nb, sh.tap[p]));
      });
    }
    float Fx = fx, Fy = fy;
    if (planes) {
      Fx += force[(int64_t)y * row + x];
      Fy += force[pitch + (int64_t)y * row + x];
    }
    const double T00 = sh.eps_ref + m00;
    e += ((double)Fx * m0x + (double)Fy * m0y) / 6.0;
    px += (double)Fx * T00 / 6.0;
    py += (double)Fy * T00 / 6.0;
  }
  __shared__ double red[4][3];
  e = wave_sum(e);
  px = wave_sum(px);
  py = wave_sum(py);
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  if (ln == 0) {
    red[wv][0] = e; red[wv][1] = px; red[wv][2] = py;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int c = threadIdx.x;
    partial[4 * blockIdx.x + c] = c == 3 ? 0.0 : (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
  }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Plain device copy for bandwidth calibration: each thread moves four
// 16-byte items, all four loads issued before the (non-temporal) stores.
constexpr int kCopyUnroll = 4;
__global__ __launch_bounds__(256) void copy_kernel(const f32x4* __restrict__ s,
                                                   f32x4* __restrict__ d, size_t n) {
  const size_t base = (size_t)blockIdx.x * (256 * kCopyUnroll) + threadIdx.x;
  f32x4 v[kCopyUnroll];
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const size_t i = base + (size_t)u * 256;
    if (i < n) v[u] = s[i];
  }
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const size_t i = base + (size_t)u * 256;
    if (i < n) __builtin_nontemporal_store(v[u], d + i);
  }
}

hipError_t launch_totals(const rlb_lattice* lat, const float* state,
                         double* result) {
  const int ncell = lat->p.nx * lat->p.ny;
  if (lat->Q == 17)
    hipLaunchKernelGGL(totals_kernel<Dir17>, dim3(kRedBlocks), dim3(256), 0,
                       lat->stream, state, lat->p.nx, lat->p.ny, lat->row,
                       lat->partials);
  else if (lat->Q == 12)
    hipLaunchKernelGGL(totals_kernel<DirP12>, dim3(kRedBlocks), dim3(256), 0,
                       lat->stream, state, lat->p.nx, lat->p.ny, lat->row,
                       lat->partials);
  else
    hipLaunchKernelGGL(totals_kernel<Dir26>, dim3(kRedBlocks), dim3(256), 0,
                       lat->stream, state, lat->p.nx, lat->p.ny, lat->row,
                       lat->partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(totals_final_kernel, dim3(1), dim3(256), 0, lat->stream,
                     lat->partials, kRedBlocks, (double)ncell, lat->p.eps_ref,
                     lat->p.n_ref, result);
  return hipGetLastError();
}

template <class DS>
static void injection_go(const rlb_lattice* lat, bool planes, const StepShared& sh) {
  const dim3 g(kRedBlocks), b(256);
  const uint8_t* mask = lat->any_solid ? lat->mask : nullptr;
  const float fx = (float)lat->fx, fy = (float)lat->fy;
  const float* st = lat->state[lat->cur];
  switch (stream_mode(lat->p.cfl)) {
    case SM_WIDE:
      hipLaunchKernelGGL((injection_kernel<DS, SM_WIDE>), g, b, 0, lat->stream, st, mask, lat->force,
                         lat->pitch, planes ? 1 : 0, fx, fy, sh, lat->p.nx, lat->p.ny, lat->row,
                         lat->partials);
      break;
    case SM_UNIT:
      hipLaunchKernelGGL((injection_kernel<DS, SM_UNIT>), g, b, 0, lat->stream, st, mask, lat->force,
                         lat->pitch, planes ? 1 : 0, fx, fy, sh, lat->p.nx, lat->p.ny, lat->row,
                         lat->partials);
      break;
    default:
      hipLaunchKernelGGL((injection_kernel<DS, SM_GENERAL>), g, b, 0, lat->stream, st, mask,
                         lat->force, lat->pitch, planes ? 1 : 0, fx, fy, sh, lat->p.nx, lat->p.ny,
                         lat->row, lat->partials);
  }
}

hipError_t launch_injection(const rlb_lattice* lat, bool planes, double* result) {
  const StepShared sh = shared_of(lat);
  if (lat->Q == 17) injection_go<Dir17>(lat, planes, sh);
  else if (lat->Q == 26) injection_go<Dir26>(lat, planes, sh);
  else return hipErrorInvalidValue;   // the planar set has no driving term
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(totals_final_kernel, dim3(1), dim3(256), 0, lat->stream, lat->partials,
                     kRedBlocks, (double)lat->p.nx * lat->p.ny, 0.0, 0.0, result);
  return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 16;
  if (n == 0) return hipSuccess;
  const size_t blocks = (n + 256 * kCopyUnroll - 1) / (256 * kCopyUnroll);
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     (const f32x4*)src, (f32x4*)dst, n);
  return hipGetLastError();
}

}  // namespace rlb
