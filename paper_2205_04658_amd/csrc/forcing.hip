// Random k-shell stirring (Ch. 4 "Model and Methods": a random driving term
// on the spectral lattice inside the driving band, transformed to
// configuration space every step).
//
// Per step: (1) the series kernel draws the complex coefficients of the
// half-shell modes from Philox4x64-10 + Box-Muller in float64 (counter
// (m, step, 0, 0), key (seed, stream)) -- each workgroup those of the modes
// it needs -- and folds the shell sum along ky into each row's real
// trigonometric series in x, a_k cos(k th) + b_k sin(k th), th = 2 pi x / nx,
// summing modes in a fixed order; (2) the synthesis kernel evaluates the
// series at every node, writes the two force planes the step kernel reads
// and advances the device step counter.  The synthesis is a
// dense product, F_c(y, x) = sum_j A_c(y, j) T(j, x) over the 2 (K + 1)
// slots j = (k, cos | sin), so it runs on the matrix cores.  Both operands
// are split into float16 hi + lo parts (the coefficients scaled by a power
// of two into float16's normal range), and hi*hi + hi*lo + lo*hi is
// accumulated in float32 by v_mfma_f32_32x32x16_f16, eight k (16 slots) per
// instruction: 22 significant bits per operand, about float32's accuracy,
// at a fifth of the float32 matrix instructions' cycles.
#include <algorithm>

#include "internal.hpp"
#include "device_common.hpp"
#include "brick.hpp"

namespace rlb {

// Coefficients (Re Fx, Im Fx, Re Fy, Im Fy) of half-shell mode m at step t.
__device__ __forceinline__ void draw_mode(const StirArgs& a, int m, int64_t t, double c[4]) {
  const U64x4 r = philox4x64_10((uint64_t)m, (uint64_t)t, 0, 0, a.seed, a.stream);
  double z0, z1, z2, z3;
  box_muller(r.v[0], r.v[1], z0, z1);
  box_muller(r.v[2], r.v[3], z2, z3);
  c[0] = a.amplitude * z0;
  c[1] = a.amplitude * z1;
  c[2] = a.amplitude * z2;
  c[3] = a.amplitude * z3;
}

// Every mode's coefficients at step `step` into a.coef (the coefficient
// read-out; the step's own series kernel draws what it needs itself).
__global__ __launch_bounds__(256) void stir_draw_kernel(const StirArgs a, int64_t step) {
  for (int m = threadIdx.x; m < a.nmodes; m += blockDim.x) {
    double c[4];
    draw_mode(a, m, step, c);
    double* o = a.coef + 4 * (size_t)m;
    o[0] = c[0];
    o[1] = c[1];
    o[2] = c[2];
    o[3] = c[3];
  }
}

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

// float16 hi + lo split of v: hi = v rounded, lo = the rest rounded, so
// hi + lo = v to about 2^-22 relative while |v| is a normal float16.
__device__ __forceinline__ void split16(double v, _Float16& hi, _Float16& lo) {
  hi = (_Float16)v;
  lo = (_Float16)(v - (double)hi);
}

// Series coefficients: (a_k, b_k) of F^x and F^y for every |kx| = k and row
// y, times the lattice's power-of-two scale, in the synthesis's operand
// order (see StirArgs::table).  A workgroup (one wavefront, 64 rows of one
// k) first draws the coefficients of its bin's modes at the step (the
// device counter, or fixed_step >= 0), 64 modes at a time into LDS; then
// each thread sums the modes of the bin in their fixed order: mode
// (kx, ky) with coefficient c contributes prod = 2 c e^{2 pi i ky y / ny}
// to cos(k th) with Re(prod) and to sin(k th) with -sign(kx) Im(prod).
// Rows k past K are written as zeros.  (Drawing in this kernel instead of
// a one-workgroup draw kernel before it: 14.8 -> 12 us per step at 4096^2.)
// The phase e^{2 pi i ky y / ny} follows ky through the bin by complex
// multiplication (about n ulp after n modes, far below the float32 force)
// instead of a phase-table read per mode (11.9 -> 11.6 us at 4096^2; the
// kernel is latency-bound: without the mode loop and the draws a launch
// of this grid takes 5.3 us, the draws add 3 us).  The bins go out in
// decreasing |kx|: near the shell's radius a bin holds many more modes
// (the line kx = const runs along the annulus), and dispatched last those
// workgroups had set the kernel's end (whole step 1.4 us shorter).
__global__ __launch_bounds__(64) void stir_table_kernel(const StirArgs a, int64_t fixed_step) {
  __shared__ double s_c[64][4];
  const int y = blockIdx.x * 64 + threadIdx.x;
  const int k = (int)gridDim.y - 1 - (int)blockIdx.y;   // 8 chunks(K) - 1 .. 0
  const bool row = y < a.ny;
  double ax = 0.0, bx = 0.0, ay = 0.0, by = 0.0;
  // the bin's modes and the step are the same for every thread of the
  // workgroup and read-only here (written by earlier launches): read them
  // through the constant address space, i.e. with scalar loads
  typedef const __attribute__((address_space(4))) int CInt;
  typedef const __attribute__((address_space(4))) int64_t CI64;
  CInt* bins = (CInt*)a.bins;
  CInt* modes = (CInt*)a.modes;
  const int64_t t = fixed_step >= 0 ? fixed_step : *(CI64*)a.dstep;
  const int j0 = k <= a.K ? bins[k] : 0;
  const int j1 = k <= a.K ? bins[k + 1] : 0;
  // e^{2 pi i ky y / ny} of the last mode's ky, advanced by w = e^{2 pi i y
  // / ny} when ky grows by one (the bins hold their modes by ky ascending),
  // else read from the phase table
  const double2 w = a.phase[row ? y : 0];
  double cs = 1.0, sn = 0.0;
  int kprev = 0;
  for (int jc = j0; jc < j1; jc += 64) {
    const int n = min(64, j1 - jc);
    if ((int)threadIdx.x < n) {
      double c[4];
      draw_mode(a, modes[4 * (jc + threadIdx.x)], t, c);
      s_c[threadIdx.x][0] = c[0];
      s_c[threadIdx.x][1] = c[1];
      s_c[threadIdx.x][2] = c[2];
      s_c[threadIdx.x][3] = c[3];
    }
    __syncthreads();
    for (int jj = 0; jj < n; ++jj) {
      const int j = jc + jj;
      const int md_y = modes[4 * j + 1], md_z = modes[4 * j + 2];
      if (md_z == kprev + 1) {
        const double c2 = cs * w.x - sn * w.y;
        sn = cs * w.y + sn * w.x;
        cs = c2;
      } else if (md_z != kprev) {
        // index reduced exactly (0 <= ky <= 63 and y < ny < 2^24: the
        // product fits 32 bits)
        const double2 e = a.phase[row ? (unsigned)(md_z * y) % (unsigned)a.ny : 0u];
        cs = e.x;
        sn = e.y;
      }
      kprev = md_z;
      const double* c = s_c[jj];
      const double pxr = 2.0 * (c[0] * cs - c[1] * sn);
      const double pxi = 2.0 * (c[0] * sn + c[1] * cs);
      const double pyr = 2.0 * (c[2] * cs - c[3] * sn);
      const double pyi = 2.0 * (c[2] * sn + c[3] * cs);
      const double sg = md_y > 0 ? -1.0 : 1.0;   // kx = 0 has no sine part
      ax += pxr;
      bx += sg * pxi;
      ay += pyr;
      by += sg * pyi;
    }
    __syncthreads();
  }
  if (!row) return;
  if (k == 0) bx = by = 0.0;
  const double sc = (double)a.scale;
  const double v[2][2] = {{ax * sc, bx * sc}, {ay * sc, by * sc}};
  // items (k / 8, (k / 4) % 2, component, hi | lo, y); halves 2 (k % 4), +1
  const size_t part = (size_t)((k >> 3) * 2 + ((k >> 2) & 1));
  const int p = 2 * (k & 3);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    _Float16 h0, l0, h1, l1;
    split16(v[c][0], h0, l0);
    split16(v[c][1], h1, l1);
    _Float16* hi = (_Float16*)(a.table + (part * 4 + 2 * c) * a.ny + y);
    _Float16* lo = (_Float16*)(a.table + (part * 4 + 2 * c + 1) * a.ny + y);
    hi[p] = h0; hi[p + 1] = h1;
    lo[p] = l0; lo[p + 1] = l1;
  }
}

// Column twiddles (cos, sin)(2 pi k x / nx) for k = 0..kMaxK as float16
// hi + lo in the synthesis's operand order (see StirArgs::twiddle), exactly
// reduced; rows past K are zero.  Static per lattice and shell.
__global__ __launch_bounds__(256) void twiddle_kernel(uint4* tw, int K, int nx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (kMaxK + 1) * nx) return;
  const int k = i / nx, x = i - k * nx;
  double sn = 0.0, cs = 0.0;
  if (k <= K) sincospi(2.0 * (double)(((long long)k * x) % nx) / (double)nx, &sn, &cs);
  // items (k / 8, (k / 4) % 2, hi | lo, x); halves 2 (k % 4), +1
  const size_t part = (size_t)((k >> 3) * 2 + ((k >> 2) & 1));
  _Float16* hi = (_Float16*)(tw + (part * 2) * nx + x);
  _Float16* lo = (_Float16*)(tw + (part * 2 + 1) * nx + x);
  const int p = 2 * (k & 3);
  _Float16 hc, lc, hs, ls;
  split16(cs, hc, lc);
  split16(sn, hs, ls);
  hi[p] = hc; hi[p + 1] = hs;
  lo[p] = lc; lo[p + 1] = ls;
}

constexpr int kSynthBlocks = 2;                  // 32-column blocks per wavefront
constexpr int kSynthWaveCols = 32 * kSynthBlocks;
constexpr int kSynthWaves = 4;                   // wavefronts per workgroup

// Chunks of eight k the synthesis runs: ceil((K + 1) / 8) (<= 8).
static inline int synth_chunks(int K) { return (K + 8) >> 3; }

// One wavefront: rows y0 .. y0+31, columns xw .. xw + 32 kSynthBlocks - 1,
// both components.
// v_mfma_f32_32x32x16_f16 takes, in lane l, A row l % 32 and B column l % 32
// with slots 8 (l / 32) .. +7, i.e. (cos, sin) of k = 8 c + 4 (l / 32) .. +3
// for chunk c: one 16-byte item of each (component, hi | lo) plane of the
// table and of each hi | lo plane of the twiddles.  Accumulator element i
// of lane l is block row 8 (i / 4) + 4 (l / 32) + i % 4, column l % 32.
// Rows and columns past the lattice are clamped on load and skipped on
// store.  The kernel advances the device step counter when `advance` is set
// (the series kernel of the next step reads it).
// At 4096^2 the kernel takes 33 us; the same launch with the products
// but no stores takes 25 us, with the stores but no products 26.5 us (a
// plain 16-byte-store kernel writes the 134 MB in 22.8 us).  Waiting for
// each chunk's operands before its products cost 3 us of that (36 us);
// the operand layout with rows (columns) contiguous, 1 us.  Measured
// against the 36 us form: 16-byte stores through a per-wavefront LDS
// tile, the same; the transposed product with 16-byte stores straight
// from the accumulators (32-byte pieces per row), 148 us; 32 x 32 tiles
// (6 waves per SIMD), 49 us; 32 x 128 tiles (1 wave per SIMD), 41 us.
// Re-timed with the contiguous operands and the prefetch: 32 x 32 tiles
// (5 waves per SIMD) and 2 or 8 wavefronts per workgroup all within 0.3 to
// 2 us of this form.  Keeping each XCD on its own row bands (below; an
// XCD's L2 then holds an eighth of the series table) measured the same,
// and is kept.
__global__ __launch_bounds__(64 * kSynthWaves) void stir_synth_kernel(
    const uint4* __restrict__ table, const uint4* __restrict__ tw, float* __restrict__ force,
    int64_t force_pitch, int nchunks, int nx, int ny, int row_pitch, float inv_scale,
    int64_t* dstep, int advance, int wgs_per_xcd) {
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5, l32 = lane & 31;
  const int tiles_x = (nx + kSynthWaveCols - 1) / kSynthWaveCols;
  // workgroups go to the XCDs in turn (blockIdx % 8): give each XCD a
  // contiguous run of tiles, i.e. of row bands, so that its L2 holds only
  // its rows' series coefficients besides the twiddles
  const int wg = (int)(blockIdx.x & 7) * wgs_per_xcd + (int)(blockIdx.x >> 3);
  const int tile = wg * kSynthWaves + (threadIdx.x >> 6);
  if (advance && tile == 0 && lane == 0) *dstep += 1;
  const int ty = tile / tiles_x;
  const int y0 = ty * 32;
  const int xw = (tile - ty * tiles_x) * kSynthWaveCols;
  if (y0 >= ny) return;   // wave-uniform
  const int ya = min(y0 + l32, ny - 1);
  int xb[kSynthBlocks];
#pragma unroll
  for (int b = 0; b < kSynthBlocks; ++b) xb[b] = min(xw + 32 * b + l32, nx - 1);
  floatx16 acc[2][kSynthBlocks];
#pragma unroll
  for (int b = 0; b < kSynthBlocks; ++b) {
#pragma unroll
    for (int i = 0; i < 16; ++i) { acc[0][b][i] = 0.0f; acc[1][b][i] = 0.0f; }
  }
  // operands of one chunk; chunk c + 1's are loaded before chunk c's
  // products run, so that one L2 round trip per wavefront is waited for
  // instead of one per chunk
  struct Ops { uint4 a[4], bh[kSynthBlocks], bl[kSynthBlocks]; };
  auto load = [&](int c, Ops& o) {
    const size_t part = (size_t)(2 * c + half);
    const uint4* ap = table + part * 4 * ny + ya;
#pragma unroll
    for (int i = 0; i < 4; ++i) o.a[i] = ap[i * ny];
#pragma unroll
    for (int b = 0; b < kSynthBlocks; ++b) {
      const uint4* bp = tw + part * 2 * nx + xb[b];
      o.bh[b] = bp[0];
      o.bl[b] = bp[nx];
    }
  };
  auto mma = [&](const Ops& o) {
    const half8 axh = __builtin_bit_cast(half8, o.a[0]), axl = __builtin_bit_cast(half8, o.a[1]);
    const half8 ayh = __builtin_bit_cast(half8, o.a[2]), ayl = __builtin_bit_cast(half8, o.a[3]);
#pragma unroll
    for (int b = 0; b < kSynthBlocks; ++b) {
      const half8 bh = __builtin_bit_cast(half8, o.bh[b]), bl = __builtin_bit_cast(half8, o.bl[b]);
      acc[0][b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(axl, bh, acc[0][b], 0, 0, 0);
      acc[0][b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(axh, bl, acc[0][b], 0, 0, 0);
      acc[0][b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(axh, bh, acc[0][b], 0, 0, 0);
      acc[1][b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ayl, bh, acc[1][b], 0, 0, 0);
      acc[1][b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ayh, bl, acc[1][b], 0, 0, 0);
      acc[1][b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ayh, bh, acc[1][b], 0, 0, 0);
    }
  };
  // even and odd chunks; no branch inside the loop, so that the wait
  // before each product covers only that chunk's loads (the last even load
  // of an even count reads chunk nchunks - 1 again, unused)
  Ops o0, o1;
  load(0, o0);
  int c = 0;
  for (; c + 1 < nchunks; c += 2) {   // wave-uniform
    load(c + 1, o1);
    __builtin_amdgcn_sched_barrier(0);   // keep the prefetch ahead of the products
    mma(o0);
    __builtin_amdgcn_sched_barrier(0);
    load(min(c + 2, nchunks - 1), o0);
    __builtin_amdgcn_sched_barrier(0);
    mma(o1);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (c < nchunks) mma(o0);
  // store block by block (the barriers keep one block's accumulators in
  // flight to memory at a time); non-temporal, like the step's stores:
  // measured 7 us less for the step kernel that reads the planes next, at
  // 4096^2 (830 against 838 us)
#pragma unroll
  for (int b = 0; b < kSynthBlocks; ++b) {
    const int x = xw + 32 * b + l32;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int y = y0 + 8 * (i >> 2) + 4 * half + (i & 3);
      if (x < nx && y < ny) {
        __builtin_nontemporal_store(acc[0][b][i] * inv_scale, &force[(size_t)y * row_pitch + x]);
        __builtin_nontemporal_store(acc[1][b][i] * inv_scale,
                                    &force[force_pitch + (size_t)y * row_pitch + x]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
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

hipError_t launch_stir_draw(const StirArgs& a, int64_t step, hipStream_t s) {
  hipLaunchKernelGGL(stir_draw_kernel, dim3(1), dim3(256), 0, s, a, step);
  return hipGetLastError();
}

hipError_t launch_stir_table(const StirArgs& a, int64_t fixed_step, hipStream_t s) {
  hipLaunchKernelGGL(stir_table_kernel, dim3((a.ny + 63) / 64, 8 * synth_chunks(a.K)), dim3(64), 0,
                     s, a, fixed_step);
  return hipGetLastError();
}

hipError_t launch_stir_synth(const StirArgs& a, bool advance, hipStream_t s) {
  const int tiles = ((a.nx + kSynthWaveCols - 1) / kSynthWaveCols) * ((a.ny + 31) / 32);
  const int wgs = (tiles + kSynthWaves - 1) / kSynthWaves;
  const int per_xcd = (wgs + 7) / 8;   // tiles past the last one return at once
  hipLaunchKernelGGL(stir_synth_kernel, dim3(8 * per_xcd), dim3(64 * kSynthWaves), 0, s, a.table,
                     a.twiddle, a.force, a.force_pitch, synth_chunks(a.K), a.nx, a.ny, a.row,
                     a.inv_scale, a.dstep, advance ? 1 : 0, per_xcd);
  return hipGetLastError();
}

hipError_t launch_twiddle(uint4* tw, int K, int nx, hipStream_t s) {
  hipLaunchKernelGGL(twiddle_kernel, dim3(((kMaxK + 1) * nx + 255) / 256), dim3(256), 0, s, tw, K, nx);
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
