// Node-brick layout of the population state and the bilinear pull over it.
//
// A state copy holds the 2Q planes (F then G) of every node.  Row y of the
// lattice is a run of ceil(nx / 64) bricks; brick b holds columns
// 64 b .. 64 b + 63 and, inside it, plane k of column x sits at element
// k * 64 + (x mod 64).  So the 64 nodes of one wavefront find each plane in
// one aligned 256-byte segment, all 2Q planes of the wavefront lie in one
// contiguous 2Q * 256-byte run, and a row is 2Q * row elements long
// (row = nx rounded up to 64).  Compared with whole-lattice planes this
// keeps the three rows a pull touches in three contiguous runs, which the
// memory system serves with far fewer DRAM page switches.
//
// Addresses are split into a row part (64-bit byte offset, uniform across
// a wavefront that covers one lattice row) and a column part (32-bit byte
// offset inside the row), so every access is scalar base + vector offset.
#pragma once

#include <cstdint>

#include "internal.hpp"

namespace rlb {

// Byte offset of column x inside a state row.
template <int Q>
__device__ __forceinline__ uint32_t col_bytes(int x) {
  return 4u * (uint32_t)((x >> 6) * (2 * Q * 64) + (x & 63));
}

// Element offset of plane k of node (x, y) inside a state copy.
template <int Q>
__device__ __forceinline__ int64_t state_elem(int k, int x, int y, int row) {
  return (int64_t)y * (2 * Q) * row + (int64_t)((x >> 6) * (2 * Q * 64) + k * 64 + (x & 63));
}

// Periodic 3x3 neighbourhood of (x, y): rows y-1, y, y+1 and columns
// x-1, x, x+1.
struct Nbr {
  int64_t r[3];    // byte offsets of the rows
  uint32_t c[3];   // byte offsets of the columns inside a row
};

template <int Q>
__device__ __forceinline__ Nbr neighbourhood(int x, int y, int nx, int ny, int row) {
  const int xm = x == 0 ? nx - 1 : x - 1;
  const int xp = x == nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1;
  const int yp = y == ny - 1 ? 0 : y + 1;
  const int64_t rb = (int64_t)4 * (2 * Q) * row;
  Nbr n;
  n.r[0] = ym * rb;
  n.r[1] = y * rb;
  n.r[2] = yp * rb;
  n.c[0] = col_bytes<Q>(xm);
  n.c[1] = col_bytes<Q>(x);
  n.c[2] = col_bytes<Q>(xp);
  return n;
}

// Device-memory (global address space) views, so that accesses compile to
// global loads and stores with a scalar base rather than flat ones.
using gbyte = __attribute__((address_space(1))) char;
using gfloat = __attribute__((address_space(1))) float;

// Value of plane PL at row part r, column part c.
template <int PL>
__device__ __forceinline__ float ldp(const float* base, int64_t r, uint32_t c) {
  const gbyte* b = (const gbyte*)base + r + PL * 256;
  return *(const gfloat*)(b + c);
}

// NT: a non-temporal store (large lattices); otherwise a plain one, which
// leaves the value in the last-level cache for the next step's pulls.
template <int PL, bool NT = true>
__device__ __forceinline__ void stp(float* base, int64_t r, uint32_t c, float v) {
  gbyte* b = (gbyte*)base + r + PL * 256;
  if constexpr (NT) __builtin_nontemporal_store(v, (gfloat*)(b + c));
  else *(gfloat*)(b + c) = v;
}

// Four-tap interpolation t0 a + t1 b + t2 c + t3 d with t0 + t1 + t2 + t3 = 1,
// as a + t1 (b - a) + t2 (c - a) + t3 (d - a) (exact for a = b = c = d).
// SYM: t1 = t2 (|vx| = |vy|), so t1 ((b + c) - 2a) + t3 (d - a).
template <bool SYM>
__device__ __forceinline__ float bilinear(float a, float b, float c, float d, const float* tap) {
  if constexpr (SYM) {
    return __builtin_fmaf(tap[3], d - a, __builtin_fmaf(tap[1], __builtin_fmaf(-2.0f, a, b + c), a));
  } else {
    return __builtin_fmaf(tap[3], d - a,
                          __builtin_fmaf(tap[2], c - a, __builtin_fmaf(tap[1], b - a, a)));
  }
}

template <class DS, int P>
struct Taps {
  static constexpr double vx = DS::vx[P], vy = DS::vy[P];
  static constexpr int sx = vx > 0 ? 1 : (vx < 0 ? -1 : 0);
  static constexpr int sy = vy > 0 ? 1 : (vy < 0 ? -1 : 0);
  static constexpr bool unit_x = vx == 1.0 || vx == -1.0;
  static constexpr bool unit_y = vy == 1.0 || vy == -1.0;
};

// Bilinear pull of direction P from plane PL at the node: the pre-stream
// value at the departure point (x, y) - cfl (vx, vy), with the taps
// tap[0..3] on (x, y), (x - sx, y), (x, y - sy), (x - sx, y - sy).  REV
// takes the same weights at x + delta instead (the transposed pull, used
// by the adjoint).  With UNIT (cfl = 1) a unit component is a plain shift.
// The weights sum to exactly 1, so the sum is formed as the first tap's
// value plus weighted differences, a + t1 (b - a) + t2 (c - a) + t3 (d - a)
// (with |vx| = |vy| the two middle weights are equal and share one
// product): a uniform field streams unchanged bit for bit.  (Summed as
// t0 a + t1 b + t2 c + t3 d, the float32 products moved a uniform value by
// an ulp at some values, the same at every node, and the conserved totals
// drifted at a steady rate.)
template <class DS, bool UNIT, int P, int PL, bool REV>
__device__ __forceinline__ float pull(const float* __restrict__ base, const Nbr& n,
                                      const float* tap) {
  using T = Taps<DS, P>;
  constexpr int sx = REV ? -T::sx : T::sx;
  constexpr int sy = REV ? -T::sy : T::sy;
  const int64_t r0 = n.r[1], ry = n.r[1 - sy];
  const uint32_t c0 = n.c[1], cx = n.c[1 - sx];
  if constexpr (T::sx == 0 && T::sy == 0) {
    return ldp<PL>(base, r0, c0);
  } else if constexpr (UNIT && T::unit_x) {
    return ldp<PL>(base, r0, cx);
  } else if constexpr (UNIT && T::unit_y) {
    return ldp<PL>(base, ry, c0);
  } else if constexpr (T::sy == 0) {
    const float a = ldp<PL>(base, r0, c0);
    return a + tap[1] * (ldp<PL>(base, r0, cx) - a);
  } else if constexpr (T::sx == 0) {
    const float a = ldp<PL>(base, r0, c0);
    return a + tap[2] * (ldp<PL>(base, ry, c0) - a);
  } else {
    return bilinear<DS::vx[P] == DS::vy[P] || DS::vx[P] == -DS::vy[P]>(
        ldp<PL>(base, r0, c0), ldp<PL>(base, r0, cx), ldp<PL>(base, ry, c0), ldp<PL>(base, ry, cx),
        tap);
  }
}

// Two-cell neighbourhood for 1 < cfl <= 2: rows y-2 .. y+2 and columns
// x-2 .. x+2 (periodic), index 2 is the node itself.
struct Nbr5 {
  int64_t r[5];
  uint32_t c[5];
};

template <int Q>
__device__ __forceinline__ Nbr5 neighbourhood5(int x, int y, int nx, int ny, int row) {
  const int64_t rb = (int64_t)4 * (2 * Q) * row;
  Nbr5 n;
#pragma unroll
  for (int d = -2; d <= 2; ++d) {
    int xx = x + d, yy = y + d;
    xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
    yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
    n.r[d + 2] = yy * rb;
    n.c[d + 2] = col_bytes<Q>(xx);
  }
  return n;
}

// Pull for 1 < cfl <= 2: along each axis the displacement is m whole cells
// (m = 0 or 1, uniform per plane: shift[0] for x, shift[1] for y) plus a
// fraction, so the taps sit m and m + 1 cells upstream; tap[] holds the
// bilinear weights of (near x, near y), (far x, near y), (near x, far y),
// (far x, far y).
template <class DS, int P, int PL>
__device__ __forceinline__ float pull_wide(const float* __restrict__ base, const Nbr5& n,
                                           const float* tap, const uint8_t* shift) {
  using T = Taps<DS, P>;
  constexpr int sx = T::sx, sy = T::sy;
  if constexpr (sx == 0 && sy == 0) {
    return ldp<PL>(base, n.r[2], n.c[2]);
  } else {
    const bool mx = shift[0] != 0, my = shift[1] != 0;
    const uint32_t cn = sx == 0 ? n.c[2] : (mx ? n.c[2 - sx] : n.c[2]);
    const uint32_t cf = sx == 0 ? n.c[2] : (mx ? n.c[2 - 2 * sx] : n.c[2 - sx]);
    const int64_t rn = sy == 0 ? n.r[2] : (my ? n.r[2 - sy] : n.r[2]);
    const int64_t rf = sy == 0 ? n.r[2] : (my ? n.r[2 - 2 * sy] : n.r[2 - sy]);
    const float a = ldp<PL>(base, rn, cn);   // differences from the near tap, as pull
    if constexpr (sy == 0) {
      return a + tap[1] * (ldp<PL>(base, rn, cf) - a);
    } else if constexpr (sx == 0) {
      return a + tap[2] * (ldp<PL>(base, rf, cn) - a);
    } else {
      return bilinear<DS::vx[P] == DS::vy[P] || DS::vx[P] == -DS::vy[P]>(
          a, ldp<PL>(base, rn, cf), ldp<PL>(base, rf, cn), ldp<PL>(base, rf, cf), tap);
    }
  }
}

// Streaming modes of the step kernels: general cfl < 1, cfl = 1 (unit
// components are plain shifts), 1 < cfl <= 2 (two-cell stencil).
enum StreamMode : int { SM_GENERAL = 0, SM_UNIT = 1, SM_WIDE = 2 };

}  // namespace rlb
