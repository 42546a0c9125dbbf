// Device helpers shared by the RLB kernels: compile-time loops, the float64
// Landau solve, equilibrium and driving-term coefficients, Philox4x64-10.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace rlb {

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// ---------------------------------------------------------------------------
// Landau matching on the (t, x, y) block: T^mu_nu u^nu = eps u^mu with
// T^mu_nu = T^{mu lambda} g_{lambda nu}, g = diag(1, -1, -1).  The z row and
// column decouple (T^{0z} = T^{xz} = T^{yz} = 0 for a lattice with one z node
// and no z force), so u^z = 0.
//
// eps is the largest real root of the characteristic cubic of A = T g: the
// timelike eigenvalue exceeds the spacelike ones, which are minus the
// rest-frame pressures.  Newton's method on the cubic starts from the energy
// density of the ideal conformal fluid with the same T^{00} and T^{0i},
// eps0 = sqrt(4 T00^2 - 3 |T^{0i}|^2) - T00, which differs from eps only by
// the viscous stress; two steps reach float64 precision.  The result is
// accepted when the last step was small and the deflated quadratic has no
// root above it (chi'(eps) > 0 and 3 eps > trace); otherwise the root is
// taken from the trigonometric form of the depressed cubic.  u is the cross
// product of two rows of (A - eps I), normalised to u.u = 1, u^0 > 0.
// Returns false when no timelike eigenvector exists.
// ---------------------------------------------------------------------------
struct Frame {
  double eps, u0, ux, uy;
};

__device__ __noinline__ double cubic_largest_root(double c2, double c1, double c0) {
  const double s = c2 * (1.0 / 3.0);
  const double p = c1 - c2 * s;
  const double q = (-2.0 * s * s + c1) * s - c0;
  if (!(p < 0.0)) return -1.0;
  const double r = sqrt(-p * (1.0 / 3.0));
  double arg = -q / (2.0 * r * r * r);
  arg = fmin(1.0, fmax(-1.0, arg));
  double lam = 2.0 * r * cos(acos(arg) * (1.0 / 3.0)) + s;
  for (int it = 0; it < 2; ++it) {
    const double f = ((lam - c2) * lam + c1) * lam - c0;
    const double d = (3.0 * lam - 2.0 * c2) * lam + c1;
    if (d != 0.0) lam -= f / d;
  }
  return lam;
}

// The Newton start is the ideal-fluid energy density: for P = eps/3,
// eps = sqrt(4 a^2 - 3 b^2) - a; for the planar set (P = eps/2),
// eps = (sqrt(9 a^2 - 8 b^2) - a) / 2 (a = T^00, b = |T^0i|).
template <bool PLANAR = false>
__device__ __forceinline__ bool landau3(double T00, double T0x, double T0y,
                                        double Txx, double Txy, double Tyy,
                                        Frame& fr) {
  const double a00 = T00, a01 = -T0x, a02 = -T0y;
  const double a10 = T0x, a11 = -Txx, a12 = -Txy;
  const double a20 = T0y, a21 = -Txy, a22 = -Tyy;
  const double c2 = a00 + a11 + a22;
  const double m12 = a11 * a22 - a12 * a21;
  const double c1 = (a00 * a11 - a01 * a10) + (a00 * a22 - a02 * a20) + m12;
  const double c0 = a00 * m12 - a01 * (a10 * a22 - a12 * a20) +
                    a02 * (a10 * a21 - a11 * a20);
  const double b2 = T0x * T0x + T0y * T0y;
  const double disc = PLANAR ? 9.0 * T00 * T00 - 8.0 * b2 : 4.0 * T00 * T00 - 3.0 * b2;
  double lam = disc > 0.0 ? (PLANAR ? 0.5 * (sqrt(disc) - T00) : sqrt(disc) - T00) : T00;
  double step = 0.0, d = 0.0;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double f = ((lam - c2) * lam + c1) * lam - c0;
    d = (3.0 * lam - 2.0 * c2) * lam + c1;
    step = f / d;
    lam -= step;
  }
  if (!(fabs(step) <= 1e-10 * fabs(lam)) || !(d > 0.0) || !(3.0 * lam > c2))
    lam = cubic_largest_root(c2, c1, c0);
  if (!(lam > 0.0)) return false;
  // rows of (A - lam I)
  const double r0x = a00 - lam, r0y = a01, r0z = a02;
  const double r1x = a10, r1y = a11 - lam, r1z = a12;
  const double r2x = a20, r2y = a21, r2z = a22 - lam;
  double vx = r1y * r2z - r1z * r2y;   // r1 x r2: well conditioned for |beta| < ~0.6
  double vy = r1z * r2x - r1x * r2z;
  double vz = r1x * r2y - r1y * r2x;
  double nb = vx * vx + vy * vy + vz * vz;
  double mn = vx * vx - vy * vy - vz * vz;
  if (!(mn > 0.5 * nb)) {
    const double wx = r0y * r2z - r0z * r2y;   // r0 x r2
    const double wy = r0z * r2x - r0x * r2z;
    const double wz = r0x * r2y - r0y * r2x;
    const double nw = wx * wx + wy * wy + wz * wz;
    if (nw > nb) { vx = wx; vy = wy; vz = wz; nb = nw; }
    const double ux = r0y * r1z - r0z * r1y;   // r0 x r1
    const double uy = r0z * r1x - r0x * r1z;
    const double uz = r0x * r1y - r0y * r1x;
    const double nu = ux * ux + uy * uy + uz * uz;
    if (nu > nb) { vx = ux; vy = uy; vz = uz; nb = nu; }
    mn = vx * vx - vy * vy - vz * vz;
    if (!(mn > 1e-12 * nb)) return false;
  }
  const double inv = (vx > 0.0 ? 1.0 : -1.0) / sqrt(mn);
  fr.eps = lam;
  fr.u0 = vx * inv;
  fr.ux = vy * inv;
  fr.uy = vz * inv;
  return true;
}

// ---------------------------------------------------------------------------
// Equilibrium in shifted form.  With T_eq = (4 eps/3) u u - (eps/3) g and the
// expansion coefficients 1, 3, 15/2 of the angular polynomials, the
// truncated Juttner equilibrium of a direction v (|v| = 1) is
//     F_eq = w (eps - 2 eps |u|^2 + 4 eps u^0 (u.v) + 10 eps (u.v)^2),
//     G_eq = w (n u^0 + 3 n (u.v)).
// The kernels store F - w eps_ref and G - w n_ref, so the constant terms are
// formed in float64 relative to the references before rounding.
// Planar set (P = eps/2, circle polynomials with coefficients 1, 2, 4):
//     F_eq = w (eps - 3/2 eps |u|^2 + 3 eps u^0 (u.v) + 6 eps (u.v)^2),
//     G_eq = w (n u^0 + 2 n (u.v)).
// ---------------------------------------------------------------------------
struct EqCoef {
  float A, B, C;   // F_eq - w eps_ref = w (A + B s + C s^2), s = u.v
  float Ag, Bg;    // G_eq - w n_ref   = w (Ag + Bg s)
};

// kappa: see dirset.hpp (float32 quadrature correction of the s, s^2 terms).
template <bool PLANAR = false>
__device__ __forceinline__ EqCoef eq_coef(const Frame& fr, double n,
                                          double eps_ref, double n_ref,
                                          double kappa) {
  constexpr double cu = PLANAR ? 1.5 : 2.0, cb = PLANAR ? 3.0 : 4.0;
  constexpr double cc = PLANAR ? 6.0 : 10.0, cg = PLANAR ? 2.0 : 3.0;
  EqCoef c;
  const double u2 = fr.ux * fr.ux + fr.uy * fr.uy;
  c.A = (float)((fr.eps - eps_ref) - cu * fr.eps * u2);
  c.B = (float)(cb * kappa * fr.eps * fr.u0);
  c.C = (float)(cc * kappa * fr.eps);
  c.Ag = (float)(n * fr.u0 - n_ref);
  c.Bg = (float)(cg * kappa * n);
  return c;
}

// Frame of a 3-velocity (initial fields).
__device__ __forceinline__ bool frame_from_beta(double eps, double bx,
                                                double by, Frame& fr) {
  const double b2 = bx * bx + by * by;
  if (!(b2 < 1.0) || !(eps > 0.0)) return false;
  const double g = 1.0 / sqrt(1.0 - b2);
  fr.eps = eps;
  fr.u0 = g;
  fr.ux = g * bx;
  fr.uy = g * by;
  return true;
}


// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11) and the Box-Muller transform.
// ---------------------------------------------------------------------------
struct U64x4 {
  uint64_t v[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1,
                                               uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  U64x4 o;
  o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

// ((x >> 11) + 1/2) 2^-53 in (0, 1)
__device__ __forceinline__ double uniform_open(uint64_t x) {
  return ((double)(x >> 11) + 0.5) * 1.1102230246251565404e-16;
}

__device__ __forceinline__ void box_muller(uint64_t a, uint64_t b, double& z0,
                                           double& z1) {
  const double u1 = uniform_open(a), u2 = uniform_open(b);
  const double r = sqrt(-2.0 * log(u1));
  const double th = 6.283185307179586477 * u2;
  z0 = r * cos(th);
  z1 = r * sin(th);
}

}  // namespace rlb
