// Discrete adjoint of the RLB step for gradients of time-averaged channel
// objectives with respect to the body force, the relaxation time and the
// amplitudes of a fixed stirring basis.
//
// The step is s_{t+1} = C(P s_t): P the bilinear pull (Ch. 3, linear
// interpolation of off-lattice streaming), C the local update (moments,
// Landau matching, equilibrium, Anderson-Witting relaxation, driving term
// of Ch. 4 eq. forceTerm, bounce-back).  With an objective
// J = sum_t J_t(P s_t), the adjoint is
//     mu_t = (dC/dF~)^T lambda_{t+1} + dJ_t/dF~     (local, per node)
//     lambda_t = P^T mu_t                             (transposed pull)
// and dJ/dtheta = sum_t lambda_{t+1} . dC/dtheta.  One adjoint kernel per
// step reads s_t (pulled, to recompute the forward intermediates) and
// mu_{t+1} (transpose-pulled: the same bilinear weights taken at x + delta),
// applies the hand-written local reverse sweep and writes mu_t; per-node
// float64 accumulators collect dJ/dF(x) and dJ/d(1/tau), reduced at the end.
// Landau matching is differentiated implicitly: with A = T g, l = g u,
//     d eps = u_mu u_nu dT^{mu nu},
//     [A - eps I, u; l^T, 0] [du; 0] = [d eps u - dA u; 0],
// so the adjoint solves the transposed bordered system once per node, as a
// regular 3x3 system (see the reverse sweep).
#include <algorithm>

#include "internal.hpp"
#include "device_common.hpp"
#include "dirset.hpp"
#include "brick.hpp"

namespace rlb {

struct Moments {
  double T00, T0x, T0y, Txx, Txy, Tyy, J0, Jx, Jy;
};

template <class DS>
__device__ __forceinline__ Moments moments_of(const float* f, const float* g, double eps_ref,
                                              double n_ref) {
  // plane by plane (summed by opposite pairs, as the step kernel does, the
  // adjoint run measured 1.7 ms slower at 512 x 256: a pair's sum waits for
  // both of its loads)
  float m00 = 0, m0x = 0, m0y = 0, mxx = 0, mxy = 0, myy = 0, j0 = 0, jx = 0, jy = 0;
  static_for<0, DS::Q>([&](auto P) {
    constexpr int p = decltype(P)::value;
    constexpr double vx = DS::vx[p], vy = DS::vy[p];
    m00 += f[p];
    j0 += g[p];
    if constexpr (vx != 0.0) { m0x += (float)vx * f[p]; jx += (float)vx * g[p]; mxx += (float)(vx * vx) * f[p]; }
    if constexpr (vy != 0.0) { m0y += (float)vy * f[p]; jy += (float)vy * g[p]; myy += (float)(vy * vy) * f[p]; }
    if constexpr (vx != 0.0 && vy != 0.0) mxy += (float)(vx * vy) * f[p];
  });
  Moments m;
  m.T00 = eps_ref + (double)m00;
  m.T0x = (double)m0x;
  m.T0y = (double)m0y;
  m.Txx = eps_ref * (1.0 / 3.0) + (double)mxx;
  m.Tyy = eps_ref * (1.0 / 3.0) + (double)myy;
  m.Txy = (double)mxy;
  m.J0 = n_ref + (double)j0;
  m.Jx = (double)jx;
  m.Jy = (double)jy;
  return m;
}

// Non-equilibrium stress pi^{kl} = T^{kl} - T_eq^{kl} (k, l over x, y, z)
// with T^{zz} = T^{00} - T^{xx} - T^{yy} (traceless) and T_eq^{zz} = eps/3.
struct Pi {
  double xx, yy, xy, zz;
};

__device__ __forceinline__ Pi pi_of(const Moments& m, const Frame& fr) {
  Pi q;
  const double e43 = (4.0 / 3.0) * fr.eps;
  q.xx = m.Txx - (e43 * fr.ux * fr.ux + fr.eps / 3.0);
  q.yy = m.Tyy - (e43 * fr.uy * fr.uy + fr.eps / 3.0);
  q.xy = m.Txy - e43 * fr.ux * fr.uy;
  q.zz = (m.T00 - m.Txx - m.Tyy) - fr.eps / 3.0;
  return q;
}

// Tiles of 64 x 4 nodes, ordered as the step kernel orders them: the eight
// XCDs (workgroup i runs on XCD i mod 8) each take a contiguous band of
// tiles, visited in vertical strips `strip` tiles wide and row by row
// inside a strip, so that neighbouring tiles, which share halo rows, meet in
// one L2.  (Row-major order over the XCDs in turn: 1.31x the algorithmic
// reads at 512 x 256.)
template <class DS, bool UNIT, bool MASK, bool MU>
__global__ __launch_bounds__(256) void adjoint_kernel(const AdjArgs a) {
  constexpr int Q = DS::Q;
  const int t = (int)(blockIdx.x & 7) * a.tiles_per_xcd + (int)(blockIdx.x >> 3);
  if (t >= a.ntiles) return;
  const int tiles_y = (a.ny + 3) / 4;
  const int sw = min(a.strip, a.tiles_x);
  const int full = a.tiles_x / sw;
  const int st = t / (sw * tiles_y);
  const int w = st < full ? sw : a.tiles_x - full * sw;
  const int in = t - st * sw * tiles_y;
  const int ty = in / w;
  const int x = (st * sw + (in - ty * w)) * 64 + (threadIdx.x & 63);
  const int y = __builtin_amdgcn_readfirstlane(ty * 4 + (threadIdx.x >> 6));
  if (x >= a.nx || y >= a.ny) return;
  const uint32_t node = (uint32_t)(y * a.nx + x);
  const Nbr nb = neighbourhood<Q>(x, y, a.nx, a.ny, a.row);
  const StepShared& sh = a.sh;

  // The first adjoint step has no mu_{t+1} (MU = false: lambda = 0, no
  // transposed pulls); the others pull both in one branch-free batch of
  // loads (a runtime test per plane made the compiler wait for each
  // plane's loads in turn).
  float f[Q], g[Q], lf[Q], lg[Q];
  static_for<0, Q>([&](auto P) {
    constexpr int p = decltype(P)::value;
    f[p] = pull<DS, UNIT, p, p, false>(a.state, nb, sh.tap[p]);
    g[p] = pull<DS, UNIT, p, Q + p, false>(a.state, nb, sh.tap[p]);
    if constexpr (MU) {
      lf[p] = pull<DS, UNIT, p, p, true>(a.mu_in, nb, sh.tap[p]);
      lg[p] = pull<DS, UNIT, p, Q + p, true>(a.mu_in, nb, sh.tap[p]);
    } else {
      lf[p] = 0.0f;
      lg[p] = 0.0f;
    }
  });
  // this node's force and accumulators, loaded with the populations so
  // that their latency overlaps the pulls (the accumulators would otherwise
  // be read after the adjoint's stores, at the end of the critical path)
  const gfloat* frc = (const gfloat*)a.force + (int64_t)y * a.row + x;
  const float frx = frc[0], fry = frc[a.pitch];
  double2 af = a.acc_f[node];
  double at = a.acc_itau[node];
  char* out = (char*)a.mu_out + nb.r[1] + nb.c[1];
  auto put = [&](int plane, float v) { *(float*)(out + plane * 256) = v; };

  if constexpr (MASK) {
    if (a.mask[node]) {   // f'_p = f~_opp(p): mu_q = lambda'_opp(q)
      static_for<0, Q>([&](auto P) {
        constexpr int p = decltype(P)::value;
        put(p, lf[DS::opp[p]]);
        put(Q + p, lg[DS::opp[p]]);
      });
      return;
    }
  }

  // ---- forward recomputation ----
  const Moments m = moments_of<DS>(f, g, sh.eps_ref, sh.n_ref);
  Frame fr{0.0, 1.0, 0.0, 0.0};
  const bool ok = landau3(m.T00, m.T0x, m.T0y, m.Txx, m.Txy, m.Tyy, fr);
  if (!ok) {   // forward left the node uncollided: identity
    atomicOr(sh.err, ERR_LANDAU);
    static_for<0, Q>([&](auto P) {
      constexpr int p = decltype(P)::value;
      put(p, lf[p]);
      put(Q + p, lg[p]);
    });
    return;
  }
  const double n = fr.u0 * m.J0 - fr.ux * m.Jx - fr.uy * m.Jy;
  const EqCoef ec = eq_coef(fr, n, sh.eps_ref, sh.n_ref, DS::kappa);
  const float ux = (float)fr.ux, uy = (float)fr.uy, u0 = (float)fr.u0;
  const float itau = sh.inv_tau;
  const float Fx = sh.fx + frx;
  const float Fy = sh.fy + fry;
  float q3xxx = 0, q3xxy = 0, q3xyy = 0, q3yyy = 0, q3xzz = 0, q3yzz = 0;
  static_for<0, Q>([&](auto P) {   // odd in v: from f_a - f_b of each pair
    constexpr int p = decltype(P)::value;
    constexpr int q = DS::opp[p];
    if constexpr (q > p) {
      constexpr double vx = DS::vx[p], vy = DS::vy[p], vz2 = DS::vz2[p];
      const float d = f[p] - f[q];
      q3xxx += (float)(vx * vx * vx) * d;
      q3xxy += (float)(vx * vx * vy) * d;
      q3xyy += (float)(vx * vy * vy) * d;
      q3yyy += (float)(vy * vy * vy) * d;
      q3xzz += (float)(vx * vz2) * d;
      q3yzz += (float)(vy * vz2) * d;
    }
  });
  const float M0 = (float)m.T00, M1x = (float)m.T0x, M1y = (float)m.T0y;

  // ---- reverse sweep ----
  // per-direction part: lambda of A, B, C, Ag, Bg, u, 1/tau, Phi coefficients
  float lA = 0, lB = 0, lC = 0, lAg = 0, lBg = 0, lux = 0, luy = 0, lu0 = 0, litau = 0;
  float lp0 = 0, lpx = 0, lpy = 0, lpxx = 0, lpxy = 0, lpyy = 0;
  // By opposite pairs (a, b), v_b = -v_a: s_b = -s_a, the equilibrium
  // splits into an even part e0 and an odd part e1 in s, and every
  // accumulation below is the pair's sum (even in v) or difference (odd).
  float mf[Q], mg[Q];
  static_for<0, Q>([&](auto P) {
    constexpr int p = decltype(P)::value;
    constexpr int q = DS::opp[p];
    constexpr float w = DS::w32[p];
    if constexpr (q == p) {   // v_x = v_y = 0: s = 0
      const float om = u0 * itau;
      const float lfp = lf[p], lgp = lg[p];
      mf[p] = lfp * (1.0f - om);
      mg[p] = lgp * (1.0f - om);
      const float lom = -lfp * (f[p] - w * ec.A) - lgp * (g[p] - w * ec.Ag);
      lu0 += lom * itau;
      litau += lom * u0;
      lA += w * (lfp * om);
      lAg += w * (lgp * om);
      lp0 -= w * lfp;
    } else if constexpr (q > p) {
      constexpr float vx = (float)DS::vx[p], vy = (float)DS::vy[p];
      const float s = ux * vx + uy * vy;
      const float oma = (u0 - s) * itau, omb = (u0 + s) * itau;
      const float e0 = w * (ec.A + ec.C * s * s), e1 = w * (ec.B * s);
      const float g0 = w * ec.Ag, g1 = w * (ec.Bg * s);
      const float lfa = lf[p], lfb = lf[q], lga = lg[p], lgb = lg[q];
      mf[p] = lfa * (1.0f - oma);
      mf[q] = lfb * (1.0f - omb);
      mg[p] = lga * (1.0f - oma);
      mg[q] = lgb * (1.0f - omb);
      const float loma = -lfa * (f[p] - (e0 + e1)) - lga * (g[p] - (g0 + g1));
      const float lomb = -lfb * (f[q] - (e0 - e1)) - lgb * (g[q] - (g0 - g1));
      const float los = loma + lomb, lod = loma - lomb;
      const float lfea = lfa * oma, lfeb = lfb * omb, lgea = lga * oma, lgeb = lgb * omb;
      const float fs = lfea + lfeb, fd = lfea - lfeb, gs = lgea + lgeb, gd = lgea - lgeb;
      lu0 += los * itau;
      litau += u0 * los - s * lod;
      lA += w * fs;
      lB += w * s * fd;
      lC += w * s * s * fs;
      lAg += w * gs;
      lBg += w * s * gd;
      // d/ds of pair member a minus that of b (v_b = -v_a)
      const float lsd = -lod * itau + w * ec.B * fd + 2.0f * w * ec.C * s * fs + w * ec.Bg * gd;
      lux += vx * lsd;
      luy += vy * lsd;
      const float ps = -w * (lfa + lfb), pd = -w * (lfa - lfb);
      lp0 += ps;
      lpx += vx * pd;
      lpy += vy * pd;
      lpxx += vx * vx * ps;
      lpxy += vx * vy * ps;
      lpyy += vy * vy * ps;
    }
  });
  // driving-term coefficients (vz^2 folded into p0, pxx, pyy)
  const float lpzz = lp0 - lpxx - lpyy;
  const float lQzz = 1.25f * lpzz, lQxx = 1.25f * lpxx, lQxy = 2.5f * lpxy, lQyy = 1.25f * lpyy;
  const float lFM1 = 0.25f * lp0;
  const float lM0 = -0.5f * (Fx * lpx + Fy * lpy);
  const float lFx = -0.5f * M0 * lpx - 2.5f * M1x * lpxx - 2.5f * M1y * lpxy + M1x * lFM1 +
                    q3xxx * lQxx + q3xxy * lQxy + q3xyy * lQyy + q3xzz * lQzz;
  const float lFy = -0.5f * M0 * lpy - 2.5f * M1y * lpyy - 2.5f * M1x * lpxy + M1y * lFM1 +
                    q3xxy * lQxx + q3xyy * lQxy + q3yyy * lQyy + q3yzz * lQzz;
  const float lM1x = -2.5f * Fx * lpxx - 2.5f * Fy * lpxy + Fx * lFM1;
  const float lM1y = -2.5f * Fy * lpyy - 2.5f * Fx * lpxy + Fy * lFM1;
  const float lq3xxx = Fx * lQxx, lq3xxy = Fy * lQxx + Fx * lQxy;
  const float lq3xyy = Fy * lQxy + Fx * lQyy, lq3yyy = Fy * lQyy;
  const float lq3xzz = Fx * lQzz, lq3yzz = Fy * lQzz;

  // equilibrium coefficients -> eps, u, n (float64 from here)
  const double kap = DS::kappa;
  double leps = (double)lA * (1.0 - 2.0 * (fr.ux * fr.ux + fr.uy * fr.uy)) +
                4.0 * kap * fr.u0 * (double)lB + 10.0 * kap * (double)lC;
  double lUx = (double)lux - 4.0 * fr.eps * fr.ux * (double)lA;
  double lUy = (double)luy - 4.0 * fr.eps * fr.uy * (double)lA;
  double lU0 = (double)lu0 + 4.0 * kap * fr.eps * (double)lB + n * (double)lAg;
  const double ln = fr.u0 * (double)lAg + 3.0 * kap * (double)lBg;
  lU0 += m.J0 * ln;
  lUx -= m.Jx * ln;
  lUy -= m.Jy * ln;
  double lJ0 = fr.u0 * ln, lJx = -fr.ux * ln, lJy = -fr.uy * ln;
  double lT00 = (double)lM0, lT0x = (double)lM1x, lT0y = (double)lM1y;
  double lTxx = 0.0, lTxy = 0.0, lTyy = 0.0;

  // objective density of this step
  if (a.obj_c != 0.0f) {
    const double c = (double)a.obj_c;
    if (a.kind == 0) {
      lJx += c;
    } else {
      const Pi q = pi_of(m, fr);
      const double lxx = 2.0 * c * q.xx, lyy = 2.0 * c * q.yy, lxy = 4.0 * c * q.xy,
                   lzz = 2.0 * c * q.zz;
      lTxx += lxx - lzz;
      lTyy += lyy - lzz;
      lTxy += lxy;
      lT00 += lzz;
      leps -= lxx * ((4.0 / 3.0) * fr.ux * fr.ux + 1.0 / 3.0) +
              lyy * ((4.0 / 3.0) * fr.uy * fr.uy + 1.0 / 3.0) +
              lxy * (4.0 / 3.0) * fr.ux * fr.uy + lzz / 3.0;
      lUx -= lxx * (8.0 / 3.0) * fr.eps * fr.ux + lxy * (4.0 / 3.0) * fr.eps * fr.uy;
      lUy -= lyy * (8.0 / 3.0) * fr.eps * fr.uy + lxy * (4.0 / 3.0) * fr.eps * fr.ux;
    }
  }

  // Landau matching, implicitly: solve [B, l; u^T, 0] [z; zeta] =
  // [lambda_u; 0] with B = (A - eps I)^T, then lambda_T = (lambda_eps + z.u)
  // l l^T - sym(z l^T).  Since A u = eps u, u^T B = 0, and u.l = u_mu u^mu
  // = 1: the first three rows dotted with u give zeta = u.lambda_u.  The
  // rank-one term l u^T fills B's null direction, M = B + l u^T is regular
  // (at rest its determinant is about -(4 eps / 3)^2), and M z = lambda_u -
  // zeta l has the solution of the bordered system (u.z = 0 follows from
  // u^T M z = u.z).  Solved by the adjugate: no pivoting, one division.
  {
    const double u[3] = {fr.u0, fr.ux, fr.uy};
    const double l[3] = {fr.u0, -fr.ux, -fr.uy};
    const double Am[3][3] = {{m.T00, -m.T0x, -m.T0y},
                             {m.T0x, -m.Txx, -m.Txy},
                             {m.T0y, -m.Txy, -m.Tyy}};
    double M[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int c = 0; c < 3; ++c) M[r][c] = Am[c][r] - (r == c ? fr.eps : 0.0) + l[r] * u[c];
    }
    const double zeta = u[0] * lU0 + u[1] * lUx + u[2] * lUy;
    const double rhs[3] = {lU0 - zeta * l[0], lUx - zeta * l[1], lUy - zeta * l[2]};
    // cofactors C[i][j] of M; M^{-1}[i][j] = C[j][i] / det
    const double C00 = M[1][1] * M[2][2] - M[1][2] * M[2][1];
    const double C01 = M[1][2] * M[2][0] - M[1][0] * M[2][2];
    const double C02 = M[1][0] * M[2][1] - M[1][1] * M[2][0];
    const double C10 = M[0][2] * M[2][1] - M[0][1] * M[2][2];
    const double C11 = M[0][0] * M[2][2] - M[0][2] * M[2][0];
    const double C12 = M[0][1] * M[2][0] - M[0][0] * M[2][1];
    const double C20 = M[0][1] * M[1][2] - M[0][2] * M[1][1];
    const double C21 = M[0][2] * M[1][0] - M[0][0] * M[1][2];
    const double C22 = M[0][0] * M[1][1] - M[0][1] * M[1][0];
    const double idet = 1.0 / (M[0][0] * C00 + M[0][1] * C01 + M[0][2] * C02);
    const double z[3] = {(C00 * rhs[0] + C10 * rhs[1] + C20 * rhs[2]) * idet,
                         (C01 * rhs[0] + C11 * rhs[1] + C21 * rhs[2]) * idet,
                         (C02 * rhs[0] + C12 * rhs[1] + C22 * rhs[2]) * idet};
    const double s = leps + (z[0] * u[0] + z[1] * u[1] + z[2] * u[2]);
    // symmetric-matrix entries lambda_T^{mu nu}; off-diagonals counted twice
    lT00 += s * l[0] * l[0] - z[0] * l[0];
    lTxx += s * l[1] * l[1] - z[1] * l[1];
    lTyy += s * l[2] * l[2] - z[2] * l[2];
    lT0x += 2.0 * s * l[0] * l[1] - (z[0] * l[1] + z[1] * l[0]);
    lT0y += 2.0 * s * l[0] * l[2] - (z[0] * l[2] + z[2] * l[0]);
    lTxy += 2.0 * s * l[1] * l[2] - (z[1] * l[2] + z[2] * l[1]);
  }

  // moments -> populations
  const float a00 = (float)lT00, a0x = (float)lT0x, a0y = (float)lT0y;
  const float axx = (float)lTxx, axy = (float)lTxy, ayy = (float)lTyy;
  const float b0 = (float)lJ0, bx = (float)lJx, by = (float)lJy;
  static_for<0, Q>([&](auto P) {   // even part + / - odd part per pair
    constexpr int p = decltype(P)::value;
    constexpr int q = DS::opp[p];
    if constexpr (q == p) {
      put(p, mf[p] + a00);
      put(Q + p, mg[p] + b0);
    } else if constexpr (q > p) {
      constexpr double vx = DS::vx[p], vy = DS::vy[p], vz2 = DS::vz2[p];
      const float ev = a00 + (float)(vx * vx) * axx + (float)(vx * vy) * axy + (float)(vy * vy) * ayy;
      const float od = (float)vx * a0x + (float)vy * a0y + (float)(vx * vx * vx) * lq3xxx +
                       (float)(vx * vx * vy) * lq3xxy + (float)(vx * vy * vy) * lq3xyy +
                       (float)(vy * vy * vy) * lq3yyy + (float)(vx * vz2) * lq3xzz +
                       (float)(vy * vz2) * lq3yzz;
      const float odg = (float)vx * bx + (float)vy * by;
      put(p, mf[p] + (ev + od));
      put(q, mf[q] + (ev - od));
      put(Q + p, mg[p] + (b0 + odg));
      put(Q + q, mg[q] + (b0 - odg));
    }
  });
  // parameter adjoints of this node
  af.x += (double)lFx;
  af.y += (double)lFy;
  a.acc_f[node] = af;
  a.acc_itau[node] = at + (double)litau;
}

// The transposed bilinear pull alone, out = P^T mu: the pull of the
// adjoint kernel (same weights taken at x + delta) without the local
// reverse sweep, for checking <P^T mu, v> = <mu, P v>.
template <class DS, bool UNIT>
__global__ __launch_bounds__(256) void transpose_pull_kernel(const float* __restrict__ mu,
                                                             float* __restrict__ out, int nx,
                                                             int ny, int row, int tiles_x,
                                                             int ntiles, const StepShared sh) {
  constexpr int Q = DS::Q;
  const int tile = blockIdx.x;
  if (tile >= ntiles) return;
  const int ty = tile / tiles_x;
  const int x = (tile - ty * tiles_x) * 64 + (threadIdx.x & 63);
  const int y = ty * 4 + (threadIdx.x >> 6);
  if (x >= nx || y >= ny) return;
  const Nbr nb = neighbourhood<Q>(x, y, nx, ny, row);
  char* o = (char*)out + nb.r[1] + nb.c[1];
  static_for<0, Q>([&](auto P) {
    constexpr int p = decltype(P)::value;
    *(float*)(o + p * 256) = pull<DS, UNIT, p, p, true>(mu, nb, sh.tap[p]);
    *(float*)(o + (Q + p) * 256) = pull<DS, UNIT, p, Q + p, true>(mu, nb, sh.tap[p]);
  });
}

// Objective density summed over fluid nodes, added to a per-block running
// sum (fixed grid and order: deterministic).
template <class DS, bool UNIT, bool MASK>
__global__ __launch_bounds__(256) void objective_kernel(const ObjArgs a) {
  constexpr int Q = DS::Q;
  const int ncell = a.nx * a.ny;
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ncell; i += gridDim.x * blockDim.x) {
    const int y = i / a.nx, x = i - y * a.nx;
    if constexpr (MASK) {
      if (a.mask[i]) continue;
    }
    const Nbr nb = neighbourhood<Q>(x, y, a.nx, a.ny, a.row);
    float f[Q], g[Q];
    static_for<0, Q>([&](auto P) {
      constexpr int p = decltype(P)::value;
      f[p] = pull<DS, UNIT, p, p, false>(a.state, nb, a.sh.tap[p]);
      g[p] = pull<DS, UNIT, p, Q + p, false>(a.state, nb, a.sh.tap[p]);
    });
    const Moments m = moments_of<DS>(f, g, a.sh.eps_ref, a.sh.n_ref);
    if (a.kind == 2) {
      acc += 1.0;   // fluid-node count
    } else if (a.kind == 0) {
      acc += m.Jx;
    } else {
      Frame fr{0.0, 1.0, 0.0, 0.0};
      if (landau3(m.T00, m.T0x, m.T0y, m.Txx, m.Txy, m.Tyy, fr)) {
        const Pi q = pi_of(m, fr);
        acc += q.xx * q.xx + q.yy * q.yy + 2.0 * q.xy * q.xy + q.zz * q.zz;
      } else {
        atomicOr(a.sh.err, ERR_LANDAU);
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) a.acc[blockIdx.x] += (red[0] + red[1]) + (red[2] + red[3]);
}

// Static stirring-basis force planes: F_c(x) = sum_m A_m e_mc cos(theta_m),
// theta_m = 2 pi (kx x / nx + ky y / ny) + phase_m, angle reduced exactly.
__global__ __launch_bounds__(256) void basis_force_kernel(const double* __restrict__ modes,
                                                          const double* __restrict__ amps,
                                                          int M, int nx, int ny, int row,
                                                          int64_t pitch, float* force) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nx * ny) return;
  const int y = i / nx, x = i - y * nx;
  double fx = 0.0, fy = 0.0;
  const long long NN = (long long)nx * ny;
  for (int k = 0; k < M; ++k) {
    const long long kx = (long long)modes[5 * k], ky = (long long)modes[5 * k + 1];
    long long num = (kx * x * ny + ky * y * nx) % NN;
    if (num < 0) num += NN;
    const double th = 6.283185307179586477 * ((double)num / (double)NN) + modes[5 * k + 4];
    const double c = cos(th);
    fx += amps[k] * modes[5 * k + 2] * c;
    fy += amps[k] * modes[5 * k + 3] * c;
  }
  force[(size_t)y * row + x] = (float)fx;
  force[pitch + (size_t)y * row + x] = (float)fy;
}

// Gradient reduction: row r = 0 (body force: sum of dJ/dF^x), 1 (tau:
// -sum dJ/d(1/tau) / tau^2), 2 + m (basis amplitude m: sum of dJ/dF . phi_m).
__global__ __launch_bounds__(256) void grad_reduce_kernel(const double2* __restrict__ acc_f,
                                                          const double* __restrict__ acc_itau,
                                                          const double* __restrict__ modes,
                                                          int nx, int ny, double tau,
                                                          double* partial) {
  const int r = blockIdx.y;
  const int ncell = nx * ny;
  const long long NN = (long long)ncell;
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ncell; i += gridDim.x * blockDim.x) {
    if (r == 0) {
      acc += acc_f[i].x;
    } else if (r == 1) {
      acc += acc_itau[i];
    } else {
      const int k = r - 2;
      const int y = i / nx, x = i - y * nx;
      const long long kx = (long long)modes[5 * k], ky = (long long)modes[5 * k + 1];
      long long num = (kx * x * ny + ky * y * nx) % NN;
      if (num < 0) num += NN;
      const double c = cos(6.283185307179586477 * ((double)num / (double)NN) + modes[5 * k + 4]);
      const double2 v = acc_f[i];
      acc += (v.x * modes[5 * k + 2] + v.y * modes[5 * k + 3]) * c;
    }
  }
  if (r == 1) acc *= -1.0 / (tau * tau);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[(size_t)r * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void sum_rows_kernel(const double* __restrict__ partial,
                                                       int cols, int rows, double scale,
                                                       double* out) {
  const int r = blockIdx.x;
  if (r >= rows) return;
  double acc = 0.0;
  for (int c = threadIdx.x; c < cols; c += blockDim.x) acc += partial[(size_t)r * cols + c];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[r] = scale * ((red[0] + red[1]) + (red[2] + red[3]));
}

__global__ __launch_bounds__(256) void fill_f64_kernel(double* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
template <class DS, bool UNIT, bool MU>
static void adj_go_mu(bool mask, const AdjArgs& a, hipStream_t s) {
  const dim3 grid(8 * a.tiles_per_xcd);
  if (mask)
    hipLaunchKernelGGL((adjoint_kernel<DS, UNIT, true, MU>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((adjoint_kernel<DS, UNIT, false, MU>), grid, dim3(256), 0, s, a);
}

template <class DS, bool UNIT>
static void adj_go(bool mask, const AdjArgs& a, hipStream_t s) {
  if (a.mu_in) adj_go_mu<DS, UNIT, true>(mask, a, s);
  else adj_go_mu<DS, UNIT, false>(mask, a, s);
}

hipError_t launch_adjoint(int Q, bool unit, bool mask, const AdjArgs& a, hipStream_t s) {
  if (Q == 17) {
    if (unit) adj_go<Dir17, true>(mask, a, s); else adj_go<Dir17, false>(mask, a, s);
  } else {
    if (unit) adj_go<Dir26, true>(mask, a, s); else adj_go<Dir26, false>(mask, a, s);
  }
  return hipGetLastError();
}

template <class DS, bool UNIT>
static void tpull_go(const float* mu, float* out, int nx, int ny, int row, const StepShared& sh,
                     hipStream_t s) {
  const int tiles_x = (nx + 63) / 64, ntiles = tiles_x * ((ny + 3) / 4);
  hipLaunchKernelGGL((transpose_pull_kernel<DS, UNIT>), dim3(ntiles), dim3(256), 0, s, mu, out, nx,
                     ny, row, tiles_x, ntiles, sh);
}

hipError_t launch_transpose_pull(int Q, bool unit, const float* mu, float* out, int nx, int ny,
                                 int row, const StepShared& sh, hipStream_t s) {
  if (Q == 17) {
    if (unit) tpull_go<Dir17, true>(mu, out, nx, ny, row, sh, s);
    else tpull_go<Dir17, false>(mu, out, nx, ny, row, sh, s);
  } else {
    if (unit) tpull_go<Dir26, true>(mu, out, nx, ny, row, sh, s);
    else tpull_go<Dir26, false>(mu, out, nx, ny, row, sh, s);
  }
  return hipGetLastError();
}

template <class DS, bool UNIT>
static void obj_go(bool mask, const ObjArgs& a, int grid, hipStream_t s) {
  if (mask)
    hipLaunchKernelGGL((objective_kernel<DS, UNIT, true>), dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((objective_kernel<DS, UNIT, false>), dim3(grid), dim3(256), 0, s, a);
}

hipError_t launch_objective(int Q, bool unit, bool mask, const ObjArgs& a, int grid, hipStream_t s) {
  if (Q == 17) {
    if (unit) obj_go<Dir17, true>(mask, a, grid, s); else obj_go<Dir17, false>(mask, a, grid, s);
  } else {
    if (unit) obj_go<Dir26, true>(mask, a, grid, s); else obj_go<Dir26, false>(mask, a, grid, s);
  }
  return hipGetLastError();
}

hipError_t launch_basis_force(const double* modes, const double* amps, int M, int nx, int ny,
                              int row, int64_t pitch, float* force, hipStream_t s) {
  hipLaunchKernelGGL(basis_force_kernel, dim3((nx * ny + 255) / 256), dim3(256), 0, s, modes, amps,
                     M, nx, ny, row, pitch, force);
  return hipGetLastError();
}

hipError_t launch_grad_reduce(const double2* acc_f, const double* acc_itau, const double* modes,
                              int M, int nx, int ny, double tau, double* partial, int cols,
                              double* out, hipStream_t s) {
  hipLaunchKernelGGL(grad_reduce_kernel, dim3(cols, 2 + M), dim3(256), 0, s, acc_f, acc_itau,
                     modes, nx, ny, tau, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_rows_kernel, dim3(2 + M), dim3(256), 0, s, partial, cols, 2 + M, 1.0, out);
  return hipGetLastError();
}

hipError_t launch_sum_rows(const double* partial, int cols, int rows, double scale, double* out,
                           hipStream_t s) {
  hipLaunchKernelGGL(sum_rows_kernel, dim3(rows), dim3(256), 0, s, partial, cols, rows, scale, out);
  return hipGetLastError();
}

hipError_t launch_zero_f64(double* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace rlb
