// The fused step kernel and its launch dispatch, shared by step.hip (the
// instantiations with non-temporal population stores) and step_cached.hip
// (plain stores).  The store kind is a template parameter: a launch whose
// two state copies fit the last-level cache (256 MB) takes the plain
// stores, so that the next step reads the new state from that cache
// (1024 x 256: 19.0 -> 13.8 us, 1536 x 512: 45.6 -> 33.7 us); a larger one
// takes the non-temporal stores, which keep the cache for the rows a pull
// reads (4096^2: 800 -> 831 us with plain stores).
#pragma once

#include "internal.hpp"
#include "device_common.hpp"
#include "dirset.hpp"
#include "brick.hpp"

namespace rlb {

// The plain-store launch (step_cached.hip): arguments as launch_tiles after
// the tile height and grid are fixed.
hipError_t launch_tiles_cached(int Q, int sm, bool mask, int mode, int force_mode,
                               const TileArgs& a, int ty, int grid, hipStream_t s);

// Open x borders of the new state, set by the waves that hold them (Ch. 5,
// "Model and Methods": a fixed velocity enters along the inflow border):
//   * velocity inlet, column 0: equilibrium at the prescribed 3-velocity and
//     charge density, with the energy density of column 1;
//   * pressure outlet, column nx-1: equilibrium at the prescribed energy
//     density, with the velocity and charge density of column nx-2.
// The adjacent column's frame comes from Landau matching of the moments of
// its new (post-collision) populations `fo`, `go`, which the neighbouring
// lane has just stored; the border lane then overwrites its own store.
// Moments in float32 in plane order, references added in float64.  Needs
// columns nx-2 and nx-1 in one 64-node tile (nx % 64 != 1; otherwise the
// borders are set by a kernel of their own after the step).
template <class DS, bool NT>
__device__ __forceinline__ void open_borders(const StepShared& a, int x, int nx,
                                             const float (&fo)[DS::Q], const float (&go)[DS::Q],
                                             float* __restrict__ dst, int64_t rs, uint32_t cs) {
  constexpr int Q = DS::Q;
  const int base = x & ~63;
  if (base != 0 && base + 63 < nx - 1) return;   // tile holds neither border (wave-uniform)
  float m00 = 0, m0x = 0, m0y = 0, mxx = 0, mxy = 0, myy = 0, j0 = 0, jx = 0, jy = 0;
  static_for<0, Q>([&](auto P) {
    constexpr int p = decltype(P)::value;
    constexpr double vx = DS::vx[p], vy = DS::vy[p];
    m00 += fo[p];
    j0 += go[p];
    if constexpr (vx != 0.0) { m0x += (float)vx * fo[p]; jx += (float)vx * go[p]; mxx += (float)(vx * vx) * fo[p]; }
    if constexpr (vy != 0.0) { m0y += (float)vy * fo[p]; jy += (float)vy * go[p]; myy += (float)(vy * vy) * fo[p]; }
    if constexpr (vx != 0.0 && vy != 0.0) mxy += (float)(vx * vy) * fo[p];
  });
  // border lanes take the moments of the adjacent column's lane
  const int lane = x & 63;
  const int from = x == 0 ? 1 : (lane > 0 ? lane - 1 : 0);
  m00 = __shfl(m00, from, 64); m0x = __shfl(m0x, from, 64); m0y = __shfl(m0y, from, 64);
  mxx = __shfl(mxx, from, 64); mxy = __shfl(mxy, from, 64); myy = __shfl(myy, from, 64);
  j0 = __shfl(j0, from, 64); jx = __shfl(jx, from, 64); jy = __shfl(jy, from, 64);
  if (x != 0 && x != nx - 1) return;
  const double T00 = a.eps_ref + (double)m00;
  const double Txx = a.eps_ref * (1.0 / 3.0) + (double)mxx;
  const double Tyy = a.eps_ref * (1.0 / 3.0) + (double)myy;
  Frame fr{a.eps_ref, 1.0, 0.0, 0.0};
  if (!landau3(T00, (double)m0x, (double)m0y, Txx, (double)mxy, Tyy, fr)) {
    atomicOr(a.err, ERR_LANDAU);
    fr = Frame{a.eps_ref, 1.0, 0.0, 0.0};
  }
  Frame b;
  double n;
  if (x == 0) {
    frame_from_beta(fr.eps, a.o_bx, a.o_by, b);   // |beta| < 1 checked on the host
    n = a.o_n;
  } else {
    b = Frame{a.o_eps, fr.u0, fr.ux, fr.uy};
    n = fr.u0 * (a.n_ref + (double)j0) - fr.ux * (double)jx - fr.uy * (double)jy;
  }
  const EqCoef ec = eq_coef(b, n, a.eps_ref, a.n_ref, DS::kappa);
  const float ux = (float)b.ux, uy = (float)b.uy;
  static_for<0, Q>([&](auto P) {
    constexpr int p = decltype(P)::value;
    constexpr float vx = (float)DS::vx[p], vy = (float)DS::vy[p];
    constexpr float w = DS::w32[p];
    const float s = ux * vx + uy * vy;
    stp<p, NT>(dst, rs, cs, w * (ec.A + s * (ec.B + s * ec.C)));
    stp<Q + p, NT>(dst, rs, cs, w * (ec.Ag + s * ec.Bg));
  });
}

// Kernels whose waves raise their issue priority while they issue the pulls
// (measured): the folded two-cell (cfl > 1) step at 4096^2 (+3%), the
// open-channel steps (1024x256 channel +5..9%, six-channel batch +1%), and
// the masked, stirred steps of the adjoint (forward 11.6k -> 13.0k MLUPS,
// its objective steps included).  The cfl <= 1 step at 4096^2 loses 5%
// with it and the masked batched step with a body force 0.7%.  Measured
// with the non-temporal stores; with the plain stores of the small
// lattices the raised priority costs (1024x256 channel 16.65 -> 17.05 us,
// the adjoint's 512x256 forward 13.1k -> 12.3k MLUPS), so only the
// non-temporal form raises it.
template <class DS, int SM, bool MASK, int FORCE, int MODE>
constexpr bool kLoadPriority =
    (MODE == MODE_STEP && SM == SM_WIDE && DS::Q == 17) || MODE == MODE_OPEN ||
    MODE == MODE_OBJ || (MODE == MODE_STEP && MASK && FORCE == FORCE_STIR);

template <class DS, int SM, bool MASK, int FORCE, int MODE, bool NT, class Desc>
__device__ __forceinline__ void node_update(const StepShared& sh, Desc& L,
                                            const float* __restrict__ src,
                                            float* __restrict__ dst,
                                            float* __restrict__ fields, int x, int y,
                                            double& obj) {
  constexpr int Q = DS::Q;
  const int nx = L.nx, ny = L.ny;
  const int row = L.row;   // nx rounded up to 64
  Nbr nb;
  Nbr5 nb5;
  if constexpr (SM == SM_WIDE) nb5 = neighbourhood5<Q>(x, y, nx, ny, row);
  else nb = neighbourhood<Q>(x, y, nx, ny, row);
  const int64_t rs = SM == SM_WIDE ? nb5.r[2] : nb.r[1];   // the node's own row and column
  const uint32_t cs = SM == SM_WIDE ? nb5.c[2] : nb.c[1];
  const uint32_t node = (uint32_t)(y * nx + x);   // dense index (mask, fields)
  const StepShared& a = sh;

  // 1. pull-stream every plane (at raised issue priority where that helps)
  if constexpr (NT && kLoadPriority<DS, SM, MASK, FORCE, MODE>) __builtin_amdgcn_s_setprio(2);
  float f[Q], g[Q];
  static_for<0, Q>([&](auto P) {
    constexpr int p = decltype(P)::value;
    if constexpr (SM == SM_WIDE) {
      f[p] = pull_wide<DS, p, p>(src, nb5, a.tap[p], a.shift[p]);
      g[p] = pull_wide<DS, p, Q + p>(src, nb5, a.tap[p], a.shift[p]);
    } else {
      f[p] = pull<DS, SM == SM_UNIT, p, p, false>(src, nb, a.tap[p]);
      g[p] = pull<DS, SM == SM_UNIT, p, Q + p, false>(src, nb, a.tap[p]);
    }
  });

  float Fsx = 0.0f, Fsy = 0.0f;   // stirring force, loaded with the populations
  if constexpr (FORCE == FORCE_STIR && MODE != MODE_FIELDS) {
    const gfloat* fr = (const gfloat*)L.force + (int64_t)y * row;
    Fsx = __builtin_nontemporal_load(&fr[x]);   // read once: keep L2 for the state rows
    Fsy = __builtin_nontemporal_load(&fr[L.pitch + x]);
  }
  if constexpr (NT && kLoadPriority<DS, SM, MASK, FORCE, MODE>) __builtin_amdgcn_s_setprio(0);
  // Solid nodes bounce back (F'_i = F~_opp(i)).  They run the same
  // arithmetic on a rest-frame stand-in and select at the store, so a
  // wavefront that straddles an obstacle does not diverge.
  bool solid = false;
  if constexpr (MASK) solid = ((const __attribute__((address_space(1))) uint8_t*)L.mask)[node] != 0;

  // 2. moments of the deviations from the reference: float32 sums over
  //    opposite pairs (even moments from f_a + f_b, odd from f_a - f_b),
  //    then the reference added in float64
  float m00 = 0, m0x = 0, m0y = 0, mxx = 0, mxy = 0, myy = 0;
  float j0 = 0, jx = 0, jy = 0;
  float df[Q];   // f_a - f_b of each pair head a (odd parts), reused by the force
  static_for<0, Q>([&](auto P) {
    constexpr int p = decltype(P)::value;
    constexpr int q = DS::opp[p];
    if constexpr (q == p) {
      m00 += f[p];
      j0 += g[p];
    } else if constexpr (q > p) {
      constexpr double vx = DS::vx[p], vy = DS::vy[p];
      const float sf = f[p] + f[q], sg = g[p] + g[q];
      df[p] = f[p] - f[q];
      const float dg = g[p] - g[q];
      m00 += sf;
      j0 += sg;
      if constexpr (vx != 0.0) {
        m0x += (float)vx * df[p]; jx += (float)vx * dg; mxx += (float)(vx * vx) * sf;
      }
      if constexpr (vy != 0.0) {
        m0y += (float)vy * df[p]; jy += (float)vy * dg; myy += (float)(vy * vy) * sf;
      }
      if constexpr (vx != 0.0 && vy != 0.0) mxy += (float)(vx * vy) * sf;
    }
  });
  double T00 = a.eps_ref + (double)m00;
  double T0x = (double)m0x, T0y = (double)m0y;
  double Txx = a.eps_ref * DS::cs2 + (double)mxx;
  double Tyy = a.eps_ref * DS::cs2 + (double)myy;
  double Txy = (double)mxy;
  double J0 = a.n_ref + (double)j0, Jx = (double)jx, Jy = (double)jy;
  // every streamed population enters m00 or j0, so both are finite unless
  // a population is not (solid nodes included: the test precedes their
  // rest-frame stand-in)
  const bool finite = __builtin_isfinite(m00 + j0);
  if constexpr (MASK) {
    if (solid) {
      T00 = a.eps_ref; T0x = 0.0; T0y = 0.0;
      Txx = a.eps_ref * DS::cs2; Tyy = Txx; Txy = 0.0;
      J0 = a.n_ref; Jx = 0.0; Jy = 0.0;
    }
  }
  // the current density of one column, recorded row by row (solid: zero);
  // compiled into the open-channel kernels and the full set's kernels only.
  // The branch splits the kernel's scheduling regions: measured at 4096^2,
  // that costs the folded set's step 8% and saves the full set's 6%
  if constexpr (MODE == MODE_OPEN) {
    if (a.rec != nullptr && x == (a.rec_x < 0 ? a.rec_x + L.nx : a.rec_x)) a.rec[L.rec_row + y] = Jx;
  } else if constexpr (DS::Q == 26 && MODE != MODE_FIELDS) {
    if (a.rec != nullptr && x == a.rec_x) a.rec[y] = Jx;
  }

  // 3. Landau frame and charge density
  Frame fr{0.0, 1.0, 0.0, 0.0};
  bool ok = landau3<DS::planar>(T00, T0x, T0y, Txx, Txy, Tyy, fr);
  const double n = fr.u0 * J0 - fr.ux * Jx - fr.uy * Jy;
  ok = ok && (n == n) && finite;

  // objective density of the streamed state (fluid nodes): the charge
  // current J^x, or pi:pi with pi = T^{kl} - T_eq^{kl} (spatial block)
  if constexpr (MODE == MODE_OBJ) {
    if (!solid && ok) {
      if (a.obj_kind == 0) {
        obj = Jx;
      } else {
        const double e43 = (4.0 / 3.0) * fr.eps, e3 = fr.eps / 3.0;
        const double pxx = Txx - (e43 * fr.ux * fr.ux + e3);
        const double pyy = Tyy - (e43 * fr.uy * fr.uy + e3);
        const double pxy = Txy - e43 * fr.ux * fr.uy;
        const double pzz = (T00 - Txx - Tyy) - e3;
        obj = pxx * pxx + pyy * pyy + 2.0 * pxy * pxy + pzz * pzz;
      }
    }
  }

  if constexpr (MODE == MODE_FIELDS) {
    const double vals[RLB_FIELD_COUNT] = {
        fr.eps, fr.ux / fr.u0, fr.uy / fr.u0, n, T00, T0x, T0y,
        Txx, Txy, Tyy, J0, Jx, Jy};
    if (!ok && (!solid || !finite)) atomicOr(a.err, finite ? ERR_LANDAU : ERR_NONFINITE);
    int k = 0;
    const size_t plane = (size_t)nx * ny;
#pragma unroll
    for (int fld = 0; fld < RLB_FIELD_COUNT; ++fld) {
      if (a.field_mask & (1u << fld)) {
        fields[k * plane + node] = (solid || !ok) ? 0.0f : (float)vals[fld];
        ++k;
      }
    }
    return;
  } else {
    float fo[Q], go[Q];   // the stored values (open borders only)
    if (!ok) {   // no rest frame, or a non-finite population: flag it and
                 // leave the node uncollided
      atomicOr(a.err, finite ? ERR_LANDAU : ERR_NONFINITE);
      static_for<0, Q>([&](auto P) {
        constexpr int p = decltype(P)::value;
        stp<p, NT>(dst, rs, cs, f[p]);
        stp<Q + p, NT>(dst, rs, cs, g[p]);
        if constexpr (MODE == MODE_OPEN) {
          fo[p] = f[p];
          go[p] = g[p];
        }
      });
    } else {
      // 4. equilibrium and collision-rate coefficients
      const EqCoef ec = eq_coef<DS::planar>(fr, n, a.eps_ref, a.n_ref, DS::kappa);
      const float ux = (float)fr.ux, uy = (float)fr.uy;
      // 1/tau: constant, or from eta/s at the node's temperature,
      // T ~ eps^(1/4) (tau_R = 5 (eta/s) / T with eps = 3 T^4 / pi^2); the
      // fourth root in float32 with the hardware square root (1 ulp): the
      // constant-tau path then pays a dozen instructions, not two float64
      // square roots
      const float itau = a.tau_k > 0.0
          ? (float)a.tau_k * __builtin_amdgcn_sqrtf(__builtin_amdgcn_sqrtf((float)fr.eps))
          : a.inv_tau;
      const float w0 = (float)fr.u0 * itau;

      // 5. driving term Phi(v) = p0 + px vx + py vy + pxx vx^2 + pxy vx vy
      //    + pyy vy^2 (vz^2 = 1 - vx^2 - vy^2 folded in)
      float p0 = 0, px = 0, py = 0, pxx = 0, pxy = 0, pyy = 0;
      if constexpr (FORCE != FORCE_NONE) {
        float Fx = a.fx, Fy = a.fy;
        if constexpr (FORCE == FORCE_STIR) {
          Fx += Fsx;
          Fy += Fsy;
        }
        float q3xxx = 0, q3xxy = 0, q3xyy = 0, q3yyy = 0, q3xzz = 0, q3yzz = 0;
        static_for<0, Q>([&](auto P) {
          constexpr int p = decltype(P)::value;
          if constexpr (DS::opp[p] > p) {   // third moments are odd
            constexpr double vx = DS::vx[p], vy = DS::vy[p], vz2 = DS::vz2[p];
            if constexpr (vx != 0.0) {
              q3xxx += (float)(vx * vx * vx) * df[p];
              if constexpr (vz2 != 0.0) q3xzz += (float)(vx * vz2) * df[p];
            }
            if constexpr (vy != 0.0) {
              q3yyy += (float)(vy * vy * vy) * df[p];
              if constexpr (vz2 != 0.0) q3yzz += (float)(vy * vz2) * df[p];
            }
            if constexpr (vx != 0.0 && vy != 0.0) {
              q3xxy += (float)(vx * vx * vy) * df[p];
              q3xyy += (float)(vx * vy * vy) * df[p];
            }
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

      // 6. relax and drive, per opposite pair (a, b) with v_b = -v_a: the
      //    equilibrium, rate and driving term split into even and odd parts
      //    in s = u.v_a
      static_for<0, Q>([&](auto P) {
        constexpr int p = decltype(P)::value;
        constexpr int q = DS::opp[p];
        constexpr float w = DS::w32[p];
        if constexpr (q == p) {
          const float fn = f[p] - w0 * (f[p] - w * ec.A) - w * p0;
          const float gn = g[p] - w0 * (g[p] - w * ec.Ag);
          stp<p, NT>(dst, rs, cs, solid ? f[p] : fn);
          stp<Q + p, NT>(dst, rs, cs, solid ? g[p] : gn);
          if constexpr (MODE == MODE_OPEN) {
            fo[p] = solid ? f[p] : fn;
            go[p] = solid ? g[p] : gn;
          }
        } else if constexpr (q > p) {
          constexpr float vx = (float)DS::vx[p], vy = (float)DS::vy[p];
          constexpr float vxx = (float)(DS::vx[p] * DS::vx[p]);
          constexpr float vyy = (float)(DS::vy[p] * DS::vy[p]);
          constexpr float vxy = (float)(DS::vx[p] * DS::vy[p]);
          const float s = ux * vx + uy * vy;
          const float t = s * itau;
          const float e0 = w * (ec.A + ec.C * s * s), e1 = w * (ec.B * s);
          const float g0 = w * ec.Ag, g1 = w * (ec.Bg * s);
          const float oa = w0 - t, ob = w0 + t;
          float fa = f[p] - oa * (f[p] - (e0 + e1));
          float fb = f[q] - ob * (f[q] - (e0 - e1));
          if constexpr (FORCE != FORCE_NONE) {
            const float pe = w * (p0 + vxx * pxx + vxy * pxy + vyy * pyy);
            const float po = w * (vx * px + vy * py);
            fa -= pe + po;
            fb -= pe - po;
          }
          const float ga = g[p] - oa * (g[p] - (g0 + g1));
          const float gb = g[q] - ob * (g[q] - (g0 - g1));
          stp<p, NT>(dst, rs, cs, solid ? f[q] : fa);
          stp<q, NT>(dst, rs, cs, solid ? f[p] : fb);
          stp<Q + p, NT>(dst, rs, cs, solid ? g[q] : ga);
          stp<Q + q, NT>(dst, rs, cs, solid ? g[p] : gb);
          if constexpr (MODE == MODE_OPEN) {
            fo[p] = solid ? f[q] : fa;
            fo[q] = solid ? f[p] : fb;
            go[p] = solid ? g[q] : ga;
            go[q] = solid ? g[p] : gb;
          }
        }
      });
    }
    if constexpr (MODE == MODE_OPEN) open_borders<DS, NT>(a, x, nx, fo, go, dst, rs, cs);
  }
}

// The full set's kernels are held to 3 waves per SIMD (<= 168 VGPRs): left
// alone the compiler takes ~200 registers and 2 waves, measured 4% slower
// at 4096^2.
template <class DS, int SM, bool MASK, int FORCE, int MODE, int TY, bool NT>
__global__ __launch_bounds__(64 * TY, DS::Q == 26 ? 3 : 1) void tile_kernel(const TileArgs a) {
  const int xcd = blockIdx.x & 7;
  const int per = gridDim.x >> 3;
  const int lo = xcd * a.tiles_per_xcd;
  const int hi = min(lo + a.tiles_per_xcd, a.ntiles);
  const int lane = threadIdx.x & 63;
  const int row = threadIdx.x >> 6;
  for (int t = lo + (int)(blockIdx.x >> 3); t < hi; t += per) {
    const int tile = a.tile_first + t;
    // the tile's lattice and its descriptor are wave-uniform and read-only
    // here: read through the constant address space (scalar loads, which
    // never wait on the vector-memory counter the pulls are counted on)
    typedef const __attribute__((address_space(4))) int32_t CI32;
    typedef const __attribute__((address_space(4))) LatDesc CDesc;
    const int b = a.tile_lat ? ((CI32*)a.tile_lat)[tile] : 0;
    CDesc& L = ((CDesc*)a.lats)[b];
    // tiles of a lattice run strip by strip (strips a.strip tiles wide,
    // the last one narrower), row-major inside a strip: neighbouring tiles,
    // which share halo rows and columns, are dispatched close together
    int lt = tile - L.tile_begin;
    const int tiles_y = (L.ny + TY - 1) / TY;
    const int sw = min(a.strip, L.tiles_x);
    if constexpr (MODE == MODE_OPEN) {
      // the border tiles (columns 0 and nx-1: a second Landau solve and
      // the border stores) go first within this XCD's share, so that
      // their extra work overlaps the interior tiles that start after
      // them instead of finishing last (1024 x 256 channel 16.9 -> 14.5
      // us).  Applied to a single lattice whose strip spans its width and
      // whose XCD shares are whole tile rows; otherwise the plain order.
      // Each node's arithmetic is the same in either order
      const int tx = L.tiles_x, n = hi - lo;
      if (a.tile_lat == nullptr && sw == tx && tx > 2 && lo % tx == 0 && n % tx == 0) {
        const int k = t - lo, r0 = lo / tx, nr = n / tx;
        int r, c;
        if (k < 2 * nr) {
          r = r0 + (k >> 1);
          c = (k & 1) ? tx - 1 : 0;
        } else {
          const int k2 = k - 2 * nr;
          r = r0 + k2 / (tx - 2);
          c = 1 + k2 % (tx - 2);
        }
        lt = r * tx + c;
      }
    }
    const int full = L.tiles_x / sw;
    const int st = lt / (sw * tiles_y);
    const int w = st < full ? sw : L.tiles_x - full * sw;
    const int in = lt - st * sw * tiles_y;
    const int ty = in / w;
    const int x = (st * sw + (in - ty * w)) * 64 + lane;
    const int y = __builtin_amdgcn_readfirstlane(ty * TY + row);
    double obj = 0.0;
    if (x < L.nx && y < L.ny)
      node_update<DS, SM, MASK, FORCE, MODE, NT>(a.sh, L, L.state[a.parity],
                                               const_cast<float*>(L.state[a.parity ^ 1]),
                                               a.fields, x, y, obj);
    if constexpr (MODE == MODE_OBJ) {
      if (y < L.ny) {   // wave-uniform; every lane takes part (0 past nx)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) obj += __shfl_xor(obj, o, 64);
        if (lane == 0) a.sh.obj[(size_t)y * L.tiles_x + (x >> 6)] += obj;
      }
    }
  }
}

template <class DS, int SM, bool MASK, int FORCE, int MODE, int TY, bool NT>
static void go(const TileArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((tile_kernel<DS, SM, MASK, FORCE, MODE, TY, NT>), dim3(grid),
                     dim3(64 * TY), 0, s, a);
}

// Tile heights other than 4 are compiled for the folded set's step kernels
// and the full set's plain step (2-row tiles: 1.308 -> 1.276 ms at 4096^2
// stirred; 1 and 8 rows no faster than 4); everything else uses 4.  `ty`
// comes from kernel_tile_rows, which the tile counts use too.
template <class DS, int SM, bool MASK, int FORCE, int MODE, bool NT>
static void by_rows(int ty, const TileArgs& a, int grid, hipStream_t s) {
  if constexpr (DS::Q == 17 && MODE != MODE_FIELDS) {
    switch (ty) {
      case 1: go<DS, SM, MASK, FORCE, MODE, 1, NT>(a, grid, s); return;
      case 2: go<DS, SM, MASK, FORCE, MODE, 2, NT>(a, grid, s); return;
      case 8: go<DS, SM, MASK, FORCE, MODE, 8, NT>(a, grid, s); return;
      default: break;
    }
  } else if constexpr (DS::Q == 26 && MODE == MODE_STEP) {
    if (ty == 2) {
      go<DS, SM, MASK, FORCE, MODE, 2, NT>(a, grid, s);
      return;
    }
  }
  go<DS, SM, MASK, FORCE, MODE, 4, NT>(a, grid, s);
}

template <class DS, int SM, bool MASK, bool NT>
static void by_force(int mode, int force, int ty, const TileArgs& a, int grid, hipStream_t s) {
  if (mode == MODE_FIELDS) {   // stores no populations: one instantiation
    if constexpr (NT) by_rows<DS, SM, MASK, FORCE_NONE, MODE_FIELDS, true>(4, a, grid, s);
    return;
  }
  if (mode == MODE_OBJ) {   // the adjoint's forward: stirring-basis force, cfl <= 1, 3D set
    if constexpr (!DS::planar && SM != SM_WIDE) by_rows<DS, SM, MASK, FORCE_STIR, MODE_OBJ, NT>(ty, a, grid, s);
    return;
  }
  if (mode == MODE_OPEN) {   // open borders: not with the planar set or cfl > 1 (host checks)
    if constexpr (!DS::planar && SM != SM_WIDE) {
      if (force == FORCE_NONE) return by_rows<DS, SM, MASK, FORCE_NONE, MODE_OPEN, NT>(ty, a, grid, s);
      if (force == FORCE_BODY) return by_rows<DS, SM, MASK, FORCE_BODY, MODE_OPEN, NT>(ty, a, grid, s);
      by_rows<DS, SM, MASK, FORCE_STIR, MODE_OPEN, NT>(ty, a, grid, s);
    }
    return;
  }
  if (force == FORCE_NONE) return by_rows<DS, SM, MASK, FORCE_NONE, MODE_STEP, NT>(ty, a, grid, s);
  if constexpr (!DS::planar) {   // the planar set has no driving term (rejected on the host)
    if (force == FORCE_BODY) return by_rows<DS, SM, MASK, FORCE_BODY, MODE_STEP, NT>(ty, a, grid, s);
    by_rows<DS, SM, MASK, FORCE_STIR, MODE_STEP, NT>(ty, a, grid, s);
  }
}

template <class DS, bool NT>
static void by_flags(int sm, bool mask, int mode, int force, int ty, const TileArgs& a,
                     int grid, hipStream_t s) {
  if (sm == SM_UNIT) {
    if (mask) by_force<DS, SM_UNIT, true, NT>(mode, force, ty, a, grid, s);
    else by_force<DS, SM_UNIT, false, NT>(mode, force, ty, a, grid, s);
  } else if (sm == SM_WIDE) {
    if (mask) by_force<DS, SM_WIDE, true, NT>(mode, force, ty, a, grid, s);
    else by_force<DS, SM_WIDE, false, NT>(mode, force, ty, a, grid, s);
  } else {
    if (mask) by_force<DS, SM_GENERAL, true, NT>(mode, force, ty, a, grid, s);
    else by_force<DS, SM_GENERAL, false, NT>(mode, force, ty, a, grid, s);
  }
}

}  // namespace rlb
