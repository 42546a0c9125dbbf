// Momentum sets for the step kernels.
//
// The dissertation's spherical "D3Q27" set (Ch. 3 "Boltzmann to Lattice
// Boltzmann", Ch. 4 "Model and Methods") is read as the 26 unit cube
// directions (6 faces, 12 edges, 8 corners) with the degree-7 Lebedev
// weights 1/21, 4/105, 9/280; the zero-momentum slot carries nothing for
// massless particles.  The lattice has a single z node and neither the
// initial data nor the force has a z component, so the two members of each
// z-mirror pair (vx, vy, +vz) / (vx, vy, -vz) stream by the same in-plane
// displacement, see the same collision rate and equilibrium, and stay equal.
// Dir17 stores each pair as one plane holding the pair's sum (weight 2w);
// Dir26 stores every direction.  A kernel needs per plane only (vx, vy, vz^2,
// w, opposite plane).
//
// DirP12 is the planar (2+1) variant: 12 in-plane unit momenta at 30 degree
// spacing, equal weights, for massless particles confined to the plane
// (traceless T over t, x, y: P = eps/2, c_s^2 = 1/2 instead of 1/3).  Its
// equilibrium coefficients follow from the circle's orthogonal polynomials
// (see eq_coef); it has no driving term.  Each set states `planar` and
// cs2 = sum_i w_i vx_i^2 (the reference state's T^xx / T^00).
#pragma once

namespace rlb {

constexpr double kS2 = 0.70710678118654752440;   // 1/sqrt(2)
constexpr double kS3 = 0.57735026918962576451;   // 1/sqrt(3)
constexpr double kWf = 1.0 / 21.0;
constexpr double kWe = 4.0 / 105.0;
constexpr double kWc = 9.0 / 280.0;

// float32 weights for the shifted-storage arithmetic: multiples of 2^-28
// within 5e-9 of 1/21, 4/105, 9/280 chosen so that 6 wf + 12 we + 8 wc = 1
// exactly.  Float weights that do not sum to one would make the collision
// leak energy systematically (sum_i w_i A != A for the equilibrium's
// constant term).
constexpr float kWf32 = 12782642.0f / 268435456.0f;
constexpr float kWe32 = 10226113.0f / 268435456.0f;
constexpr float kWc32 = 8628281.0f / 268435456.0f;
static_assert(6.0 * 12782642 + 12.0 * 10226113 + 8.0 * 8628281 == 268435456.0,
              "float weights must sum to one");

// kappa = cs2 / sum_i w32_i vx_i^2 with the float32 weights and float32
// direction components the kernels use.  The equilibrium's first- and
// second-order coefficients are scaled by kappa so that, in the kernels'
// own float32 arithmetic, the equilibrium carries exactly the momentum of
// the Landau frame: otherwise the collision would change the momentum by
// (kappa - 1) ~ 2.5e-8 of itself every step.
constexpr double kappa_of(const float* w, const double* vx, int q, double cs2 = 1.0 / 3.0) {
  double s = 0.0;
  for (int i = 0; i < q; ++i) {
    const double v = (double)(float)vx[i];
    s += (double)w[i] * v * v;
  }
  return cs2 / s;
}

struct Dir17 {
  static constexpr int Q = 17;
  static constexpr double vx[Q] = {1, -1, 0, 0, kS2, -kS2, kS2, -kS2,
                                   0, kS2, -kS2, 0, 0, kS3, -kS3, kS3, -kS3};
  static constexpr double vy[Q] = {0, 0, 1, -1, kS2, kS2, -kS2, -kS2,
                                   0, 0, 0, kS2, -kS2, kS3, kS3, -kS3, -kS3};
  static constexpr double vz2[Q] = {0, 0, 0, 0, 0, 0, 0, 0,
                                    1, 0.5, 0.5, 0.5, 0.5,
                                    1.0 / 3, 1.0 / 3, 1.0 / 3, 1.0 / 3};
  static constexpr double w[Q] = {kWf, kWf, kWf, kWf, kWe, kWe, kWe, kWe,
                                  2 * kWf, 2 * kWe, 2 * kWe, 2 * kWe, 2 * kWe,
                                  2 * kWc, 2 * kWc, 2 * kWc, 2 * kWc};
  static constexpr float w32[Q] = {kWf32, kWf32, kWf32, kWf32, kWe32, kWe32, kWe32, kWe32,
                                   2 * kWf32, 2 * kWe32, 2 * kWe32, 2 * kWe32, 2 * kWe32,
                                   2 * kWc32, 2 * kWc32, 2 * kWc32, 2 * kWc32};
  static constexpr int opp[Q] = {1, 0, 3, 2, 7, 6, 5, 4,
                                 8, 10, 9, 12, 11, 16, 15, 14, 13};
  static constexpr double kappa = kappa_of(w32, vx, Q);
  static constexpr bool planar = false;
  static constexpr double cs2 = 1.0 / 3.0;
};

struct Dir26 {
  static constexpr int Q = 26;
  // in-plane (8), then vz = +1 group (9), then vz = -1 group (9)
  static constexpr double vx[Q] = {1, -1, 0, 0, kS2, -kS2, kS2, -kS2,
                                   0, kS2, -kS2, 0, 0, kS3, -kS3, kS3, -kS3,
                                   0, kS2, -kS2, 0, 0, kS3, -kS3, kS3, -kS3};
  static constexpr double vy[Q] = {0, 0, 1, -1, kS2, kS2, -kS2, -kS2,
                                   0, 0, 0, kS2, -kS2, kS3, kS3, -kS3, -kS3,
                                   0, 0, 0, kS2, -kS2, kS3, kS3, -kS3, -kS3};
  static constexpr double vz2[Q] = {0, 0, 0, 0, 0, 0, 0, 0,
                                    1, 0.5, 0.5, 0.5, 0.5,
                                    1.0 / 3, 1.0 / 3, 1.0 / 3, 1.0 / 3,
                                    1, 0.5, 0.5, 0.5, 0.5,
                                    1.0 / 3, 1.0 / 3, 1.0 / 3, 1.0 / 3};
  static constexpr double w[Q] = {kWf, kWf, kWf, kWf, kWe, kWe, kWe, kWe,
                                  kWf, kWe, kWe, kWe, kWe, kWc, kWc, kWc, kWc,
                                  kWf, kWe, kWe, kWe, kWe, kWc, kWc, kWc, kWc};
  static constexpr float w32[Q] = {kWf32, kWf32, kWf32, kWf32, kWe32, kWe32, kWe32, kWe32,
                                   kWf32, kWe32, kWe32, kWe32, kWe32, kWc32, kWc32, kWc32, kWc32,
                                   kWf32, kWe32, kWe32, kWe32, kWe32, kWc32, kWc32, kWc32, kWc32};
  // opposite of (vx, vy, +vz) is (-vx, -vy, -vz): in the other vz group
  static constexpr int opp[Q] = {1, 0, 3, 2, 7, 6, 5, 4,
                                 17, 19, 18, 21, 20, 25, 24, 23, 22,
                                 8, 10, 9, 12, 11, 16, 15, 14, 13};
  static constexpr double kappa = kappa_of(w32, vx, Q);
  static constexpr bool planar = false;
  static constexpr double cs2 = 1.0 / 3.0;
};

constexpr double kC30 = 0.86602540378443864676;   // cos 30 deg = sqrt(3)/2
// float32 weights of the planar set: multiples of 2^-28 next to 1/12 summing
// to one exactly (the four axis directions take the extra unit, which keeps
// the set symmetric under quarter turns and axis reflections)
constexpr float kWp32 = 22369621.0f / 268435456.0f;
constexpr float kWa32 = 22369622.0f / 268435456.0f;
static_assert(8.0 * 22369621 + 4.0 * 22369622 == 268435456.0, "float weights must sum to one");

struct DirP12 {
  static constexpr int Q = 12;
  // angle 30 j degrees, j = 0 .. 11
  static constexpr double vx[Q] = {1, kC30, 0.5, 0, -0.5, -kC30, -1, -kC30, -0.5, 0, 0.5, kC30};
  static constexpr double vy[Q] = {0, 0.5, kC30, 1, kC30, 0.5, 0, -0.5, -kC30, -1, -kC30, -0.5};
  static constexpr double vz2[Q] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr double w[Q] = {1.0 / 12, 1.0 / 12, 1.0 / 12, 1.0 / 12, 1.0 / 12, 1.0 / 12,
                                  1.0 / 12, 1.0 / 12, 1.0 / 12, 1.0 / 12, 1.0 / 12, 1.0 / 12};
  static constexpr float w32[Q] = {kWa32, kWp32, kWp32, kWa32, kWp32, kWp32,
                                   kWa32, kWp32, kWp32, kWa32, kWp32, kWp32};
  static constexpr int opp[Q] = {6, 7, 8, 9, 10, 11, 0, 1, 2, 3, 4, 5};
  static constexpr double kappa = kappa_of(w32, vx, Q, 0.5);
  static constexpr bool planar = true;
  static constexpr double cs2 = 0.5;
};

}  // namespace rlb
