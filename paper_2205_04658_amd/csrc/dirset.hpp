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
#pragma once

namespace rlb {

constexpr double kS2 = 0.70710678118654752440;   // 1/sqrt(2)
constexpr double kS3 = 0.57735026918962576451;   // 1/sqrt(3)
constexpr double kWf = 1.0 / 21.0;
constexpr double kWe = 4.0 / 105.0;
constexpr double kWc = 9.0 / 280.0;

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
  static constexpr int opp[Q] = {1, 0, 3, 2, 7, 6, 5, 4,
                                 8, 10, 9, 12, 11, 16, 15, 14, 13};
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
  // opposite of (vx, vy, +vz) is (-vx, -vy, -vz): in the other vz group
  static constexpr int opp[Q] = {1, 0, 3, 2, 7, 6, 5, 4,
                                 17, 19, 18, 21, 20, 25, 24, 23, 22,
                                 8, 10, 9, 12, 11, 16, 15, 14, 13};
};

}  // namespace rlb
