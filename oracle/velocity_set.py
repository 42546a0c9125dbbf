"""Spherical momentum set and angular polynomials (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Ch. 3, "Boltzmann to Lattice Boltzmann": the momentum directions come from a
quadrature that is exact for angular integrals (dOmega / 4 pi) of the
polynomials used; the dissertation names the set a spherical "D3Q27" (Ch. 4,
"Model and Methods") without listing it.  Reading used here: the 26 unit
vectors of the cube directions (6 faces, 12 edges, 8 corners) with the
degree-7 Lebedev weights 1/21, 4/105, 9/280.  The 27th (zero-momentum) slot
carries nothing for massless particles and is omitted.

Appendix "Three Dimensional Orthogonal Polynomials" defines P^(0..3); they are
written out below exactly as listed there.
"""
import itertools

import numpy as np

W_FACE = 1.0 / 21.0
W_EDGE = 4.0 / 105.0
W_CORNER = 9.0 / 280.0


def velocity_set():
    """Return (v, w, opp): v (26, 3) unit vectors, w (26,) weights, opp (26,)
    index of the direction -v_i."""
    dirs, weights = [], []
    for c in itertools.product((-1, 0, 1), repeat=3):
        nz = sum(abs(a) for a in c)
        if nz == 0:
            continue
        dirs.append(np.array(c, dtype=np.float64) / np.sqrt(nz))
        weights.append({1: W_FACE, 2: W_EDGE, 3: W_CORNER}[nz])
    v = np.array(dirs)
    w = np.array(weights)
    opp = np.array([int(np.argmin(np.abs(v + vi).sum(axis=1))) for vi in v])
    return v, w, opp


def four_velocity(v):
    """v_i^mu = (1, v_i) for massless momenta p^mu = |p| (1, v)."""
    return np.concatenate([np.ones((v.shape[0], 1)), v], axis=1)


# Appendix "Three Dimensional Orthogonal Polynomials".
def P0(v):
    return np.ones(v.shape[0])


def P1(v):
    return v.copy()                                  # P_i = v_i


def P2(v):
    d = np.eye(3)
    return v[:, :, None] * v[:, None, :] - d / 3.0   # v_i v_j - delta_ij / 3


def P3(v):
    d = np.eye(3)
    vvv = v[:, :, None, None] * v[:, None, :, None] * v[:, None, None, :]
    corr = (d[None, :, :, None] * v[:, None, None, :]
            + d[None, :, None, :] * v[:, None, :, None]
            + d[None, None, :, :] * v[:, :, None, None])
    return vvv - corr / 5.0
