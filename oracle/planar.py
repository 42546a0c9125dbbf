"""The scheme on a planar (2+1) momentum set (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The dissertation's momentum set is three-dimensional: on its one-z-node
lattice the equation of state stays that of a 3D massless gas, P = eps / 3,
so the sound speed is c_s^2 = 1/3 (Ch. 4 "Model and Methods"; Appendix
"Determination of the Equation of State").  Massless particles confined to
the plane instead give a traceless 3 x 3 T^{mu nu} over (t, x, y): the
ideal-fluid tensor T_eq = (eps + P) u u - P g with T^mu_mu = 0 has
P = eps / 2 and c_s^2 = 1/2.  This module builds that variant from the same
definitions (Ch. 3, "Relativistic Lattice Boltzmann" and "Boltzmann to
Lattice Boltzmann"), with in-plane unit momenta:

* momenta: n equally spaced directions v_j = (cos 2 pi j / n, sin 2 pi j / n),
  weights 1/n (n = 12: angular sums exact for polynomials of degree < 12);
* equilibrium: the expansion of T_eq in the circle's orthogonal polynomials
  1, v^a, v^a v^b - delta^{ab}/2 (norms 1, 1/2, 1/8):
      F_eq,i = w_i [T^00 + 2 T^{0a} v^a + 4 (T^{ab} - delta^{ab} T^00 / 2) v^a v^b]
             = w_i eps (1 - 3/2 |u|^2 + 3 u^0 (u.v_i) + 6 (u.v_i)^2),
      G_eq,i = w_i (J^0 + 2 J^a v^a) = w_i n (u^0 + 2 u.v_i);
* streaming, moments, Landau matching, the Anderson-Witting rate and
  bounce-back as in `rlb` (shared functions, this set's momenta).

No driving term: the dissertation derives its bracket for the 3D set only.
"""
import numpy as np

from . import rlb
from .velocity_set import four_velocity


def velocity_set(n=12):
    """(v (n, 3) with v_z = 0, w (n,), opp (n,))."""
    if n % 2 or n < 6:
        raise ValueError("n must be even and >= 6")
    th = 2.0 * np.pi * np.arange(n) / n
    v = np.stack([np.cos(th), np.sin(th), np.zeros(n)], axis=1)
    w = np.full(n, 1.0 / n)
    opp = (np.arange(n) + n // 2) % n
    return v, w, opp


V, W, OPP = velocity_set()
VMU = four_velocity(V)
Q = V.shape[0]


def ideal_tensor(eps, u):
    """T_eq^{mu nu} = (3/2) eps u^mu u^nu - (eps/2) g^{mu nu} (P = eps / 2)."""
    return 1.5 * eps[None, None] * u[:, None] * u[None, :] \
        - 0.5 * eps[None, None] * rlb.METRIC[:, :, None, None]


def equilibrium_F(eps, u):
    T = ideal_tensor(eps, u)
    t00 = T[0, 0]
    t0 = T[0, 1:3]
    tab = T[1:3, 1:3] - 0.5 * np.eye(2)[:, :, None, None] * t00[None, None]
    v2 = V[:, :2]
    return W[:, None, None] * (t00[None] + 2.0 * np.einsum("ia,ayx->iyx", v2, t0)
                               + 4.0 * np.einsum("ia,ib,abyx->iyx", v2, v2, tab))


def equilibrium_G(n, u):
    J = n[None] * u
    return W[:, None, None] * (J[0][None] + 2.0 * np.einsum("ia,ayx->iyx", V[:, :2], J[1:3]))


def initial_state(eps, bx, by, n):
    u = rlb.four_velocity_from_beta(bx, by)
    return equilibrium_F(eps, u), equilibrium_G(n, u)


def step(F, G, tau, cfl=1.0, solid=None):
    """Stream, (bounce-back), moments, Landau, equilibrium, collide."""
    Ft = rlb.stream(F, cfl, v=V)
    Gt = rlb.stream(G, cfl, v=V)
    T = rlb.energy_momentum(Ft, v=V)
    J = rlb.charge_current(Gt, v=V)
    eps, u = rlb.landau(T, skip=solid)
    n = rlb.charge_density(J, u)
    om = rlb.collision_rate(u, tau, v=V)
    Fn = Ft - om * (Ft - equilibrium_F(eps, u))
    Gn = Gt - om * (Gt - equilibrium_G(n, u))
    if solid is not None:
        Fn[:, solid] = Ft[OPP][:, solid]
        Gn[:, solid] = Gt[OPP][:, solid]
    return Fn, Gn


def fields(F, G, cfl=1.0, solid=None):
    Ft, Gt = rlb.stream(F, cfl, v=V), rlb.stream(G, cfl, v=V)
    T = rlb.energy_momentum(Ft, v=V)
    J = rlb.charge_current(Gt, v=V)
    eps, u = rlb.landau(T, skip=solid)
    n = rlb.charge_density(J, u)
    out = {"eps": eps, "beta_x": u[1] / u[0], "beta_y": u[2] / u[0], "n": n,
           "T00": T[0, 0], "T0x": T[0, 1], "T0y": T[0, 2],
           "Txx": T[1, 1], "Txy": T[1, 2], "Tyy": T[2, 2],
           "J0": J[0], "Jx": J[1], "Jy": J[2]}
    if solid is not None:
        for k in out:
            out[k] = np.where(solid, 0.0, out[k])
    return out


def totals(F, G):
    return np.array([F.sum(), np.einsum("i,iyx->", V[:, 0], F),
                     np.einsum("i,iyx->", V[:, 1], F), G.sum()])
