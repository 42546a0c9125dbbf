"""The planar (2+1) momentum set (oracle.planar), pinned by closed forms and
textbook integrals rather than by its own formulas:

* circle quadrature: sum_j w_j cos^a sin^b of the 12 directions equals the
  exact circle average (a-1)!!(b-1)!!/(a+b)!! for every a + b <= 10;
* equilibrium moments equal the angular integrals of the exact 2D massless
  Juttner distributions, eps / (gamma (1 - beta.v))^3 for energy-momentum
  and n / (gamma (1 - beta.v))^2 for charge (fine quadrature on the circle);
  in particular T^{mu}_{mu} = 0, i.e. P = eps / 2;
* Landau matching returns (eps, u) from the equilibrium moments;
* a uniform moving equilibrium is a fixed point, and E, P, Q are conserved;
* small modes follow the linear theory of this set, whose sound speed is
  c_s^2 = 1/2 and whose viscosity changes by (tau1 - tau2) / 4 (the 2D
  kinetic value tau (eps + P) / 4 instead of the 3D tau (eps + P) / 5)."""
import numpy as np
import pytest

from oracle import linear, planar, rlb


def dfact(n):
    return 1.0 if n <= 0 else n * dfact(n - 2)


def test_circle_quadrature():
    v, w = planar.V, planar.W
    assert abs(w.sum() - 1.0) < 1e-15
    for a in range(11):
        for b in range(11 - a):
            got = np.sum(w * v[:, 0] ** a * v[:, 1] ** b)
            want = 0.0 if (a % 2 or b % 2) else dfact(a - 1) * dfact(b - 1) / dfact(a + b)
            assert abs(got - want) < 1e-15, (a, b)


@pytest.mark.parametrize("beta", [(0.0, 0.0), (0.6, 0.3), (-0.2, 0.85)])
def test_equilibrium_matches_2d_juttner(beta):
    eps, n = 1.7, 0.3
    bx, by = (np.full((1, 1), b) for b in beta)
    u = rlb.four_velocity_from_beta(bx, by)
    F = planar.equilibrium_F(np.full((1, 1), eps), u)
    G = planar.equilibrium_G(np.full((1, 1), n), u)
    T = rlb.energy_momentum(F, v=planar.V)[..., 0, 0]
    J = rlb.charge_current(G, v=planar.V)[..., 0, 0]
    th = 2 * np.pi * np.arange(4096) / 4096
    vm = np.stack([np.ones_like(th), np.cos(th), np.sin(th), 0 * th])
    g = 1.0 / np.sqrt(1 - beta[0] ** 2 - beta[1] ** 2)
    d = g * (1 - beta[0] * vm[1] - beta[1] * vm[2])
    Tw = np.einsum("mt,nt,t->mn", vm, vm, eps / d ** 3) / th.size
    Jw = np.einsum("mt,t->m", vm, n / d ** 2) / th.size
    assert np.abs(T - Tw).max() < 1e-12 * np.abs(Tw).max()
    assert np.abs(J - Jw).max() < 1e-12 * np.abs(Jw).max()
    g_mn = np.diag([1.0, -1.0, -1.0, -1.0])
    assert abs(np.sum(T * g_mn)) < 1e-12 * T[0, 0]          # traceless: P = eps / 2


def test_landau_round_trip():
    e = np.array([[1.3, 0.7]])
    u = rlb.four_velocity_from_beta(np.array([[0.5, -0.1]]), np.array([[0.2, 0.8]]))
    T = rlb.energy_momentum(planar.equilibrium_F(e, u), v=planar.V)
    eps, uu = rlb.landau(T)
    assert np.abs(eps - e).max() < 1e-12 and np.abs(uu - u).max() < 1e-11


def test_fixed_point_and_conservation():
    one = np.ones((6, 8))
    F0, G0 = planar.initial_state(one, 0.3 * one, -0.2 * one, 0.1 * one)
    F, G = F0, G0
    for _ in range(10):
        F, G = planar.step(F, G, 0.8)
    assert np.abs(F - F0).max() < 1e-14 and np.abs(G - G0).max() < 1e-15
    rng = np.random.default_rng(5)
    F, G = planar.initial_state(1 + 0.05 * rng.normal(size=(10, 12)), 0.03 * rng.normal(size=(10, 12)),
                                0.03 * rng.normal(size=(10, 12)), 0.1 + 0 * rng.normal(size=(10, 12)))
    t0 = planar.totals(F, G)
    for _ in range(40):
        F, G = planar.step(F, G, 0.7, cfl=0.8)
    assert np.abs(planar.totals(F, G) - t0).max() < 1e-12 * t0[0]


@pytest.mark.parametrize("kind,kvec,tau,cfl", [
    ("shear", (0, 1), 0.8, 1.0), ("sound", (1, 0), 0.8, 1.0), ("sound", (1, 2), 0.6, 0.5)])
def test_small_mode_follows_linear_theory(kind, kvec, tau, cfl):
    nx = ny = 16
    k = 2 * np.pi * np.array(kvec) / np.array([nx, ny])
    y, x = np.mgrid[0:ny, 0:nx]
    ph = k[0] * x + k[1] * y
    d = 1e-6
    e = np.ones((ny, nx))
    if kind == "shear":
        t = np.array([-k[1], k[0]]) / np.linalg.norm(k)
        F, G = planar.initial_state(e, d * t[0] * np.sin(ph), d * t[1] * np.sin(ph), 0.1 * e)
    else:
        F, G = planar.initial_state(e + d * np.cos(ph), 0 * e, 0 * e, 0.1 * e)
    M = linear.update_matrix(k, tau, cfl, planar=True)
    c0 = np.einsum("iyx,yx->i", F, np.exp(-1j * ph)) / (nx * ny)
    c = c0.copy()
    for _ in range(30):
        F, G = planar.step(F, G, tau, cfl=cfl)
        c = M @ c
    got = np.einsum("iyx,yx->i", F, np.exp(-1j * ph)) / (nx * ny)
    assert np.abs(got - c).max() < 1e-6 * np.abs(c0).max()


def test_sound_speed_and_viscosity_of_the_planar_set():
    k = 2 * np.pi / 512
    nus = []
    for tau in (0.6, 1.0):
        ls, lc = linear.hydrodynamic_modes(np.array([k, 0.0]), tau, planar=True)
        assert abs((np.angle(lc) / k) ** 2 - 0.5) < 1e-4
        nus.append(-np.log(abs(ls)) / k ** 2)
    assert abs((nus[1] - nus[0]) - 0.4 / 4) < 1e-4
    # the 3D set at the same tau values: 1/3 and (tau1 - tau2) / 5
    ls0, lc0 = linear.hydrodynamic_modes(np.array([k, 0.0]), 0.6)
    ls1, _ = linear.hydrodynamic_modes(np.array([k, 0.0]), 1.0)
    assert abs((np.angle(lc0) / k) ** 2 - 1.0 / 3.0) < 1e-4
    assert abs((np.log(abs(ls0)) - np.log(abs(ls1))) / k ** 2 - 0.4 / 5) < 1e-4
