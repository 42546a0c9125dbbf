"""P3 / P5: the truncated equilibrium against the exact Juttner moments, and
equilibrium as a fixed point of the collision and of the full step."""
import numpy as np
import pytest

from oracle import rlb


def exact_juttner_moments(eps, n, beta, order=64):
    """Continuum moments of the massless Juttner distribution, by Gauss-Legendre
    in cos(theta) and the trapezoid rule in phi (exact for these smooth
    periodic integrands): the angular densities are eps / (gamma^4 (1 - v.b)^4)
    for T^{mu nu} and n / (gamma^3 (1 - v.b)^3) for J^mu."""
    x, wx = np.polynomial.legendre.leggauss(order)
    phi = np.arange(2 * order) * np.pi / order
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    v = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wq = (np.outer(wx, np.full(2 * order, np.pi / order)) / (4 * np.pi)).ravel()
    g = 1.0 / np.sqrt(1 - beta @ beta)
    fT = eps / (g ** 4 * (1 - v @ beta) ** 4)
    fJ = n / (g ** 3 * (1 - v @ beta) ** 3)
    vmu = np.concatenate([np.ones((len(v), 1)), v], 1)
    return (np.einsum("q,qm,qn->mn", wq * fT, vmu, vmu), np.einsum("q,qm->m", wq * fJ, vmu))


@pytest.mark.parametrize("beta", [(0.0, 0.0), (0.01, 0.0), (0.6, 0.3), (0.3, -0.8), (0.9, 0.0)])
def test_equilibrium_moments_match_juttner(beta):
    eps = np.full((1, 1), 1.7)
    n = np.full((1, 1), 0.3)
    b = np.array([beta[0], beta[1], 0.0])
    u = rlb.four_velocity_from_beta(np.full((1, 1), beta[0]), np.full((1, 1), beta[1]))
    T = rlb.energy_momentum(rlb.equilibrium_F(eps, u))[:, :, 0, 0]
    J = rlb.charge_current(rlb.equilibrium_G(n, u))[:, 0, 0]
    Tx, Jx = exact_juttner_moments(1.7, 0.3, b)
    np.testing.assert_allclose(T, Tx, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(J, Jx, rtol=1e-12, atol=1e-12)


def test_worked_example_t00():
    """beta = (0.6, 0.3), eps = 1: T^00 = (4/3) gamma^2 - 1/3 = 2.0909..."""
    u = rlb.four_velocity_from_beta(np.full((1, 1), 0.6), np.full((1, 1), 0.3))
    T = rlb.energy_momentum(rlb.equilibrium_F(np.ones((1, 1)), u))
    assert abs(T[0, 0, 0, 0] - (4.0 / 3.0 / 0.55 - 1.0 / 3.0)) < 1e-14
    assert abs(T[0, 0, 0, 0] - 2.0909090909090909) < 1e-14


def test_collision_fixed_point_random_cells():
    """Per node: equilibrium -> moments -> Landau -> equilibrium reproduces itself."""
    rng = np.random.default_rng(1)
    eps = rng.uniform(0.5, 2.0, (4, 5))
    bx = rng.uniform(-0.6, 0.6, (4, 5))
    by = rng.uniform(-0.6, 0.6, (4, 5))
    n = rng.uniform(0.05, 0.5, (4, 5))
    F, G = rlb.initial_state(eps, bx, by, n)
    e2, u2 = rlb.landau(rlb.energy_momentum(F))
    n2 = rlb.charge_density(rlb.charge_current(G), u2)
    np.testing.assert_allclose(e2, eps, rtol=1e-12)
    np.testing.assert_allclose(u2[1] / u2[0], bx, atol=1e-12)
    np.testing.assert_allclose(n2, n, rtol=1e-12)
    np.testing.assert_allclose(rlb.equilibrium_F(e2, u2), F, atol=1e-13)
    np.testing.assert_allclose(rlb.equilibrium_G(n2, u2), G, atol=1e-13)


@pytest.mark.parametrize("beta", [(0.0, 0.0), (0.3, 0.2), (0.9, 0.0), (-0.5, 0.6)])
def test_uniform_equilibrium_is_fixed_point_of_step(beta):
    e = np.ones((6, 7))
    F, G = rlb.initial_state(1.3 * e, beta[0] * e, beta[1] * e, 0.2 * e)
    F2, G2 = rlb.step(F, G, tau=0.6)
    np.testing.assert_allclose(F2, F, atol=1e-14)
    np.testing.assert_allclose(G2, G, atol=1e-14)
