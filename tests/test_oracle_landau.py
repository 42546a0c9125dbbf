"""P4: Landau matching against closed forms (boosted tensors)."""
import numpy as np
import pytest

from oracle import rlb


def boost(beta):
    b = np.asarray(beta, float)
    g = 1.0 / np.sqrt(1 - b @ b)
    L = np.eye(4)
    L[0, 0] = g
    L[0, 1:] = L[1:, 0] = g * b
    bb = b @ b
    if bb > 0:
        L[1:, 1:] += (g - 1) * np.outer(b, b) / bb
    return L


@pytest.mark.parametrize("seed", range(5))
def test_boosted_anisotropic_tensor(seed):
    """T = L diag(eps, p1, p2, p3) L^T with arbitrary rest-frame pressures:
    the Landau frame is exactly the boost, u = L (1,0,0,0), eps exact."""
    rng = np.random.default_rng(seed)
    b = rng.uniform(-0.6, 0.6, 2)
    beta = np.array([b[0], b[1], 0.0])
    eps = rng.uniform(0.5, 3.0)
    p = rng.uniform(0.05, 0.6, 3) * eps
    L = boost(beta)
    T = L @ np.diag([eps, *p]) @ L.T
    e, u = rlb.landau(T[:, :, None, None])
    assert abs(e[0, 0] - eps) < 1e-12 * eps
    np.testing.assert_allclose(u[:, 0, 0], L[:, 0], atol=1e-12)


@pytest.mark.parametrize("speed", [0.0, 0.5, 0.9, 0.99])
def test_round_trip_equilibrium(speed):
    ang = np.linspace(0, 2 * np.pi, 7)[None, :]
    bx = speed * np.cos(ang)
    by = speed * np.sin(ang)
    eps = np.full_like(bx, 0.8)
    u = rlb.four_velocity_from_beta(bx, by)
    e, u2 = rlb.landau(rlb.ideal_tensor(eps, u))
    np.testing.assert_allclose(e, eps, rtol=1e-11)
    np.testing.assert_allclose(u2, u, atol=1e-12 * (1 + np.abs(u).max()))


def test_random_positive_populations_give_timelike_frame():
    rng = np.random.default_rng(5)
    F = rng.uniform(0.0, 1.0, size=(26, 8, 8))
    T = rlb.energy_momentum(F)
    e, u = rlb.landau(T)
    norm = u[0] ** 2 - (u[1:] ** 2).sum(0)
    np.testing.assert_allclose(norm, 1.0, atol=1e-12)
    assert np.all(e > 0)
    resid = np.einsum("mlyx,l,lyx->myx", T, [1, -1, -1, -1], u) - e * u
    assert np.abs(resid).max() < 1e-12


def test_rejects_spacelike():
    """A beam of populations moving in a single direction has no rest frame."""
    F = np.zeros((26, 1, 1))
    F[0] = 1.0
    T = rlb.energy_momentum(F)
    with pytest.raises(rlb.LandauError):
        rlb.landau(T)
