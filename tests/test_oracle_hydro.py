"""P8, P9, P11: hydrodynamics of the oracle against the linear theory of the
scheme (oracle.linear, built from the definitions, independently of
rlb.step) and against closed forms: shear-wave decay at nu_eff = (tau-1/2)/5
+ nu_interp, sound at c_s^2 = 1/3 (the paper's 3D momentum set and P = eps/3;
a planar 2+1 set would give 1/2), and Poiseuille flow between bounce-back
walls with curvature -F/(8 nu_eff) (effective acceleration F/8: the driving
term adds F T^00/6 to a momentum density (4/3) eps beta)."""
import numpy as np
import pytest

from oracle import geometry, linear, rlb
from oracle.velocity_set import velocity_set

V, W, _ = velocity_set()
NU_INTERP = 1.5 * np.sum(W * V[:, 0] ** 2 * (np.abs(V[:, 1]) - V[:, 1] ** 2))


def fourier(F, k):
    ny, nx = F.shape[1:]
    y, x = np.mgrid[0:ny, 0:nx]
    return np.einsum("iyx,yx->i", F, np.exp(-1j * (k[0] * x + k[1] * y))) / (nx * ny)


@pytest.mark.parametrize("kind,kvec,tau", [
    ("shear", (0, 1), 0.8), ("shear", (1, 1), 0.6),
    ("sound", (1, 0), 0.8), ("sound", (1, 2), 0.55)])
def test_small_mode_follows_linear_theory(kind, kvec, tau):
    """A 1e-6 single-mode perturbation evolves as M(k)^t (to O(delta^3))."""
    nx = ny = 16
    k = 2 * np.pi * np.array(kvec) / np.array([nx, ny])
    y, x = np.mgrid[0:ny, 0:nx]
    ph = k[0] * x + k[1] * y
    d = 1e-6
    e = np.ones((ny, nx))
    if kind == "shear":
        t = np.array([-k[1], k[0]]) / np.linalg.norm(k)
        F, G = rlb.initial_state(e, d * t[0] * np.sin(ph), d * t[1] * np.sin(ph), 0.1 * e)
    else:
        F, G = rlb.initial_state(e + d * np.cos(ph), 0 * e, 0 * e, 0.1 * e)
    c0 = fourier(F, k)
    M = linear.update_matrix(k, tau)
    c = c0.copy()
    for _ in range(40):
        F, G = rlb.step(F, G, tau)
        c = M @ c
    got = fourier(F, k)
    assert np.abs(got - c).max() < 1e-6 * np.abs(c0).max()


def test_viscosity_and_sound_speed_of_linear_theory():
    for tau in (0.55, 0.8, 1.0):
        k = 2 * np.pi / 256
        ls, lc = linear.hydrodynamic_modes(np.array([0.0, k]), tau)
        nu = -np.log(abs(ls)) / k ** 2
        assert abs(nu - ((tau - 0.5) / 5 + NU_INTERP)) < 1e-3 * nu
        cs2 = (np.angle(lc) / k) ** 2
        assert abs(cs2 - 1.0 / 3.0) < 1e-4


def test_shear_wave_decay_rate():
    """The shear-wave workload (beta_x = 0.01 sin(2 pi y / 64), tau = 0.8),
    reduced to 4 columns (the flow does not depend on x)."""
    nx, ny, tau = 4, 64, 0.8
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    e = np.ones((ny, nx))
    F, G = rlb.initial_state(e, 0.01 * np.sin(2 * np.pi * y / ny), 0 * e, 0.1 * e)
    amps = []
    for s in range(1, 301):
        F, G = rlb.step(F, G, tau)
        if s in (100, 300):
            T = rlb.energy_momentum(F)
            amps.append(2.0 / (nx * ny) * np.sum(T[0, 1] * np.sin(2 * np.pi * y / ny)))
    k = 2 * np.pi / ny
    ls, _ = linear.hydrodynamic_modes(np.array([0.0, k]), tau)
    assert abs(amps[1] / amps[0] - abs(ls) ** 200) < 2e-4
    nu = -np.log(amps[1] / amps[0]) / (200 * k * k)
    assert abs(nu - ((tau - 0.5) / 5 + NU_INTERP)) < 2e-3 * nu


def test_poiseuille_channel():
    nx, ny, tau, fb = 4, 18, 1.2, 1e-5
    solid = geometry.channel_mask(nx, ny)
    e = np.ones((ny, nx))
    F, G = rlb.initial_state(e, 0 * e, 0 * e, 0.1 * e)
    force = np.zeros((3, ny, nx))
    force[0] = fb
    for _ in range(2500):
        F, G = rlb.step(F, G, tau, force=force, solid=solid)
    b = rlb.fields(F, G, solid=solid)["beta_x"][:, 0]
    ys = np.arange(3, ny - 3)
    c2, c1, c0 = np.polyfit(ys, b[3:ny - 3], 2)
    k = 2 * np.pi / 256
    ls, _ = linear.hydrodynamic_modes(np.array([0.0, k]), tau)
    nu = -np.log(abs(ls)) / k ** 2
    assert abs(c2 - (-fb / (16 * nu))) < 1e-3 * abs(c2)
    y0, y1 = sorted(np.roots([c2, c1, c0]).real)
    assert abs(y0 - 0.5) < 0.2 and abs(y1 - (ny - 1.5)) < 0.2
