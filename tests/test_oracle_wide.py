"""Streaming with cfl up to 2 (Ch. 4 "Model and Methods": dt = 0.05 against
lattice spacings down to 0.04, i.e. cfl = dt/dx up to 1.25), pinned by:

* where a unit pulse lands: a face direction at cfl = 2 moves exactly two
  cells; at cfl = 1.25 it splits 3/4 : 1/4 between one and two cells;
  an edge direction at cfl = 1.5 (1.0607 cells per axis) lands on the 2x2
  block one and two cells away with the product weights;
* exact conservation of E, P and Q over a periodic run at cfl = 1.25;
* a uniform moving equilibrium stays a fixed point;
* small shear and sound modes follow the linear theory of the scheme
  (oracle.linear, built from the Fourier symbol), and the sound phase speed
  per step is cfl / sqrt(3)."""
import numpy as np
import pytest

from oracle import linear, rlb

V = rlb.V


def pulse(n=9):
    F = np.zeros((rlb.Q, n, n))
    F[:, 4, 4] = 1.0
    return F


def direction(vx, vy):
    return int(np.argmin(np.abs(V[:, 0] - vx) + np.abs(V[:, 1] - vy) + np.abs(V[:, 2])))


def test_face_pulse_at_cfl_2_and_1_25():
    i = direction(1.0, 0.0)
    out = rlb.stream(pulse(), 2.0)[i]
    assert out[4, 6] == 1.0 and out.sum() == 1.0
    out = rlb.stream(pulse(), 1.25)[i]
    assert abs(out[4, 5] - 0.75) < 1e-15 and abs(out[4, 6] - 0.25) < 1e-15
    assert abs(out.sum() - 1.0) < 1e-15


def test_edge_pulse_at_cfl_1_5():
    i = direction(-1 / np.sqrt(2), 1 / np.sqrt(2))
    d = 1.5 / np.sqrt(2)            # 1.0607 cells per axis
    a = d - 1.0
    out = rlb.stream(pulse(), 1.5)[i]
    # moving (-x, +y): lands at x = 4 - 1, 4 - 2 and y = 4 + 1, 4 + 2
    want = {(5, 3): (1 - a) ** 2, (5, 2): (1 - a) * a, (6, 3): a * (1 - a), (6, 2): a * a}
    for (y, x), w in want.items():
        assert abs(out[y, x] - w) < 1e-15
    assert abs(out.sum() - 1.0) < 1e-15


def test_conservation_at_cfl_1_25():
    rng = np.random.default_rng(4)
    ny, nx = 12, 10
    e = 1.0 + 0.05 * rng.normal(size=(ny, nx))
    F, G = rlb.initial_state(e, 0.02 * rng.normal(size=(ny, nx)),
                             0.02 * rng.normal(size=(ny, nx)), 0.1 + 0 * e)
    t0 = rlb.totals(F, G)
    for _ in range(50):
        F, G = rlb.step(F, G, 0.8, cfl=1.25)
    t1 = rlb.totals(F, G)
    assert np.abs(t1 - t0).max() < 1e-12 * t0[0]


def test_uniform_flow_is_a_fixed_point_at_cfl_1_25():
    one = np.ones((6, 7))
    F0, G0 = rlb.initial_state(one, 0.3 * one, -0.2 * one, 0.1 * one)
    F, G = F0, G0
    for _ in range(10):
        F, G = rlb.step(F, G, 0.9, cfl=1.25)
    assert np.abs(F - F0).max() < 1e-14 and np.abs(G - G0).max() < 1e-15


@pytest.mark.parametrize("kind,kvec,tau,cfl", [
    ("shear", (0, 1), 0.8, 1.25), ("sound", (1, 0), 0.8, 1.25), ("sound", (1, 1), 0.7, 1.6)])
def test_small_mode_follows_linear_theory(kind, kvec, tau, cfl):
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
    M = linear.update_matrix(k, tau, cfl)
    c0 = np.einsum("iyx,yx->i", F, np.exp(-1j * ph)) / (nx * ny)
    c = c0.copy()
    for _ in range(30):
        F, G = rlb.step(F, G, tau, cfl=cfl)
        c = M @ c
    got = np.einsum("iyx,yx->i", F, np.exp(-1j * ph)) / (nx * ny)
    assert np.abs(got - c).max() < 1e-6 * np.abs(c0).max()


@pytest.mark.parametrize("cfl", [0.625, 1.25])
def test_sound_speed_per_step(cfl):
    k = 2 * np.pi / 512
    _, lc = linear.hydrodynamic_modes(np.array([k, 0.0]), 0.8, cfl)
    assert abs(np.angle(lc) / k - cfl / np.sqrt(3.0)) < 1e-4 * cfl
