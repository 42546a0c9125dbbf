"""Per-node relaxation time from eta/s (Ch. 3, "Relativistic Lattice
Boltzmann": tau_R = 5 (eta/s) / T; "Boltzmann to Lattice Boltzmann":
eps = 3 T^4 / pi^2), pinned without retyping the formula:

* the equation of state at hand-computed points (T = 1 and T = 2);
* a uniform state reduces the per-node step to the constant-tau step at the
  hand-computed tau (eta/s = 0.02, dt = 0.05, T = 1: tau = 5 * 0.02 / 0.05
  = 2), and not to a neighbouring tau;
* shear-wave decay at two background temperatures follows the linear theory
  of the scheme (oracle.linear, independent of rlb.step) at tau = 2 and
  tau = 1: sixteen times the energy density doubles T and halves tau."""
import numpy as np
import pytest

from oracle import linear, rlb

E_T1 = 3.0 / np.pi ** 2          # energy density at T = 1
RELAX = rlb.ViscosityRelaxation(eta_s=0.02, dt=0.05)


def test_temperature_at_hand_points():
    assert abs(rlb.temperature(E_T1) - 1.0) < 1e-15
    assert abs(rlb.temperature(16 * E_T1) - 2.0) < 1e-15
    assert abs(RELAX(E_T1) - 2.0) < 1e-14
    assert abs(RELAX(16 * E_T1) - 1.0) < 1e-14


def test_relaxation_rejects_nonpositive_parameters():
    with pytest.raises(ValueError):
        rlb.ViscosityRelaxation(0.0, 0.05)
    with pytest.raises(ValueError):
        rlb.ViscosityRelaxation(0.02, -1.0)


def test_uniform_state_reduces_to_constant_tau():
    """A uniform moving state, pushed off equilibrium by a population vector
    with no energy-momentum (a null vector of the moment map), keeps
    eps = E_T1 at every node, so its first step has per-node tau = 2."""
    ny, nx = 3, 4
    e = np.full((ny, nx), E_T1)
    F, G = rlb.initial_state(e, 0.3 + 0 * e, 0.1 + 0 * e, 0.1 * e)
    vmu = np.hstack([np.ones((rlb.Q, 1)), rlb.V])
    moments = np.stack([vmu[:, a] * vmu[:, b] for a in range(4) for b in range(a, 4)])
    d = np.linalg.svd(moments)[2][-1]            # sum_i d_i v^mu v^nu = 0
    assert np.abs(moments @ d).max() < 1e-14
    F = F + 1e-3 * d[:, None, None]
    G = G + 1e-4 * d[:, None, None]
    force = np.zeros((3, ny, nx))
    force[0] = 2e-3
    force[1] = -1e-3
    a = rlb.step(F, G, RELAX, force=force)
    b = rlb.step(F, G, 2.0, force=force)
    c = rlb.step(F, G, 2.02, force=force)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() < 1e-14 * np.abs(y).max()
    assert np.abs(a[0] - c[0]).max() > 1e-9   # tau matters in this set-up


@pytest.mark.parametrize("scale,tau", [(1.0, 2.0), (16.0, 1.0)])
def test_shear_decay_follows_temperature(scale, tau):
    """beta_x = 1e-3 sin(2 pi y / 32) on a background eps = scale * E_T1:
    the T^{0x} mode decays as the shear eigenvalue of the linear update at
    the tau the background temperature gives (the mode leaves eps uniform
    to first order)."""
    nx, ny = 2, 32
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    e = np.full((ny, nx), scale * E_T1)
    F, G = rlb.initial_state(e, 1e-3 * np.sin(2 * np.pi * y / ny), 0 * e, 0.1 * e)
    amps = []
    for s in range(1, 121):
        F, G = rlb.step(F, G, RELAX)
        if s in (20, 120):
            T = rlb.energy_momentum(F)
            amps.append(2.0 / (nx * ny) * np.sum(T[0, 1] * np.sin(2 * np.pi * y / ny)))
    k = 2 * np.pi / ny
    ls, _ = linear.hydrodynamic_modes(np.array([0.0, k]), tau)
    assert abs(amps[1] / amps[0] - abs(ls) ** 100) < 1e-5
    # and not the other background's tau
    lo, _ = linear.hydrodynamic_modes(np.array([0.0, k]), 3.0 - tau)
    assert abs(amps[1] / amps[0] - abs(lo) ** 100) > 1e-3
