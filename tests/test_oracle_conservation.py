"""P6: exact global conservation of energy, momentum and charge (periodic,
no force); energy and charge with solids; the driving term's injection
(dP^j = sum F^j T^00 / 6, dE = sum F.T^{0.} / 6 per step); and a negative
control showing that the classical rate 1/tau would break momentum
conservation, which the Anderson-Witting rate does not."""
import numpy as np

from oracle import rlb, geometry
from paper_2205_04658_amd import workloads


def perturbed_state(nx, ny, seed, amp=0.02):
    f = workloads.random_fields(nx, ny, seed)
    F, G = rlb.initial_state(f["eps"], f["bx"], f["by"], f["n"])
    rng = np.random.default_rng(seed + 100)
    F = F * (1 + amp * rng.uniform(-1, 1, F.shape))     # non-equilibrium stress
    G = G * (1 + amp * rng.uniform(-1, 1, G.shape))
    return F, G


def test_periodic_conservation():
    F, G = perturbed_state(12, 10, 1)
    t0 = rlb.totals(F, G)
    for _ in range(200):
        F, G = rlb.step(F, G, tau=0.7)
    t1 = rlb.totals(F, G)
    scale = np.array([t0[0], t0[0], t0[0], t0[3]])
    assert np.all(np.abs(t1 - t0) <= 1e-12 * scale), (t1 - t0) / scale


def test_conservation_with_solids():
    nx, ny = 16, 12
    solid = geometry.channel_mask(nx, ny, [(5.0, 6.0, 2.0)])
    F, G = perturbed_state(nx, ny, 2)
    t0 = rlb.totals(F, G)
    for _ in range(100):
        F, G = rlb.step(F, G, tau=0.8, solid=solid)
    t1 = rlb.totals(F, G)
    assert abs(t1[0] - t0[0]) <= 1e-12 * t0[0]
    assert abs(t1[3] - t0[3]) <= 1e-12 * t0[3]


def test_force_injection_per_step():
    nx, ny = 12, 10
    F, G = perturbed_state(nx, ny, 3)
    rng = np.random.default_rng(9)
    for _ in range(5):
        force = np.zeros((3, ny, nx))
        force[:2] = 1e-3 * rng.normal(size=(2, ny, nx))
        inj = rlb.force_injection(F, force)
        t0 = rlb.totals(F, G)
        F, G = rlb.step(F, G, tau=0.7, force=force)
        d = rlb.totals(F, G) - t0
        np.testing.assert_allclose(d[:3], inj, rtol=1e-9, atol=1e-13 * t0[0])
        assert abs(d[3]) < 1e-13 * t0[3]
        assert inj[1] != 0.0


def test_uniform_force_accelerates_along_force():
    e = np.ones((4, 4))
    F, G = rlb.initial_state(e, 0 * e, 0 * e, 0.1 * e)
    force = np.zeros((3, 4, 4))
    force[0] = 1e-4
    for _ in range(3):
        F, G = rlb.step(F, G, tau=0.8, force=force)
    f = rlb.fields(F, G)
    assert np.all(f["beta_x"] > 0)
    np.testing.assert_allclose(f["beta_y"], 0, atol=1e-15)


def test_negative_control_classical_rate_breaks_momentum():
    F, G = perturbed_state(12, 10, 4, amp=0.1)
    t0 = rlb.totals(F, G)
    Fa, Ga = rlb.step(F, G, tau=0.7)
    Fb, Gb = rlb.step(F, G, tau=0.7, collision="bgk")
    da = np.abs(rlb.totals(Fa, Ga) - t0)
    db = np.abs(rlb.totals(Fb, Gb) - t0)
    assert da[1:3].max() < 1e-13 * t0[0]
    assert db[1:3].max() > 1e-6 * t0[0]
