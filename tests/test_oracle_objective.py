"""Pins of the gradient-workload oracle: the objectives respond to the body
force as linear response predicts (the charge current linearly, the squared
non-equilibrium stress quadratically), and the central differences recover
that closed-form derivative."""
import numpy as np

from oracle import geometry, objective
from paper_2205_04658_amd import workloads

NX, NY, N = 8, 12, 40


def rest():
    return workloads.uniform(NX, NY)


def test_basis_force_closed_form():
    modes = np.array([[1.0, 2.0, 0.6, 0.8, 0.3]])
    F = objective.basis_force(NX, NY, modes, [2.0], 0.5)
    y, x = np.mgrid[0:NY, 0:NX]
    c = np.cos(2 * np.pi * (x / NX + 2 * y / NY) + 0.3)
    np.testing.assert_allclose(F[0], 0.5 + 2.0 * 0.6 * c, atol=1e-15)
    np.testing.assert_allclose(F[1], 2.0 * 0.8 * c, atol=1e-15)
    assert abs(F[1].mean()) < 1e-15


def test_current_linear_and_dissipation_quadratic_in_body_force():
    solid = geometry.channel_mask(NX, NY)
    j1 = objective.run_objective(rest(), N, 0.8, 1e-6, [], [], "current", solid)
    j2 = objective.run_objective(rest(), N, 0.8, 2e-6, [], [], "current", solid)
    assert j1 > 0 and abs(j2 / j1 - 2.0) < 1e-4
    d1 = objective.run_objective(rest(), N, 0.8, 1e-6, [], [], "dissipation", solid)
    d2 = objective.run_objective(rest(), N, 0.8, 2e-6, [], [], "dissipation", solid)
    assert d1 > 0 and abs(d2 / d1 - 4.0) < 1e-3


def test_fd_gradient_recovers_linear_response():
    solid = geometry.channel_mask(NX, NY)
    j = objective.run_objective(rest(), N, 0.8, 1e-6, [], [], "current", solid)
    g = objective.fd_gradient(rest(), N, 0.8, 1e-6, [], [], "current", solid, which=[0])
    assert abs(g[0] - j / 1e-6) < 1e-5 * abs(g[0])
