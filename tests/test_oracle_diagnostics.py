"""Diagnostics pins: Parseval for E(k), a single mode lands in its shell, and
the enstrophy of a known field."""
import numpy as np

from oracle import diagnostics


def test_single_mode_spectrum():
    n = 32
    y, x = np.mgrid[0:n, 0:n]
    bx = 0.01 * np.cos(2 * np.pi * 3 * y / n)
    E = diagnostics.energy_spectrum(bx, 0 * bx)
    assert abs(E[3] - 0.5 * 2 * (0.005) ** 2) < 1e-18
    assert abs(E.sum() - E[3]) < 1e-18


def test_parseval():
    rng = np.random.default_rng(0)
    bx, by = rng.normal(size=(2, 16, 16))
    E = diagnostics.energy_spectrum(bx, by, kmax=12)
    assert abs(E.sum() - 0.5 * (bx ** 2 + by ** 2).mean()) < 1e-12


def test_enstrophy_of_shear():
    n = 64
    y = np.arange(n)[:, None] * np.ones((1, n))
    k = 2 * np.pi / n
    bx = np.sin(k * y)
    # omega = -d_y beta_x = -sin(k) cos(k y) by central differences
    Z = diagnostics.enstrophy(bx, 0 * bx)
    assert abs(Z - np.sin(k) ** 2 * n * n / 2) < 1e-9
