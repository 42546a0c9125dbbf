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


def test_filtered_velocity_keeps_only_the_inertial_modes():
    """A low mode (|k| = 2) and a driven one (|k| = 9): the filter at k_cut
    = 6 keeps exactly the first; its speed is |A| |cos|, mean 2|A|/pi,
    rms |A|/sqrt(2)."""
    n = 64
    y, x = np.mgrid[0:n, 0:n]
    low = 0.02 * np.cos(2 * np.pi * 2 * x / n + 0.4)
    high = 0.05 * np.sin(2 * np.pi * (9 * y) / n)
    fx, fy, mean, rms = diagnostics.filtered_velocity(0 * low + high, low, 6.0)
    assert np.abs(fx).max() < 1e-15
    assert np.abs(fy - low).max() < 1e-15
    assert abs(rms - 0.02 / np.sqrt(2)) < 1e-15
    assert abs(mean - np.abs(low).mean()) < 1e-15
    assert abs(mean - 2 * 0.02 / np.pi) < 2e-3 * 0.02    # the continuum value


def test_spectrum_average_and_error():
    s = np.array([[1.0, 10.0], [3.0, 10.0], [2.0, 10.0]])
    mean, err = diagnostics.spectrum_average(s)
    assert np.allclose(mean, [2.0, 10.0])
    assert abs(err[0] - np.sqrt(2.0 / 6.0)) < 1e-15 and err[1] == 0.0


def test_power_law_fit_recovers_kolmogorov():
    k = np.arange(2, 12, dtype=np.float64)
    slope, a = diagnostics.power_law_fit(k, 3.5 * k ** (-5.0 / 3.0))
    assert abs(slope + 5.0 / 3.0) < 1e-13 and abs(a - np.log(3.5)) < 1e-13
