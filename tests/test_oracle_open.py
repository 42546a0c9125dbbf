"""Open x borders (Ch. 5, "Model and Methods": a fixed velocity enters along
the inflow border, the lateral borders are periodic) and the current-density
spectra, pinned by:

* a uniform state equal to the border states is a fixed point of the open
  step (the borders add nothing to a uniform flow), at rest and moving;
* an empty channel started at rest becomes plug flow at the inlet velocity,
  the outlet pressure and the inlet charge density (velocity inlet and
  pressure outlet together fix the uniform state);
* with a disc on the channel's mirror line the flow stays mirror-symmetric;
* the spectrum: a pure cosine puts A^2/4 in its own bin and nothing else,
  Parseval's sum, and agreement with numpy's real FFT."""
import numpy as np
import pytest

from oracle import diagnostics, geometry, rlb


def uniform(ny, nx, e, bx, by, n):
    one = np.ones((ny, nx))
    return rlb.initial_state(e * one, bx * one, by * one, n * one)


@pytest.mark.parametrize("beta", [(0.0, 0.0), (0.1, 0.0), (0.05, -0.02)])
def test_uniform_inflow_state_is_a_fixed_point(beta):
    F0, G0 = uniform(6, 20, 1.0, beta[0], beta[1], 0.1)
    F, G = F0, G0
    for _ in range(25):
        F, G = rlb.step(F, G, 0.8, open_x=(beta[0], beta[1], 0.1, 1.0))
    assert np.abs(F - F0).max() < 1e-13
    assert np.abs(G - G0).max() < 1e-14


def test_empty_channel_fills_with_the_inflow_state():
    """Rest at eps = 1.2, n = 0.1 -> plug flow at beta = 0.1, eps = 1,
    n = 0.15 (a y-independent 1-row channel, 12 long, tau = 1.5, so the
    acoustic transients damp within a few thousand steps); interior columns
    only (the border columns' own read-out mixes the two borders)."""
    F, G = uniform(1, 12, 1.2, 0.0, 0.0, 0.1)
    for _ in range(4000):
        F, G = rlb.step(F, G, 1.5, open_x=(0.1, 0.0, 0.15, 1.0))
    f = rlb.fields(F, G)
    inner = slice(2, -2)
    assert np.abs(f["beta_x"][:, inner] - 0.1).max() < 1e-9
    assert np.abs(f["beta_y"][:, inner]).max() < 1e-14
    assert np.abs(f["eps"][:, inner] - 1.0).max() < 1e-9
    assert np.abs(f["n"][:, inner] - 0.15).max() < 1e-9


def test_disc_on_the_mirror_line_keeps_the_flow_symmetric():
    ny, nx = 21, 40
    solid = geometry.disc_mask(nx, ny, [(12.0, 10.0, 3.5)])
    assert np.array_equal(solid, solid[::-1])
    F, G = uniform(ny, nx, 1.0, 0.0, 0.0, 0.1)
    for _ in range(40):
        F, G = rlb.step(F, G, 0.7, solid=solid, open_x=(0.08, 0.0, 0.1, 1.0))
    f = rlb.fields(F, G, solid=solid)
    assert np.abs(f["beta_x"]).max() > 1e-2
    assert np.abs(f["beta_x"] - f["beta_x"][::-1]).max() < 1e-13
    assert np.abs(f["beta_y"] + f["beta_y"][::-1]).max() < 1e-13
    assert np.abs(f["beta_y"]).max() > 1e-4


def test_power_spectrum_pins():
    n = 96
    t = np.arange(n)
    s = 2.0 + 0.7 * np.cos(2 * np.pi * 5 * t / n + 0.3)
    p = diagnostics.power_spectrum(s)
    assert p.shape == (n // 2 + 1,)
    assert abs(p[5] - 0.7 ** 2 / 4) < 1e-15
    assert np.delete(p, 5).max() < 1e-30
    r = np.random.default_rng(3).normal(size=n)
    p = diagnostics.power_spectrum(r)
    d = r - r.mean()
    assert abs(p[0] + 2 * p[1:n // 2].sum() + p[n // 2] - np.mean(d * d)) < 1e-14
    want = np.abs(np.fft.rfft(d)) ** 2 / n ** 2
    assert np.abs(p - want).max() < 1e-15 * want.max() + 1e-18


def test_column_current():
    f = {"Jx": np.arange(12.0).reshape(3, 4)}
    assert diagnostics.column_current(f, 1) == 5.0
