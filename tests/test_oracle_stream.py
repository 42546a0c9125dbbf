"""Streaming pins: a single population moves by exactly delta_i = v_i (cfl=1)
with the bilinear weights, and streaming conserves every population's sum."""
import numpy as np
import pytest

from oracle import rlb

V = rlb.V


@pytest.mark.parametrize("i", range(26))
def test_delta_moves_by_velocity(i):
    ny, nx = 9, 11
    F = np.zeros((26, ny, nx))
    F[i, 4, 5] = 1.0
    out = rlb.stream(F)[i]
    dx, dy = V[i, 0], V[i, 1]
    assert abs(out.sum() - 1.0) < 1e-15
    y, x = np.mgrid[0:ny, 0:nx]
    assert abs((out * x).sum() - (5 + dx)) < 1e-14
    assert abs((out * y).sum() - (4 + dy)) < 1e-14
    # explicit bilinear weights
    sx, sy = int(np.sign(dx)), int(np.sign(dy))
    ax, ay = abs(dx), abs(dy)
    want = np.zeros((ny, nx))
    want[4, 5] += (1 - ax) * (1 - ay)
    want[4, 5 + sx] += ax * (1 - ay)
    want[4 + sy, 5] += (1 - ax) * ay
    want[4 + sy, 5 + sx] += ax * ay
    np.testing.assert_allclose(out, want, atol=1e-16)


def test_periodic_wrap():
    F = np.zeros((26, 4, 4))
    F[:, 0, 0] = 1.0
    out = rlb.stream(F)
    np.testing.assert_allclose(out.sum(axis=(1, 2)), 1.0, atol=1e-15)


def test_cfl_half_moves_half():
    F = np.zeros((26, 9, 9))
    F[:, 4, 4] = 1.0
    out = rlb.stream(F, cfl=0.5)
    x = np.arange(9)[None, :]
    for i in range(26):
        assert abs((out[i] * x).sum() - (4 + 0.5 * V[i, 0])) < 1e-14
