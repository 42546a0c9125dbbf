"""P10: the counter-based generator against its published known answers and
an independent library implementation; the shell synthesis against an
inverse FFT of the Hermitian-filled coefficient grid."""
import os

import numpy as np
import pytest

from oracle import forcing

KAT = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")


def kat_rows():
    rows = []
    for line in open(KAT):
        if line.startswith("#") or not line.strip():
            continue
        h = [int(t, 16) for t in line.split()]
        rows.append((h[0:4], h[4:6], h[6:10]))
    return rows


@pytest.mark.parametrize("row", kat_rows())
def test_philox_known_answers(row):
    ctr, key, out = row
    assert list(forcing.philox4x64_10(ctr, key)) == out


def test_philox_matches_numpy_bit_generator():
    """numpy.random.Philox (4x64, 10 rounds) increments its counter before
    each block, so its first block is philox(counter + 1, key)."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        key = [int(x) for x in rng.integers(0, 2**63, size=2)]
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4)]
        bg = np.random.Philox(key=np.array(key, np.uint64), counter=np.array(ctr, np.uint64))
        got = [int(x) for x in bg.random_raw(4)]
        c1 = [ctr[0] + 1] + ctr[1:]
        assert list(forcing.philox4x64_10(c1, key)) == got


def test_box_muller_statistics():
    z = []
    for m in range(4000):
        r = forcing.philox4x64_10((m, 0, 0, 0), (1, 0))
        z += list(forcing.box_muller(r[0], r[1])) + list(forcing.box_muller(r[2], r[3]))
    z = np.array(z)
    assert abs(z.mean()) < 0.03 and abs(z.var() - 1) < 0.05
    assert abs(np.mean(z ** 4) - 3) < 0.2


def test_shell_counts():
    assert len(forcing.shell_modes(7, 9)) == 54
    assert len(forcing.shell_modes(31, 33)) == 206
    full = forcing.shell_modes(7, 9)
    assert len({kx for kx, _ in full} | {-kx for kx, _ in full}) == 19


def test_synthesis_equals_inverse_fft():
    nx, ny = 32, 24
    modes = forcing.shell_modes(3, 5)
    cx, cy = forcing.stirring_coefficients(modes, seed=5, step=17, amplitude=0.3)
    f = forcing.synthesize(modes, cx, cy, nx, ny)
    for comp, c in ((0, cx), (1, cy)):
        grid = np.zeros((ny, nx), np.complex128)
        for (kx, ky), a in zip(modes, c):
            grid[ky % ny, kx % nx] += a
            grid[(-ky) % ny, (-kx) % nx] += np.conj(a)
        ref = np.fft.ifft2(grid) * (nx * ny)
        assert np.abs(ref.imag).max() < 1e-12
        np.testing.assert_allclose(f[comp], ref.real, atol=1e-12)
        assert abs(f[comp].mean()) < 1e-13


def test_point_synthesis_equals_inverse_fft():
    """field_at (the sum at chosen nodes, for lattices too large to
    synthesise whole) against the inverse FFT of the Hermitian grid."""
    nx, ny = 40, 30
    st = forcing.Stirring(nx, ny, 2, 6, 0.2, 9)
    cx, cy = forcing.stirring_coefficients(st.modes, 9, 4, 0.2)
    rng = np.random.default_rng(3)
    xs, ys = rng.integers(0, nx, 25), rng.integers(0, ny, 25)
    got = st.field_at(4, xs, ys)
    for comp, c in ((0, cx), (1, cy)):
        grid = np.zeros((ny, nx), np.complex128)
        for (kx, ky), a in zip(st.modes, c):
            grid[ky % ny, kx % nx] += a
            grid[(-ky) % ny, (-kx) % nx] += np.conj(a)
        ref = (np.fft.ifft2(grid) * (nx * ny)).real
        np.testing.assert_allclose(got[comp], ref[ys, xs], atol=1e-12)


def test_fresh_draw_every_step():
    modes = forcing.shell_modes(7, 9)
    a = forcing.stirring_coefficients(modes, 2205, 0, 1.0)
    b = forcing.stirring_coefficients(modes, 2205, 1, 1.0)
    c = forcing.stirring_coefficients(modes, 2205, 0, 1.0)
    assert np.all(a[0] != b[0])
    np.testing.assert_array_equal(a[0], c[0])
