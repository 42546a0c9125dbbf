"""Random k-shell stirring force (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Ch. 4, "Model and Methods": every step a random driving term is set on the
spectral lattice inside the driving band, then transformed to configuration
space and fed to the driving term.  The band, law and amplitude used here are
the ones of the forced-turbulence workloads (a closed shell kmin <= |k| <=
kmax of integer modes, i.i.d. Gaussian coefficients of standard deviation
`amplitude` for the real and imaginary parts of each in-plane component, a
fresh draw every step, Hermitian symmetry so the field is real and has zero
mean).

Random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11), written from its published definition,
and the Box-Muller transform.  Counter = (mode index, step, 0, 0), key =
(seed, stream).
"""
import math

import numpy as np

_M64 = (1 << 64) - 1
_PHILOX_MUL = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
_PHILOX_WEYL = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)


def philox4x64_10(counter, key):
    """Philox4x64 with 10 rounds.  counter: 4 ints < 2^64, key: 2 ints."""
    c0, c1, c2, c3 = (int(x) & _M64 for x in counter)
    k0, k1 = (int(x) & _M64 for x in key)
    for r in range(10):
        if r:
            k0 = (k0 + _PHILOX_WEYL[0]) & _M64
            k1 = (k1 + _PHILOX_WEYL[1]) & _M64
        p0 = _PHILOX_MUL[0] * c0
        p1 = _PHILOX_MUL[1] * c2
        c0, c1, c2, c3 = ((p1 >> 64) ^ c1 ^ k0, p1 & _M64,
                          (p0 >> 64) ^ c3 ^ k1, p0 & _M64)
    return c0, c1, c2, c3


def uniform_open(x):
    """Map a 64-bit integer to a double in (0, 1): ((x >> 11) + 1/2) 2^-53."""
    return ((x >> 11) + 0.5) * 2.0 ** -53


def box_muller(x0, x1):
    """Two independent standard normals from two 64-bit integers."""
    u1, u2 = uniform_open(x0), uniform_open(x1)
    r = math.sqrt(-2.0 * math.log(u1))
    return r * math.cos(2.0 * math.pi * u2), r * math.sin(2.0 * math.pi * u2)


def shell_modes(kmin, kmax):
    """Integer modes (kx, ky) with kmin <= |k| <= kmax on the half plane
    ky > 0 or (ky = 0 and kx > 0), ordered by ky, then kx.  The other half
    of the shell is the complex conjugate."""
    K = int(math.floor(kmax))
    out = []
    for ky in range(0, K + 1):
        for kx in range(-K, K + 1):
            if ky == 0 and kx <= 0:
                continue
            k2 = kx * kx + ky * ky
            if kmin * kmin <= k2 <= kmax * kmax:
                out.append((kx, ky))
    return out


def stirring_coefficients(modes, seed, step, amplitude, stream=0):
    """Complex coefficients (Fx_hat, Fy_hat) of every half-shell mode for one
    step: Fx_hat = A (z0 + i z1), Fy_hat = A (z2 + i z3), with z the four
    normals of one Philox block (counter (m, step, 0, 0), key (seed, stream))."""
    cx = np.zeros(len(modes), np.complex128)
    cy = np.zeros(len(modes), np.complex128)
    for m in range(len(modes)):
        r = philox4x64_10((m, step, 0, 0), (seed, stream))
        z0, z1 = box_muller(r[0], r[1])
        z2, z3 = box_muller(r[2], r[3])
        cx[m] = amplitude * complex(z0, z1)
        cy[m] = amplitude * complex(z2, z3)
    return cx, cy


def synthesize(modes, cx, cy, nx, ny):
    """Real-space force F_c(x, y) = sum over the full shell of
    F_c_hat(k) exp(2 pi i (kx x / Nx + ky y / Ny)), the -k half being the
    complex conjugate of the +k half.  Returns (2, Ny, Nx)."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    out = np.zeros((2, ny, nx))
    for (kx, ky), ax, ay in zip(modes, cx, cy):
        ph = np.exp(2j * np.pi * (kx * x / nx + ky * y / ny))
        out[0] += 2.0 * (ax * ph).real
        out[1] += 2.0 * (ay * ph).real
    return out


def synthesize_at(modes, cx, cy, nx, ny, xs, ys):
    """The same sum as `synthesize`, evaluated only at the nodes (xs[j],
    ys[j]) (for lattices too large to synthesise whole).  Returns (2, J)."""
    xs = np.asarray(xs, np.float64)
    ys = np.asarray(ys, np.float64)
    out = np.zeros((2, xs.size))
    for (kx, ky), ax, ay in zip(modes, cx, cy):
        ph = np.exp(2j * np.pi * (kx * xs / nx + ky * ys / ny))
        out[0] += 2.0 * (ax * ph).real
        out[1] += 2.0 * (ay * ph).real
    return out


class Stirring:
    """The per-step stirring field of a lattice: shell, amplitude, seed."""

    def __init__(self, nx, ny, kmin, kmax, amplitude, seed, stream=0):
        self.nx, self.ny = nx, ny
        self.modes = shell_modes(kmin, kmax)
        self.amplitude, self.seed, self.stream = amplitude, seed, stream

    def field(self, step):
        cx, cy = stirring_coefficients(self.modes, self.seed, step,
                                       self.amplitude, self.stream)
        return synthesize(self.modes, cx, cy, self.nx, self.ny)

    def field_at(self, step, xs, ys):
        """field(step)[:, ys, xs] without synthesising the whole lattice."""
        cx, cy = stirring_coefficients(self.modes, self.seed, step,
                                       self.amplitude, self.stream)
        return synthesize_at(self.modes, cx, cy, self.nx, self.ny, xs, ys)
