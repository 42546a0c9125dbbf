"""Seeded synthetic inputs for the RLB workloads.

This module holds input recipes only (initial fields, obstacle positions,
lattice-size draws, stirring-basis draws): none of the method's arithmetic.
Both the HIP path and the FP64 oracle are fed from here so that they start
from bit-identical inputs.  Every array is float32 (the library's input type)
unless stated; the oracle widens to float64.

Workloads (sizes of the dissertation's runs, Ch. 4 and Ch. 5; the data of
those runs is not public, so these synthetic inputs stand in for them):

* shear wave   64 x 64 periodic, eps = 1, n = 0.1,
               beta_x = 0.01 sin(2 pi y / 64), tau = 0.8
* forced 1024  1024^2 periodic, rest, tau = 0.55, shell 7 <= |k| <= 9,
               amplitude 1e-5, seed 2205
* forced 4096  4096^2 periodic, rest, tau = 0.52, shell 31 <= |k| <= 33,
               amplitude 5e-6, seed 4658
* channels     64 channel lattices W ~ U{256..2048}, H ~ U{128..512}, walls,
               body force 1e-6 along x, tau = 0.8, discs of radius 6 at area
               fraction 1 / 5 / 10 % (index mod 3), seed 2022
* adjoint      512 x 256 channel, 5 % discs, seed 7, 2000 steps, K = 100
"""
import math

import numpy as np

SHEAR = dict(nx=64, ny=64, tau=0.8, amp=0.01, eps=1.0, n=0.1, steps=1000)
FORCED_1024 = dict(nx=1024, ny=1024, tau=0.55, kmin=7.0, kmax=9.0,
                   amplitude=1e-5, seed=2205, eps=1.0, n=0.1, steps=20000)
FORCED_4096 = dict(nx=4096, ny=4096, tau=0.52, kmin=31.0, kmax=33.0,
                   amplitude=5e-6, seed=4658, eps=1.0, n=0.1, steps=50000)
CHANNELS = dict(count=64, wmin=256, wmax=2048, hmin=128, hmax=512,
                body_force=1e-6, tau=0.8, radius=6.0,
                fractions=(0.01, 0.05, 0.10), seed=2022, eps=1.0, n=0.1)
ADJOINT = dict(nx=512, ny=256, fraction=0.05, radius=6.0, seed=7, tau=0.8,
               body_force=1e-6, steps=2000, checkpoint=100, eps=1.0, n=0.1,
               nmodes=32, kmin=7.0, kmax=9.0, mode_amplitude=1e-6)

# Part II channel (Ch. 5 "Model and Methods"): a 40 x 10 um sample on a
# 1024 x 256 lattice (spacing 0.038 um), flow entering at 0.1 v_F (lattice
# speed 1 = v_F) through the inlet column, periodic lateral borders, one or
# two rigid impurities of diameter 0.5 um (radius 0.25 / 0.038 nodes) in the
# obstruction region near the inlet, the second one behind and to the side
# of the first at a chosen separation.  tau is chosen (the paper's graphene
# viscosity is below the scheme's interpolation viscosity at cfl = 1):
# tau = 0.6 gives Re = U D / nu_eff = 0.1 * 13.2 / 0.075 = 17.5, near the
# paper's 6.4 - 12.7, and the run starts from the uniform inflow state (an
# impulsive start from rest, or tau <= 0.55, is not stable with these
# borders).
PART2 = dict(nx=1024, ny=256, tau=0.6, eps=1.0, n=0.1, beta_in=0.1, eps_out=1.0,
             spacing_um=0.038, diameter_um=0.5, first=(128.0, 128.0), angle_deg=25.0,
             separations_um=(1.68, 2.34, 3.38, 6.02, 8.39), steps=20000)


def part2_discs(separation_um=None, angle_deg=None, cfg=PART2):
    """[(x, y, r)] of the Part II impurities: the first at cfg['first'], the
    second (if a separation in um is given) at that distance, rotated
    angle_deg from the flow direction."""
    r = 0.5 * cfg["diameter_um"] / cfg["spacing_um"]
    x0, y0 = cfg["first"]
    out = [(x0, y0, r)]
    if separation_um is not None:
        a = np.deg2rad(cfg["angle_deg"] if angle_deg is None else angle_deg)
        d = separation_um / cfg["spacing_um"]
        out.append((x0 + d * np.cos(a), y0 + d * np.sin(a), r))
    return out


def uniform(nx, ny, eps=1.0, n=0.1):
    """Fluid at rest: eps, beta_x, beta_y, n arrays (Ny, Nx) float32."""
    z = np.zeros((ny, nx), np.float32)
    return dict(eps=z + np.float32(eps), bx=z.copy(), by=z.copy(), n=z + np.float32(n))


def shear_wave(nx=64, ny=64, amp=0.01, eps=1.0, n=0.1):
    """beta_x = amp sin(2 pi y / ny), uniform eps and n."""
    f = uniform(nx, ny, eps, n)
    y = np.arange(ny, dtype=np.float64)[:, None]
    f["bx"] = np.broadcast_to(amp * np.sin(2 * np.pi * y / ny), (ny, nx)).astype(np.float32)
    return f


def random_fields(nx, ny, seed, beta=0.05, deps=0.05, dn=0.02, eps=1.0, n=0.1):
    """Smooth-ish random fields for parity tests: a few random Fourier modes
    per field with the given amplitudes around (eps, 0, 0, n)."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)

    def field(a):
        out = np.zeros((ny, nx))
        for _ in range(4):
            kx, ky = rng.integers(-3, 4, size=2)
            ph = rng.uniform(0, 2 * np.pi)
            out += np.cos(2 * np.pi * (kx * x / nx + ky * y / ny) + ph)
        return a * out / 4.0

    return dict(eps=(eps + field(deps)).astype(np.float32),
                bx=field(beta).astype(np.float32),
                by=field(beta).astype(np.float32),
                n=(n + field(dn)).astype(np.float32))


def boosted(nx, ny, bx, by, eps=1.0, n=0.1):
    """Uniform flow at 3-velocity (bx, by)."""
    f = uniform(nx, ny, eps, n)
    f["bx"][:] = np.float32(bx)
    f["by"][:] = np.float32(by)
    return f


def disc_count(nx, ny, radius, fraction):
    """Number of discs for a target area fraction of the fluid region
    between the walls: round(fraction Nx (Ny - 2) / (pi r^2))."""
    return int(round(fraction * nx * (ny - 2) / (math.pi * radius * radius)))


def channel_discs(nx, ny, radius, fraction, seed, stream=0):
    """Disc centres uniform in [0, Nx) x [1, Ny - 1), overlaps allowed.
    Returns an (m, 3) float64 array of (cx, cy, r)."""
    rng = np.random.default_rng([seed, stream])
    m = disc_count(nx, ny, radius, fraction)
    cx = rng.uniform(0.0, nx, size=m)
    cy = rng.uniform(1.0, ny - 1.0, size=m)
    return np.stack([cx, cy, np.full(m, float(radius))], axis=1)


def channel_batch(count=64, seed=2022, wmin=256, wmax=2048, hmin=128, hmax=512,
                  radius=6.0, fractions=(0.01, 0.05, 0.10)):
    """Sizes and disc lists of the batched channel workload."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        w = int(rng.integers(wmin, wmax + 1))
        h = int(rng.integers(hmin, hmax + 1))
        frac = fractions[b % len(fractions)]
        out.append(dict(nx=w, ny=h, fraction=frac,
                        discs=channel_discs(w, h, radius, frac, seed, stream=b + 1)))
    return out


def stirring_basis(nx, ny, nmodes=32, kmin=7.0, kmax=9.0, seed=7):
    """Fixed stirring basis for the adjoint workload: modes m = 0..nmodes-1
    with integer (kx, ky), kmin <= |k| <= kmax, unit in-plane direction e_m
    and phase phi_m.  Basis field phi_m(x) = e_m cos(2 pi (kx x / Nx + ky y /
    Ny) + phi_m).  Returns (nmodes, 5) float64 rows (kx, ky, ex, ey, phi)."""
    rng = np.random.default_rng([seed, 99])
    K = int(kmax)
    cand = [(kx, ky) for ky in range(0, K + 1) for kx in range(-K, K + 1)
            if kmin * kmin <= kx * kx + ky * ky <= kmax * kmax and (ky > 0 or kx > 0)]
    pick = rng.choice(len(cand), size=nmodes, replace=False)
    rows = []
    for p in pick:
        kx, ky = cand[p]
        a = rng.uniform(0, 2 * np.pi)
        rows.append((kx, ky, math.cos(a), math.sin(a), rng.uniform(0, 2 * np.pi)))
    return np.array(rows, np.float64)
