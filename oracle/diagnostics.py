"""Turbulence diagnostics (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Ch. 2, "Turbulence": the energy spectrum E(k) = dE/dk with the spectral
energy density 1/2 <|v~(k)|^2> averaged over directions, and the enstrophy
Z = int |curl u|^2.
"""
import numpy as np


def energy_spectrum(bx, by, kmax=None):
    """E(k) for integer shells k - 1/2 <= |k| < k + 1/2 (k = 0, 1, ...):
    1/2 sum |v_hat(k)|^2 / (Nx Ny)^2 with numpy.fft's unnormalised forward
    transform."""
    ny, nx = bx.shape
    fx = np.fft.fft2(bx)
    fy = np.fft.fft2(by)
    p = 0.5 * (np.abs(fx) ** 2 + np.abs(fy) ** 2) / float(nx * ny) ** 2
    kx = np.fft.fftfreq(nx, 1.0 / nx)
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    kk = np.sqrt(kx[None, :] ** 2 + ky[:, None] ** 2)
    shell = np.floor(kk + 0.5).astype(int)
    if kmax is None:
        kmax = min(nx, ny) // 2
    return np.bincount(shell.ravel(), weights=p.ravel(), minlength=kmax + 1)[:kmax + 1]


def vorticity(bx, by):
    """omega = d_x beta_y - d_y beta_x by periodic central differences."""
    dby_dx = 0.5 * (np.roll(by, -1, axis=1) - np.roll(by, 1, axis=1))
    dbx_dy = 0.5 * (np.roll(bx, -1, axis=0) - np.roll(bx, 1, axis=0))
    return dby_dx - dbx_dy


def enstrophy(bx, by):
    """Z = sum over nodes of omega^2."""
    return float((vorticity(bx, by) ** 2).sum())
