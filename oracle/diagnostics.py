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


# --------------------------------------------------------------------------
# Current-density fluctuations (Ch. 5, "Model and Methods": j(t) at the
# outflow border, j(x) along the sampling region, and their spectra)
# --------------------------------------------------------------------------
def column_current(fields, x):
    """j at column x: the charge current J^x averaged over the column's
    nodes (solid nodes count as zero), from a dict of fields."""
    return float(np.mean(fields["Jx"][:, x]))


def power_spectrum(series):
    """One-sided power spectrum of the fluctuations of a real series s of
    length n: P(k) = |sum_t (s_t - mean s) exp(-2 pi i k t / n)|^2 / n^2 for
    k = 0 .. n // 2, evaluated as the plain sum (no FFT)."""
    s = np.asarray(series, np.float64)
    n = s.size
    d = s - s.mean()
    t = np.arange(n)
    out = np.empty(n // 2 + 1)
    for k in range(n // 2 + 1):
        ph = 2.0 * np.pi * ((k * t) % n) / n
        out[k] = (np.dot(d, np.cos(ph)) ** 2 + np.dot(d, np.sin(ph)) ** 2) / float(n) ** 2
    return out


# --------------------------------------------------------------------------
# Part I analysis (Ch. 4, "Model and Methods" and "Results"): velocities
# filtered to the inertial range, E(k) averaged over decorrelated samples,
# and the power-law slope of the inertial range
# --------------------------------------------------------------------------
def filtered_velocity(bx, by, k_cut):
    """The velocity with its driven range removed: beta keeps only the
    Fourier modes with |k| < k_cut (integer wave numbers, numpy.fft
    frequencies).  Returns (bx_f, by_f, mean |beta_f|, rms |beta_f|)."""
    ny, nx = bx.shape
    kx = np.fft.fftfreq(nx, 1.0 / nx)
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    keep = (kx[None, :] ** 2 + ky[:, None] ** 2) < k_cut ** 2
    fx = np.real(np.fft.ifft2(np.fft.fft2(bx) * keep))
    fy = np.real(np.fft.ifft2(np.fft.fft2(by) * keep))
    speed = np.sqrt(fx * fx + fy * fy)
    return fx, fy, float(speed.mean()), float(np.sqrt((speed * speed).mean()))


def spectrum_average(samples):
    """Mean and standard error of E(k) over M samples taken a
    decorrelation stride apart: samples (M, K) -> (mean (K,), stderr (K,)),
    stderr = sqrt(sum_m (E_m - mean)^2 / (M (M - 1)))."""
    s = np.asarray(samples, np.float64)
    m = s.shape[0]
    mean = s.mean(axis=0)
    err = np.sqrt(((s - mean) ** 2).sum(axis=0) / (m * (m - 1))) if m > 1 else np.zeros_like(mean)
    return mean, err


def power_law_fit(k, E):
    """Least-squares fit of log E = a + slope log k; returns (slope, a)."""
    x = np.log(np.asarray(k, np.float64))
    y = np.log(np.asarray(E, np.float64))
    A = np.stack([x, np.ones_like(x)], axis=1)
    (slope, a), *_ = np.linalg.lstsq(A, y, rcond=None)
    return float(slope), float(a)
