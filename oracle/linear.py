"""Linearised single-mode update matrix (oracle, for the hydrodynamic pins).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Around a uniform rest state (eps0, u = (1,0,0,0)) a small perturbation
dF ~ exp(i k.x) of the energy-momentum populations evolves, to first order,
as dF(t+1) = M(k) dF(t) with

    M(k) = [I - (1/tau) (I - E)] S(k)

(stream, then collide: the state is the post-collision population),

built here directly from the definitions, independently of `rlb.step`:

* S(k) = diag(s_i(k)), the Fourier symbol of the bilinear pull of direction
  i (Ch. 3, linear interpolation of off-lattice streaming);
* the Anderson-Witting rate (u^0 - u.v_i)/tau is 1/tau at rest; its
  perturbation multiplies F - F_eq, which vanishes at rest;
* E is the linearised equilibrium: d(F_eq,i) = w_i (dT^{00} + 3 v_i.dT^{0.})
  because the second-order coefficient (15/2)(T_eq^{kl} - delta^{kl}
  T_eq^{00}/3) is quadratic in u (Ch. 3, eqs. stressEnergyT, rel_pdf_exp_coef).
"""
import numpy as np

from .velocity_set import velocity_set


def momentum_set(planar=False):
    """(v, w, c1): the momenta, weights and the first-order equilibrium
    coefficient (3 for the 3D set, 2 for the planar set)."""
    if planar:
        from .planar import V, W
        return V, W, 2.0
    v, w, _ = velocity_set()
    return v, w, 3.0


def stream_symbol(k, cfl=1.0, planar=False):
    """s_i(k) = sum over the 4 bilinear taps of weight * exp(-i k.offset):
    along each axis the displacement |d| = m + a has taps m and m + 1 cells
    upstream with weights 1 - a and a."""
    v, _, _ = momentum_set(planar)
    s = np.zeros(v.shape[0], np.complex128)
    for i in range(v.shape[0]):
        f = 1.0 + 0j
        for ax_, kk in ((0, k[0]), (1, k[1])):
            d = cfl * v[i, ax_]
            sg, m = np.sign(d), np.floor(abs(d))
            a = abs(d) - m
            f *= np.exp(-1j * kk * sg * m) * ((1 - a) + a * np.exp(-1j * kk * sg))
        s[i] = f
    return s


def update_matrix(k, tau, cfl=1.0, planar=False):
    v, w, c1 = momentum_set(planar)
    q = v.shape[0]
    E = w[:, None] * (1.0 + c1 * v @ v.T)             # E_ij = w_i (1 + c1 v_i.v_j)
    C = np.eye(q) - (np.eye(q) - E) / tau
    return C @ np.diag(stream_symbol(k, cfl, planar))


def hydrodynamic_modes(k, tau, cfl=1.0, planar=False):
    """Return (lambda_shear, lambda_sound) for a wavevector k.  The shear mode
    is the eigenvector with the largest transverse momentum weight, the sound
    mode the one (Im lambda > 0) with the largest energy weight."""
    v, _, _ = momentum_set(planar)
    M = update_matrix(k, tau, cfl, planar)
    lam, vec = np.linalg.eig(M)
    kh = np.array([k[0], k[1], 0.0]) / np.linalg.norm(k)
    th = np.array([-kh[1], kh[0], 0.0])
    trans = np.abs(vec.T @ (v @ th))                  # |sum_i dF_i v_i.t|
    energy = np.abs(vec.sum(axis=0))                  # |sum_i dF_i|
    norm = np.linalg.norm(vec, axis=0)
    i_shear = int(np.argmax(trans / norm * (np.abs(lam) > 0.5)))
    cand = (lam.imag > 0) & (np.abs(lam) > 0.5)
    i_sound = int(np.argmax(energy / norm * cand))
    return lam[i_shear], lam[i_sound]
