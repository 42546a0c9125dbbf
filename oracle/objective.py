"""Time-averaged objectives of a driven channel run and their parameters
(oracle for the gradient workload).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The dissertation computes no gradients; these definitions fix what the
adjoint of the step differentiates.  Parameters theta = (F_b, tau,
A_1..A_M): a uniform body force F_b along x, the relaxation time and the
amplitudes of a fixed stirring basis phi_m(x) = e_m cos(2 pi (kx x / Nx +
ky y / Ny) + phase_m) (a static form of the k-space stirring of Ch. 4,
"Model and Methods").  The driving force is F(x) = F_b x_hat +
sum_m A_m phi_m(x).

Objectives, averaged over the steps t = N/2 + 1 .. N and over fluid nodes,
from the fields of step t (post-stream moments, Ch. 3 LBM procedure step 3):

* current:      J^x, the charge current along the channel;
* dissipation:  pi^{kl} pi^{kl} with pi = T^{kl} - T_eq^{kl}(eps, u) the
                non-equilibrium stress (k, l over x, y, z), a proxy for the
                viscous dissipation.
"""
import numpy as np

from . import rlb


def basis_force(nx, ny, modes, amps, body):
    """F(x) = F_b x_hat + sum_m A_m e_m cos(2 pi (kx x/nx + ky y/ny) + phase),
    shape (3, ny, nx).  modes rows: (kx, ky, ex, ey, phase)."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    F = np.zeros((3, ny, nx))
    F[0] += body
    for (kx, ky, ex, ey, ph), A in zip(modes, amps):
        c = np.cos(2.0 * np.pi * (kx * x / nx + ky * y / ny) + ph)
        F[0] += A * ex * c
        F[1] += A * ey * c
    return F


def node_objective(F, G, kind, solid=None, cfl=1.0):
    """Mean over fluid nodes of the objective density of the current state."""
    Ft, Gt = rlb.stream(F, cfl), rlb.stream(G, cfl)
    fluid = np.ones(F.shape[1:], bool) if solid is None else ~solid
    if kind == "current":
        j = rlb.charge_current(Gt)[1]
    elif kind == "dissipation":
        T = rlb.energy_momentum(Ft)
        eps, u = rlb.landau(T, skip=solid)
        Teq = rlb.ideal_tensor(eps, u)
        pi = T[1:, 1:] - Teq[1:, 1:]
        j = np.einsum("klyx,klyx->yx", pi, pi)
    else:
        raise ValueError(kind)
    return j[fluid].mean()


def run_objectives(fields, nsteps, tau, body, modes, amps, kinds, solid=None, cfl=1.0):
    """J(theta) for each objective in `kinds` from one run: initialise from
    float32 fields, take nsteps steps with the basis-driven force and
    average each objective over steps N/2+1..N."""
    ny, nx = fields["eps"].shape
    F, G = rlb.initial_state(*(fields[k].astype(np.float64) for k in ("eps", "bx", "by", "n")))
    force = basis_force(nx, ny, modes, amps, body)
    acc = np.zeros(len(kinds))
    for t in range(nsteps):
        F, G = rlb.step(F, G, tau, cfl=cfl, force=force, solid=solid)
        if t + 1 > nsteps // 2:
            for j, kind in enumerate(kinds):
                acc[j] += node_objective(F, G, kind, solid, cfl)
    return acc / (nsteps - nsteps // 2)


def run_objective(fields, nsteps, tau, body, modes, amps, kind, solid=None, cfl=1.0):
    """J(theta) of one objective (see run_objectives)."""
    return float(run_objectives(fields, nsteps, tau, body, modes, amps, (kind,), solid, cfl)[0])


def fd_gradient(fields, nsteps, tau, body, modes, amps, kind, solid=None, rel=1e-4, which=None):
    """Central finite differences of run_objective with relative steps
    theta (1 +- rel).  Returns an array over (F_b, tau, A_1..A_M) (entries
    not in `which` are NaN)."""
    theta = np.concatenate([[body, tau], np.asarray(amps, np.float64)])
    out = np.full(theta.shape, np.nan)
    idx = range(len(theta)) if which is None else which
    for i in idx:
        h = rel * theta[i]
        vals = []
        for sgn in (+1, -1):
            th = theta.copy()
            th[i] += sgn * h
            vals.append(run_objective(fields, nsteps, th[1], th[0], modes, th[2:], kind, solid))
        out[i] = (vals[0] - vals[1]) / (2 * h)
    return out
