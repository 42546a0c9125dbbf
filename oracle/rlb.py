"""The relativistic lattice-Boltzmann step, written out plainly (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

State: two families of 26 populations on an Ny x Nx lattice (one z node),
float64, unshifted, arrays of shape (26, Ny, Nx) indexed [i][y][x]:

* F_i carries energy and momentum, T^{mu nu} = sum_i F_i v_i^mu v_i^nu
  (Ch. 3, eq. energyMomentumIntegral, with the quadrature weight absorbed
  into F_i as in Ch. 3, "The Standard/Classical LBM");
* G_i carries charge, J^mu = sum_i G_i v_i^mu.  The dissertation has no
  charge distribution; it is added with the reading documented at
  `equilibrium_G`.

One step follows the LBM procedure of Ch. 3 (stream, moments, equilibrium,
collide), with the relativistic pieces of Ch. 3 "Relativistic Lattice
Boltzmann" / "Boltzmann to Lattice Boltzmann" and the driving term of Ch. 4
(eq. forceTerm, Appendix "Discrete the Forcing Term").  Lattice units:
dx = 1, dt = cfl * dx, tau is the relaxation time in time steps.
"""
import numpy as np

from .velocity_set import velocity_set, four_velocity, P1, P2

V, W, OPP = velocity_set()
VMU = four_velocity(V)                      # (26, 4): v_i^mu = (1, v_i)
METRIC = np.diag([1.0, -1.0, -1.0, -1.0])   # g_{mu nu}, Ch. 2 (Minkowski)
Q = V.shape[0]


class LandauError(ArithmeticError):
    """Landau matching found no timelike eigenvector with eps > 0."""


# --------------------------------------------------------------------------
# Streaming (Ch. 3, LBM procedure step 2; "linear interpolation scheme")
# --------------------------------------------------------------------------
def stream(F, cfl=1.0, v=None):
    """Pull-stream every population along its in-plane displacement.

    Population i moves by delta_i = cfl * (v_ix, v_iy) per step.  The momentum
    set is off-lattice, so the value arriving at node x is the bilinear
    interpolation of the pre-stream field at the departure point x - delta_i,
    between the two lattice nodes that bracket it along each axis: with
    |delta| = m + a (m whole cells, 0 <= a < 1), the taps sit m and m + 1
    cells upstream with weights 1 - a and a (for cfl <= 1, m = 0 except a
    displacement of exactly one cell; cfl up to 2 reaches two cells, the
    paper's time steps giving cfl = dt / dx up to 1.25, Ch. 4 "Model and
    Methods").  The lattice has one z node, so the z displacement is the
    identity.
    Borders are periodic in x and y (walls are solid nodes, and open x
    borders overwrite their columns after the update, see `step`).  `v`
    (Q, 3) selects another momentum set (default: the 26 directions).
    """
    V = globals()["V"] if v is None else v
    if not (0.0 < cfl <= 2.0):
        raise ValueError("the bilinear pull supports 0 < cfl <= 2")
    out = np.empty_like(F)
    for i in range(F.shape[0]):
        dx, dy = cfl * V[i, 0], cfl * V[i, 1]
        sx, sy = int(np.sign(dx)), int(np.sign(dy))
        mx, my = int(np.floor(abs(dx))), int(np.floor(abs(dy)))
        ax, ay = abs(dx) - mx, abs(dy) - my
        f = np.roll(F[i], (my * sy, mx * sx), axis=(0, 1))   # F(x - m s): the nearer taps
        f_x = np.roll(f, sx, axis=1)        # one cell further along x
        f_y = np.roll(f, sy, axis=0)        # f(x, y - sy)
        f_xy = np.roll(f_x, sy, axis=0)     # f(x - sx, y - sy)
        out[i] = ((1 - ax) * (1 - ay) * f + ax * (1 - ay) * f_x
                  + (1 - ax) * ay * f_y + ax * ay * f_xy)
    return out


# --------------------------------------------------------------------------
# Moments (Ch. 3, eq. energyMomentumIntegral and the T^{mu nu} matrix)
# --------------------------------------------------------------------------
def energy_momentum(F, v=None):
    """T^{mu nu}(x) = sum_i F_i v_i^mu v_i^nu, shape (4, 4, Ny, Nx); `v`
    selects another momentum set."""
    vmu = VMU if v is None else four_velocity(v)
    return np.einsum("im,in,iyx->mnyx", vmu, vmu, F)


def charge_current(G, v=None):
    """J^mu(x) = sum_i G_i v_i^mu, shape (4, Ny, Nx)."""
    vmu = VMU if v is None else four_velocity(v)
    return np.einsum("im,iyx->myx", vmu, G)


def third_moment(F):
    """M3^{abc} = sum_i F_i v_i^a v_i^b v_i^c (spatial), shape (3,3,3,Ny,Nx)."""
    return np.einsum("ia,ib,ic,iyx->abcyx", V, V, V, F)


# --------------------------------------------------------------------------
# Landau matching (Ch. 3 end of "Relativistic Lattice Boltzmann" and of
# "Boltzmann to Lattice Boltzmann"): u_mu T^{mu nu} = eps u^nu.
# --------------------------------------------------------------------------
def landau(T, skip=None):
    """Return (eps, u) with T^mu_nu u^nu = eps u^nu, u.u = 1, u^0 > 0.

    T^mu_nu = T^{mu lambda} g_{lambda nu}.  The eigenproblem is solved with
    LAPACK (numpy.linalg.eig) per node; eps is the largest real eigenvalue
    whose eigenvector is timelike (v^T g v > 0).  `skip` (bool Ny x Nx) marks
    nodes to leave out (solid nodes): they get eps = 0, u = (1, 0, 0, 0).
    Raises LandauError where no such eigenpair exists or eps <= 0.
    """
    ny, nx = T.shape[2:]
    A = np.moveaxis(T, (0, 1), (2, 3)) @ METRIC          # (Ny, Nx, 4, 4)
    if skip is not None:
        A = A.copy()
        A[skip] = np.diag([1.0, -1.0 / 3, -1.0 / 3, -1.0 / 3])
    lam, vec = np.linalg.eig(A)                          # columns = eigvecs
    vr = vec.real
    mnorm = np.einsum("yxmk,mn,yxnk->yxk", vr, METRIC, vr)
    scale = np.abs(lam).max(axis=-1, keepdims=True)
    # timelike with margin: for a unit (Euclidean) eigenvector, v^T g v > 1e-6
    # means |beta| < 1 - 5e-7; a lightlike beam has no rest frame.
    ok = (np.abs(lam.imag) <= 1e-9 * scale) & (np.abs(vec.imag).max(axis=2) <= 1e-9) \
        & (mnorm > 1e-6)
    score = np.where(ok, lam.real, -np.inf)
    k = np.argmax(score, axis=-1)
    if not np.all(np.isfinite(np.take_along_axis(score, k[..., None], -1))):
        raise LandauError("no timelike eigenvector")
    eps = np.take_along_axis(lam.real, k[..., None], -1)[..., 0]
    u = np.take_along_axis(vr, k[:, :, None, None].repeat(4, 2), -1)[..., 0]
    u = u / np.sqrt(np.take_along_axis(mnorm, k[..., None], -1))
    u = u * np.sign(u[..., :1])
    eps = np.where(skip, 0.0, eps) if skip is not None else eps
    if skip is not None:
        u[skip] = np.array([1.0, 0.0, 0.0, 0.0])
    fluid = ~skip if skip is not None else np.ones((ny, nx), bool)
    if np.any(eps[fluid] <= 0.0) or not np.all(np.isfinite(u)):
        raise LandauError("eps <= 0 or non-finite velocity")
    return eps, np.moveaxis(u, 2, 0)                     # u: (4, Ny, Nx)


def charge_density(J, u):
    """n = u_mu J^mu (Landau matching for the charge current)."""
    return np.einsum("m,myx,myx->yx", np.diag(METRIC), u, J)


def four_velocity_from_beta(bx, by):
    """u^mu = gamma (1, beta), gamma = (1 - beta^2)^(-1/2) (Ch. 3)."""
    g = 1.0 / np.sqrt(1.0 - bx * bx - by * by)
    return np.stack([g, g * bx, g * by, np.zeros_like(g)])


# --------------------------------------------------------------------------
# Equilibrium (Ch. 3, eqs. stressEnergyT, rel_pdf_exp, rel_pdf_exp_coef)
# --------------------------------------------------------------------------
def ideal_tensor(eps, u):
    """T_eq^{mu nu} = (eps + P) u^mu u^nu - P g^{mu nu}, P = eps / 3.

    The dissertation prints "+ P g" with g = diag(1,-1,-1,-1); the sign is
    read as "- P g" so that the rest frame gives diag(eps, P, P, P) with
    positive pressure (Appendix "Determination of the Equation of State":
    P = eps / 3).
    """
    P = eps / 3.0
    return ((eps + P) * u[:, None] * u[None, :]
            - P * METRIC[:, :, None, None])


def expansion_coefficients(T):
    """a^(0), a^(1), a^(2) of the angular expansion from the moments.

    Ch. 3, eq. rel_pdf_exp_coef: a^(n) = c_n * int f P^(n) with c_0 = 1,
    c_1 = 3, c_2 = 15/2 (alpha = 3; the radial integral and the quadrature
    weight are absorbed into the lattice moments, so int f P^(n) is
    T^{00}, T^{0i} and T^{ij} - delta_ij T^{00} / 3).
    """
    a0 = T[0, 0]
    a1 = 3.0 * T[0, 1:]
    a2 = 7.5 * (T[1:, 1:] - np.eye(3)[:, :, None, None] * T[0, 0] / 3.0)
    return a0, a1, a2


def from_coefficients(a0, a1, a2):
    """f_i = w_i sum_n P^(n)(v_i) a^(n) (Ch. 3, eq. rel_pdf_exp, n <= 2)."""
    return W[:, None, None] * (a0[None]
                               + np.einsum("ik,kyx->iyx", P1(V), a1)
                               + np.einsum("ikl,klyx->iyx", P2(V), a2))


def equilibrium_F(eps, u):
    """F_eq,i: the truncated Juttner equilibrium for energy-momentum."""
    return from_coefficients(*expansion_coefficients(ideal_tensor(eps, u)))


def equilibrium_G(n, u):
    """G_eq,i = w_i (a^(0) + a^(1) . v_i) with a^(0) = n u^0, a^(1) = 3 n u.

    Reading: the charge distribution is expanded like F to first order, with
    the equilibrium current J_eq^mu = n u^mu (Landau matching n = u_mu J^mu).
    """
    a0 = n * u[0]
    a1 = 3.0 * n[None] * u[1:]
    return W[:, None, None] * (a0[None] + np.einsum("ik,kyx->iyx", P1(V), a1))


# --------------------------------------------------------------------------
# Collision (Ch. 3, eq. boltzmanneq_rel: Anderson-Witting rate p.u / tau_R)
# --------------------------------------------------------------------------
def collision_rate(u, tau, v=None):
    """omega_i = p^mu u_mu / (p^0 tau) = (u^0 - u . v_i) / tau; tau is a
    number or an (Ny, Nx) array (per-node relaxation time)."""
    vmu = VMU if v is None else four_velocity(v)
    return np.einsum("im,m,myx->iyx", vmu, np.diag(METRIC), u) / tau


def temperature(eps):
    """T from the massless ideal-gas energy density eps = 3 T^4 / pi^2
    (Ch. 3, "Boltzmann to Lattice Boltzmann", natural units)."""
    return (np.pi ** 2 * np.asarray(eps, np.float64) / 3.0) ** 0.25


class ViscosityRelaxation:
    """Per-node relaxation time from a fixed eta/s (Ch. 3, "Relativistic
    Lattice Boltzmann"): tau_R = 5 (eta/s) / T, in steps of length dt,
        tau(x) = 5 (eta/s) / (T(x) dt),
    with T(x) from the node's Landau energy density.  Passed to `step` in
    place of a constant tau."""

    def __init__(self, eta_s, dt):
        if not (eta_s > 0 and dt > 0):
            raise ValueError("eta/s and dt must be positive")
        self.eta_s, self.dt = float(eta_s), float(dt)

    def __call__(self, eps):
        return 5.0 * self.eta_s / (temperature(eps) * self.dt)


# --------------------------------------------------------------------------
# Driving term (Ch. 4 eq. forceTerm; Appendix "Discrete the Forcing Term")
# --------------------------------------------------------------------------
def driving_term(Ft, force):
    """Phi_i, the bracket of the projected driving term with T_0 = 1.

    Phi_i = 3/12 F.M1 - 1/2 (F.v_i) M0 + 5/4 F_a v_ib v_ic M3^{abc}
            - 5/2 (F.v_i)(v_i.M1)
    with M0 = sum F~, M1^k = sum F~ v^k, M3^{abc} = sum F~ v^a v^b v^c taken
    over the post-stream (pre-collision) populations F~.  `force` has shape
    (3, Ny, Nx) (the z component is zero for the 2D workloads).
    """
    M0 = Ft.sum(axis=0)
    M1 = np.einsum("ik,iyx->kyx", V, Ft)
    M3 = third_moment(Ft)
    FM1 = np.einsum("kyx,kyx->yx", force, M1)
    Fv = np.einsum("ik,kyx->iyx", V, force)
    vM1 = np.einsum("ik,kyx->iyx", V, M1)
    FM3vv = np.einsum("ayx,ib,ic,abcyx->iyx", force, V, V, M3)
    return (3.0 / 12.0) * FM1[None] - 0.5 * Fv * M0[None] \
        + 1.25 * FM3vv - 2.5 * Fv * vM1


# --------------------------------------------------------------------------
# The full step
# --------------------------------------------------------------------------
def step(F, G, tau, cfl=1.0, force=None, solid=None, collision="aw", open_x=None):
    """One time step: stream, (bounce-back), moments, Landau, equilibrium,
    collide and drive.  Returns the post-collision (F, G).

    * solid nodes (Ch. 5 "Model and Methods", bounce-back at impurities):
      F'_i = F~_opp(i), G'_i = G~_opp(i); no collision, no force there.
      Fluid nodes stream from solid nodes like from any other node.
    * update (Ch. 4, "The Driving Term"): f* = f + dt C[f] + dt F.grad f,
      read as F'_i = F~_i - omega_i (F~_i - F_eq,i) - w_i Phi_i, the sign
      chosen so the flow accelerates along +F.
    * collision="bgk" replaces omega_i by 1/tau (the classical rate of
      Ch. 3 eq. lbe_coll_term); used only as a negative control.
    * tau: a constant, or a ViscosityRelaxation giving tau(x) from the
      node's Landau energy density.
    * open_x = (beta_x, beta_y, n_in, eps_out): open x borders (Ch. 5
      "Model and Methods": a fixed velocity enters along the inflow border,
      the lateral borders are periodic); see `open_borders`.
    """
    Ft = stream(F, cfl)
    Gt = stream(G, cfl)
    T = energy_momentum(Ft)
    J = charge_current(Gt)
    eps, u = landau(T, skip=solid)
    n = charge_density(J, u)
    Feq = equilibrium_F(eps, u)
    Geq = equilibrium_G(n, u)
    if callable(tau):
        e = eps if solid is None else np.where(solid, 1.0, eps)   # solid nodes do not collide
        tau = tau(e)
    if collision == "aw":
        om = collision_rate(u, tau)
    elif collision == "bgk":
        om = np.broadcast_to(1.0 / tau, Ft.shape)
    else:
        raise ValueError(collision)
    Fn = Ft - om * (Ft - Feq)
    Gn = Gt - om * (Gt - Geq)
    if force is not None:
        Fn = Fn - W[:, None, None] * driving_term(Ft, force)
    if solid is not None:
        Fn[:, solid] = Ft[OPP][:, solid]
        Gn[:, solid] = Gt[OPP][:, solid]
    if open_x is not None:
        open_borders(Fn, Gn, *open_x)
    return Fn, Gn


def open_borders(F, G, bx, by, n_in, eps_out):
    """Open x borders, applied in place to a post-collision state:

    * velocity inlet, column x = 0: F_eq, G_eq at the prescribed 3-velocity
      (bx, by) and charge density n_in, with the energy density of the
      adjacent column x = 1;
    * pressure outlet, column x = Nx-1: F_eq, G_eq at the prescribed energy
      density eps_out (pressure eps_out / 3), with the velocity and charge
      density of the adjacent column x = Nx-2.

    The adjacent columns' eps, u and n come from Landau matching of their
    (post-collision) moments.  Streaming stays periodic: the wrapped values
    only ever reach the two border columns, which this overwrites."""
    ny = F.shape[1]
    T1 = energy_momentum(F[:, :, 1:2])
    e1, _ = landau(T1)
    u_in = four_velocity_from_beta(np.full((ny, 1), float(bx)), np.full((ny, 1), float(by)))
    F[:, :, 0] = equilibrium_F(e1, u_in)[:, :, 0]
    G[:, :, 0] = equilibrium_G(np.full((ny, 1), float(n_in)), u_in)[:, :, 0]
    Tm = energy_momentum(F[:, :, -2:-1])
    Jm = charge_current(G[:, :, -2:-1])
    _, um = landau(Tm)
    nm = charge_density(Jm, um)
    F[:, :, -1] = equilibrium_F(np.full((ny, 1), float(eps_out)), um)[:, :, 0]
    G[:, :, -1] = equilibrium_G(nm, um)[:, :, 0]


def initial_state(eps, bx, by, n):
    """F = F_eq(eps, u), G = G_eq(n, u) from initial fields (Ch. 3, LBM
    procedure step 1).  Inputs are arrays (Ny, Nx); beta is the 3-velocity."""
    u = four_velocity_from_beta(np.asarray(bx, np.float64), np.asarray(by, np.float64))
    eps = np.asarray(eps, np.float64)
    n = np.asarray(n, np.float64)
    return equilibrium_F(eps, u), equilibrium_G(n, u)


def fields(F, G, cfl=1.0, solid=None):
    """Macroscopic fields at the current step: the populations are streamed,
    then moments and Landau matching are taken (Ch. 3, LBM procedure step 3;
    no collision).  Solid nodes report zeros."""
    Ft, Gt = stream(F, cfl), stream(G, cfl)
    T = energy_momentum(Ft)
    J = charge_current(Gt)
    eps, u = landau(T, skip=solid)
    n = charge_density(J, u)
    out = {"eps": eps, "beta_x": u[1] / u[0], "beta_y": u[2] / u[0], "n": n,
           "T00": T[0, 0], "T0x": T[0, 1], "T0y": T[0, 2],
           "Txx": T[1, 1], "Txy": T[1, 2], "Tyy": T[2, 2],
           "J0": J[0], "Jx": J[1], "Jy": J[2]}
    if solid is not None:
        for k in out:
            out[k] = np.where(solid, 0.0, out[k])
    return out


def totals(F, G):
    """Global E = sum F, P^x = sum F v_x, P^y = sum F v_y, Q = sum G over all
    nodes and directions (energy, momentum and charge, Ch. 2: d_mu T^{mu nu}
    = 0 and current conservation)."""
    return np.array([F.sum(), np.einsum("i,iyx->", V[:, 0], F),
                     np.einsum("i,iyx->", V[:, 1], F), G.sum()])


def force_injection(F, force, cfl=1.0, solid=None):
    """Energy and momentum the driving term injects in the next step:
    (sum_x F.T^{0.} / 6, sum_x F^x T^{00} / 6, sum_x F^y T^{00} / 6) over fluid
    nodes, from the post-stream moments."""
    Ft = stream(F, cfl)
    T = energy_momentum(Ft)
    fl = np.ones(T.shape[2:], bool) if solid is None else ~solid
    dE = (np.einsum("kyx,kyx->yx", force, T[0, 1:]) / 6.0)[fl].sum()
    dPx = (force[0] * T[0, 0] / 6.0)[fl].sum()
    dPy = (force[1] * T[0, 0] / 6.0)[fl].sum()
    return np.array([dE, dPx, dPy])
