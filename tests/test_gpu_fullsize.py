"""Parity at the workloads' full sizes, in the launch shapes the benchmark
times.  The oracle cannot run these lattices, but the step is local: with
cfl = 1 a node's new populations depend only on its 3 x 3 neighbourhood of
the previous state.  So the GPU's own state before one step is gathered
around sampled nodes, the FP64 oracle steps each patch (with its solid
nodes), and the patch centre is compared with the GPU's state after the
step.  Samples include lattice corners (periodic wrap), both sides of
64-node tile edges, wall rows and random nodes.  Covered: the forced 4096^2
headline (from rest, from a random flow, full set) and its variants (cfl
0.15625 and 1.25, the latter from 5 x 5 patches; per-node tau from eta/s;
the planar set, by its fields), the forced 1024^2 run after 200 steps, and
members of the 64-channel batch.  The 1024 x 256 Part II channel is small
enough for the oracle to run whole, every node compared.  The adjoint at
512 x 256 over 2000 steps is checked through properties that hold at any
size: its gradient along a random direction against a central difference
of its own forward objective, and invariance under the checkpoint
interval.  The widest rows the library accepts are sampled the same way
(column offsets at the top of their 32-bit range)."""
import json
import os

import numpy as np
import pytest

from oracle import forcing, geometry, planar, rlb
from paper_2205_04658_amd import workloads
from rlbtest import _folded_dirs, _full_dirs, compare, need_gpu, scales

pytestmark = pytest.mark.gpu

C = workloads.FORCED_4096
N = C["nx"]
TOL = 2e-8     # absolute, on populations of magnitude ~w_i eps ~ 0.05


def samples():
    fixed = [(0, 0), (N - 1, N - 1), (0, N - 1), (N - 1, 0), (63, 100), (64, 100),
             (127, 2047), (128, 2048), (2047, 1), (2048, N - 2), (4031, 3000), (4032, 3001)]
    rng = np.random.default_rng(4096)
    rand = list(zip(rng.integers(0, N, 52).tolist(), rng.integers(0, N, 52).tolist()))
    xs, ys = np.array([p[0] for p in fixed + rand]), np.array([p[1] for p in fixed + rand])
    return xs, ys


def oracle_order(full):
    """For each oracle direction: (library plane, share) -- folded planes
    hold both z mirrors, which stay equal, so each gets half."""
    dirs = _full_dirs() if full else _folded_dirs()
    out = []
    for v in rlb.V:
        for k, d in enumerate(dirs):
            if np.allclose(v[:2], d[:2]) and (np.isclose(v[2], d[2]) if full
                                              else np.isclose(abs(v[2]), d[2])):
                out.append((k, 1.0 if (full or v[2] == 0) else 0.5))
                break
    assert len(out) == 26
    return out


def to_oracle(p, order, ref):
    """Library planes (Q, ...) of shifted values -> oracle (26, ...) totals."""
    return np.stack([p[k] * s for k, s in order]) + rlb.W.reshape((26,) + (1,) * (p.ndim - 1)) * ref


def to_library(F, order, q, ref):
    out = np.zeros((q,) + F.shape[1:])
    for i, (k, _) in enumerate(order):
        out[k] += F[i] - rlb.W[i] * ref
    return out


def gather(planes, xs, ys, nx, ny, torch, r=1):
    """(Q, M, 2r+1, 2r+1) float64 patches around (xs, ys), periodic."""
    d = torch.arange(-r, r + 1, device=planes.device)
    iy = (torch.tensor(ys, device=planes.device)[:, None, None] + d[None, :, None]) % ny
    ix = (torch.tensor(xs, device=planes.device)[:, None, None] + d[None, None, :]) % nx
    return planes[:, iy, ix].double().cpu().numpy()


def at(planes, xs, ys, torch):
    return planes[:, torch.tensor(ys, device=planes.device),
                  torch.tensor(xs, device=planes.device)].double().cpu().numpy()


def sampled_step_error(lat, xs, ys, tau, force_at, full, eps_ref, n_ref, solid=None, cfl=1.0):
    """Take one GPU step of `lat`; return (max error F, max error G, largest
    one-step change) of the sampled nodes against the oracle patch step."""
    import torch
    nx, ny = lat.nx, lat.ny
    r = 2 if cfl > 1 else 1        # the two-cell stencil pulls from a 5 x 5 patch
    F0, G0 = lat.planes()
    pf, pg = gather(F0, xs, ys, nx, ny, torch, r), gather(G0, xs, ys, nx, ny, torch, r)
    del F0, G0
    lat.step(1)
    lat.sync()
    F1, G1 = lat.planes()
    got_f, got_g = at(F1, xs, ys, torch), at(G1, xs, ys, torch)
    del F1, G1
    q = pf.shape[0]
    order = oracle_order(full)
    err_f = err_g = change = 0.0
    for m in range(len(xs)):
        F = to_oracle(pf[:, m], order, eps_ref)
        G = to_oracle(pg[:, m], order, n_ref)
        w = 2 * r + 1
        fo = np.zeros((3, w, w))
        if force_at is not None:
            fo[0, r, r], fo[1, r, r] = force_at[0, m], force_at[1, m]
        sp = None
        if solid is not None:
            sp = solid[(ys[m] + np.arange(-r, r + 1))[:, None] % ny,
                       (xs[m] + np.arange(-r, r + 1))[None, :] % nx]
        Fn, Gn = rlb.step(F, G, tau, cfl=cfl, force=fo, solid=sp)
        want_f = to_library(Fn[:, r:r + 1, r:r + 1], order, q, eps_ref)[:, 0, 0]
        want_g = to_library(Gn[:, r:r + 1, r:r + 1], order, q, n_ref)[:, 0, 0]
        err_f = max(err_f, np.abs(got_f[:, m] - want_f).max())
        err_g = max(err_g, np.abs(got_g[:, m] - want_g).max())
        change = max(change, np.abs(want_f - pf[:, m, r, r]).max())
    print(f"max |gpu - oracle|: F {err_f:.3e}  G {err_g:.3e}; one-step change {change:.3e}")
    return err_f, err_g, change


@pytest.mark.parametrize("start,full,cfl,eta_s", [
    ("rest", False, 1.0, None), ("random", False, 1.0, None), ("random", True, 1.0, None),
    ("random", False, 0.15625, None), ("random", False, 1.25, None),
    ("random", False, 1.0, (0.007, 0.05))],
    ids=["workload_rest", "random_flow", "random_flow_full26", "random_flow_cfl_0_15625",
         "random_flow_cfl_1_25", "random_flow_eta_s"])
def test_headline_step_sampled(start, full, cfl, eta_s):
    """The 4096^2 stirred workload in the launch shape bench.py times, and
    its single-lattice variants: the paper's smallest and largest cfl
    (0.05 / 0.32 and 0.05 / 0.04, the latter a 5 x 5 pull) and per-node
    tau from eta/s."""
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import Lattice
    eps_ref, n_ref = C["eps"], C["n"]
    lat = Lattice(N, N, C["tau"], cfl=cfl, full26=full, eps_ref=eps_ref, n_ref=n_ref)
    if start == "rest":
        f = workloads.uniform(N, N, eps_ref, n_ref)
    else:
        f = workloads.random_fields(N, N, seed=C["seed"], beta=0.05)
    lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
    del f
    stir = (C["kmin"], C["kmax"], C["amplitude"], C["seed"])
    lat.set_stirring(*stir)
    tau = C["tau"]
    if eta_s is not None:
        lat.set_relaxation_eta_s(*eta_s)
        tau = rlb.ViscosityRelaxation(*eta_s)
    lat.set_launch_shape(*((4, 0, 16) if full else (2, 0, 16)))
    t0 = 20
    lat.step(t0)
    xs, ys = samples()
    force = forcing.Stirring(N, N, *stir).field_at(t0, xs, ys)   # (2, M)
    ef, eg, change = sampled_step_error(lat, xs, ys, tau, force, full, eps_ref, n_ref,
                                        cfl=cfl)
    assert ef < TOL and eg < TOL, (ef, eg)
    assert change > 10 * TOL          # the step moved the sampled populations


@pytest.mark.parametrize("full", [False, True], ids=["folded17", "full26"])
def test_widest_rows_step_sampled(full):
    """The widest rows the library accepts, 4 rows high (nx = 31,580,608
    folded, 20,648,832 full set: one row of state just under 2^32 bytes,
    so column offsets reach the top of their 32-bit range), forced by a
    k-shell stirring: sampled one-step parity at both ends of the row,
    around tile edges near the end, and in between."""
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import Lattice
    nx, ny = (20648832 if full else 31580608), 4
    eps_ref, n_ref = 1.0, 0.1
    lat = Lattice(nx, ny, 0.6, full26=full, eps_ref=eps_ref, n_ref=n_ref)
    f = workloads.uniform(nx, ny, eps_ref, n_ref)
    lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
    del f
    stir = (0.5, 1.5, 2e-4, 11)          # |k| = 1 and sqrt(2) (kmax < ny / 2)
    lat.set_stirring(*stir)
    lat.set_launch_shape(*((4, 0, 16) if full else (2, 0, 16)))
    t0 = 5
    lat.step(t0)
    xs = np.array([0, 1, 63, 64, 1000003, nx // 2 - 1, nx // 2, nx - 193, nx - 129, nx - 128,
                   nx - 65, nx - 64, nx - 63, nx - 2, nx - 1, nx - 1])
    ys = np.arange(len(xs)) % ny
    force = forcing.Stirring(nx, ny, *stir).field_at(t0, xs, ys)
    ef, eg, change = sampled_step_error(lat, xs, ys, 0.6, force, full, eps_ref, n_ref)
    assert ef < TOL and eg < TOL, (ef, eg)
    assert change > 10 * TOL


def test_planar_step_sampled():
    """The planar (2+1) set on the 4096^2 seeded random flow that bench.py
    times: one GPU step from the initial fields, then the fields at sampled
    nodes against the oracle's planar step of a 5 x 5 patch of the same
    float32 fields (a step, then the fields' own pull: two cells)."""
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import Lattice
    f = workloads.random_fields(N, N, seed=C["seed"], beta=0.01)
    lat = Lattice(N, N, C["tau"], planar=True, eps_ref=C["eps"], n_ref=C["n"])
    lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
    lat.step(1)
    lat.sync()
    xs, ys = samples()
    g = lat.fields()
    names = ("eps", "beta_x", "beta_y", "n")
    got = {k: g[k][torch.tensor(ys, device=g[k].device), torch.tensor(xs, device=g[k].device)]
           .double().cpu().numpy() for k in names}
    del g
    sc = scales(beta=0.05)
    worst = dict.fromkeys(names, 0.0)
    change = 0.0
    for m in range(len(xs)):
        iy = (ys[m] + np.arange(-2, 3))[:, None] % N
        ix = (xs[m] + np.arange(-2, 3))[None, :] % N
        F, G = planar.initial_state(*(f[k][iy, ix].astype(np.float64) for k in ("eps", "bx", "by", "n")))
        o0 = planar.fields(F, G)
        F, G = planar.step(F, G, C["tau"])
        o = planar.fields(F, G)
        for k in names:
            worst[k] = max(worst[k], abs(got[k][m] - o[k][2, 2]) / sc[k])
            change = max(change, abs(o[k][2, 2] - o0[k][2, 2]) / sc[k])
    print(f"planar 4096^2, max scaled field error over {len(xs)} nodes: {worst}; "
          f"one-step change {change:.3e}")
    assert max(worst.values()) < 1e-5, worst
    assert change > 1e-4              # the step moved the sampled fields


def test_part2_channel_full_size():
    """The Part II channel at its full 1024 x 256 size: two discs 3.38 um
    apart, velocity inlet and pressure outlet, in the launch shape the
    autotuner picks for it (8-row tiles).  Small enough for the oracle to
    run whole: after 4 steps from the inlet flow every node's fields,
    the border columns and the solid nodes included, against it."""
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import Lattice
    c = workloads.PART2
    nx, ny = c["nx"], c["ny"]
    discs = workloads.part2_discs(3.38)
    borders = (c["beta_in"], 0.0, c["n"], c["eps_out"])
    f = workloads.uniform(nx, ny, c["eps"], c["n"])
    f["bx"][:] = c["beta_in"]
    lat = Lattice(nx, ny, c["tau"], open_x=True, eps_ref=c["eps"], n_ref=c["n"])
    lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
    lat.add_disks(np.array(discs))
    lat.set_open_borders(*borders)
    lat.set_launch_shape(8, 0, 16)
    steps = 4
    lat.step(steps)
    lat.sync()
    solid = geometry.disc_mask(nx, ny, discs)
    F, G = rlb.initial_state(*(f[k].astype(np.float64) for k in ("eps", "bx", "by", "n")))
    for _ in range(steps):
        F, G = rlb.step(F, G, c["tau"], solid=solid, open_x=borders)
    o = rlb.fields(F, G, solid=solid)
    g = lat.fields()
    err = compare(g, o, scales(beta=0.1, n=0.1))
    print(f"Part II 1024 x 256 after {steps} steps, max scaled field error: {err}")
    assert max(err.values()) < 1e-5, err
    # the step moved the flow: the discs' wakes and the borders
    assert np.abs(o["beta_y"]).max() > 1e-3


def test_forced_1024_step_sampled_after_200_steps():
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import Lattice
    c = workloads.FORCED_1024
    n = c["nx"]
    lat = Lattice(n, n, c["tau"], eps_ref=c["eps"], n_ref=c["n"])
    f = workloads.uniform(n, n, c["eps"], c["n"])
    lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
    stir = (c["kmin"], c["kmax"], c["amplitude"], c["seed"])
    lat.set_stirring(*stir)
    lat.autotune(trials=2)
    t0 = 200
    lat.step(t0)
    rng = np.random.default_rng(1024)
    xs = np.concatenate([[0, n - 1, 63, 64, 511, 512], rng.integers(0, n, 42)])
    ys = np.concatenate([[n - 1, 0, 10, 11, 512, 513], rng.integers(0, n, 42)])
    force = forcing.Stirring(n, n, *stir).field_at(t0, xs, ys)
    ef, eg, change = sampled_step_error(lat, xs, ys, c["tau"], force, False, c["eps"], c["n"])
    assert ef < TOL and eg < TOL, (ef, eg)
    assert change > 10 * TOL


def test_batched_channels_step_sampled():
    """The 64-channel batch (walls, discs, body force) in the autotuned
    shape, from random flows: sampled nodes of several members, solid ones
    included."""
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import Batch
    c = workloads.CHANNELS
    lats = workloads.channel_batch(c["count"], c["seed"], c["wmin"], c["wmax"], c["hmin"],
                                   c["hmax"], c["radius"], c["fractions"])
    B = Batch([(d["nx"], d["ny"]) for d in lats], c["tau"], walls=True, eps_ref=c["eps"],
              n_ref=c["n"])
    for b, d in enumerate(lats):
        f = workloads.random_fields(d["nx"], d["ny"], seed=300 + b, beta=0.02)
        B[b].init_fields(f["eps"], f["bx"], f["by"], f["n"])
        B[b].add_disks(d["discs"])
    B.set_body_force(c["body_force"], 0.0)
    B.autotune(trials=1)
    B.step(10)
    B.sync()
    rng = np.random.default_rng(64)
    worst = [0.0, 0.0]
    for b in (0, 1, 2, 31, 63):
        lat, d = B[b], lats[b]
        nx, ny = d["nx"], d["ny"]
        solid = geometry.channel_mask(nx, ny, d["discs"])
        sx, sy = np.nonzero(solid[1:-1].T)               # a few disc nodes
        pick = rng.choice(len(sx), size=min(4, len(sx)), replace=False)
        xs = np.concatenate([[0, nx - 1, 63, 64, 5], sx[pick], rng.integers(0, nx, 8)])
        ys = np.concatenate([[0, ny - 1, 1, ny - 2, ny // 2], sy[pick] + 1, rng.integers(0, ny, 8)])
        # the batch steps every member: save, step the batch once, compare
        F0, G0 = lat.planes()
        pf, pg = gather(F0, xs, ys, nx, ny, torch), gather(G0, xs, ys, nx, ny, torch)
        del F0, G0
        B.step(1)
        B.sync()
        F1, G1 = lat.planes()
        got_f, got_g = at(F1, xs, ys, torch), at(G1, xs, ys, torch)
        del F1, G1
        order = oracle_order(False)
        for m in range(len(xs)):
            F = to_oracle(pf[:, m], order, c["eps"])
            G = to_oracle(pg[:, m], order, c["n"])
            fo = np.zeros((3, 3, 3))
            fo[0] = c["body_force"]
            sp = solid[(ys[m] + np.arange(-1, 2))[:, None] % ny, (xs[m] + np.arange(-1, 2))[None, :] % nx]
            Fn, Gn = rlb.step(F, G, c["tau"], force=fo, solid=sp)
            wf = to_library(Fn[:, 1:2, 1:2], order, 17, c["eps"])[:, 0, 0]
            wg = to_library(Gn[:, 1:2, 1:2], order, 17, c["n"])[:, 0, 0]
            worst[0] = max(worst[0], np.abs(got_f[:, m] - wf).max())
            worst[1] = max(worst[1], np.abs(got_g[:, m] - wg).max())
    print("batch max |gpu - oracle|:", worst)
    assert worst[0] < TOL and worst[1] < TOL, worst


ADJOINT512 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                          "adjoint512_oracle.json")


@pytest.mark.parametrize("kind", ["current", "dissipation"])
def test_adjoint_full_size_directional_derivative(kind):
    """512 x 256 channel, 2000 steps, checkpoints every 100, 32 modes, both
    objectives: the adjoint gradient along a seeded direction d equals the
    central difference (J(theta + h d) - J(theta - h d)) / 2h of the
    forward objective to 1e-3, and that of the FP64 oracle's runs (stored
    by tests/golden/make_golden.py) to 1e-3; the objective matches the
    oracle's to 1e-5; the gradient does not depend on the checkpoint
    interval."""
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import Lattice
    c = workloads.ADJOINT
    nx, ny = c["nx"], c["ny"]
    modes = workloads.stirring_basis(nx, ny, c["nmodes"], c["kmin"], c["kmax"], c["seed"])
    amps = np.full(c["nmodes"], c["mode_amplitude"])
    discs = workloads.channel_discs(nx, ny, c["radius"], c["fraction"], c["seed"])

    def run(fb, tau, a, K=c["checkpoint"], grad=True):
        lat = Lattice(nx, ny, tau, walls=True, eps_ref=c["eps"], n_ref=c["n"])
        f = workloads.uniform(nx, ny, c["eps"], c["n"])
        lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
        lat.add_disks(discs)
        return lat.adjoint_run(c["steps"], K, kind, modes, a, fb, grad=grad)

    J, g = run(c["body_force"], c["tau"], amps)
    J2, g2 = run(c["body_force"], c["tau"], amps, K=40)
    assert J2 == J
    np.testing.assert_array_equal(g2, g)
    theta = np.concatenate([[c["body_force"], c["tau"]], amps])
    d = np.random.default_rng(5).normal(size=theta.size) * np.abs(theta)
    h = 1e-3
    Jp, _ = run(*(lambda t: (t[0], t[1], t[2:]))(theta + h * d), grad=False)
    Jm, _ = run(*(lambda t: (t[0], t[1], t[2:]))(theta - h * d), grad=False)
    fd = (Jp - Jm) / (2 * h)
    ad = float(g @ d)
    gold = json.load(open(ADJOINT512))
    assert gold["config"]["h"] == h and np.allclose(gold["direction"], d, rtol=1e-15, atol=0)
    ref = gold[kind]
    print(f"{kind}: directional derivative: adjoint {ad:.9e}  forward difference {fd:.9e}  "
          f"oracle {ref['directional']:.9e}; J {J:.9e} oracle {ref['J']:.9e}")
    assert abs(ad - fd) < 1e-3 * abs(fd), (ad, fd)
    assert abs(ad - ref["directional"]) < 1e-3 * abs(ref["directional"]), (ad, ref)
    assert abs(J - ref["J"]) < 1e-5 * abs(ref["J"]), (J, ref["J"])
