"""Write the stored FP64 oracle results that the long GPU parity tests
compare against (runs too long to repeat inside a test).

Calls only the oracle (`oracle/`) and the seeded input recipes
(`paper_2205_04658_amd/workloads.py`); nothing here reads a GPU result.
Each output records the configuration it was made with, and the tests build
their GPU inputs from that record.

    python tests/golden/make_golden.py forced128 [--procs N]
    python tests/golden/make_golden.py stats256
    python tests/golden/make_golden.py adjoint64 [--procs N]
    python tests/golden/make_golden.py adjoint512 [--procs N]

forced128  the forced-turbulence workload of the 4096^2 run (shell
           31 <= |k| <= 33, amplitude 5e-6, seed 4658, tau 0.52, at rest)
           on a 128^2 lattice, 1000 steps: fields and totals at step 1000
           (Ch. 4 "Model and Methods": 1000-8000 step runs).
stats256   the same workload on a 256^2 crop, 2000 steps: the energy
           spectrum E(k) and the enstrophy of the fields every 10 steps from
           step 200 to 2000 (Ch. 2 "Turbulence"), their time averages.
adjoint512 the gradient workload itself (512 x 256 walled channel, discs of
           radius 6 at 5 % area, seed 7, tau 0.8, F_b = 1e-6, 32 basis modes
           7 <= |k| <= 9 at 1e-6, 2000 steps, from rest): both objectives at
           theta and at theta +- h d along one seeded direction d (h = 1e-3),
           in float64 -- the oracle's directional derivative.
adjoint64  a 64 x 32 walled channel with two discs, at rest, driven by
           F = F_b x_hat + sum_m A_m phi_m (32 basis modes 7 <= |k| <= 9,
           F_b = A_m = 1e-6; Ch. 4 eq. forceTerm), tau 0.8, 200 steps: both
           objectives and their central finite-difference gradients with
           respect to (F_b, tau, A_1..A_32), relative step 1e-4, in float64.
"""
import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import diagnostics, forcing, geometry, objective, rlb  # noqa: E402
from paper_2205_04658_amd import workloads  # noqa: E402

_F4 = workloads.FORCED_4096
FORCED128 = dict(nx=128, ny=128, tau=_F4["tau"], kmin=_F4["kmin"], kmax=_F4["kmax"],
                 amplitude=_F4["amplitude"], seed=_F4["seed"], eps=_F4["eps"], n=_F4["n"],
                 steps=1000, checkpoints=[1000])
STATS256 = dict(nx=256, ny=256, tau=_F4["tau"], kmin=_F4["kmin"], kmax=_F4["kmax"],
                amplitude=_F4["amplitude"], seed=_F4["seed"], eps=_F4["eps"], n=_F4["n"],
                steps=2000, first=200, stride=10)
ADJOINT64 = dict(nx=64, ny=32, tau=0.8, body_force=1e-6, steps=200, eps=1.0, n=0.1,
                 discs=[[20.0, 16.0, 4.0], [45.5, 10.0, 3.0]], nmodes=32, kmin=7.0, kmax=9.0,
                 basis_seed=7, mode_amplitude=1e-6, rel_step=1e-4)

_A = workloads.ADJOINT
ADJOINT512 = dict(nx=_A["nx"], ny=_A["ny"], tau=_A["tau"], body_force=_A["body_force"],
                  steps=_A["steps"], eps=_A["eps"], n=_A["n"], fraction=_A["fraction"],
                  radius=_A["radius"], seed=_A["seed"], nmodes=_A["nmodes"], kmin=_A["kmin"],
                  kmax=_A["kmax"], mode_amplitude=_A["mode_amplitude"], direction_seed=5, h=1e-3)

FIELDS = ("eps", "beta_x", "beta_y", "n")


def _forced_run(cfg, on_step):
    """Step the FP64 oracle from rest with the stirring of cfg; call
    on_step(t, F, G) after every step t = 1 .. steps."""
    nx, ny = cfg["nx"], cfg["ny"]
    f = workloads.uniform(nx, ny, cfg["eps"], cfg["n"])
    F, G = rlb.initial_state(*(f[k].astype(np.float64) for k in ("eps", "bx", "by", "n")))
    st = forcing.Stirring(nx, ny, cfg["kmin"], cfg["kmax"], cfg["amplitude"], cfg["seed"])
    for t in range(cfg["steps"]):
        force = np.zeros((3, ny, nx))
        force[:2] = st.field(t)
        F, G = rlb.step(F, G, cfg["tau"], force=force)
        on_step(t + 1, F, G)


def make_forced128(out):
    cfg = FORCED128
    saved = {}
    t0 = time.time()

    def on_step(t, F, G):
        if t in cfg["checkpoints"]:
            fl = rlb.fields(F, G)
            for k in FIELDS:
                saved[f"{k}_{t}"] = fl[k]
            saved[f"totals_{t}"] = rlb.totals(F, G)
        if t % 100 == 0:
            print(f"forced128 step {t} ({time.time() - t0:.0f} s)", flush=True)

    _forced_run(cfg, on_step)
    np.savez_compressed(out, config=json.dumps(cfg), **saved)


def make_stats256(out):
    cfg = STATS256
    n = cfg["nx"]
    kmax = n // 2
    E, Z, ts = [], [], []
    t0 = time.time()

    def on_step(t, F, G):
        if t >= cfg["first"] and (t - cfg["first"]) % cfg["stride"] == 0:
            fl = rlb.fields(F, G)
            E.append(diagnostics.energy_spectrum(fl["beta_x"], fl["beta_y"], kmax))
            Z.append(diagnostics.enstrophy(fl["beta_x"], fl["beta_y"]))
            ts.append(t)
        if t % 100 == 0:
            print(f"stats256 step {t} ({time.time() - t0:.0f} s)", flush=True)

    _forced_run(cfg, on_step)
    mean, err = diagnostics.spectrum_average(np.array(E))
    np.savez_compressed(out, config=json.dumps(cfg), steps=np.array(ts), E=np.array(E),
                        Z=np.array(Z), E_mean=mean, E_err=err, Z_mean=np.mean(Z))


def adjoint64_inputs(cfg=ADJOINT64):
    """Fields, solid mask and stirring basis of the adjoint64 instance."""
    f = workloads.uniform(cfg["nx"], cfg["ny"], cfg["eps"], cfg["n"])
    solid = geometry.channel_mask(cfg["nx"], cfg["ny"], cfg["discs"])
    modes = workloads.stirring_basis(cfg["nx"], cfg["ny"], cfg["nmodes"], cfg["kmin"],
                                     cfg["kmax"], cfg["basis_seed"])
    amps = np.full(cfg["nmodes"], cfg["mode_amplitude"])
    return f, solid, modes, amps


def _adjoint_job(args):
    kind, i = args
    cfg = ADJOINT64
    f, solid, modes, amps = adjoint64_inputs(cfg)
    if i < 0:
        return kind, i, objective.run_objective(f, cfg["steps"], cfg["tau"], cfg["body_force"],
                                                modes, amps, kind, solid)
    g = objective.fd_gradient(f, cfg["steps"], cfg["tau"], cfg["body_force"], modes, amps,
                              kind, solid, rel=cfg["rel_step"], which=[i])
    return kind, i, float(g[i])


def make_adjoint64(out, procs):
    cfg = ADJOINT64
    npar = 2 + cfg["nmodes"]
    jobs = [(k, i) for k in ("current", "dissipation") for i in range(-1, npar)]
    res = {"current": {}, "dissipation": {}}
    t0 = time.time()
    with cf.ProcessPoolExecutor(procs) as ex:
        for kind, i, v in ex.map(_adjoint_job, jobs):
            res[kind][i] = v
            print(f"adjoint64 {kind} {i}: {v:.12e} ({time.time() - t0:.0f} s)", flush=True)
    doc = {"_doc": "FP64 oracle objectives and central finite-difference gradients of the "
                   "adjoint64 instance; written by tests/golden/make_golden.py",
           "config": cfg, "params": ["F_b", "tau"] + [f"A_{m + 1}" for m in range(cfg["nmodes"])]}
    for kind in res:
        doc[kind] = {"J": res[kind][-1], "fd_grad": [res[kind][i] for i in range(npar)]}
    with open(out, "w") as fh:
        json.dump(doc, fh, indent=1)


def adjoint512_inputs(cfg=ADJOINT512):
    """Fields, solid mask, basis, amplitudes and the direction d (one entry
    per parameter, scaled by |theta|) of the adjoint512 instance."""
    nx, ny = cfg["nx"], cfg["ny"]
    f = workloads.uniform(nx, ny, cfg["eps"], cfg["n"])
    discs = workloads.channel_discs(nx, ny, cfg["radius"], cfg["fraction"], cfg["seed"])
    solid = geometry.channel_mask(nx, ny, discs)
    modes = workloads.stirring_basis(nx, ny, cfg["nmodes"], cfg["kmin"], cfg["kmax"], cfg["seed"])
    amps = np.full(cfg["nmodes"], cfg["mode_amplitude"])
    theta = np.concatenate([[cfg["body_force"], cfg["tau"]], amps])
    d = np.random.default_rng(cfg["direction_seed"]).normal(size=theta.size) * np.abs(theta)
    return f, solid, modes, theta, d


def _adjoint512_job(sign):
    cfg = ADJOINT512
    f, solid, modes, theta, d = adjoint512_inputs(cfg)
    th = theta + sign * cfg["h"] * d
    kinds = ("current", "dissipation")
    J = objective.run_objectives(f, cfg["steps"], th[1], th[0], modes, th[2:], kinds, solid)
    return sign, dict(zip(kinds, (float(v) for v in J)))


def make_adjoint512(out, procs):
    cfg = ADJOINT512
    t0 = time.time()
    res = {}
    with cf.ProcessPoolExecutor(min(procs, 3)) as ex:
        for sign, J in ex.map(_adjoint512_job, (0, 1, -1)):
            res[sign] = J
            print(f"adjoint512 sign {sign}: {J} ({time.time() - t0:.0f} s)", flush=True)
    doc = {"_doc": "FP64 oracle objectives of the adjoint512 instance at theta and theta +- h d, "
                   "and the central difference (J(theta + h d) - J(theta - h d)) / 2h; written by "
                   "tests/golden/make_golden.py",
           "config": cfg, "direction": adjoint512_inputs(cfg)[4].tolist()}
    for kind in ("current", "dissipation"):
        doc[kind] = {"J": res[0][kind], "J_plus": res[1][kind], "J_minus": res[-1][kind],
                     "directional": (res[1][kind] - res[-1][kind]) / (2 * cfg["h"])}
    with open(out, "w") as fh:
        json.dump(doc, fh, indent=1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("case", choices=["forced128", "stats256", "adjoint64", "adjoint512"])
    ap.add_argument("--procs", type=int, default=4)
    a = ap.parse_args()
    if a.case == "forced128":
        make_forced128(os.path.join(HERE, "forced128_oracle.npz"))
    elif a.case == "stats256":
        make_stats256(os.path.join(HERE, "stats256_oracle.npz"))
    elif a.case == "adjoint64":
        make_adjoint64(os.path.join(HERE, "adjoint64_oracle.json"), a.procs)
    else:
        make_adjoint512(os.path.join(HERE, "adjoint512_oracle.json"), a.procs)


if __name__ == "__main__":
    main()
