"""Forced-turbulence parity over whole runs (Ch. 4 "Model and Methods": the
stirred runs are 1000-8000 steps), against FP64 oracle runs stored by
tests/golden/make_golden.py from the same seeded inputs:

* the 4096^2 workload's stirring (shell 31 <= |k| <= 33, amplitude 5e-6,
  seed 4658, tau 0.52, from rest) on a 128^2 lattice for 1000 steps, every
  field within 1e-5 of its scale, both storage layouts;
* the same workload on a 256^2 crop over 2000 steps: the time-averaged
  energy spectrum E(k) per shell for 1 <= k < kmin within 5 %, and the mean
  enstrophy within 5 %, over the samples taken every 10 steps from step 200
  (Ch. 2 "Turbulence": E(k) and Z)."""
import json
import os

import numpy as np
import pytest

from paper_2205_04658_amd import workloads
from rlbtest import need_gpu

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    d = np.load(os.path.join(HERE, name))
    return json.loads(str(d["config"])), d


def _forced_lattice(cfg, full26=False):
    from paper_2205_04658_amd.rlb import Lattice
    n = cfg["nx"]
    lat = Lattice(n, cfg["ny"], cfg["tau"], full26=full26, eps_ref=cfg["eps"], n_ref=cfg["n"])
    f = workloads.uniform(n, cfg["ny"], cfg["eps"], cfg["n"])
    lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
    lat.set_stirring(cfg["kmin"], cfg["kmax"], cfg["amplitude"], cfg["seed"])
    return lat


@pytest.mark.parametrize("full", [False, True], ids=["folded17", "full26"])
def test_forced_run_1000_steps(full):
    """Every field after 1000 stirred steps within 1e-5 of its scale: 1 for
    eps, n for n, and the flow amplitude (max |beta| of the oracle run) for
    beta.  Also the totals: energy and charge to 1e-8 relative, momentum to
    1e-8 of the energy (the stirring has zero mean, so momentum stays
    near zero)."""
    need_gpu()
    cfg, d = _load("forced128_oracle.npz")
    lat = _forced_lattice(cfg, full)
    lat.step(cfg["steps"])
    lat.sync()
    g = {k: v.double().cpu().numpy() for k, v in lat.fields().items()}
    t = cfg["steps"]
    amp = max(np.abs(d[f"beta_x_{t}"]).max(), np.abs(d[f"beta_y_{t}"]).max())
    scale = {"eps": 1.0, "n": cfg["n"], "beta_x": amp, "beta_y": amp}
    err = {k: float(np.abs(g[k] - d[f"{k}_{t}"]).max() / s) for k, s in scale.items()}
    # the deviations themselves, on their own amplitude (reported)
    dev = {k: float(np.abs(g[k] - d[f"{k}_{t}"]).max() / np.abs(d[f"{k}_{t}"] - c).max())
           for k, c in (("eps", cfg["eps"]), ("n", cfg["n"]))}
    print(f"forced 128^2 x {t}: flow amplitude {amp:.3e}, errors {err}, on deviations {dev}")
    assert max(err.values()) < 1e-5, err
    tot = lat.conserved()
    want = d[f"totals_{t}"]
    print(f"totals: relative differences {(tot - want) / want[[0, 0, 0, 3]]}")
    assert abs(tot[0] - want[0]) < 1e-8 * want[0]
    assert abs(tot[3] - want[3]) < 1e-8 * want[3]
    assert np.abs(tot[1:3] - want[1:3]).max() < 1e-8 * want[0]


def test_forced_statistics_window():
    """256^2 crop of the 4096^2 workload, 2000 steps: time averages of E(k)
    over 1 <= k < kmin and of the enstrophy Z over the samples every 10
    steps from step 200 agree with the oracle run's within 5 %."""
    torch = need_gpu()
    cfg, d = _load("stats256_oracle.npz")
    lat = _forced_lattice(cfg)
    kmax = cfg["nx"] // 2
    acc = torch.zeros(2 * (kmax + 1), dtype=torch.float64, device="cuda")
    Z = []
    t = 0
    for ts in d["steps"]:
        lat.step(int(ts) - t)
        t = int(ts)
        _, sp = lat.energy_spectrum(kmax, 6.0, acc=acc)
        Z.append(sp[2].item())
    from paper_2205_04658_amd.rlb import spectrum_average
    mean, _ = spectrum_average(acc, len(d["steps"]))
    lo, hi = 1, int(np.ceil(cfg["kmin"]))
    rel = np.abs(mean[lo:hi] - d["E_mean"][lo:hi]) / d["E_mean"][lo:hi]
    relZ = abs(np.mean(Z) - float(d["Z_mean"])) / float(d["Z_mean"])
    band = slice(hi, int(cfg["kmax"]) + 1)
    rel_band = np.abs(mean[band] - d["E_mean"][band]) / d["E_mean"][band]
    print(f"stats 256^2: E(k) 1..{hi - 1} max rel {rel.max():.2e}; driven band max rel "
          f"{rel_band.max():.2e}; mean Z rel {relZ:.2e}")
    assert rel.max() < 0.05, rel
    assert relZ < 0.05, relZ
    assert rel_band.max() < 0.05, rel_band
