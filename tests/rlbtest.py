"""Shared helpers of the GPU parity tests: running the FP64 oracle on the
same seeded inputs as the HIP path, and scaled field comparisons."""
import numpy as np
import pytest

from oracle import forcing, geometry, rlb

# Field scales for the parity tolerance: max |gpu - oracle| / S.  S is the
# magnitude of the quantity (1 for energy densities, the charge density for
# n and J0) or, for quantities that vanish at rest, the flow amplitude.
def scales(beta=0.01, n=0.1):
    return {"eps": 1.0, "T00": 1.0, "Txx": 1.0, "Tyy": 1.0, "Txy": beta,
            "beta_x": beta, "beta_y": beta, "T0x": beta, "T0y": beta,
            "n": n, "J0": n, "Jx": n * beta, "Jy": n * beta}


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_04658_amd import rlb as binding
    binding.lib()     # raises if the library is not built
    return torch


def oracle_run(f, nsteps, tau, cfl=1.0, solid=None, body=(0.0, 0.0), stir=None, start=0):
    """Initialise from float32 fields f (dict eps, bx, by, n) and take nsteps.
    stir = (kmin, kmax, amplitude, seed) or None.  Returns (F, G)."""
    F, G = rlb.initial_state(f["eps"].astype(np.float64), f["bx"].astype(np.float64),
                             f["by"].astype(np.float64), f["n"].astype(np.float64))
    ny, nx = f["eps"].shape
    st = forcing.Stirring(nx, ny, *stir) if stir is not None else None
    for t in range(start, start + nsteps):
        force = None
        if body != (0.0, 0.0) or st is not None:
            force = np.zeros((3, ny, nx))
            force[0] += body[0]
            force[1] += body[1]
            if st is not None:
                force[:2] += st.field(t)
        F, G = rlb.step(F, G, tau, cfl=cfl, force=force, solid=solid)
    return F, G


def fold(F):
    """Oracle 26 populations -> (17, ...) planes of the z-mirror-folded
    layout, in the library's plane order (in-plane faces and edges, then the
    mirror pairs): plane = sum of the directions with its (vx, vy) and |vz|."""
    out = []
    for vx, vy, az in _folded_dirs():
        idx = [i for i in range(26) if np.allclose(rlb.V[i, :2], (vx, vy)) and
               np.isclose(abs(rlb.V[i, 2]), az)]
        out.append(F[idx].sum(axis=0))
    return np.stack(out)


def unfold26(F):
    """Oracle 26 populations in the library's RLB_FULL26 plane order."""
    order = []
    for vx, vy, vz in _full_dirs():
        order.append(int(np.argmin(np.abs(rlb.V - np.array([vx, vy, vz])).sum(axis=1))))
    return F[order]


def _folded_dirs():
    s2, s3 = 1 / np.sqrt(2), 1 / np.sqrt(3)
    inplane = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
               (s2, s2, 0), (-s2, s2, 0), (s2, -s2, 0), (-s2, -s2, 0)]
    pairs = [(0, 0, 1), (s2, 0, s2), (-s2, 0, s2), (0, s2, s2), (0, -s2, s2),
             (s3, s3, s3), (-s3, s3, s3), (s3, -s3, s3), (-s3, -s3, s3)]
    return inplane + pairs


def _full_dirs():
    d = _folded_dirs()
    return d + [(vx, vy, -vz) for vx, vy, vz in d[8:]]


def _dir_index(vx, vy, vz):
    return int(np.argmin(np.abs(rlb.V - np.array([vx, vy, vz])).sum(axis=1)))


def expand(P, full):
    """Library planes (Q, ...) of one family -> the oracle's 26 populations:
    the full set's planes reordered, or each folded plane split evenly over
    its z-mirror pair (the states the folded layout represents are
    z-symmetric)."""
    out = np.zeros((26,) + P.shape[1:])
    if full:
        for k, d in enumerate(_full_dirs()):
            out[_dir_index(*d)] = P[k]
    else:
        for k, (vx, vy, az) in enumerate(_folded_dirs()):
            idx = [i for i in range(26) if np.allclose(rlb.V[i, :2], (vx, vy)) and
                   np.isclose(abs(rlb.V[i, 2]), az)]
            for i in idx:
                out[i] = P[k] / len(idx)
    return out


def contract(F, full):
    """Oracle 26 populations -> library planes of one family (inverse of
    expand on z-symmetric populations)."""
    return unfold26(F) if full else fold(F)


def compare(gpu, ora, sc, names=None):
    """Max scaled error per field (gpu: dict of tensors, ora: dict of arrays)."""
    names = names or list(gpu)
    return {k: float(np.abs(gpu[k].double().cpu().numpy() - ora[k]).max() / sc[k]) for k in names}
