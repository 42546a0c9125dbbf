"""The C-ABI library loads, exports every symbol include/rlb.h declares, and
rejects bad arguments with the documented status codes.  Runs without a GPU
(no compute calls)."""
import ctypes
import os
import re

import pytest

from paper_2205_04658_amd import rlb as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rlb.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(B.LIB_PATH):
        from paper_2205_04658_amd import build
        build.build()
    return B.lib()


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rlb_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(L):
    names = declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(B.SYMBOLS) == names


def test_version(L):
    assert b"gfx950" in L.rlb_version()


def P(**kw):
    d = dict(nx=64, ny=32, tau=0.8, cfl=1.0, flags=0, eps_ref=1.0, n_ref=0.1)
    d.update(kw)
    return B.Params(**d)


@pytest.mark.parametrize("kw,status", [
    (dict(nx=3), B.EINVAL), (dict(ny=0), B.EINVAL), (dict(nx=70000, ny=70000), B.EINVAL),
    (dict(tau=0.5), B.EINVAL), (dict(tau=float("nan")), B.EINVAL),
    (dict(cfl=0.0), B.EINVAL), (dict(cfl=2.5), B.EUNSUPPORTED),
    (dict(cfl=1.25, flags=0x1), B.EUNSUPPORTED), (dict(cfl=1.25, flags=0x4), B.EUNSUPPORTED),
    (dict(flags=0x10), B.EINVAL), (dict(eps_ref=float("inf")), B.EINVAL),
    (dict(nx=31580609, ny=4), B.EINVAL), (dict(nx=20648833, ny=4, flags=0x2), B.EINVAL),
    (dict(nx=44739201, ny=4, flags=0x8), B.EINVAL)])
def test_bad_params(L, kw, status):
    n = ctypes.c_size_t(123)
    assert L.rlb_workspace_bytes(ctypes.byref(P(**kw)), ctypes.byref(n)) == status
    assert n.value == 123            # nothing written on failure
    assert len(L.rlb_last_error()) > 0


def test_widest_rows_are_accepted(L):
    """The widest rows whose state still fits 32-bit column offsets (one
    row of 2 x Q float32 planes, nx rounded up to 64, below 2^32 bytes)."""
    n = ctypes.c_size_t()
    for nx, flags, q in ((31580608, 0, 17), (20648832, 0x2, 26), (44739200, 0x8, 12)):
        assert nx * 2 * q * 4 < 2 ** 32 <= (nx + 64) * 2 * q * 4
        assert L.rlb_workspace_bytes(ctypes.byref(P(nx=nx, ny=4, flags=flags)), ctypes.byref(n)) == B.OK


def test_wide_cfl_is_accepted_on_periodic_lattices(L):
    n = ctypes.c_size_t()
    for cfl in (1.25, 2.0):
        assert L.rlb_workspace_bytes(ctypes.byref(P(cfl=cfl)), ctypes.byref(n)) == B.OK


def test_workspace_size(L):
    n = ctypes.c_size_t()
    assert L.rlb_workspace_bytes(ctypes.byref(P(nx=4096, ny=4096)), ctypes.byref(n)) == B.OK
    state = 2 * 2 * 17 * 4096 * 4096 * 4
    assert state < n.value < state + 256 * 2**20
    n26 = ctypes.c_size_t()
    assert L.rlb_workspace_bytes(ctypes.byref(P(nx=4096, ny=4096, flags=B.FULL26)), ctypes.byref(n26)) == B.OK
    assert n26.value > n.value


def test_create_rejects_bad_workspace(L):
    n = ctypes.c_size_t()
    L.rlb_workspace_bytes(ctypes.byref(P()), ctypes.byref(n))
    h = ctypes.c_void_p()
    assert L.rlb_create(ctypes.byref(P()), None, n.value, None, ctypes.byref(h)) == B.EINVAL
    assert L.rlb_create(ctypes.byref(P()), ctypes.c_void_p(4096 + 8), n.value, None,
                        ctypes.byref(h)) == B.EINVAL
    assert L.rlb_create(ctypes.byref(P()), ctypes.c_void_p(4096 * 256), 16, None,
                        ctypes.byref(h)) == B.ENOMEM
    assert h.value is None


def test_create_without_gpu_reports_device(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    n = ctypes.c_size_t()
    L.rlb_workspace_bytes(ctypes.byref(P()), ctypes.byref(n))
    h = ctypes.c_void_p()
    assert L.rlb_create(ctypes.byref(P()), ctypes.c_void_p(4096 * 256), n.value, None,
                        ctypes.byref(h)) == B.EDEVICE


def test_null_handle_calls(L):
    assert L.rlb_destroy(None) == B.OK
    assert L.rlb_step(None, 1) == B.EINVAL
    assert L.rlb_sync(None) == B.EINVAL
    assert L.rlb_set_body_force(None, 0.0, 0.0) == B.EINVAL
    assert L.rlb_read_fields(None, 1, None) == B.EINVAL
    d = (ctypes.c_double * 4)()
    assert L.rlb_conserved(None, d) == B.EINVAL
    assert L.rlb_philox(0, 0, 0, -1, None, None) == B.EINVAL
    assert L.rlb_copy_probe(ctypes.c_void_p(256), ctypes.c_void_p(512 + 4), 32, None) == B.EINVAL
    assert L.rlb_copy_probe(ctypes.c_void_p(256), ctypes.c_void_p(512), 30, None) == B.EINVAL
    assert L.rlb_use_graph(None, 2) == B.EINVAL
    n = ctypes.c_size_t(7)
    assert L.rlb_record_workspace_bytes(None, 16, ctypes.byref(n)) == B.EINVAL and n.value == 7
    assert L.rlb_record_current(None, 4, 0, None, None, 0) == B.EINVAL
    assert L.rlb_batch_set_open_borders(None, 0.1, 0.0, 0.1, 1.0) == B.EINVAL
    assert L.rlb_set_open_borders(None, 0.1, 0.0, 0.1, 1.0) == B.EINVAL
    assert b"null" in L.rlb_last_error() or len(L.rlb_last_error()) > 0


@pytest.mark.parametrize("cls,cname", [(B.AdjointCfg, "rlb_adjoint_cfg"), (B.Params, "rlb_params")])
def test_binding_structs_match_the_header(cls, cname, tmp_path):
    """The ctypes structures the binding passes by pointer have the header's
    size and field offsets (checked with the host C compiler)."""
    fields = [f for f, _ in cls._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "rlb.h"\nint main(void) {\n'
                   f'  printf("%zu\\n", sizeof({cname}));\n'
                   + "".join(f'  printf("%zu\\n", offsetof({cname}, {f}));\n' for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got == [ctypes.sizeof(cls)] + [getattr(cls, f).offset for f in fields]
