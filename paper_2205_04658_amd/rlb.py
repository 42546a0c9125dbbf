"""ctypes binding of librlb (C ABI in include/rlb.h).

Argument marshalling only: every computation runs in the HIP kernels of
librlb.so.  PyTorch supplies device memory (the workspace and I/O tensors)
and the stream.  If the library is not built, every entry point raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RLB_LIB_PATH names another build of the same library (the host-sanitizer
# build of the CPU boundary tests); by default the in-tree librlb.so
LIB_PATH = os.environ.get("RLB_LIB_PATH") or os.path.join(_HERE, "librlb.so")

OK, EINVAL, EDEVICE, ENOMEM, ENONFINITE, ELANDAU, ESTATE, EUNSUPPORTED = range(8)
STATUS_NAMES = ["RLB_OK", "RLB_EINVAL", "RLB_EDEVICE", "RLB_ENOMEM", "RLB_ENONFINITE",
                "RLB_ELANDAU", "RLB_ESTATE", "RLB_EUNSUPPORTED"]
WALLS_Y = 0x1
FULL26 = 0x2
OPEN_X = 0x4
PLANAR = 0x8
FIELDS = ["eps", "beta_x", "beta_y", "n", "T00", "T0x", "T0y", "Txx", "Txy", "Tyy",
          "J0", "Jx", "Jy"]

# Every symbol include/rlb.h declares.
SYMBOLS = [
    "rlb_workspace_bytes", "rlb_create", "rlb_destroy", "rlb_init_fields",
    "rlb_set_obstacles", "rlb_add_disks", "rlb_clear_obstacles", "rlb_set_body_force",
    "rlb_set_stirring", "rlb_step", "rlb_use_graph", "rlb_read_fields", "rlb_conserved",
    "rlb_force_injection", "rlb_sync",
    "rlb_get_step", "rlb_state_bytes", "rlb_save_state", "rlb_load_state", "rlb_layout",
    "rlb_stirring_coefficients", "rlb_stirring_field", "rlb_philox", "rlb_timing",
    "rlb_timing_read", "rlb_copy_probe", "rlb_last_error", "rlb_version",
    "rlb_set_launch_shape", "rlb_get_launch_shape", "rlb_autotune",
    "rlb_batch_workspace_bytes", "rlb_batch_create", "rlb_batch_destroy", "rlb_batch_member",
    "rlb_batch_set_body_force", "rlb_batch_set_open_borders", "rlb_batch_step", "rlb_batch_sync", "rlb_batch_info",
    "rlb_batch_record_workspace_bytes", "rlb_batch_record_current",
    "rlb_batch_set_launch_shape", "rlb_batch_get_launch_shape", "rlb_batch_autotune",
    "rlb_batch_use_graph", "rlb_batch_timing", "rlb_batch_timing_read",
    "rlb_set_relaxation_time", "rlb_set_relaxation_eta_s", "rlb_adjoint_workspace_bytes",
    "rlb_adjoint_run", "rlb_adjoint_apply", "rlb_set_open_borders", "rlb_column_current", "rlb_record_workspace_bytes", "rlb_record_current",
    "rlb_record_current_noalloc", "rlb_power_spectrum",
    "rlb_spectrum_workspace_bytes", "rlb_energy_spectrum", "rlb_spectrum_average",
    "rlb_power_law_fit",
]
OBJECTIVES = {"current": 0, "dissipation": 1}


def _tune_rows(out):
    rows = [(int(out[4 * i]), int(out[4 * i + 1]), int(out[4 * i + 2]), out[4 * i + 3])
            for i in range(len(out) // 4)]
    return [r for r in rows if r[3] > 0]


class RLBError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {message}")


class AdjointCfg(ctypes.Structure):
    _fields_ = [("nsteps", ctypes.c_int64), ("checkpoint", ctypes.c_int32),
                ("objective", ctypes.c_int32), ("nmodes", ctypes.c_int32),
                ("h_modes", ctypes.c_void_p), ("h_amps", ctypes.c_void_p),
                ("body_force", ctypes.c_double), ("resident", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("tau", ctypes.c_double),
                ("cfl", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("eps_ref", ctypes.c_double), ("n_ref", ctypes.c_double)]


_lib = None
_vp = ctypes.c_void_p
_i32, _i64, _u32, _u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
_sz, _d = ctypes.c_size_t, ctypes.c_double
_P = ctypes.POINTER


def lib():
    """Load librlb.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2205_04658_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "rlb_workspace_bytes": [_P(Params), _P(_sz)],
        "rlb_create": [_P(Params), _vp, _sz, _vp, _P(_vp)],
        "rlb_destroy": [_vp],
        "rlb_init_fields": [_vp, _vp, _vp, _vp, _vp],
        "rlb_set_obstacles": [_vp, _vp],
        "rlb_add_disks": [_vp, _i32, _vp],
        "rlb_clear_obstacles": [_vp],
        "rlb_set_body_force": [_vp, _d, _d],
        "rlb_set_stirring": [_vp, _d, _d, _d, _u64],
        "rlb_step": [_vp, _i64],
        "rlb_use_graph": [_vp, _i32],
        "rlb_read_fields": [_vp, _u32, _vp],
        "rlb_conserved": [_vp, _P(_d)],
        "rlb_force_injection": [_vp, _P(_d)],
        "rlb_sync": [_vp],
        "rlb_get_step": [_vp, _P(_i64)],
        "rlb_state_bytes": [_vp, _P(_sz)],
        "rlb_save_state": [_vp, _vp, _sz],
        "rlb_load_state": [_vp, _vp, _sz],
        "rlb_layout": [_vp, _P(_i32), _P(_i32), _P(_i64), _P(_sz)],
        "rlb_stirring_coefficients": [_vp, _i64, _vp, _P(_i32)],
        "rlb_stirring_field": [_vp, _i64, _vp],
        "rlb_philox": [_u64, _u64, _u64, _i64, _vp, _vp],
        "rlb_timing": [_vp, _i32],
        "rlb_timing_read": [_vp, _P(_d), _P(_i64)],
        "rlb_copy_probe": [_vp, _vp, _sz, _vp],
        "rlb_set_launch_shape": [_vp, _i32, _i32, _i32],
        "rlb_get_launch_shape": [_vp, _P(_i32), _P(_i32), _P(_i32)],
        "rlb_autotune": [_vp, _i32, _P(_d), _i32],
        "rlb_batch_workspace_bytes": [_P(Params), _i32, _vp, _vp, _P(_sz)],
        "rlb_batch_create": [_P(Params), _i32, _vp, _vp, _vp, _sz, _vp, _P(_vp)],
        "rlb_batch_destroy": [_vp],
        "rlb_batch_member": [_vp, _i32, _P(_vp)],
        "rlb_batch_set_body_force": [_vp, _d, _d],
        "rlb_batch_set_open_borders": [_vp, _d, _d, _d, _d],
        "rlb_batch_step": [_vp, _i64],
        "rlb_batch_sync": [_vp],
        "rlb_batch_record_workspace_bytes": [_vp, _i32, _P(_sz)],
        "rlb_batch_record_current": [_vp, _i64, _i32, _vp, _i64, _vp, _sz],
        "rlb_batch_info": [_vp, _P(_i32), _P(_i64), _P(_i32), _P(_i64)],
        "rlb_batch_set_launch_shape": [_vp, _i32, _i32, _i32],
        "rlb_batch_get_launch_shape": [_vp, _P(_i32), _P(_i32), _P(_i32)],
        "rlb_batch_autotune": [_vp, _i32, _P(_d), _i32],
        "rlb_batch_use_graph": [_vp, _i32],
        "rlb_batch_timing": [_vp, _i32],
        "rlb_batch_timing_read": [_vp, _P(_d), _P(_i64)],
        "rlb_set_relaxation_time": [_vp, _d],
        "rlb_set_relaxation_eta_s": [_vp, _d, _d],
        "rlb_set_open_borders": [_vp, _d, _d, _d, _d],
        "rlb_column_current": [_vp, _i32, _vp],
        "rlb_record_workspace_bytes": [_vp, _i32, _P(_sz)],
        "rlb_record_current": [_vp, _i64, _i32, _vp, _vp, _sz],
        "rlb_record_current_noalloc": [_vp, _i64, _i32, _vp],
        "rlb_power_spectrum": [_vp, _i64, _vp, _vp],
        "rlb_spectrum_workspace_bytes": [_vp, _i32, _P(_sz)],
        "rlb_energy_spectrum": [_vp, _i32, _d, _vp, _vp, _vp, _sz],
        "rlb_spectrum_average": [_vp, _i32, _i64, _vp, _vp],
        "rlb_power_law_fit": [_vp, _vp, _i32, _P(_d), _P(_d)],
        "rlb_adjoint_workspace_bytes": [_vp, _P(AdjointCfg), _P(_sz)],
        "rlb_adjoint_run": [_vp, _P(AdjointCfg), _vp, _sz, _P(_d), _vp],
        "rlb_adjoint_apply": [_vp, _i32, _vp, _vp, _vp, _vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.rlb_last_error.restype = ctypes.c_char_p
    L.rlb_last_error.argtypes = []
    L.rlb_version.restype = ctypes.c_char_p
    L.rlb_version.argtypes = []
    _lib = L
    return L


def check(status):
    if status != OK:
        raise RLBError(status, lib().rlb_last_error().decode())


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    return _vp(stream.cuda_stream if stream is not None else 0)


def workspace_bytes(nx, ny, tau, cfl=1.0, flags=0, eps_ref=1.0, n_ref=0.1):
    p = Params(nx, ny, tau, cfl, flags, eps_ref, n_ref)
    n = _sz()
    check(lib().rlb_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
    return n.value


def philox(k0, k1, c1, count, device="cuda"):
    """Raw Philox4x64-10 blocks from the device generator: (count, 4) uint64
    (as int64 storage) for counters (m, c1, 0, 0), m < count."""
    torch = _torch()
    out = torch.empty((max(count, 1), 4), dtype=torch.int64, device=device)
    check(lib().rlb_philox(k0, k1, c1, count, _vp(out.data_ptr()),
                           _stream_ptr(torch.cuda.current_stream())))
    return out[:count]


def copy_probe(src, dst):
    torch = _torch()
    check(lib().rlb_copy_probe(_vp(src.data_ptr()), _vp(dst.data_ptr()),
                               src.numel() * src.element_size(),
                               _stream_ptr(torch.cuda.current_stream())))


def _dev_f32(a, device, shape):
    torch = _torch()
    t = torch.as_tensor(np.asarray(a) if not isinstance(a, torch.Tensor) else a)
    t = t.to(device=device, dtype=torch.float32).contiguous()
    if tuple(t.shape) != shape:
        raise ValueError(f"field has shape {tuple(t.shape)}, expected {shape}")
    return t


class Lattice:
    """One lattice on one GPU.  The workspace is a torch uint8 tensor owned by
    this object; all work goes to the torch stream current at creation."""

    def __init__(self, nx, ny, tau, cfl=1.0, walls=False, full26=False,
                 eps_ref=1.0, n_ref=0.1, device=None, open_x=False, planar=False, _member=None):
        torch = _torch()
        if _member is not None:          # a batch member: handle owned by the batch
            batch, h = _member
            self.nx, self.ny = int(nx), int(ny)
            self.device, self.stream, self.workspace = batch.device, batch.stream, None
            self._h, self._owned, self._batch, self._keep = h, False, batch, []
            return
        self.nx, self.ny = int(nx), int(ny)
        flags = (WALLS_Y if walls else 0) | (FULL26 if full26 else 0) | (OPEN_X if open_x else 0) \
            | (PLANAR if planar else 0)
        self.params = Params(self.nx, self.ny, float(tau), float(cfl), flags,
                             float(eps_ref), float(n_ref))
        n = _sz()
        check(lib().rlb_workspace_bytes(ctypes.byref(self.params), ctypes.byref(n)))
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.workspace = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = _vp()
        check(lib().rlb_create(ctypes.byref(self.params), _vp(self.workspace.data_ptr()), n.value,
                               _stream_ptr(self.stream), ctypes.byref(h)))
        self._h = h
        self._owned = True
        self._keep = []

    # -- streams ------------------------------------------------------------
    def _in(self, *tensors):
        """Order the lattice stream after the caller's stream (inputs ready)."""
        torch = _torch()
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)
            for t in tensors:
                t.record_stream(self.stream)

    def _out(self):
        """Order the caller's stream after the lattice stream (outputs ready)."""
        torch = _torch()
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) and getattr(self, "_owned", False):
            lib().rlb_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup --------------------------------------------------------------
    def init_fields(self, eps, bx, by, n):
        shape = (self.ny, self.nx)
        ts = [_dev_f32(a, self.device, shape) for a in (eps, bx, by, n)]
        self._in(*ts)
        check(lib().rlb_init_fields(self._h, *[_vp(t.data_ptr()) for t in ts]))
        self._keep = ts

    def set_obstacles(self, mask):
        torch = _torch()
        m = torch.as_tensor(np.asarray(mask) if not isinstance(mask, torch.Tensor) else mask)
        m = m.to(device=self.device, dtype=torch.uint8).contiguous()
        self._in(m)
        check(lib().rlb_set_obstacles(self._h, _vp(m.data_ptr())))
        self._keep = [m]

    def add_disks(self, discs):
        d = np.ascontiguousarray(np.asarray(discs, np.float64).reshape(-1, 3))
        check(lib().rlb_add_disks(self._h, d.shape[0], d.ctypes.data_as(_vp)))

    def clear_obstacles(self):
        check(lib().rlb_clear_obstacles(self._h))

    def set_body_force(self, fx, fy=0.0):
        check(lib().rlb_set_body_force(self._h, float(fx), float(fy)))

    def set_stirring(self, kmin, kmax, amplitude, seed):
        check(lib().rlb_set_stirring(self._h, float(kmin), float(kmax), float(amplitude), int(seed)))

    # -- stepping -----------------------------------------------------------
    def step(self, n=1):
        check(lib().rlb_step(self._h, int(n)))

    def use_graph(self, steps_per_graph):
        """Replay steps_per_graph steps as one HIP graph (0 = off, even)."""
        check(lib().rlb_use_graph(self._h, int(steps_per_graph)))

    def sync(self):
        check(lib().rlb_sync(self._h))

    @property
    def step_count(self):
        s = _i64()
        check(lib().rlb_get_step(self._h, ctypes.byref(s)))
        return s.value

    # -- read-out -----------------------------------------------------------
    def fields(self, names=None):
        """Dict name -> float32 tensor (ny, nx) of the current fields."""
        torch = _torch()
        names = FIELDS if names is None else list(names)
        mask = 0
        for nm in names:
            mask |= 1 << FIELDS.index(nm)
        order = [f for f in FIELDS if mask & (1 << FIELDS.index(f))]
        out = torch.empty((len(order), self.ny, self.nx), dtype=torch.float32, device=self.device)
        self._in(out)
        check(lib().rlb_read_fields(self._h, mask, _vp(out.data_ptr())))
        self._out()
        return {nm: out[i] for i, nm in enumerate(order)}

    def conserved(self):
        out = (_d * 4)()
        check(lib().rlb_conserved(self._h, out))
        return np.array(out[:])

    def force_injection(self):
        """(dE, dP^x, dP^y) the next step's driving term adds (rlb_force_injection)."""
        out = (_d * 3)()
        check(lib().rlb_force_injection(self._h, out))
        return np.array(out[:])

    def layout(self):
        """(planes per family, row pitch, state row stride, header bytes); see
        rlb_layout for the node-brick addressing."""
        q, row, pitch, hb = _i32(), _i32(), _i64(), _sz()
        check(lib().rlb_layout(self._h, ctypes.byref(q), ctypes.byref(row), ctypes.byref(pitch),
                               ctypes.byref(hb)))
        return q.value, row.value, pitch.value, hb.value

    def save_state(self):
        torch = _torch()
        n = _sz()
        check(lib().rlb_state_bytes(self._h, ctypes.byref(n)))
        buf = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        self._in(buf)
        check(lib().rlb_save_state(self._h, _vp(buf.data_ptr()), n.value))
        self._out()
        return buf

    def load_state(self, buf):
        self._in(buf)
        check(lib().rlb_load_state(self._h, _vp(buf.data_ptr()), buf.numel()))

    def planes(self, buf=None):
        """Shifted population planes of a saved state: (F, G) float32 tensors
        of shape (Q, ny, nx) holding F_i - w_i eps_ref and G_i - w_i n_ref."""
        torch = _torch()
        buf = self.save_state() if buf is None else buf
        q, row, stride, hb = self.layout()
        f = buf[hb:hb + 4 * self.ny * stride].view(torch.float32)
        f = f.view(self.ny, row // 64, 2 * q, 64).permute(2, 0, 1, 3).reshape(2 * q, self.ny, row)
        f = f[:, :, :self.nx]
        return f[:q], f[q:]

    def bricks(self, planes):
        """A population copy in the lattice's node-brick layout (rlb_layout)
        from planes of shape (2Q, ny, nx): a float32 device tensor of
        row_stride * ny elements, padding columns zero."""
        torch = _torch()
        q, row, stride, _ = self.layout()
        planes = planes.to(device=self.device, dtype=torch.float32)
        if tuple(planes.shape) != (2 * q, self.ny, self.nx):
            raise ValueError(f"planes must have shape {(2 * q, self.ny, self.nx)}")
        full = torch.zeros((2 * q, self.ny, row), dtype=torch.float32, device=self.device)
        full[:, :, :self.nx] = planes
        return full.view(2 * q, self.ny, row // 64, 64).permute(1, 2, 0, 3).contiguous().view(-1)

    def unbricks(self, buf):
        """Inverse of bricks: (2Q, ny, nx) planes of a node-brick copy."""
        q, row, stride, _ = self.layout()
        f = buf[:self.ny * stride].view(self.ny, row // 64, 2 * q, 64).permute(2, 0, 1, 3)
        return f.reshape(2 * q, self.ny, row)[:, :, :self.nx]

    def adjoint_apply(self, op, mu, state=None):
        """rlb_adjoint_apply on planes of shape (2Q, ny, nx): op "pull_t"
        returns P^T mu; op "step" returns ((dC/dF~)^T P^T mu at the given
        shifted state, per-node adjoints (ny, nx, 3) of (F^x, F^y, 1/tau))."""
        torch = _torch()
        code = {"step": 0, "pull_t": 1}[op]
        m = self.bricks(mu)
        out = torch.zeros_like(m)
        st = self.bricks(state) if code == 0 else None
        acc = torch.zeros(3 * self.nx * self.ny + 32, dtype=torch.float64, device=self.device) \
            if code == 0 else None
        self._in(*(t for t in (m, out, st, acc) if t is not None))
        check(lib().rlb_adjoint_apply(self._h, code, _vp(st.data_ptr()) if st is not None else None,
                                      _vp(m.data_ptr()), _vp(out.data_ptr()),
                                      _vp(acc.data_ptr()) if acc is not None else None))
        self._out()
        res = self.unbricks(out)
        if code == 1:
            return res
        n = self.nx * self.ny
        a = torch.stack([acc[0:2 * n:2], acc[1:2 * n:2], acc[2 * n:3 * n]], 1).view(self.ny, self.nx, 3)
        return res, a

    def stirring_coefficients(self, step):
        torch = _torch()
        out = torch.empty((8192, 4), dtype=torch.float64, device=self.device)
        cnt = _i32()
        check(lib().rlb_stirring_coefficients(self._h, int(step), _vp(out.data_ptr()),
                                              ctypes.byref(cnt)))
        return out[:cnt.value]

    def stirring_field(self, step):
        torch = _torch()
        out = torch.empty((2, self.ny, self.nx), dtype=torch.float32, device=self.device)
        check(lib().rlb_stirring_field(self._h, int(step), _vp(out.data_ptr())))
        return out

    def set_launch_shape(self, tile_rows, grid_per_cu=0, strip=16):
        check(lib().rlb_set_launch_shape(self._h, int(tile_rows), int(grid_per_cu), int(strip)))

    def launch_shape(self):
        """(tile_rows, grid_per_cu, strip)."""
        a, b, c = _i32(), _i32(), _i32()
        check(lib().rlb_get_launch_shape(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def autotune(self, trials=5):
        """Time every launch shape on the current state (which does not
        advance), keep the fastest; returns [(tile_rows, grid_per_cu, strip, ms)]."""
        out = (_d * (4 * 64))()
        check(lib().rlb_autotune(self._h, int(trials), out, 64))
        return _tune_rows(out)

    def timing(self, enable=True, every=1):
        """Time the step kernel of every `every`-th step (rlb_timing)."""
        check(lib().rlb_timing(self._h, int(every) if enable else 0))

    def timing_read(self):
        ms, n = _d(), _i64()
        check(lib().rlb_timing_read(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def set_relaxation_time(self, tau):
        check(lib().rlb_set_relaxation_time(self._h, float(tau)))

    def set_open_borders(self, bx, by, n_in, eps_out):
        """Velocity inlet at x = 0 (beta, n_in), pressure outlet at x = nx-1
        (eps_out); the lattice must be created with open_x=True."""
        check(lib().rlb_set_open_borders(self._h, float(bx), float(by), float(n_in), float(eps_out)))

    def column_current(self, x, out=None):
        """j at column x of the current step into out[0] (a float64 device
        tensor; a new 1-element tensor if None), asynchronously."""
        torch = _torch()
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.device)
        if out.dtype != torch.float64 or not out.is_cuda:
            raise ValueError("out must be a float64 device tensor")
        self._in(out)
        check(lib().rlb_column_current(self._h, int(x), _vp(out.data_ptr())))
        self._out()
        return out

    def record_current(self, steps, x, out=None, chunk=1024):
        """`steps` steps; out[t] = j at column x of the state before step
        t + 1 (a float64 device tensor of >= steps elements; new if None).
        The row workspace holds `chunk` steps."""
        torch = _torch()
        if out is None:
            out = torch.empty(steps, dtype=torch.float64, device=self.device)
        if out.dtype != torch.float64 or not out.is_cuda or out.numel() < steps \
                or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 device tensor of >= steps elements")
        n = _sz()
        check(lib().rlb_record_workspace_bytes(self._h, int(max(1, min(chunk, steps))),
                                               ctypes.byref(n)))
        work = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        self._in(out, work)
        check(lib().rlb_record_current(self._h, int(steps), int(x), _vp(out.data_ptr()),
                                       _vp(work.data_ptr()), n.value))
        self._out()
        return out

    def record_current_noalloc(self, steps, x, out=None):
        """As record_current, through rlb_record_current_noalloc: the rows
        go to the library's fixed device scratch instead of a workspace."""
        torch = _torch()
        if out is None:
            out = torch.empty(steps, dtype=torch.float64, device=self.device)
        if out.dtype != torch.float64 or not out.is_cuda or out.numel() < steps \
                or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 device tensor of >= steps elements")
        self._in(out)
        check(lib().rlb_record_current_noalloc(self._h, int(steps), int(x), _vp(out.data_ptr())))
        self._out()
        return out

    def energy_spectrum(self, kmax=None, k_cut=0.0, acc=None):
        """E(k) of the current velocity (rlb_energy_spectrum): returns
        (E tensor [kmax+1], a 3-element tensor: rms and mean speed of the
        field filtered to |k| < k_cut, and the enstrophy), all float64 on
        the device; acc (a float64 tensor [2 (kmax+1)]) collects running
        sums."""
        torch = _torch()
        kmax = min(self.nx, self.ny) // 2 if kmax is None else int(kmax)
        n = _sz()
        check(lib().rlb_spectrum_workspace_bytes(self._h, kmax, ctypes.byref(n)))
        work = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        out = torch.empty(kmax + 4, dtype=torch.float64, device=self.device)
        if acc is not None and (acc.dtype != torch.float64 or acc.numel() != 2 * (kmax + 1)):
            raise ValueError("acc must be a float64 tensor of 2 (kmax + 1) elements")
        self._in(out, work, *([acc] if acc is not None else []))
        check(lib().rlb_energy_spectrum(self._h, kmax, float(k_cut), _vp(out.data_ptr()),
                                        _vp(acc.data_ptr()) if acc is not None else None,
                                        _vp(work.data_ptr()), n.value))
        self._out()
        return out[:kmax + 1], out[kmax + 1:]

    def set_relaxation_eta_s(self, eta_over_s, dt):
        """Per-node tau(x) = 5 (eta/s) / (T(x) dt), T = (pi^2 eps / 3)^(1/4)."""
        check(lib().rlb_set_relaxation_eta_s(self._h, float(eta_over_s), float(dt)))

    def adjoint_run(self, nsteps, checkpoint, objective, modes, amps, body_force, grad=True,
                    resident=0):
        """Run nsteps from the current state with F = F_b x_hat + sum_m A_m
        phi_m; return (J, dJ/d(F_b, tau, A_1..A_M) or None).  `resident`:
        segments of `checkpoint` states kept in device memory (0: the
        minimum; ceil(nsteps / checkpoint) or more: all, nothing recomputed)."""
        torch = _torch()
        modes = np.ascontiguousarray(np.asarray(modes, np.float64).reshape(-1, 5))
        amps = np.ascontiguousarray(np.asarray(amps, np.float64).reshape(-1))
        cfg = AdjointCfg(int(nsteps), int(checkpoint), OBJECTIVES[objective], modes.shape[0],
                         modes.ctypes.data, amps.ctypes.data, float(body_force), int(resident))
        nb = _sz()
        check(lib().rlb_adjoint_workspace_bytes(self._h, ctypes.byref(cfg), ctypes.byref(nb)))
        ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        self._in(ws)
        J = _d()
        g = np.zeros(2 + modes.shape[0], np.float64)
        check(lib().rlb_adjoint_run(self._h, ctypes.byref(cfg), _vp(ws.data_ptr()), nb.value,
                                    ctypes.byref(J), g.ctypes.data if grad else None))
        return J.value, (g if grad else None)


class Batch:
    """Many lattices of uneven sizes advanced by one launch per step (hipGraph
    replay on a dedicated stream).  `sizes` is a list of (nx, ny); members
    are Lattice objects (`batch[b]`) for initialisation and read-out."""

    def __init__(self, sizes, tau, cfl=1.0, walls=False, full26=False, eps_ref=1.0,
                 n_ref=0.1, device=None, open_x=False):
        torch = _torch()
        self.sizes = [(int(a), int(b)) for a, b in sizes]
        n = len(self.sizes)
        flags = (WALLS_Y if walls else 0) | (FULL26 if full26 else 0) | (OPEN_X if open_x else 0)
        self.params = Params(0, 0, float(tau), float(cfl), flags, float(eps_ref), float(n_ref))
        self._nx = (_i32 * n)(*[a for a, _ in self.sizes])
        self._ny = (_i32 * n)(*[b for _, b in self.sizes])
        nb = _sz()
        check(lib().rlb_batch_workspace_bytes(ctypes.byref(self.params), n, self._nx, self._ny,
                                              ctypes.byref(nb)))
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = torch.cuda.Stream(self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(self.stream):
            self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        h = _vp()
        check(lib().rlb_batch_create(ctypes.byref(self.params), n, self._nx, self._ny,
                                     _vp(self.workspace.data_ptr()), nb.value,
                                     _stream_ptr(self.stream), ctypes.byref(h)))
        self._h = h
        self.members = []
        for b, (a, c) in enumerate(self.sizes):
            mh = _vp()
            check(lib().rlb_batch_member(self._h, b, ctypes.byref(mh)))
            self.members.append(Lattice(a, c, tau, _member=(self, mh)))

    def __getitem__(self, b):
        return self.members[b]

    def __len__(self):
        return len(self.members)

    def close(self):
        if getattr(self, "_h", None):
            for m in self.members:
                m._h = None
            lib().rlb_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_open_borders(self, bx, by, n_in, eps_out):
        check(lib().rlb_batch_set_open_borders(self._h, float(bx), float(by), float(n_in),
                                               float(eps_out)))

    def set_body_force(self, fx, fy=0.0):
        check(lib().rlb_batch_set_body_force(self._h, float(fx), float(fy)))

    def step(self, n=1):
        torch = _torch()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        check(lib().rlb_batch_step(self._h, int(n)))

    def sync(self):
        check(lib().rlb_batch_sync(self._h))

    def record_current(self, steps, x, out=None, chunk=1024):
        """`steps` batched steps; out[b, t] = j at column x of member b's
        state before step t + 1 (x < 0 counts from each member's last
        column: -2 is the column before the outlet).  out: a float64 device
        tensor of shape (members, >= steps) with unit column stride; a new
        (members, steps) tensor if None.  The row workspace holds `chunk`
        steps."""
        torch = _torch()
        n = len(self.members)
        if out is None:
            out = torch.empty((n, steps), dtype=torch.float64, device=self.device)
        if out.dtype != torch.float64 or not out.is_cuda or out.dim() != 2 or out.shape[0] != n \
                or out.shape[1] < steps or (steps > 1 and out.stride(1) != 1):
            raise ValueError("out must be a float64 device tensor of shape (members, >= steps)")
        nb = _sz()
        check(lib().rlb_batch_record_workspace_bytes(self._h, int(max(1, min(chunk, steps, 32768))),
                                                     ctypes.byref(nb)))
        m = self.members[0]
        with torch.cuda.stream(self.stream):
            work = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        m._in(out)
        check(lib().rlb_batch_record_current(self._h, int(steps), int(x), _vp(out.data_ptr()),
                                              int(out.stride(0)) if steps else 0,
                                              _vp(work.data_ptr()), nb.value))
        m._out()
        return out

    def info(self):
        c, cells, q, st = _i32(), _i64(), _i32(), _i64()
        check(lib().rlb_batch_info(self._h, ctypes.byref(c), ctypes.byref(cells), ctypes.byref(q),
                                   ctypes.byref(st)))
        return dict(count=c.value, cells=cells.value, planes=q.value, step=st.value)

    def set_launch_shape(self, tile_rows, grid_per_cu=0, strip=16):
        check(lib().rlb_batch_set_launch_shape(self._h, int(tile_rows), int(grid_per_cu), int(strip)))

    def launch_shape(self):
        """(tile_rows, grid_per_cu, strip)."""
        a, b, c = _i32(), _i32(), _i32()
        check(lib().rlb_batch_get_launch_shape(self._h, ctypes.byref(a), ctypes.byref(b),
                                               ctypes.byref(c)))
        return a.value, b.value, c.value

    def autotune(self, trials=5):
        """As Lattice.autotune, for the batched step."""
        out = (_d * (4 * 64))()
        check(lib().rlb_batch_autotune(self._h, int(trials), out, 64))
        return _tune_rows(out)

    def use_graph(self, steps_per_graph=64):
        check(lib().rlb_batch_use_graph(self._h, int(steps_per_graph)))

    def timing(self, enable=True):
        check(lib().rlb_batch_timing(self._h, 1 if enable else 0))

    def timing_read(self):
        ms, n = _d(), _i64()
        check(lib().rlb_batch_timing_read(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


def _autograd():
    import torch

    class RLBObjective(torch.autograd.Function):
        """J(theta), theta = (F_b, tau, A_1..A_M) as a float64 tensor.  The
        forward resets the lattice to `fields`, runs the step `nsteps` times
        and evaluates the objective; the gradient comes from the library's
        adjoint run (checkpoint every `checkpoint` steps, `resident` segments
        kept in device memory)."""

        @staticmethod
        def forward(ctx, theta, lattice, fields, modes, nsteps, checkpoint, objective, resident):
            th = theta.detach().cpu().double().numpy()
            lattice.init_fields(fields["eps"], fields["bx"], fields["by"], fields["n"])
            lattice.set_relaxation_time(th[1])
            J, g = lattice.adjoint_run(nsteps, checkpoint, objective, modes, th[2:], th[0],
                                       grad=True, resident=resident)
            ctx.save_for_backward(torch.as_tensor(g, dtype=theta.dtype))
            return torch.tensor(J, dtype=theta.dtype)

        @staticmethod
        def backward(ctx, gout):
            (g,) = ctx.saved_tensors
            return gout * g.to(gout.device), None, None, None, None, None, None, None

    return RLBObjective


def power_spectrum(series):
    """One-sided power spectrum of a float64 device series' fluctuations
    (rlb_power_spectrum): a tensor of n // 2 + 1 bins on the series' device,
    computed on the current stream."""
    torch = _torch()
    s = series.contiguous()
    if s.dtype != torch.float64 or not s.is_cuda or s.dim() != 1:
        raise ValueError("series must be a 1-D float64 device tensor")
    out = torch.empty(s.numel() // 2 + 1, dtype=torch.float64, device=s.device)
    check(lib().rlb_power_spectrum(_vp(s.data_ptr()), s.numel(), _vp(out.data_ptr()),
                                   _stream_ptr(torch.cuda.current_stream(s.device))))
    return out


def spectrum_average(acc, count):
    """(mean, standard error) per shell from energy_spectrum's running sums
    of `count` samples (rlb_spectrum_average, host)."""
    a = np.ascontiguousarray(np.asarray(acc.cpu() if hasattr(acc, "cpu") else acc, np.float64))
    kmax = a.size // 2 - 1
    mean, err = np.empty(kmax + 1), np.empty(kmax + 1)
    check(lib().rlb_spectrum_average(a.ctypes.data_as(_vp), kmax, int(count),
                                     mean.ctypes.data_as(_vp), err.ctypes.data_as(_vp)))
    return mean, err


def power_law_fit(k, y):
    """(slope, intercept) of log y = intercept + slope log k (rlb_power_law_fit, host)."""
    k = np.ascontiguousarray(np.asarray(k, np.float64))
    y = np.ascontiguousarray(np.asarray(y, np.float64))
    slope, icpt = _d(), _d()
    check(lib().rlb_power_law_fit(k.ctypes.data_as(_vp), y.ctypes.data_as(_vp), k.size,
                                  ctypes.byref(slope), ctypes.byref(icpt)))
    return slope.value, icpt.value


def rlb_objective(theta, lattice, fields, modes, nsteps, checkpoint, objective="current",
                  resident=0):
    """Differentiable objective of a driven run (torch.autograd); `resident`
    as in Lattice.adjoint_run."""
    return _autograd().apply(theta, lattice, fields, modes, nsteps, checkpoint, objective,
                             resident)
