"""Thin ctypes binding of libtclbm.so (C ABI in include/tclbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels.
PyTorch supplies the device memory (a uint8 tensor of tclbm_state_bytes bytes)
and the stream (a torch stream per lattice).  If the library is
missing this module raises at import; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# TCLBM_LIB may name another build of the same library (A/B of kernel variants)
LIB_PATH = os.environ.get("TCLBM_LIB") or os.path.join(_HERE, "_lib", "libtclbm.so")

OK, E_INVALID, E_NOMEM, E_DEVICE, E_STATE, E_UNSTABLE = range(6)
STORE = {"f32": 0, "f16": 1, "bf16": 2, "f64": 3}
PERIODIC, BOUNCEBACK, WALL, WALL_ADIABATIC = 0, 1, 2, 3
XLO, XHI, YLO, YHI = 0, 1, 2, 3


class tclbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("R", ctypes.c_double), ("T0", ctypes.c_double),
        ("gamma", ctypes.c_double), ("Pr", ctypes.c_double),
        ("tau_f", ctypes.c_double),
        ("w2", ctypes.c_double), ("w3", ctypes.c_double), ("w4", ctypes.c_double),
        ("ax", ctypes.c_double), ("ay", ctypes.c_double),
        ("thermal", ctypes.c_int32), ("correction", ctypes.c_int32), ("storage", ctypes.c_int32),
        ("wall_rho", ctypes.c_int32), ("heq_moments", ctypes.c_int32), ("h_collision", ctypes.c_int32),
        ("h_force", ctypes.c_int32), ("accel_field", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 4),
        ("wall_ux", ctypes.c_double * 4), ("wall_uy", ctypes.c_double * 4), ("wall_T", ctypes.c_double * 4),
        ("viscosity_mode", ctypes.c_int32), ("mu0", ctypes.c_double),
        ("energy_df", ctypes.c_int32),
    ]


class tclbm_sums(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("momx", ctypes.c_double), ("momy", ctypes.c_double),
        ("energy", ctypes.c_double), ("kinetic", ctypes.c_double), ("nu_num", ctypes.c_double),
        ("rho_min", ctypes.c_double), ("T_min", ctypes.c_double), ("nonfinite", ctypes.c_int64),
    ]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


EXPORTS = ["tclbm_default_params", "tclbm_state_bytes", "tclbm_create", "tclbm_set_bc", "tclbm_step",
           "tclbm_step_timed", "tclbm_moments", "tclbm_moments_noalloc", "tclbm_steps_done", "tclbm_read_state", "tclbm_set_tuning",
           "tclbm_step_kernel", "tclbm_destroy", "tclbm_status_str", "tclbm_last_error", "tclbm_hbm_copy",
           "tclbm_batch_create", "tclbm_batch_step", "tclbm_batch_step_timed", "tclbm_batch_size",
           "tclbm_batch_waves", "tclbm_batch_set_graph_chunk", "tclbm_batch_set_strip_rows",
           "tclbm_batch_strip_rows", "tclbm_batch_set_persistent", "tclbm_batch_persistent",
           "tclbm_batch_step_kernel", "tclbm_batch_destroy"]


def _load():
    # torch first: its HIP runtime (same soname) must be the one the library
    # binds to, so that torch-allocated device pointers and streams are valid
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libtclbm.so not built ({LIB_PATH}); run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    d = ctypes.POINTER(ctypes.c_double)
    P = ctypes.POINTER(tclbm_params)
    H = ctypes.c_void_p
    lib.tclbm_default_params.argtypes = [ctypes.c_int32, ctypes.c_int32, P]
    lib.tclbm_default_params.restype = None
    lib.tclbm_state_bytes.argtypes = [P]
    lib.tclbm_state_bytes.restype = ctypes.c_size_t
    lib.tclbm_create.argtypes = [P, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, d, d, d, d, d, d,
                                 ctypes.POINTER(H)]
    lib.tclbm_create.restype = ctypes.c_int
    lib.tclbm_set_bc.argtypes = [H, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double]
    lib.tclbm_set_bc.restype = ctypes.c_int
    lib.tclbm_step.argtypes = [H, ctypes.c_int64]
    lib.tclbm_step.restype = ctypes.c_int
    lib.tclbm_step_timed.argtypes = [H, ctypes.c_int64, d]
    lib.tclbm_step_timed.restype = ctypes.c_int
    lib.tclbm_moments.argtypes = [H, d, d, d, d, ctypes.POINTER(tclbm_sums)]
    lib.tclbm_moments.restype = ctypes.c_int
    lib.tclbm_moments_noalloc.argtypes = [H, d, d, d, d, ctypes.POINTER(tclbm_sums)]
    lib.tclbm_moments_noalloc.restype = ctypes.c_int
    lib.tclbm_steps_done.argtypes = [H]
    lib.tclbm_steps_done.restype = ctypes.c_int64
    lib.tclbm_step_kernel.argtypes = [H]
    lib.tclbm_step_kernel.restype = ctypes.c_char_p
    lib.tclbm_read_state.argtypes = [H, d]
    lib.tclbm_read_state.restype = ctypes.c_int
    lib.tclbm_set_tuning.argtypes = [H, ctypes.c_int32, ctypes.c_int32]
    lib.tclbm_set_tuning.restype = ctypes.c_int
    lib.tclbm_destroy.argtypes = [H]
    lib.tclbm_destroy.restype = ctypes.c_int
    lib.tclbm_status_str.argtypes = [ctypes.c_int]
    lib.tclbm_status_str.restype = ctypes.c_char_p
    lib.tclbm_last_error.argtypes = [H]
    lib.tclbm_last_error.restype = ctypes.c_char_p
    lib.tclbm_hbm_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.tclbm_hbm_copy.restype = ctypes.c_int
    lib.tclbm_batch_create.argtypes = [ctypes.POINTER(H), ctypes.c_int32, ctypes.POINTER(H)]
    lib.tclbm_batch_create.restype = ctypes.c_int
    lib.tclbm_batch_step.argtypes = [H, ctypes.c_int64]
    lib.tclbm_batch_step.restype = ctypes.c_int
    lib.tclbm_batch_step_timed.argtypes = [H, ctypes.c_int64, d]
    lib.tclbm_batch_step_timed.restype = ctypes.c_int
    lib.tclbm_batch_size.argtypes = [H]
    lib.tclbm_batch_size.restype = ctypes.c_int32
    lib.tclbm_batch_waves.argtypes = [H]
    lib.tclbm_batch_waves.restype = ctypes.c_int64
    lib.tclbm_batch_set_graph_chunk.argtypes = [H, ctypes.c_int32]
    lib.tclbm_batch_set_graph_chunk.restype = ctypes.c_int
    lib.tclbm_batch_set_strip_rows.argtypes = [H, ctypes.c_int32]
    lib.tclbm_batch_set_strip_rows.restype = ctypes.c_int
    lib.tclbm_batch_strip_rows.argtypes = [H]
    lib.tclbm_batch_strip_rows.restype = ctypes.c_int32
    lib.tclbm_batch_set_persistent.argtypes = [H, ctypes.c_int32, ctypes.c_int32]
    lib.tclbm_batch_set_persistent.restype = ctypes.c_int
    lib.tclbm_batch_persistent.argtypes = [H]
    lib.tclbm_batch_persistent.restype = ctypes.c_int32
    lib.tclbm_batch_step_kernel.argtypes = [H]
    lib.tclbm_batch_step_kernel.restype = ctypes.c_char_p
    lib.tclbm_batch_destroy.argtypes = [H]
    lib.tclbm_batch_destroy.restype = ctypes.c_int
    return lib


_lib = _load()


class TclbmError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        self.status = status
        super().__init__(f"{_lib.tclbm_status_str(status).decode()} ({status}) {msg}".strip())


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _chk(st: int, h=None):
    if st != OK:
        raise TclbmError(st, _lib.tclbm_last_error(h).decode() if h else "")


# ---- the C entry points, same names ------------------------------------------------

def tclbm_default_params(nx: int, ny: int) -> tclbm_params:
    p = tclbm_params()
    _lib.tclbm_default_params(nx, ny, ctypes.byref(p))
    return p


def tclbm_state_bytes(p: tclbm_params) -> int:
    return int(_lib.tclbm_state_bytes(ctypes.byref(p)))


def tclbm_create(p: tclbm_params, dev_ptr: int, dev_bytes: int, stream: int, rho, ux, uy, T,
                 ax_field=None, ay_field=None):
    h = ctypes.c_void_p()
    arrs = [None if v is None else np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
            for v in (rho, ux, uy, T, ax_field, ay_field)]
    _chk(_lib.tclbm_create(ctypes.byref(p), ctypes.c_void_p(dev_ptr), dev_bytes, ctypes.c_void_p(stream),
                           *[_dp(a) for a in arrs], ctypes.byref(h)))
    return h


def tclbm_set_bc(h, side: int, kind: int, ux_w: float = 0.0, uy_w: float = 0.0, T_w: float = 1.0):
    _chk(_lib.tclbm_set_bc(h, side, kind, ux_w, uy_w, T_w), h)


def tclbm_step(h, n: int):
    _chk(_lib.tclbm_step(h, int(n)), h)


def tclbm_step_timed(h, n: int) -> float:
    ms = ctypes.c_double()
    _chk(_lib.tclbm_step_timed(h, int(n), ctypes.byref(ms)), h)
    return ms.value


def tclbm_moments(h, nx: int, ny: int, fields: bool = True, check: bool = True):
    out = [np.empty(nx * ny) for _ in range(4)] if fields else [None] * 4
    s = tclbm_sums()
    st = _lib.tclbm_moments(h, *[_dp(o) for o in out], ctypes.byref(s))
    if check:
        _chk(st, h)
    res = [None if o is None else o.reshape(ny, nx) for o in out]
    return (*res, s, st)


def tclbm_moments_noalloc(h, nx: int, ny: int, fields: bool = True, check: bool = True):
    out = [np.empty(nx * ny) for _ in range(4)] if fields else [None] * 4
    s = tclbm_sums()
    st = _lib.tclbm_moments_noalloc(h, *[_dp(o) for o in out], ctypes.byref(s))
    if check:
        _chk(st, h)
    res = [None if o is None else o.reshape(ny, nx) for o in out]
    return (*res, s, st)


def tclbm_steps_done(h) -> int:
    return int(_lib.tclbm_steps_done(h))


def tclbm_step_kernel(h) -> str:
    return _lib.tclbm_step_kernel(h).decode()


def tclbm_read_state(h, nplanes: int, nx: int, ny: int) -> np.ndarray:
    out = np.empty(nplanes * nx * ny)
    _chk(_lib.tclbm_read_state(h, _dp(out)), h)
    return out.reshape(nplanes, ny, nx)


def tclbm_set_tuning(h, strip_rows: int, graph_chunk: int):
    _chk(_lib.tclbm_set_tuning(h, int(strip_rows), int(graph_chunk)), h)


def tclbm_destroy(h):
    _chk(_lib.tclbm_destroy(h))


def tclbm_hbm_copy(dst_ptr: int, src_ptr: int, nbytes: int, stream: int):
    _chk(_lib.tclbm_hbm_copy(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr), nbytes, ctypes.c_void_p(stream)))


def tclbm_batch_create(handles) -> ctypes.c_void_p:
    arr = (ctypes.c_void_p * len(handles))(*[h.value for h in handles])
    b = ctypes.c_void_p()
    _chk(_lib.tclbm_batch_create(arr, len(handles), ctypes.byref(b)))
    return b


def tclbm_batch_step(b, n: int):
    _chk(_lib.tclbm_batch_step(b, int(n)))


def tclbm_batch_step_timed(b, n: int) -> float:
    ms = ctypes.c_double()
    _chk(_lib.tclbm_batch_step_timed(b, int(n), ctypes.byref(ms)))
    return ms.value


def tclbm_batch_size(b) -> int:
    return int(_lib.tclbm_batch_size(b))


def tclbm_batch_waves(b) -> int:
    return int(_lib.tclbm_batch_waves(b))


def tclbm_batch_set_graph_chunk(b, chunk: int):
    _chk(_lib.tclbm_batch_set_graph_chunk(b, int(chunk)))


def tclbm_batch_set_strip_rows(b, rows: int):
    _chk(_lib.tclbm_batch_set_strip_rows(b, int(rows)))


def tclbm_batch_strip_rows(b) -> int:
    return int(_lib.tclbm_batch_strip_rows(b))


def tclbm_batch_set_persistent(b, steps_per_launch: int, wait_us: int = 0):
    _chk(_lib.tclbm_batch_set_persistent(b, int(steps_per_launch), int(wait_us)))


def tclbm_batch_persistent(b) -> int:
    return int(_lib.tclbm_batch_persistent(b))


def tclbm_batch_step_kernel(b) -> str:
    return _lib.tclbm_batch_step_kernel(b).decode()


def tclbm_batch_destroy(b):
    _chk(_lib.tclbm_batch_destroy(b))


# ---- convenience wrappers ------------------------------------------------------------

class Lattice:
    """One lattice resident on a GPU.  `case` is a workloads.Case."""

    def __init__(self, case, storage: str = "f32", device: str = "cuda:0", stream=None, **over):
        import torch
        self.case = case
        p = tclbm_default_params(case.nx, case.ny)
        for name in ("R", "T0", "gamma", "Pr", "tau_f", "w2", "w3", "w4", "ax", "ay", "thermal", "correction",
                     "viscosity_mode", "mu0", "energy_df"):
            setattr(p, name, getattr(case, name))
        p.storage = STORE[storage]
        p.accel_field = 1 if case.ax_field is not None else 0
        for side in range(4):
            p.bc[side] = int(case.bc[side])
            p.wall_ux[side] = float(case.wall_ux[side])
            p.wall_uy[side] = float(case.wall_uy[side])
            p.wall_T[side] = float(case.wall_T[side])
        for k, v in over.items():
            setattr(p, k, v)
        self.params = p
        self.nbytes = tclbm_state_bytes(p)
        if self.nbytes == 0:
            raise TclbmError(E_INVALID, "invalid parameters")
        self.device = torch.device(device)
        # a stream of its own (default priority): the legacy default stream
        # cannot be captured into HIP graphs.  The buffer is allocated with that
        # stream current, so torch's caching allocator does not hand its memory
        # to work on another stream while the library's kernels may still use it.
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        with torch.cuda.stream(self.stream):
            self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self.h = tclbm_create(p, self.buf.data_ptr(), self.nbytes, self.stream.cuda_stream, case.rho, case.ux,
                              case.uy, case.T if case.T is not None else case.rho, case.ax_field, case.ay_field)

    def step(self, n: int = 1) -> "Lattice":
        tclbm_step(self.h, n)
        return self

    def step_timed(self, n: int) -> float:
        return tclbm_step_timed(self.h, n)

    def moments(self, fields: bool = True, check: bool = True):
        rho, ux, uy, T, s, st = tclbm_moments(self.h, self.case.nx, self.case.ny, fields, check)
        return rho, ux, uy, T, s

    def read_state(self) -> np.ndarray:
        return tclbm_read_state(self.h, 18 if self.params.thermal else 9, self.case.nx, self.case.ny)

    def set_tuning(self, strip_rows: int = 0, graph_chunk: int = 32):
        tclbm_set_tuning(self.h, strip_rows, graph_chunk)

    @property
    def steps(self) -> int:
        return tclbm_steps_done(self.h)

    @property
    def kernel(self) -> str:
        """Name of the kernel one step launches (as in a kernel trace)."""
        return tclbm_step_kernel(self.h)

    def close(self):
        if self.h is not None:
            tclbm_destroy(self.h)
            self.h = None
            self.buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Lattices advanced together, one kernel launch per step.  All members
    must share the storage form and the stream."""

    def __init__(self, lattices):
        self.members = list(lattices)
        self.h = tclbm_batch_create([m.h for m in self.members])

    def step(self, n: int = 1) -> "Batch":
        tclbm_batch_step(self.h, n)
        return self

    def step_timed(self, n: int) -> float:
        return tclbm_batch_step_timed(self.h, n)

    @property
    def waves(self) -> int:
        return tclbm_batch_waves(self.h)

    def set_graph_chunk(self, chunk: int):
        tclbm_batch_set_graph_chunk(self.h, chunk)

    def set_strip_rows(self, rows: int):
        tclbm_batch_set_strip_rows(self.h, rows)

    @property
    def strip_rows(self) -> int:
        return tclbm_batch_strip_rows(self.h)

    def set_persistent(self, steps_per_launch: int, wait_us: int = 0):
        """Run up to steps_per_launch steps per (cooperative) launch; 0: one
        launch per step."""
        tclbm_batch_set_persistent(self.h, steps_per_launch, wait_us)

    @property
    def persistent(self) -> int:
        return tclbm_batch_persistent(self.h)

    @property
    def kernel(self) -> str:
        """Name of the kernel one batch step launches (as in a kernel trace)."""
        return tclbm_batch_step_kernel(self.h)

    def close(self):
        if self.h is not None:
            tclbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
