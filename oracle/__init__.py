"""FP64 CPU oracle of the thermal cascaded lattice Boltzmann method (TCLBM).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  It wraps the
plain C reference in ``tclbm_oracle.c`` (Fei & Luo, arXiv:1610.07114,
Sections 2-4) through ctypes and shares no code with the HIP library.

Arrays are numpy float64.  Lattice fields are indexed ``[y, x]``; distribution
functions ``[a, y, x]`` with the D2Q9 order of Section 2
(0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW, 7 SW, 8 SE).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tclbm_oracle.c")
_LIB = os.path.join(_HERE, "libtclbm_oracle.so")

PERIODIC, BOUNCEBACK, WALL, WALL_ADIABATIC = 0, 1, 2, 3
XLO, XHI, YLO, YHI = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain IEEE FP64, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("R", ctypes.c_double), ("T0", ctypes.c_double),
        ("gamma", ctypes.c_double), ("Pr", ctypes.c_double),
        ("tau_f", ctypes.c_double),
        ("w2", ctypes.c_double), ("w3", ctypes.c_double), ("w4", ctypes.c_double),
        ("ax", ctypes.c_double), ("ay", ctypes.c_double),
        ("thermal", ctypes.c_int32), ("correction", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 4),
        ("wall_ux", ctypes.c_double * 4), ("wall_uy", ctypes.c_double * 4), ("wall_T", ctypes.c_double * 4),
        ("wall_rho", ctypes.c_int32), ("heq_moments", ctypes.c_int32), ("h_collision", ctypes.c_int32),
        ("ax_field", ctypes.POINTER(ctypes.c_double)), ("ay_field", ctypes.POINTER(ctypes.c_double)),
        ("h_force", ctypes.c_int32),
        ("viscosity_mode", ctypes.c_int32), ("mu0", ctypes.c_double),
        ("energy_df", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        d = ctypes.POINTER(ctypes.c_double)
        P = ctypes.POINTER(_Params)
        _lib.orc_pops_from_moments.argtypes = [ctypes.c_double, d, d]
        _lib.orc_raw_moments.argtypes = [d, d, d]
        _lib.orc_central_moments.argtypes = [d, ctypes.c_double, ctypes.c_double, d, d]
        _lib.orc_raw_from_central.argtypes = [d, ctypes.c_double, ctypes.c_double, d]
        _lib.orc_post_collision_raw.argtypes = [d] + [ctypes.c_double] * 4 + [d]
        _lib.orc_source_moments.argtypes = [ctypes.c_double] * 4 + [d]
        _lib.orc_correction_moments.argtypes = [ctypes.c_double] * 4 + [d]
        _lib.orc_feq.argtypes = [ctypes.c_double] * 4 + [d]
        _lib.orc_heq.argtypes = [ctypes.c_double] * 5 + [d]
        _lib.orc_heq_mode.argtypes = [ctypes.c_double] * 5 + [ctypes.c_int, d]
        _lib.orc_geq.argtypes = [ctypes.c_double] * 5 + [d]
        _lib.orc_node_macros.argtypes = [P, d, d, ctypes.c_double, ctypes.c_double, d, d, d, d]
        _lib.orc_collide_node.argtypes = [P, d, d] + [ctypes.c_double] * 8 + [d, d]
        _lib.orc_init.argtypes = [P, d, d, d, d, d, d]
        _lib.orc_init.restype = ctypes.c_int
        _lib.orc_macros.argtypes = [P, d, d, d, d, d, d]
        _lib.orc_macros.restype = ctypes.c_int
        _lib.orc_gradients.argtypes = [P, d, d, d, d]
        _lib.orc_gradients.restype = ctypes.c_int
        _lib.orc_step.argtypes = [P, d, d, ctypes.c_int64]
        _lib.orc_step.restype = ctypes.c_int
        _lib.orc_check_params.argtypes = [P]
        _lib.orc_check_params.restype = ctypes.c_int
        _lib.orc_num_threads.restype = ctypes.c_int
        _lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vec(v) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64))


# ---- per-node primitives (exposed for the pins) ---------------------------------

def pops_from_moments(rho: float, m: Sequence[float]) -> np.ndarray:
    """Eq. (3)."""
    m = _vec(m)
    out = np.zeros(9)
    lib().orc_pops_from_moments(rho, _p(m), _p(out))
    return out


def raw_moments(f: Sequence[float]):
    """Eq. (1)-(2): returns (rho, [M00, M10, M01, E, N, Pi, M21, M12, M22])."""
    f = _vec(f)
    rho = np.zeros(1)
    m = np.zeros(9)
    lib().orc_raw_moments(_p(f), _p(rho), _p(m))
    return float(rho[0]), m


def central_moments(f: Sequence[float], ux: float, uy: float):
    """Eq. (4)."""
    f = _vec(f)
    rho = np.zeros(1)
    m = np.zeros(9)
    lib().orc_central_moments(_p(f), ux, uy, _p(rho), _p(m))
    return float(rho[0]), m


def raw_from_central(c: Sequence[float], ux: float, uy: float) -> np.ndarray:
    """Eq. (9)."""
    c = _vec(c)
    out = np.zeros(9)
    lib().orc_raw_from_central(_p(c), ux, uy, _p(out))
    return out


def post_collision_raw(c: Sequence[float], ux, uy, ax, ay) -> np.ndarray:
    """Eq. (18)."""
    c = _vec(c)
    out = np.zeros(9)
    lib().orc_post_collision_raw(_p(c), ux, uy, ax, ay, _p(out))
    return out


def source_moments(ax, ay, ux, uy) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_source_moments(ax, ay, ux, uy, _p(out))
    return out


def correction_moments(Dx, Dy, ux, uy) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_correction_moments(Dx, Dy, ux, uy, _p(out))
    return out


def feq(rho, ux, uy, RT) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_feq(rho, ux, uy, RT, _p(out))
    return out


def heq(rho, ux, uy, RT, b, mode: int = 1) -> np.ndarray:
    """Energy-DF equilibrium; mode 1 the paper's explicit form, mode 0 the
    continuous-moment form."""
    out = np.zeros(9)
    lib().orc_heq_mode(rho, ux, uy, RT, b, int(mode), _p(out))
    return out


def geq(rho, ux, uy, RT, b) -> np.ndarray:
    """Internal-energy DF equilibrium (Section 5D reading): e f^eq, e = b RT/2."""
    out = np.zeros(9)
    lib().orc_geq(rho, ux, uy, RT, b, _p(out))
    return out


# ---- lattice -------------------------------------------------------------------

@dataclass
class Params:
    nx: int
    ny: int
    R: float = 1.0 / 3.0
    T0: float = 1.0
    gamma: float = 1.4
    Pr: float = 0.71
    tau_f: float = 0.8
    w2: float = 1.0
    w3: float = 1.0
    w4: float = 1.0
    ax: float = 0.0
    ay: float = 0.0
    thermal: int = 1
    correction: int = 1
    bc: Sequence[int] = (PERIODIC, PERIODIC, PERIODIC, PERIODIC)
    wall_ux: Sequence[float] = (0.0, 0.0, 0.0, 0.0)
    wall_uy: Sequence[float] = (0.0, 0.0, 0.0, 0.0)
    wall_T: Sequence[float] = (1.0, 1.0, 1.0, 1.0)
    wall_rho: int = 0
    heq_moments: int = 0
    h_collision: int = 0
    h_force: int = 1
    viscosity_mode: int = 0   # 1: mu = mu0 T/T0 (Section 5B), per-node w1 from Eq. (29)
    mu0: float = 0.0
    energy_df: int = 0        # 1: the internal-energy DF of Section 5D (orc_geq)
    ax_field: Optional[np.ndarray] = None
    ay_field: Optional[np.ndarray] = None
    _keep: list = field(default_factory=list, repr=False)

    def to_c(self) -> _Params:
        c = _Params()
        for name in ("nx", "ny", "R", "T0", "gamma", "Pr", "tau_f", "w2", "w3", "w4", "ax", "ay",
                     "thermal", "correction", "wall_rho", "heq_moments", "h_collision", "h_force",
                     "viscosity_mode", "mu0", "energy_df"):
            setattr(c, name, getattr(self, name))
        for i in range(4):
            c.bc[i] = int(self.bc[i])
            c.wall_ux[i] = float(self.wall_ux[i])
            c.wall_uy[i] = float(self.wall_uy[i])
            c.wall_T[i] = float(self.wall_T[i])
        self._keep = []
        if self.ax_field is not None:
            a = np.ascontiguousarray(self.ax_field, dtype=np.float64).reshape(-1)
            self._keep.append(a)
            c.ax_field = _p(a)
        if self.ay_field is not None:
            a = np.ascontiguousarray(self.ay_field, dtype=np.float64).reshape(-1)
            self._keep.append(a)
            c.ay_field = _p(a)
        return c


class Lattice:
    """An oracle lattice: state (f, h) of shape [9, ny, nx], FP64."""

    def __init__(self, params: Params, rho, ux, uy, T):
        self.params = params
        self._c = params.to_c()
        if lib().orc_check_params(ctypes.byref(self._c)):
            raise ValueError("invalid oracle parameters")
        nx, ny = params.nx, params.ny
        self.f = np.zeros((9, ny, nx))
        self.h = np.zeros((9, ny, nx))
        fields = [np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.float64), (ny, nx)))
                  for v in (rho, ux, uy, T)]
        rc = lib().orc_init(ctypes.byref(self._c), *[_p(v) for v in fields], _p(self.f), _p(self.h))
        if rc:
            raise RuntimeError(f"orc_init failed ({rc})")
        self.steps = 0

    def step(self, n: int = 1) -> "Lattice":
        rc = lib().orc_step(ctypes.byref(self._c), _p(self.f), _p(self.h), int(n))
        if rc:
            raise RuntimeError(f"orc_step failed ({rc})")
        self.steps += n
        return self

    def gradients(self):
        """(Dx, Dy), each [ny, nx]: the correction-term derivatives
        d/dx[u_x (1 - theta)], d/dy[u_y (1 - theta)] (Section 4) that the next
        collision of the current state uses."""
        ny, nx = self.params.ny, self.params.nx
        out = [np.zeros((ny, nx)) for _ in range(2)]
        rc = lib().orc_gradients(ctypes.byref(self._c), _p(self.f), _p(self.h), *[_p(v) for v in out])
        if rc:
            raise RuntimeError(f"orc_gradients failed ({rc})")
        return tuple(out)

    def macros(self):
        """(rho, ux, uy, T), each [ny, nx]."""
        ny, nx = self.params.ny, self.params.nx
        out = [np.zeros((ny, nx)) for _ in range(4)]
        rc = lib().orc_macros(ctypes.byref(self._c), _p(self.f), _p(self.h), *[_p(v) for v in out])
        if rc:
            raise RuntimeError(f"orc_macros failed ({rc})")
        return tuple(out)


def collide_node(params: Params, fb, hb, rho, ux, uy, T, Dx, Dy, ax, ay):
    c = params.to_c()
    fb, hb = _vec(fb), _vec(hb)
    fo, ho = np.zeros(9), np.zeros(9)
    lib().orc_collide_node(ctypes.byref(c), _p(fb), _p(hb), rho, ux, uy, T, Dx, Dy, ax, ay, _p(fo), _p(ho))
    return fo, ho


def node_macros(params: Params, fb, hb, ax=0.0, ay=0.0):
    c = params.to_c()
    fb, hb = _vec(fb), _vec(hb)
    out = [np.zeros(1) for _ in range(4)]
    lib().orc_node_macros(ctypes.byref(c), _p(fb), _p(hb), ax, ay, *[_p(v) for v in out])
    return tuple(float(v[0]) for v in out)


def nusselt(uy: np.ndarray, T: np.ndarray, T0: float, H: float, kappa: float, dT: float) -> float:
    """Nusselt number of a Rayleigh-Benard state (Section 5D): one plus the
    mean over all nodes of u_y (T - T0), scaled by H / (kappa dT), with kappa
    the thermal diffusivity nu/Pr at the reference state."""
    return 1.0 + float(np.mean(uy * (T - T0))) * H / (kappa * dT)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))
