"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point include/tclbm.h declares, sizes its state exactly, and
rejects invalid input with status codes before touching device memory.  Also
the node-level arithmetic of the kernels, compiled for the host, against the
oracle's node collision in FP64."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def T():
    from paper_1610_07114_amd import build as B
    if B.stale():
        B.build()
    from paper_1610_07114_amd import tclbm
    return tclbm


def _header_functions():
    src = open(os.path.join(ROOT, "include", "tclbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tclbm_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(T):
    declared = _header_functions()
    assert len(declared) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", T.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (tclbm_\w+)", out))
    assert set(declared) <= exported, set(declared) - exported
    assert sorted(T.EXPORTS) == declared


def test_null_handle_queries(T):
    """Queries on a NULL handle answer without touching a device."""
    assert T._lib.tclbm_step_kernel(None) is None
    assert T._lib.tclbm_steps_done(None) == -1


def test_state_bytes_plan(T):
    p = T.tclbm_default_params(512, 256)
    nb = T.tclbm_state_bytes(p)
    # one 64-slot block per x tile of 62 columns (periodic x) and plane
    slots, planes = -(-512 // 62) * 64, 18
    buf = slots * 256 * planes * 4
    assert nb >= 2 * buf
    assert nb - 2 * buf < 64 * 1024
    p.storage = T.STORE["f16"]
    assert T.tclbm_state_bytes(p) - 2 * buf // 2 < 64 * 1024
    p.storage = T.STORE["f64"]
    assert T.tclbm_state_bytes(p) >= 4 * buf
    p.thermal = 0
    p.storage = T.STORE["f32"]
    assert T.tclbm_state_bytes(p) < nb // 2 + 64 * 1024   # no h planes


@pytest.mark.parametrize("field,value", [("nx", 2), ("ny", 0), ("tau_f", 0.5), ("gamma", 1.0), ("Pr", 0.0),
                                         ("w2", 2.0), ("w3", 0.0), ("storage", 7), ("R", 0.5),
                                         ("wall_rho", 3), ("h_collision", 2), ("h_force", 2), ("thermal", 2),
                                         ("bc", (2, 2, 0, 0)), ("bc", (1, 0, 0, 0)), ("bc", (0, 0, 2, 0)),
                                         ("bc", (3, 3, 0, 0)), ("bc", (0, 0, 4, 4)), ("viscosity_mode", 2)])
def test_invalid_parameters_rejected(T, field, value):
    p = T.tclbm_default_params(16, 16)
    if field == "bc":
        for i, v in enumerate(value):
            p.bc[i] = v
    else:
        setattr(p, field, value)
    assert T.tclbm_state_bytes(p) == 0
    h = ctypes.c_void_p()
    n = 256
    z = np.zeros(n)
    o = np.ones(n)
    st = T._lib.tclbm_create(ctypes.byref(p), ctypes.c_void_p(1 << 20), 1 << 30, None, T._dp(o), T._dp(z),
                             T._dp(z), T._dp(o), None, None, ctypes.byref(h))
    assert st == T.E_INVALID and not h.value


def test_viscosity_law_and_adiabatic_wall_validation(T):
    """mu = mu0 T/T0 needs mu0 > 0; an adiabatic wall needs ny >= 4 (its
    temperature uses the two rows inside) and a y side."""
    p = T.tclbm_default_params(16, 16)
    p.viscosity_mode = 1
    assert T.tclbm_state_bytes(p) == 0
    p.mu0 = 0.35
    assert T.tclbm_state_bytes(p) > 0
    q = T.tclbm_default_params(5, 3)
    q.bc[2], q.bc[3] = T.WALL_ADIABATIC, T.WALL
    assert T.tclbm_state_bytes(q) == 0
    q.ny = 4
    assert T.tclbm_state_bytes(q) > 0


def test_small_buffer_and_bad_fields_rejected(T):
    p = T.tclbm_default_params(16, 16)
    need = T.tclbm_state_bytes(p)
    n = 256
    z, o = np.zeros(n), np.ones(n)
    h = ctypes.c_void_p()
    args = lambda r, t: (T._dp(r), T._dp(z), T._dp(z), T._dp(t), None, None, ctypes.byref(h))
    assert T._lib.tclbm_create(ctypes.byref(p), ctypes.c_void_p(1 << 20), need - 1, None, *args(o, o)) == T.E_NOMEM
    bad = o.copy()
    bad[7] = np.nan
    assert T._lib.tclbm_create(ctypes.byref(p), ctypes.c_void_p(1 << 20), need, None, *args(bad, o)) == T.E_INVALID
    neg = o.copy()
    neg[3] = -1.0
    assert T._lib.tclbm_create(ctypes.byref(p), ctypes.c_void_p(1 << 20), need, None, *args(o, neg)) == T.E_INVALID
    # misaligned device buffer
    assert T._lib.tclbm_create(ctypes.byref(p), ctypes.c_void_p((1 << 20) + 4), need, None, *args(o, o)) == T.E_INVALID
    assert T._lib.tclbm_status_str(T.E_UNSTABLE) == b"unstable state"


def test_product_path_does_not_use_the_oracle():
    pkg = os.path.join(ROOT, "paper_1610_07114_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "tclbm_oracle" not in txt and "orc_" not in txt, f


# ---- node-level arithmetic of the kernels, host build, vs the oracle ------------------

@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("shim") / "libnode_shim.so")
    subprocess.check_call(["g++", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", out,
                           os.path.join(ROOT, "tests", "node_shim.cpp")])
    L = ctypes.CDLL(out)
    d = ctypes.POINTER(ctypes.c_double)
    L.shim_macros.argtypes = [d, d, d, d, ctypes.c_double, ctypes.c_double, d]
    L.shim_collide.argtypes = [d, d, d, d] + [ctypes.c_double] * 4 + [d, d]
    L.shim_feq.argtypes = [d, d] + [ctypes.c_double] * 4 + [d]
    L.shim_heq.argtypes = [d, d] + [ctypes.c_double] * 4 + [d]
    return L


def _node_case(seed):
    import oracle as O
    from helpers import random_pops
    rng = np.random.default_rng(seed)
    tau = rng.uniform(0.52, 1.5)
    w2, w3, w4 = rng.uniform(0.3, 1.9, 3)
    g = float(rng.choice([1.4, 5 / 3, 1.3]))
    Pr = rng.uniform(0.5, 7)
    hm, hc, hfo = int(rng.integers(0, 2)), int(rng.integers(0, 2)), int(rng.integers(0, 2))
    th = 0 if seed % 7 == 3 else 1
    edf = 1 if seed % 5 == 1 else 0     # internal-energy DF (Section 5D)
    p = O.Params(nx=3, ny=3, tau_f=tau, w2=w2, w3=w3, w4=w4, gamma=g, Pr=Pr, heq_moments=hm, h_collision=hc,
                 h_force=hfo, thermal=th, energy_df=edf)
    b, R, w1 = 2 / (g - 1), 1 / 3, 1 / tau
    wh = 1 / ((tau - 0.5) / Pr + 0.5)
    if edf:  # the library's internal encoding: equilibrium mode 2, BGK, no total-energy force term
        hm, hc, hfo = 2, 1, 0
    cst = np.array([R, 1.0, b, w1, w2, w3, w4, wh, w1 * (Pr - 1), th, 1, hm, hc, hfo])
    fb = random_pops(rng, rng.uniform(0.7, 1.3), 0.4)
    hb = random_pops(rng, rng.uniform(0.7, 1.3), 0.4) * 0.8
    # a row reference near, not at, the node state (athermal: theta_r = R T0)
    ref = np.array([rng.uniform(0.8, 1.2), R * (rng.uniform(0.9, 1.1) if th else 1.0)])
    return O, p, cst, fb, hb, ref, rng


@pytest.mark.parametrize("seed", range(40))
def test_kernel_node_math_matches_oracle_fp64(shim, seed):
    """The kernels' per-node arithmetic (deviation form, central moments in a
    factored 3-point route) reproduces the oracle's node step in FP64."""
    O, p, cst, fb, hb, ref, rng = _node_case(seed)
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    ax, ay, Dx, Dy = rng.uniform(-0.02, 0.02, 4)
    mo = np.array(O.node_macros(p, fb, hb, ax, ay))
    mg = np.zeros(4)
    shim.shim_macros(P(cst), P(ref), P(fb), P(hb), ax, ay, P(mg))
    np.testing.assert_allclose(mg, mo, rtol=0, atol=2e-15)
    fo, ho = O.collide_node(p, fb, hb, *mo, Dx, Dy, ax, ay)
    Pg, Qg = np.zeros(9), np.zeros(9)
    shim.shim_collide(P(cst), P(ref), P(fb), P(hb), Dx, Dy, ax, ay, P(Pg), P(Qg))
    np.testing.assert_allclose(Pg, fo, rtol=0, atol=3e-15)
    if p.thermal:
        np.testing.assert_allclose(Qg, ho, rtol=0, atol=3e-15)


@pytest.mark.parametrize("seed", range(10))
def test_kernel_equilibria_match_oracle_fp64(shim, seed):
    O, p, cst, fb, hb, ref, rng = _node_case(100 + seed)
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    rho, T = rng.uniform(0.7, 1.3), rng.uniform(0.9, 1.1)
    ux, uy = rng.uniform(-0.1, 0.1, 2)
    f, h = np.zeros(9), np.zeros(9)
    shim.shim_feq(P(cst), P(ref), rho, ux, uy, T, P(f))
    np.testing.assert_allclose(f, O.feq(rho, ux, uy, T / 3), atol=2e-15)
    if p.thermal:  # no energy DF in the athermal scheme
        shim.shim_heq(P(cst), P(ref), rho, ux, uy, T, P(h))
        want = O.geq(rho, ux, uy, T / 3, cst[2]) if p.energy_df else O.heq(rho, ux, uy, T / 3, cst[2], int(cst[11]))
        np.testing.assert_allclose(h, want, atol=3e-15)
