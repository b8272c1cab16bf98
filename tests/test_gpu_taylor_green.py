"""The steady forced Taylor-Green study of Section 5A on the HIP path: E2 at
N = 64 for the four amplitudes of Table 1 (row 'Present'), FP64, the FP32
offset from it, and the second-order grid convergence of Fig. 2 at Re ~ 20
with equal and with unequal rates w2-w4 (the paper: the slope does not change
with them).  Runs stop at the paper's criterion E_R < 1e-8 over 1000 steps."""
import os
import sys

import numpy as np
import pytest

from helpers import oracle_lattice
from paper_1610_07114_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1610_07114_amd import tclbm
    return tclbm


def _table1():
    rows = []
    for line in open(os.path.join(GOLD, "taylor_green_table1.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            u0, e2 = line.split()
            rows.append((float(u0), float(e2)))
    return rows


def _e2(T, N, u0, storage, rates=None, max_blocks=600):
    """E2 of the converged GPU solution and the steps it took."""
    case = W.taylor_green(N=N, u0=u0)
    if rates:
        case = case.with_(w2=rates[0], w3=rates[1], w4=rates[2])
    lat = T.Lattice(case, storage=storage)
    prev, steps = None, 0
    for _ in range(max_blocks):
        lat.step(1000)
        steps += 1000
        _, ux, uy, _, _ = lat.moments()
        if prev is not None:
            er = np.sqrt(((ux - prev[0]) ** 2 + (uy - prev[1]) ** 2).sum() / (ux ** 2 + uy ** 2).sum())
            if er < 1e-8:
                break
        prev = (ux, uy)
    lat.close()
    ue, ve = case.meta["ux_exact"], case.meta["uy_exact"]
    return float(np.sqrt(((ux - ue) ** 2 + (uy - ve) ** 2).sum() / (ue ** 2 + ve ** 2).sum())), steps


@pytest.mark.parametrize("u0,e2_paper", _table1())
def test_taylor_green_table1_on_gpu(T, u0, e2_paper):
    """Table 1 'Present', N = 64, FP64: E2 within 1% of the printed value
    (measured 1.59222e-3, 1.55734e-3, 1.52133e-3, 1.52007e-3)."""
    e64, n64 = _e2(T, 64, u0, "f64")
    say(f"case taylor-green 64x64 u0 {u0}: E2 fp64 {e64:.5e} ({n64} steps), paper {e2_paper:.4e}")
    assert e64 == pytest.approx(e2_paper, rel=0.01)


@pytest.mark.parametrize("u0", [0.0125, 0.025])
def test_taylor_green_fp32_floor(T, u0):
    """FP32 storage and arithmetic on the same study at the two lower
    amplitudes: the converged velocity stays within 1e-4 of u0 of the FP64
    path's (4.5e-5 measured, a steady offset: round-to-nearest in the force
    and velocity terms biases every step the same way, and the slowest mode
    integrates that bias over its decay time 1/(2 nu k^2), about 1300 steps
    here), which puts E2 within 5% of Table 1 (3% above it).  At the two
    higher amplitudes the steady flow itself does not persist: a perturbation
    of 1e-6 grows in the FP64 oracle too, so FP32 rounding carries the flow
    to another state and only the FP64 path reproduces those rows."""
    case = W.taylor_green(N=64, u0=u0)
    lats = {s: T.Lattice(case, storage=s) for s in ("f64", "f32")}
    for L in lats.values():
        L.step(60000)
    out = {s: L.moments() for s, L in lats.items()}
    for L in lats.values():
        L.close()
    d = max(np.abs(out["f32"][1] - out["f64"][1]).max(), np.abs(out["f32"][2] - out["f64"][2]).max()) / u0
    ue, ve = case.meta["ux_exact"], case.meta["uy_exact"]
    e32 = float(np.sqrt(((out["f32"][1] - ue) ** 2 + (out["f32"][2] - ve) ** 2).sum() / (ue ** 2 + ve ** 2).sum()))
    e2_paper = dict(_table1())[u0]
    say(f"case taylor-green 64x64 u0 {u0} 60000 steps: max|u32 - u64|/u0 {d:.3e}, E2 fp32 {e32:.5e}, "
        f"paper {e2_paper:.4e}")
    assert d < 1e-4
    assert e32 == pytest.approx(e2_paper, rel=0.05)


@pytest.mark.parametrize("rates", [None, (1.1, 1.6, 0.3)])
def test_taylor_green_second_order_on_gpu(T, rates):
    """Fig. 2: E2 falls with the square of the grid spacing (slope 1.9953 in
    the paper) at u0 = 0.0125 (Re = 19.6) over N = 16, 32, 64, FP64, with
    equal rates and with w2, w3, w4 = 1.1, 1.6, 0.3."""
    Ns = (16, 32, 64)
    e = [_e2(T, N, 0.0125, "f64", rates)[0] for N in Ns]
    slope = -np.polyfit(np.log(Ns), np.log(e), 1)[0]
    say(f"case taylor-green convergence, rates {rates}: E2 {e}, slope {slope:.4f}")
    assert 1.95 < slope < 2.05


def test_taylor_green_unequal_rates_parity_fp64(T):
    """Per-node force field with unequal w2-w4 (64 x 64, 400 steps), FP64,
    against the oracle with the same rates within 1e-10."""
    case = W.taylor_green(N=64, u0=0.05).with_(w2=1.1, w3=1.6, w4=0.3)
    say("case taylor-green 64x64 fp64 400 steps, w2-w4 = 1.1, 1.6, 0.3")
    lat = T.Lattice(case, storage="f64")
    lat.step(400)
    r, u, v, _, _ = lat.moments()
    lat.close()
    r0, u0, v0, _ = oracle_lattice(case).step(400).macros()
    us = max(np.abs(u0).max(), np.abs(v0).max())
    e = dict(rho=np.abs(r - r0).max() / np.abs(r0).max(), ux=np.abs(u - u0).max() / us,
             uy=np.abs(v - v0).max() / us)
    say(f"  errors {e}")
    assert max(e.values()) < 1e-10
