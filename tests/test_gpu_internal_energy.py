"""The internal-energy DF (Section 5D's Rayleigh-Benard runs) on the HIP path:
FP64 parity with the oracle, FP32 parity with the bounds of the total-energy
path, a Couette flow without viscous heating, and Table 3's Nu(Ra) sweep at
the paper's resolutions against the stored FP64 oracle histories and against
the printed values."""
import json
import os
import sys

import numpy as np
import pytest

from helpers import oracle_lattice
from paper_1610_07114_amd import workloads as W
from test_gpu_parity import PERT_TOL_FP32, U_TOL_FP32_FORCED, pert_err, rel_err

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


def _pair(T, case, steps, storage):
    lat = T.Lattice(case, storage=storage)
    lat.step(steps)
    g = lat.moments()[:4]
    lat.close()
    return g, oracle_lattice(case).step(steps).macros()


def test_internal_energy_rb_fp64(T):
    """Rayleigh-Benard at the Section 5D setting (130 x 67, Ra 1e4), 300
    steps, FP64: every field within 1e-10 of the oracle."""
    case = W.rayleigh_benard(nx=130, ny=67, Ra=1e4, Pr=0.71, dT=0.06, seed=3, noise=1e-3).with_(energy_df=1)
    say("case internal-energy rayleigh-benard 130x67 fp64 300 steps")
    g, o = _pair(T, case, 300, "f64")
    e = rel_err(g, o, case)
    say(f"  errors {e}")
    assert max(e.values()) < 1e-10


def test_internal_energy_rb_fp32(T):
    """The same at 256 x 128, FP32, 100 steps: fields within 1e-5,
    perturbations within the FP32 bound, the early velocity within the forced
    FP32 bound."""
    case = W.rayleigh_benard(nx=256, ny=128, Ra=1e4, Pr=0.71, dT=0.06, seed=4, noise=1e-3).with_(energy_df=1)
    say("case internal-energy rayleigh-benard 256x128 fp32 100 steps")
    g, o = _pair(T, case, 100, "f32")
    e, p = rel_err(g, o, case), pert_err(g, o, case)
    say(f"  errors {e}; perturbation errors {p}")
    assert max(e["rho"], e["T"]) < 1e-5
    assert max(e["ux"], e["uy"]) < U_TOL_FP32_FORCED
    assert max(p.values()) < PERT_TOL_FP32


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_internal_energy_couette(T, storage, tol):
    """Thermal Couette flow (8 x 32, u0 0.108, 20000 steps in FP64, 100 in
    FP32 as every FP32 field check) against the oracle; the FP64 steady
    temperature is the linear conduction profile (no viscous heating) within
    1e-3 of the heating amplitude the total-energy DF shows."""
    case = W.couette(u0=0.108012345).with_(energy_df=1)
    n = case.steps if storage == "f64" else 100
    say(f"case internal-energy couette 8x32 {storage} {n} steps")
    g, o = _pair(T, case, n, storage)
    e = rel_err(g, o, case)
    say(f"  errors {e}")
    assert max(e.values()) < tol
    if storage == "f64":
        _, Ta = W.couette_closed_form(case)
        Tlin = 1.0 + 0.02 * np.arange(case.ny) / case.meta["H"]
        assert np.abs(g[3] - Tlin[:, None]).max() < 1e-3 * np.abs(Ta - Tlin).max()


def _table3_printed():
    rows = {}
    for line in open(os.path.join(GOLD, "rb_nusselt_table3.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            ra, nu_n, nu_ref = line.split()[:3]
            rows[float(ra)] = (float(nu_n), float(nu_ref))
    return rows


def test_table3_sweep(T):
    """Table 3's five Rayleigh numbers at the paper's resolutions (2N x N,
    N = 80/100/150), started from a density perturbation of the critical
    mode's shape (one pair of rolls across the 2:1 box, the state Table 3
    describes), all five lattices stepped as one FP32 batch for as long as
    the stored FP64 oracle runs (100 flow times, 150 at Ra 2500), Nu sampled
    on the oracle's schedule and averaged over its last 10 flow times.  Each
    Nu is within 1e-3 of the oracle's, every run keeps two rolls, Nu grows
    with Ra, and against the printed values the sweep is low by 2.1-3.4%
    (the oracle: 1.4372, 2.0527, 2.5805, 3.5046, 4.0393 against 1.468, 2.106,
    2.650, 3.629, 4.181), checked within 5%.  The total-energy DF gives the
    same Nu within 0.3% at Ra 1e4, so the deficit is not the energy DF's."""
    path = os.path.join(GOLD, "rb_table3_internal_fp64.json")
    if not os.path.exists(path):
        pytest.skip("rb_table3_internal_fp64.json not generated")
    import torch
    from paper_1610_07114_amd import serving as S
    g = json.load(open(path))
    printed = _table3_printed()
    runs = g["runs"]
    cases = [W.rb_table3(r["Ra"]) for r in runs]
    for r, c in zip(runs, cases):
        assert (c.nx, c.ny) == (r["nx"], r["ny"])
    say("case table 3 sweep fp32 batch: " + ", ".join(f"Ra {r['Ra']:g} {r['nx']}x{r['ny']}" for r in runs))
    stream = torch.cuda.Stream()
    lats = [T.Lattice(c, storage="f32", stream=stream) for c in cases]
    b = T.Batch(lats)
    b.set_graph_chunk(16)
    points = sorted({s for r in runs for s in range(r["every"], r["total"] + 1, r["every"])})
    samples = [[] for _ in runs]
    done = 0
    for p in points:
        b.step(p - done)
        done = p
        for k, (r, lat, c) in enumerate(zip(runs, lats, cases)):
            if p % r["every"] == 0 and r["avg_from"] < p <= r["total"]:
                _, _, _, _, s = lat.moments(fields=False)
                samples[k].append(S.nusselt_from_sums(c, s))
    b.close()
    from test_gpu_serving import _rolls
    rolls = [_rolls(lat.moments()[2]) for lat in lats]
    for lat in lats:
        lat.close()
    nus = []
    for r, smp, nr in zip(runs, samples, rolls):
        nu = float(np.mean(smp))
        nus.append(nu)
        pn, pref = printed[r["Ra"]]
        say(f"  Ra {r['Ra']:g}: Nu {nu:.5f}, oracle {r['nu_mean']:.5f} ({abs(nu / r['nu_mean'] - 1):.1e}), "
            f"paper {pn} ({nu / pn - 1:+.2%}), reference {pref} ({nu / pref - 1:+.2%}); rolls {nr}")
        assert abs(nu - r["nu_mean"]) / r["nu_mean"] < 1e-3
        assert abs(nu - pn) / pn < 0.05
        assert nr == 2
    assert all(a < b for a, b in zip(nus, nus[1:]))


def test_internal_energy_16bit_storage(T):
    """The internal-energy DF with FP16 storage (the generic 16-bit
    instantiation), RB 256 x 128 from near rest, 100 steps: rho and T within
    the FP16 bound of their maxima and the perturbations within the FP16
    perturbation bound of the total-energy path."""
    from test_gpu_parity import PERT_TOL_16
    case = W.rayleigh_benard(nx=256, ny=128, Ra=1e4, Pr=0.71, dT=0.06, seed=4, noise=1e-3).with_(energy_df=1)
    say("case internal-energy rayleigh-benard 256x128 f16 storage 100 steps")
    g, o = _pair(T, case, 100, "f16")
    e, p = rel_err(g, o, case), pert_err(g, o, case)
    say(f"  errors {e}; perturbation errors {p}")
    assert max(e["rho"], e["T"]) < 2e-3
    assert max(p.values()) < PERT_TOL_16["f16"]


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_mixed_batch_equals_members_alone(T, storage):
    """A batch whose members run the internal-energy DF and the default
    total-energy DF side by side (the batch kernel picks the scheme per
    member) leaves every member bitwise where it would be alone."""
    import torch
    cases = [W.rayleigh_benard(nx=130, ny=67, Ra=1e4, Pr=0.71, dT=0.06, seed=5, noise=1e-3).with_(energy_df=1),
             W.rayleigh_benard(nx=200, ny=41, Ra=2e4, Pr=0.71, seed=6, noise=1e-3),
             W.couette(u0=0.05, w2=1.0, w3=1.0, w4=1.0).with_(energy_df=1)]
    say(f"case mixed batch {storage}: internal-energy and total-energy members, 53 steps")
    stream = torch.cuda.Stream()
    alone = []
    for c in cases:
        lat = T.Lattice(c, storage=storage, stream=stream)
        lat.step(53)
        alone.append(lat.read_state())
        lat.close()
    lats = [T.Lattice(c, storage=storage, stream=stream) for c in cases]
    b = T.Batch(lats)
    b.set_graph_chunk(16)
    b.step(53)
    b.close()
    for k, lat in enumerate(lats):
        assert np.array_equal(lat.read_state(), alone[k]), k
        lat.close()
