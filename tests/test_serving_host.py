"""Host logic of the serving loop and the batched workload generator (no GPU):
seeded request streams have the stated distributions, run lengths follow the
flow's time scale, and the latency summary is computed from the results."""
import math

import numpy as np
import pytest

from paper_1610_07114_amd import workloads as W


@pytest.fixture(scope="module")
def S():
    from paper_1610_07114_amd import serving
    return serving


def test_request_stream_is_seeded_and_shaped(S):
    # the unconditioned draws (every RB draw kept) carry the stated distributions
    a = S.make_requests(2000, rate=50.0, seed=11, tau_min=0.0)
    b = S.make_requests(2000, rate=50.0, seed=11, tau_min=0.0)
    assert [(r.nx, r.ny, r.kind, r.Ra, r.Pr, r.arrival) for r in a] == \
           [(r.nx, r.ny, r.kind, r.Ra, r.Pr, r.arrival) for r in b]
    N = np.array([r.ny for r in a])
    assert N.min() >= 32 and N.max() <= 1024
    assert all(r.nx == 2 * r.ny for r in a)
    # log-uniform: the median of log N sits mid-way between log 32 and log 1024
    assert abs(np.median(np.log(N)) - 0.5 * (math.log(32) + math.log(1024))) < 0.15
    frac_rb = np.mean([r.kind == "rb" for r in a])
    assert abs(frac_rb - 0.8) < 0.03
    gaps = np.diff([0.0] + [r.arrival for r in a])
    assert abs(gaps.mean() - 1 / 50.0) < 0.1 / 50.0          # Poisson rate
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.1          # exponential gaps
    Pr = np.array([r.Pr for r in a])
    assert Pr.min() >= 0.5 and Pr.max() <= 7.0
    Ra = np.array([r.Ra for r in a])
    assert Ra.min() >= 1e4 and Ra.max() <= 1e6


def test_rb_requests_are_above_the_stability_limit(S):
    """By default an RB draw below 1/w1 = 0.55 is drawn again; Couette
    requests are untouched (1/w1 = 0.65)."""
    a = S.make_requests(2000, rate=50.0, seed=11)
    raw = S.make_requests(2000, rate=50.0, seed=11, tau_min=0.0)
    assert min(W.rb_tau_f(r.ny, r.Ra, r.Pr) for r in a if r.kind == "rb") >= W.TAU_STABLE
    assert any(W.rb_tau_f(r.ny, r.Ra, r.Pr) < W.TAU_STABLE for r in raw if r.kind == "rb")
    # arrivals and kinds do not depend on the redraws
    assert [(r.arrival, r.kind) for r in a] == [(r.arrival, r.kind) for r in raw]
    assert all((x.ny, x.Ra, x.Pr) == (y.ny, y.Ra, y.Pr) for x, y in zip(a, raw)
               if x.kind == "couette" or W.rb_tau_f(y.ny, y.Ra, y.Pr) >= W.TAU_STABLE)


def test_restart_request_uses_its_fields(S):
    ny, nx = 6, 12
    f = {"rho": np.full((ny, nx), 1.01), "ux": np.full((ny, nx), 0.002), "uy": np.zeros((ny, nx)),
         "T": np.full((ny, nx), 1.003)}
    q = S.Request(0, "rb", nx, ny, 2e4, 0.71, 10, 0.0, 3, init=f)
    c = q.case()
    for k in ("rho", "ux", "uy", "T"):
        assert np.array_equal(getattr(c, k), f[k])
    assert c.meta["Ra"] == 2e4 and c.bc == (W.PERIODIC, W.PERIODIC, W.WALL, W.WALL)


def test_run_length_follows_time_scale(S):
    assert S.solve_steps("rb", 33, 1.0) == round(32 / 0.08)
    assert S.solve_steps("couette", 33, 2.0) == round(2 * 32 / 0.05)
    assert S.solve_steps("rb", 3, 1e-6) == 1


def test_request_cases(S):
    r = S.make_requests(5, rate=1.0, seed=2, nmin=32, nmax=40)
    for q in r:
        c = q.case()
        assert (c.nx, c.ny) == (q.nx, q.ny)
        if q.kind == "rb":
            assert c.name == "rayleigh_benard" and c.meta["Ra"] == q.Ra and c.Pr == q.Pr
        else:
            assert c.name == "couette" and c.Pr == q.Pr


def test_summary(S):
    res = [S.Result(i, "rb", 64, 32, 100, arrival=float(i), admitted=float(i), finished=float(i) + 0.5 + 0.01 * i,
                    nu=1.0, status="ok") for i in range(101)]
    s = S.summarize(res, wall=10.0)
    assert s["requests"] == 101
    assert s["solves_per_s"] == pytest.approx(10.1)
    assert s["p50_latency_s"] == pytest.approx(1.0)
    assert s["p99_latency_s"] == pytest.approx(0.5 + 0.99, abs=1e-9)
    assert s["mlups"] == pytest.approx(101 * 64 * 32 * 100 / 10.0 / 1e6, rel=1e-3)


def test_batched_specs_shape():
    raw = W.batched_rb_specs(256, seed=0, tau_min=0.0)
    assert raw == W.batched_rb_specs(256, seed=0, tau_min=0.0)
    N = np.array([s["ny"] for s in raw])
    assert N.min() >= 32 and N.max() <= 512
    assert all(s["nx"] == 2 * s["ny"] for s in raw)
    assert [s["seed"] for s in raw] == list(range(256))
    nodes = sum(s["nx"] * s["ny"] for s in raw)
    # E[2N^2] for N log-uniform on [32, 512] is about 94,000 nodes per lattice
    assert 0.7 * 256 * 94180 < nodes < 1.3 * 256 * 94180


def test_batched_specs_are_conditioned_on_stability():
    """The default list is the draw sequence with the draws below the scheme's
    linear stability limit (1/w1 < 0.55) left out and 256 kept."""
    rejected = []
    specs = W.batched_rb_specs(256, seed=0, rejected=rejected)
    assert len(specs) == 256 and len(rejected) > 0
    assert all(W.rb_tau_f(s["ny"], s["Ra"], s["Pr"]) >= W.TAU_STABLE for s in specs)
    assert all(W.rb_tau_f(s["ny"], s["Ra"], s["Pr"]) < W.TAU_STABLE for s in rejected)
    long_raw = W.batched_rb_specs(256 + len(rejected), seed=0, tau_min=0.0)
    key = lambda s: (s["nx"], s["ny"], s["Ra"], s["Pr"])
    assert [key(s) for s in long_raw if W.rb_tau_f(s["ny"], s["Ra"], s["Pr"]) >= W.TAU_STABLE] == \
           [key(s) for s in specs]
    assert [s["seed"] for s in specs] == list(range(256))
