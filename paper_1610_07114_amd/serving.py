"""Continuous-batching solve server and the batched-lattice autotuner.

Requests (Rayleigh-Benard or thermal Couette solves of different sizes and
Rayleigh/Prandtl numbers) arrive over time.  The server admits each one as
soon as its device footprint (tclbm_state_bytes) fits the HBM budget and a slot
is free, keeps every admitted lattice resident on the GPU, and advances all
resident lattices together with one batched kernel launch per time step
(tclbm_batch_*), in quanta that end exactly when the next request completes.
A finished request is reduced to its FP64 Nusselt number and its memory is
released, which lets queued requests in.  Because every lattice's arithmetic
is independent of the others and of the batch composition, a result is the
same whether a request ran alone or in the mix.

The autotuner times the batch's launch shape (rows per wave strip, HIP-graph
chunk) and keeps the fastest.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import tclbm
from . import workloads as W


# ------------------------------------------------------------------ requests ---
@dataclass
class Request:
    rid: int
    kind: str          # "rb" or "couette"
    nx: int
    ny: int
    Ra: float
    Pr: float
    steps: int
    arrival: float     # seconds after the start of the run
    seed: int
    # restart: initial rho, ux, uy, T ([ny, nx] float64) in place of the
    # seeded conduction state (RB only)
    init: Optional[dict] = field(default=None, repr=False)

    def case(self) -> W.Case:
        if self.kind == "rb":
            c = W.rayleigh_benard(nx=self.nx, ny=self.ny, Ra=self.Ra, Pr=self.Pr, seed=self.seed)
            if self.init is not None:
                c = c.with_(**{k: np.ascontiguousarray(self.init[k], dtype=np.float64)
                               for k in ("rho", "ux", "uy", "T")})
            return c
        # w2 = w3 = w4 = 1 as in the paper's other thermal cases: its Couette
        # set (1.1, 1.6, 0.3) is unstable to 2-D perturbations, which a
        # Couette lattice wider than it is periodic only escapes while it
        # stays exactly 1-D
        return W.couette(nx=self.nx, ny=self.ny, u0=0.05, Pr=self.Pr, w2=1.0, w3=1.0, w4=1.0)


def solve_steps(kind: str, ny: int, time_units: float) -> int:
    """Run length: time_units of the flow's own time scale, H/u_c for RB
    (u_c = 0.08) and H/u0 for Couette (u0 = 0.05)."""
    u = 0.08 if kind == "rb" else 0.05
    return max(1, int(round(time_units * (ny - 1) / u)))


def make_requests(n: int, rate: float, seed: int = 0, nmin: int = 32, nmax: int = 1024, rb_frac: float = 0.8,
                  time_units: float = 1.0, Ra_range=(1e4, 1e6), Pr_range=(0.5, 7.0),
                  tau_min: float = W.TAU_STABLE) -> List[Request]:
    """Seeded Poisson arrivals (rate per second) of 2N x N solves, N log-uniform
    on [nmin, nmax], Ra log-uniform, Pr uniform, 80% RB / 20% Couette.  As in
    the batched workload, an RB draw whose 1/w1 falls below `tau_min` (the
    scheme's linear stability limit) is drawn again."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        N = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        kind = "rb" if rng.uniform() < rb_frac else "couette"
        Ra = math.exp(rng.uniform(math.log(Ra_range[0]), math.log(Ra_range[1])))
        Pr = float(rng.uniform(*Pr_range))
        if kind == "rb" and W.rb_tau_f(N, Ra, Pr) < tau_min:
            # redraws come from a generator of their own (keyed by the stream
            # seed and the request index), so arrivals, kinds and the other
            # requests do not depend on them
            r2 = np.random.default_rng([seed, i])
            while W.rb_tau_f(N, Ra, Pr) < tau_min:
                N = int(round(math.exp(r2.uniform(math.log(nmin), math.log(nmax)))))
                Ra = math.exp(r2.uniform(math.log(Ra_range[0]), math.log(Ra_range[1])))
                Pr = float(r2.uniform(*Pr_range))
        out.append(Request(i, kind, 2 * N, N, Ra, Pr, solve_steps(kind, N, time_units), t, seed * 100003 + i))
    return out


def mean_work(requests: Sequence[Request]) -> float:
    """Mean lattice updates per request (nodes x steps)."""
    return sum(r.nx * r.ny * r.steps for r in requests) / max(1, len(requests))


def nusselt_from_sums(case: W.Case, sums) -> float:
    """Nu = 1 + <u_y (T - T0)> H / (kappa dT) from the FP64 device sums."""
    if case.name != "rayleigh_benard":
        return float("nan")
    m = case.meta
    return 1.0 + sums.nu_num / case.nodes * m["H"] / (m["kappa"] * m["dT"])


@dataclass
class Result:
    rid: int
    kind: str
    nx: int
    ny: int
    steps: int
    arrival: float
    admitted: float
    finished: float
    nu: float
    status: str
    state: Optional[np.ndarray] = field(default=None, repr=False)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


# -------------------------------------------------------------------- server ---
class Server:
    """Continuous batching of resident lattices on one GPU."""

    def __init__(self, storage: str = "f16", hbm_budget: Optional[int] = None, max_slots: int = 512,
                 quantum: int = 4096, quantum_s: float = 0.02, device: str = "cuda:0", graph_chunk: int = 16,
                 strip_rows: int = 0, keep_states: Sequence[int] = ()):
        """storage: "f32", "f16" or "bf16" (16-bit forms store deviations from
        the rest equilibrium).  hbm_budget: bytes of lattice state allowed at
        once (default 80% of free device memory).  max_slots: resident lattices
        at most.  A quantum (steps between admission/retirement points) lasts
        about quantum_s seconds, at most `quantum` steps, and never runs past
        the next completion.  strip_rows, graph_chunk: batch launch shape
        (strip_rows 0 = the batch's automatic choice).  keep_states: request
        ids whose final states are read back (for tests)."""
        import torch
        self.torch = torch
        self.storage = storage
        self.device = torch.device(device)
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            hbm_budget = int(free * 0.8)
        self.budget = hbm_budget
        self.max_slots = max_slots
        self.quantum = quantum
        self.quantum_s = quantum_s
        self.graph_chunk = graph_chunk
        self.strip_rows = strip_rows
        self.keep = set(keep_states)
        self.stream = torch.cuda.Stream(self.device)
        self.phase_s: Dict[str, float] = {}   # host seconds per phase of the last run
        self.rebatches = 0
        self.quanta = 0

    def footprint(self, req: Request) -> int:
        p = tclbm.tclbm_default_params(req.nx, req.ny)
        p.storage = tclbm.STORE[self.storage]
        return tclbm.tclbm_state_bytes(p)

    def run(self, requests: Sequence[Request], realtime: bool = True, log=None) -> List[Result]:
        pending = sorted(requests, key=lambda r: r.arrival)
        active: Dict[int, list] = {}   # rid -> [lattice, remaining, req, admitted, bytes]
        used = 0
        results: List[Result] = []
        batch = None
        dirty = True
        step_s = None    # measured seconds per step of the latest quantum
        ph = {"admit": 0.0, "rebatch": 0.0, "step": 0.0, "retire": 0.0, "idle": 0.0}
        self.phase_s = ph
        self.rebatches = 0
        self.quanta = 0
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        while pending or active:
            # admission: first come, first served, by footprint
            ta = time.perf_counter()
            while pending and (not realtime or pending[0].arrival <= now()) and len(active) < self.max_slots:
                req = pending[0]
                nb = self.footprint(req)
                if used + nb > self.budget and active:
                    break
                pending.pop(0)
                lat = tclbm.Lattice(req.case(), storage=self.storage, device=str(self.device), stream=self.stream)
                active[req.rid] = [lat, req.steps, req, now(), lat.nbytes]
                used += lat.nbytes
                dirty = True
            ph["admit"] += time.perf_counter() - ta
            if not active:
                if pending and realtime:
                    ti = time.perf_counter()
                    time.sleep(max(0.0, min(pending[0].arrival - now(), 0.01)))
                    ph["idle"] += time.perf_counter() - ti
                continue
            tb = time.perf_counter()
            if dirty:
                self.rebatches += 1
                if batch is not None:
                    batch.close()
                batch = tclbm.Batch([a[0] for a in active.values()])
                batch.set_graph_chunk(self.graph_chunk)
                if self.strip_rows:
                    batch.set_strip_rows(self.strip_rows)
                dirty = False
            ph["rebatch"] += time.perf_counter() - tb
            # quantum: about quantum_s of device time, ending at the next completion
            q = min(self.quantum, min(a[1] for a in active.values()))
            q = min(q, 64 if step_s is None else max(16, int(self.quantum_s / step_s)))
            tq = time.perf_counter()
            batch.step(q)
            self.stream.synchronize()
            step_s = (time.perf_counter() - tq) / q
            ph["step"] += time.perf_counter() - tq
            self.quanta += 1
            tr = time.perf_counter()
            done = []
            for rid, a in active.items():
                a[1] -= q
                if a[1] <= 0:
                    done.append(rid)
            if done:
                batch.close()
                batch = None
                dirty = True
            for rid in done:
                lat, _, req, adm, nb = active.pop(rid)
                _, _, _, _, s, st = tclbm.tclbm_moments(lat.h, req.nx, req.ny, fields=False, check=False)
                status = "ok" if st == tclbm.OK else "unstable"
                nu = nusselt_from_sums(lat.case, s) if status == "ok" else float("nan")
                state = lat.read_state() if rid in self.keep else None
                results.append(Result(rid, req.kind, req.nx, req.ny, req.steps, req.arrival, adm, now(), nu, status,
                                      state))
                lat.close()
                used -= nb
                if log:
                    log(f"done {rid} {req.kind} {req.nx}x{req.ny} steps {req.steps} nu {nu:.5f} {status} "
                        f"latency {results[-1].latency:.3f}s active {len(active)}")
            ph["retire"] += time.perf_counter() - tr
        if batch is not None:
            batch.close()
        return sorted(results, key=lambda r: r.rid)


def summarize(results: Sequence[Result], wall: float) -> dict:
    lat = np.array([r.latency for r in results])
    lups = sum(r.nx * r.ny * r.steps for r in results)
    return {
        "requests": len(results),
        "solves_per_s": round(len(results) / wall, 3),
        "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
        "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
        "mlups": round(lups / wall / 1e6, 3),
        "unstable": int(sum(r.status != "ok" for r in results)),
        "wall_s": round(wall, 2),
    }


# ----------------------------------------------------------------- autotuner ---
def autotune_batch(batch, rows=(0, 2, 4, 8, 16, 32), chunks=(8, 16, 32), steps: int = 40, log=None) -> dict:
    """Time `batch` with every strip height (rows per wave strip, 0 = the
    batch's automatic choice) and HIP-graph chunk, keep the fastest on the
    batch and return it.  Advances the members by
    len(rows) * len(chunks) * (steps + 2 * chunk) steps, so tune throw-away
    copies where the state matters."""
    best = None
    for r in rows:
        batch.set_strip_rows(r)
        for ch in chunks:
            batch.set_graph_chunk(ch)
            batch.step(2 * ch)                      # capture the graph, warm up
            ms = batch.step_timed(steps)
            if log:
                log(f"autotune strip rows {r} (in use {batch.strip_rows}) graph chunk {ch}: "
                    f"{ms / steps * 1e3:.1f} us/step")
            if best is None or ms < best[0]:
                best = (ms, r, ch, batch.strip_rows)
    batch.set_strip_rows(best[1])
    batch.set_graph_chunk(best[2])
    return {"strip_rows": best[1], "strip_rows_in_use": best[3], "graph_chunk": best[2],
            "us_per_step": round(best[0] / steps * 1e3, 2)}


def autotune_cases(cases: Sequence[W.Case], storage: str = "f32", cache: Optional[str] = None, device="cuda:0",
                   log=None, **kw) -> dict:
    """autotune_batch on throw-away lattices built from `cases`; the choice is
    stored in `cache` (JSON, keyed by storage and the multiset of shapes)."""
    import torch
    shapes = sorted((c.nx, c.ny) for c in cases)
    key = f"{storage}:{len(shapes)}:{hash(tuple(shapes)) & 0xffffffff:x}"
    if cache and os.path.exists(cache):
        try:
            got = json.load(open(cache)).get(key)
            if got:
                return got
        except Exception:
            pass
    stream = torch.cuda.Stream(torch.device(device))
    lats = [tclbm.Lattice(c, storage=storage, device=device, stream=stream) for c in cases]
    b = tclbm.Batch(lats)
    choice = autotune_batch(b, log=log, **kw)
    b.close()
    for lat in lats:
        lat.close()
    if cache:
        data = {}
        if os.path.exists(cache):
            try:
                data = json.load(open(cache))
            except Exception:
                data = {}
        data[key] = choice
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        json.dump(data, open(cache, "w"), indent=1)
    return choice
