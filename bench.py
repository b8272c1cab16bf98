#!/usr/bin/env python3
"""Benchmark of the fused TCLBM step on one MI355X.

One "step" is one time step of the whole hot path over every lattice of the
workload: pull streaming, wall treatment, macroscopic variables, correction
gradients, cascaded collision of f with force and correction sources,
energy-DF collision with the coupling source, store (one fused kernel per step
for all lattices), plus the FP64 reductions (mass, energy, Nusselt numerator)
every `--reduce-every` steps.  Inputs are seeded and synthetic and resident in
HBM before timing starts.

Prints one JSON line on stdout.  The default workload is the batched
Rayleigh-Benard configuration: 256 seeded uneven 2N x N lattices (N
log-uniform on [32, 512], Ra log-uniform on [1e4, 1e6], Pr uniform on
[0.5, 7], FP32 storage) advanced together by one launch per step, replayed
from HIP graphs, with the launch shape picked by the autotuner during the
warm-up.  `value` is its whole-job MLUPS (wall clock around exactly --steps
steps); `roofline` is the HBM roofline of its kernel (algorithmic bytes per
launch / average launch time from HIP events on the batch's stream over the
timed steps); `cpu_baseline` is the FP64 CPU reference timed on the host cores
over a bounded sample of the same batch.  The line also carries, measured in
the same run (unless --no-extras):
  rb512x256       the single 512x256 Rayleigh-Benard lattice (cache-resident)
  shock_tube      the 8192x4 shock tube
  roofline_large  the step kernel on an 8192x4096 lattice (HBM-resident
                  state) with FP32, FP16 and BF16 storage
  table3          Section 5D's Nu(Ra) sweep with the internal-energy DF
  persistent_batch  persistent batched launches against per-step graph replays
  hbm_ceiling     a 2 GiB streaming copy on the same GPU with the step kernels'
                  access types; the HBM-resident figures also state their
                  fraction of it
  serving         seeded Poisson streams of RB/Couette solve requests served
                  with continuous batching and FP16 or BF16 storage (solves/s,
                  p50/p99 latency, Nu error of requests restarted from FP64
                  steady states), and the same stream through the plain
                  one-lattice-at-a-time FP32 path
  cpu_baseline_detail  the FP64 oracle on one thread and on all threads for the
                  Couette, shock-tube and 512x256 Rayleigh-Benard workloads,
                  with the host's CPU count and model
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
GOLDEN_BATCH_NU = os.path.join(ROOT, "tests", "golden", "rb_batch_nu_fp64.json")
GOLDEN_STEADY_FIELDS = os.path.join(ROOT, "tests", "golden", "rb_batch_steady_fields.npz")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload_case(name: str):
    from paper_1610_07114_amd import workloads as W
    if name == "rb":
        return W.rayleigh_benard(nx=512, ny=256, Ra=1e5, Pr=0.71, seed=0), "rayleigh_benard_512x256"
    if name == "shock":
        return W.shock_tube(), "shock_tube_8192x4"
    if name == "couette":
        return W.couette(), "couette_8x32"
    if name == "large":
        return W.rayleigh_benard(nx=8192, ny=4096, Ra=1e5, Pr=0.71, seed=0), "rayleigh_benard_8192x4096"
    raise SystemExit(f"unknown workload {name}")


def bytes_per_lup(storage: str, thermal: int = 1) -> int:
    per = {"f32": 4, "f16": 2, "bf16": 2, "f64": 8}[storage]
    planes = 18 if thermal else 9
    return 2 * planes * per  # each population read once and written once


def roofline(bpl: int, nodes: int, avg_launch_s: float, traffic=None, kernel="step_kernel"):
    achieved = bpl * nodes / avg_launch_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
            "bytes_per_lup": bpl, "lups_per_launch": nodes, "avg_launch_us": round(avg_launch_s * 1e6, 3)}


def load_traffic(path, key):
    """Per-launch HBM bytes from the rocprofv3 counter runs, if taken for this
    kernel build and workload (null otherwise)."""
    try:
        tj = json.load(open(path))
        from paper_1610_07114_amd import build as B
        ent = tj.get(key)
        if ent and ent.get("kernel_sources") == B.source_digest():
            return ent["bytes_per_launch"]
    except Exception:
        pass
    return None


# ------------------------------------------------------------------ CPU baseline ---
def _time_oracle(cases, seconds_target: float):
    """Steps the FP64 oracle over the given lattices (round robin, whole
    lattices) for about `seconds_target` seconds: (MLUPS, steps, seconds)."""
    import oracle as O
    lats = []
    for case in cases:
        p = O.Params(nx=case.nx, ny=case.ny, R=case.R, T0=case.T0, gamma=case.gamma, Pr=case.Pr,
                     tau_f=case.tau_f, w2=case.w2, w3=case.w3, w4=case.w4, ax=case.ax, ay=case.ay,
                     thermal=case.thermal, correction=case.correction, bc=case.bc, wall_ux=case.wall_ux,
                     wall_uy=case.wall_uy, wall_T=case.wall_T, ax_field=case.ax_field, ay_field=case.ay_field)
        lats.append((case, O.Lattice(p, case.rho, case.ux, case.uy, case.T)))
    nodes = sum(c.nx * c.ny for c, _ in lats)
    t0 = time.perf_counter()
    for _, L in lats:
        L.step(2)
    dt = max(time.perf_counter() - t0, 1e-6)
    n = max(2, min(5000, int(seconds_target / (dt / 2))))
    t0 = time.perf_counter()
    for _, L in lats:
        L.step(n)
    dt = time.perf_counter() - t0
    return nodes * n / dt / 1e6, n, dt


def cpu_baseline(cases, seconds_target: float = 12.0, label=None):
    """The FP64 oracle as it stands, on the host cores, over a bounded number of
    steps of the given lattices (round robin, whole lattices)."""
    import oracle as O
    mlups, n, dt = _time_oracle(cases, seconds_target)
    what = label or f"{cases[0].name} {cases[0].nx}x{cases[0].ny}"
    return {"value": round(mlups, 3), "unit": "MLUPS", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{what}, {n} steps from the seeded initial state, FP64, {dt:.1f} s"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline_detail(seconds_target: float = 3.0) -> dict:
    """The FP64 oracle on one thread and on all its threads for the Couette,
    shock-tube and Rayleigh-Benard workloads (each timed over about
    `seconds_target` seconds), with the host's CPU count and model."""
    import oracle as O
    full = O.num_threads()
    out = {"nproc": os.cpu_count(), "cpu_model": cpu_model(), "unit": "MLUPS", "threads": sorted({1, full}),
           "seconds_per_sample": seconds_target, "cases": {}}
    try:
        for name in ("couette", "shock", "rb"):
            case, wname = workload_case(name)
            row = {}
            for t in out["threads"]:
                O.set_num_threads(t)
                mlups, n, _ = _time_oracle([case], seconds_target)
                row[f"threads_{t}"] = round(mlups, 3)
                row[f"steps_{t}"] = n
            out["cases"][wname] = row
    finally:
        O.set_num_threads(full)
    return out


# ------------------------------------------------------------------- probes ---
def copy_probe(torch, tclbm, nbytes: int = 2 << 30, reps: int = 20):
    """Achievable HBM bandwidth of a streaming copy with the step kernels'
    access types (one 16-byte element per thread, plain load, non-temporal
    store; read + write bytes per launch / launch time), the measured ceiling
    beside the 8 TB/s peak."""
    dev = torch.device("cuda:0")
    s = torch.cuda.Stream(dev)
    with torch.cuda.stream(s):
        a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        b = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        a.fill_(1)
    for _ in range(3):
        tclbm.tclbm_hbm_copy(b.data_ptr(), a.data_ptr(), nbytes, s.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        tclbm.tclbm_hbm_copy(b.data_ptr(), a.data_ptr(), nbytes, s.cuda_stream)
    e1.record(s)
    torch.cuda.synchronize(dev)
    ms = e0.elapsed_time(e1) / reps
    return {"probe": "hbm_copy", "bytes_per_launch": 2 * nbytes, "avg_launch_us": round(ms * 1e3, 2),
            "GBs": round(2 * nbytes / (ms / 1e3) / 1e9, 1), "peak_GBs": HBM_PEAK_GBS}


# ---------------------------------------------------------------- one lattice ---
def bench_single(torch, tclbm, case, storage, steps, warmup, reduce_every, strip_rows, graph_chunk):
    dev = torch.device("cuda:0")
    lat = tclbm.Lattice(case, storage=storage, device="cuda:0")
    lat.set_tuning(strip_rows, graph_chunk)
    nodes = case.nx * case.ny

    def run(nsteps):
        done = 0
        while done < nsteps:
            k = min(reduce_every, nsteps - done)
            lat.step(k)
            done += k
            if done % reduce_every == 0:
                lat.moments(fields=False)   # FP64 sums (mass, energy, Nusselt numerator)

    run(warmup)
    torch.cuda.synchronize(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(lat.stream)
    run(steps)
    ev1.record(lat.stream)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    dev_ms = ev0.elapsed_time(ev1)
    # kernel-only average: a separate pass of pure steps timed with HIP events
    # on the library's stream (graph replays of the same kernel)
    kern_ms = lat.step_timed(steps)
    _, _, _, _, sums = lat.moments(fields=False)
    kernel = lat.kernel
    lat.close()
    return dict(wall=wall, dev_ms=dev_ms, avg_launch_s=kern_ms / 1e3 / steps, nodes=nodes, sums=sums, kernel=kernel)


# -------------------------------------------------------------------- batch ---
def bench_batch(torch, tclbm, n=256, seed=0, storage="f32", steps=1000, warmup=200, reduce_every=1000,
                strip_rows=0, graph_chunk=None, traffic_json=None, persistent=0):
    """The batched workload: n seeded 2N x N Rayleigh-Benard lattices (N
    log-uniform on [32, 512], Ra log-uniform on [1e4, 1e6], Pr uniform on
    [0.5, 7]; draws below the scheme's linear stability limit 1/w1 = 0.55 are
    drawn again) advanced together, one launch per step, HIP-graph chunks.  The
    autotuner's trial steps (strip height x graph chunk) are part of the
    warm-up; a given strip height (and graph chunk) replaces the autotuner.
    The graph chunk is capped at half the timed steps, so that the timed steps
    replay graphs.  Timed: exactly `steps` steps, with the FP64 sums of every
    member after each `reduce_every` of them; HIP events on the batch's stream
    bracket the same steps.  `traffic` is the stored counter measurement for
    the strip height in use.  persistent > 0: persistent launches of up to
    that many steps each instead (no traffic figure: the counters were taken
    on the per-step kernel)."""
    from paper_1610_07114_amd import serving as S
    from paper_1610_07114_amd import workloads as W
    rejected = []
    specs = W.batched_rb_specs(n, seed=seed, rejected=rejected)
    t0 = time.perf_counter()
    cases = [W.rb_from_spec(s) for s in specs]
    nodes = sum(c.nx * c.ny for c in cases)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    lats = [tclbm.Lattice(c, storage=storage, stream=stream) for c in cases]
    del cases
    log(f"batch: {n} seeded lattices resident, {nodes} nodes ({time.perf_counter() - t0:.1f} s; "
        f"{len(rejected)} draws below the stability limit drawn again)")
    b = tclbm.Batch(lats)
    tune = None
    if strip_rows > 0:
        b.set_strip_rows(strip_rows)
        chunk = graph_chunk if graph_chunk is not None else 16
    else:
        tune = S.autotune_batch(b, log=log)
        log(f"batch autotune: {tune}")
        chunk = tune["graph_chunk"]
    cap = (steps // 2) // 2 * 2
    chunk = min(chunk, cap) if cap >= 2 else 0
    b.set_graph_chunk(chunk)
    if persistent > 0:
        b.set_persistent(persistent)
    rows_in_use = b.strip_rows
    b.step(warmup)
    torch.cuda.synchronize(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reductions = 0
    t0 = time.perf_counter()
    ev0.record(stream)
    done = 0
    while done < steps:
        k = min(reduce_every, steps - done)
        b.step(k)
        done += k
        if done % reduce_every == 0:
            for lat in lats:   # FP64 sums (mass, energy, Nusselt numerator)
                tclbm.tclbm_moments(lat.h, lat.case.nx, lat.case.ny, fields=False, check=False)
            reductions += 1
    ev1.record(stream)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    dev_ms = ev0.elapsed_time(ev1)
    waves = b.waves
    kernel = b.kernel
    b.close()
    unstable = 0
    for lat in lats:
        _, _, _, _, _, st = tclbm.tclbm_moments(lat.h, lat.case.nx, lat.case.ny, fields=False, check=False)
        unstable += st != tclbm.OK
        lat.close()
    bpl = bytes_per_lup(storage)
    return {"workload": f"batched_rayleigh_benard_{n}x(2N x N, N log-uniform 32..512, seed {seed})",
            "instances": n, "nodes": nodes, "storage": storage, "steps": steps, "warmup": warmup,
            "mlups": round(nodes * steps / wall / 1e6, 1), "ms_per_step": round(wall * 1e3 / steps, 4),
            "device_ms": round(dev_ms, 3), "graph_chunk": chunk, "fp64_reductions_timed": reductions,
            "autotune": tune, "waves_per_step": waves, "unstable_instances": int(unstable),
            "redrawn_below_stability_limit": len(rejected), "strip_rows": rows_in_use,
            "roofline": roofline(bpl, nodes, dev_ms / 1e3 / steps,
                                 load_traffic(traffic_json, f"batched_rayleigh_benard_{n}_{storage}_rows{rows_in_use}")
                                 if traffic_json and persistent <= 0 else None, kernel=kernel),
            "persistent_steps_per_launch": persistent}


# ------------------------------------------------------------------ serving ---
def restart_requests(S, start_id, rate_span, seed=7, time_units=30.0):
    """Requests that restart the batched-subset instances whose FP64 oracle Nu
    ended steady from the oracle's final fields (populations rebuilt at
    equilibrium), at seeded arrival times inside the stream, for `time_units`
    flow times.  Starting on the FP64 steady state fixes the roll pattern, so
    the final Nu measures the storage precision; the reference is the stored
    FP64 time average."""
    import numpy as np
    try:
        g = json.load(open(GOLDEN_BATCH_NU))
        fields = np.load(GOLDEN_STEADY_FIELDS, allow_pickle=False)
    except Exception:
        return [], {}
    rng = np.random.default_rng(seed)
    out, ref = [], {}
    for k, inst in enumerate(g["instances"]):
        if not (math.isfinite(inst["nu_mean"]) and inst["unsteadiness"] < 2e-3
                and f"i{inst['index']}_rho" in fields):
            continue
        s = inst["spec"]
        rid = start_id + k
        init = {q: np.array(fields[f"i{inst['index']}_{q}"]) for q in ("rho", "ux", "uy", "T")}
        out.append(S.Request(rid, "rb", s["nx"], s["ny"], s["Ra"], s["Pr"], S.solve_steps("rb", s["ny"], time_units),
                             float(rng.uniform(0, rate_span)), s["seed"], init=init))
        ref[rid] = inst["nu_mean"]
    return out, ref


def _nu_errors(res, ref):
    import numpy as np
    errs = [abs(r.nu - ref[r.rid]) / abs(ref[r.rid]) for r in res if r.rid in ref]
    return {"max": max(errs) if errs else None, "median": float(np.median(errs)) if errs else None, "n": len(errs)}


def bench_serving(torch, tclbm, n_requests=500, storages=("f16",), seed=0, load=0.8, time_units=1.0,
                  sequential_fp32=True):
    """One seeded Poisson stream of `n_requests` RB/Couette solves per storage
    form, at `load` times the capacity measured in a closed-loop calibration
    run of the same distribution, served with continuous batching; plus the
    restart requests (Nu error), which are excluded from the latency figures.
    Optionally the same stream through the plain one-lattice-at-a-time FP32
    path."""
    from paper_1610_07114_amd import serving as S
    out = {"run_length": f"{time_units} H/u_c per request (u_c = 0.08 RB, u0 = 0.05 Couette)"}
    reqs_unit = S.make_requests(n_requests, rate=1.0, seed=seed, time_units=time_units)
    work = S.mean_work(reqs_unit)
    work_c4 = S.mean_work(S.make_requests(n_requests, rate=1.0, seed=seed, time_units=50.0))
    nu_fp32 = None
    for storage in storages:
        # capacity: the aggregate lattice-update rate of a closed-loop run
        # (everything queued at t = 0) of a calibration stream from the same
        # distribution, divided by the mean work of the stream's own requests
        # (the work per request is heavy-tailed, ~N^3)
        # (fewer calibration requests when each one is long)
        n_cal = max(40, n_requests // 8) if time_units <= 1.0 else max(8, n_requests // 4)
        calib = S.make_requests(n_cal, rate=1.0, seed=seed + 1000, time_units=time_units)
        for r in calib:
            r.arrival = 0.0
        srv = S.Server(storage=storage)
        t0 = time.perf_counter()
        res = srv.run(calib, realtime=False, log=log if time_units > 1.0 else None)
        cap_wall = time.perf_counter() - t0
        cal_lups = sum(r.nx * r.ny * r.steps for r in res) / cap_wall
        capacity = cal_lups / work
        rate = load * capacity
        reqs = S.make_requests(n_requests, rate=rate, seed=seed, time_units=time_units)
        span = reqs[-1].arrival
        gold, ref = restart_requests(S, n_requests, span)
        reqs = sorted(reqs + gold, key=lambda r: r.arrival)
        log(f"serving {storage}: closed loop {cal_lups / 1e6:.0f} MLUPS ({len(calib)} calibration requests, "
            f"{cap_wall:.1f} s), mean work {work:.3g} LUP -> capacity {capacity:.2f} solves/s; stream of "
            f"{len(reqs)} requests at {rate:.2f}/s over {span:.1f} s")
        t0 = time.perf_counter()
        # long requests: one line per completed request (progress of the run)
        res = srv.run(reqs, realtime=True, log=log if time_units > 1.0 else None)
        wall = time.perf_counter() - t0
        summ = S.summarize([r for r in res if r.rid not in ref], wall)
        out[storage] = {"arrival_rate_per_s": round(rate, 3), "load_vs_capacity": load,
                        "capacity_solves_per_s": round(capacity, 3), "closed_loop_mlups": round(cal_lups / 1e6, 1),
                        "mean_work_lup": round(work), **summ,
                        "capacity_solves_per_s_at_50_Huc": round(cal_lups / work_c4, 4),
                        "phases_s": {k: round(v, 2) for k, v in srv.phase_s.items()}, "rebatches": srv.rebatches,
                        "nu_restart_requests": len(gold),
                        "nu_rel_err_vs_fp64": _nu_errors(res, ref),
                        "_nu": {r.rid: r.nu for r in res if r.rid in ref}}
    if sequential_fp32:
        # the plain path: one FP32 lattice at a time, first come first served,
        # the last stream's arrivals
        srv1 = S.Server(storage="f32", max_slots=1)
        t0 = time.perf_counter()
        res1 = srv1.run(reqs, realtime=True, log=log if time_units > 1.0 else None)
        wall1 = time.perf_counter() - t0
        nu_fp32 = {r.rid: r.nu for r in res1 if r.rid in ref}
        out["single_lattice_fp32"] = {**S.summarize([r for r in res1 if r.rid not in ref], wall1),
                                      "nu_rel_err_vs_fp64": _nu_errors(res1, ref)}
    for storage in storages:
        nus = out[storage].pop("_nu")
        if nu_fp32:
            e = [abs(nus[k] - nu_fp32[k]) / abs(nu_fp32[k]) for k in nus if k in nu_fp32]
            m = max(e) if e else None
            # the 16-bit precision target: steady Nu within 5e-3 of the FP32
            # run from the identical start (the FP32 run's own offset from the
            # FP64 time average is the restart transient, the same in every
            # storage form)
            out[storage]["nu_rel_err_vs_fp32_same_start"] = {"max": m, "n": len(e),
                                                             "meets_5e-3": (m < 5e-3) if m is not None else None}
    out["restart_length"] = "restart requests run 30 H/u_c from the FP64 steady fields"
    return out


def bench_table3(torch, tclbm):
    """Section 5D's Nu(Ra) sweep with the internal-energy DF: the five Table 3
    lattices (2N x N, N = 80/100/150) as one FP32 batch from the critical-mode
    start, 100 flow times (150 at Ra 2500), Nu averaged over the last 10 flow
    times, against the printed values."""
    import numpy as np
    from paper_1610_07114_amd import serving as S
    from paper_1610_07114_amd import workloads as W
    cases = [W.rb_table3(Ra) for Ra in W.TABLE3_RA]
    sched = []
    for c in cases:
        tu = c.meta["H"] / c.meta["uc"]
        every = max(1, int(round(tu / 4)))
        total = int(round((150.0 if c.meta["Ra"] < 3000 else 100.0) * tu / every)) * every
        sched.append((every, total, total - int(round(10.0 * tu / every)) * every))
    stream = torch.cuda.Stream()
    lats = [tclbm.Lattice(c, storage="f32", stream=stream) for c in cases]
    b = tclbm.Batch(lats)
    b.set_graph_chunk(16)
    points = sorted({p for ev, tot, _ in sched for p in range(ev, tot + 1, ev)})
    samples = [[] for _ in cases]
    t0 = time.perf_counter()
    done = 0
    for p in points:
        b.step(p - done)
        done = p
        for k, (c, lat, (ev, tot, frm)) in enumerate(zip(cases, lats, sched)):
            if p % ev == 0 and frm < p <= tot:
                _, _, _, _, sm = lat.moments(fields=False)
                samples[k].append(S.nusselt_from_sums(c, sm))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b.close()
    for lat in lats:
        lat.close()
    out = {"workload": "rb_table3: 2N x N, N 80/100/150, dT 0.06, u_c 0.08, Pr 0.71, internal-energy DF, "
                       "FP32 batch of the five", "steps": done, "wall_s": round(wall, 2),
           "mlups": round(sum(c.nx * c.ny for c in cases) * done / wall / 1e6, 1), "nu": {}}
    for c, smp in zip(cases, samples):
        nu = float(np.mean(smp))
        pn, pref = W.TABLE3_NU[c.meta["Ra"]]
        out["nu"][f"{c.meta['Ra']:g}"] = {"nu": round(nu, 5), "paper": pn, "reference": pref,
                                           "rel_vs_paper": round(nu / pn - 1.0, 4)}
    return out


def bench_persistent(torch, tclbm):
    """Persistent batched launches (up to 256 steps per cooperative launch,
    a grid barrier between steps) against the default per-step launches
    replayed from 32-step graphs, on a small serving-sized batch, RB 512x256
    and the 256-lattice batch: device microseconds per step, best of two."""
    from paper_1610_07114_amd import workloads as W
    sets = [("8 x RB 64x32, f16", [W.rayleigh_benard(nx=64, ny=32, seed=i, noise=1e-3) for i in range(8)], "f16",
             2048),
            ("RB 512x256, f32", [W.rayleigh_benard(nx=512, ny=256, seed=0)], "f32", 2048),
            ("256 batched RB lattices, f32", [W.rb_from_spec(x) for x in W.batched_rb_specs(256, seed=0)], "f32",
             128)]
    stream = torch.cuda.Stream()
    out = {}
    for name, cases, storage, n in sets:
        lats = [tclbm.Lattice(c, storage=storage, stream=stream) for c in cases]
        b = tclbm.Batch(lats)
        b.set_graph_chunk(32)
        r = {}
        for mode, steps in (("graph_us_per_step", 0), ("persistent_us_per_step", 256)):
            b.set_persistent(steps)
            b.step(64)
            r[mode] = round(min(b.step_timed(n) for _ in range(2)) / n * 1e3, 2)
        r["persistent_kernel"] = b.kernel
        out[name] = r
        b.close()
        for lat in lats:
            lat.close()
    return out


def single_extra(torch, tclbm, name, storage, steps, warmup, traffic_json, reduce_every=1000):
    """A single-lattice figure measured beside the headline: MLUPS over `steps`
    steps (FP64 sums every `reduce_every`) and the roofline of its kernel."""
    case, wname = workload_case(name)
    r = bench_single(torch, tclbm, case, storage, steps, warmup, reduce_every, 0, 32)
    out = {"workload": wname, "storage": storage, "steps": steps,
           "mlups": round(r["nodes"] * steps / r["wall"] / 1e6, 1),
           **roofline(bytes_per_lup(storage, case.thermal), r["nodes"], r["avg_launch_s"],
                      load_traffic(traffic_json, f"{wname}_{storage}"), kernel=r["kernel"])}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="batch", choices=["batch", "rb", "shock", "couette", "large", "serve"])
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16", "f64"])
    ap.add_argument("--reduce-every", type=int, default=1000)
    ap.add_argument("--strip-rows", type=int, default=0)
    ap.add_argument("--batch-strip-rows", type=int, default=0,
                    help="batch workload: fixed strip height (with --graph-chunk) instead of the autotuner")
    ap.add_argument("--graph-chunk", type=int, default=32)
    ap.add_argument("--persistent", type=int, default=0,
                    help="batch workload: persistent launches of up to this many steps each")
    ap.add_argument("--requests", type=int, default=500, help="serving stream length")
    ap.add_argument("--serve-storage", default="f16,bf16", help="storage forms of the serving streams")
    ap.add_argument("--time-units", type=float, default=1.0, help="serving request length in flow times")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the selected workload (no other lattices, rooflines or serving figures)")
    ap.add_argument("--no-serving", action="store_true", help="extras without the serving streams")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="time the plain HBM copy kernel (2 x 2 GiB) instead and exit")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="per-launch HBM traffic from rocprofv3 counters (if measured for this kernel)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (the batched and single-lattice paths would shard by "
              "instance or by slab across GPUs, but no multi-GPU path is built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1610_07114_amd import tclbm

    if args.copy_probe:
        print(json.dumps(copy_probe(torch, tclbm)), flush=True)
        return

    serve_storages = tuple(x for x in args.serve_storage.split(",") if x)

    if args.workload == "serve":
        s = bench_serving(torch, tclbm, n_requests=args.requests, storages=serve_storages,
                          time_units=args.time_units)
        first = s[serve_storages[0]]
        out = {"metric": "batched serving solves/s", "value": first["solves_per_s"], "unit": "solves/s",
               "n_gpus": 1, "steps": first["requests"], "warmup": 0,
               "ms_per_step": round(1e3 / max(first["solves_per_s"], 1e-9), 3), "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded)",
               "config": {"workload": f"serving stream, {args.requests} requests, {args.time_units} H/u_c",
                          "storage": serve_storages[0]},
               "serving": s}
        print(json.dumps(out), flush=True)
        return

    if args.workload == "batch":
        log(f"bench: batched RB workload, 256 instances, {args.storage}, warmup {args.warmup}, steps {args.steps}")
        b = bench_batch(torch, tclbm, storage=args.storage, steps=args.steps, warmup=args.warmup,
                        reduce_every=args.reduce_every, strip_rows=args.batch_strip_rows,
                        graph_chunk=args.graph_chunk if args.batch_strip_rows > 0 else None,
                        traffic_json=args.traffic_json, persistent=args.persistent)
        out = {"metric": "TCLBM MLUPS", "value": b["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": b["ms_per_step"], "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.storage == "f64" else "f32",
               "data": "synthetic (seeded)",
               "config": {"workload": b["workload"], "storage": args.storage, "instances": b["instances"],
                          "nodes": b["nodes"], "steps_per_reduction": args.reduce_every,
                          "unstable_instances": b["unstable_instances"],
                          "redrawn_below_stability_limit": b["redrawn_below_stability_limit"],
                          "strip_rows": b["strip_rows"], "graph_chunk": b["graph_chunk"],
                          "device_ms": b["device_ms"], "autotune": b["autotune"],
                          **({"persistent_steps_per_launch": args.persistent} if args.persistent > 0 else {})},
               "roofline": b["roofline"]}
        if not args.no_extras:
            log("bench: RB 512x256 fp32, 2000 steps")
            out["rb512x256"] = single_extra(torch, tclbm, "rb", "f32", 2000, 200, args.traffic_json)
            log("bench: shock tube 8192x4 fp32, 4000 steps")
            out["shock_tube"] = single_extra(torch, tclbm, "shock", "f32", 4000, 200, args.traffic_json)
            out["roofline_large"] = {}
            for st in ("f32", "f16", "bf16"):
                log(f"bench: RB 8192x4096 {st}, 200 warmup + 1000 timed steps")
                out["roofline_large"][st] = single_extra(torch, tclbm, "large", st, 1000, 200, args.traffic_json)
            log("bench: Section 5D Table 3 sweep, internal-energy DF, FP32 batch of five lattices")
            out["table3"] = bench_table3(torch, tclbm)
            log("bench: persistent batched launches vs per-step graph replays")
            out["persistent_batch"] = bench_persistent(torch, tclbm)
            log("bench: HBM copy ceiling, 2 GiB -> 2 GiB")
            ceil = copy_probe(torch, tclbm)
            out["hbm_ceiling"] = ceil
            out["roofline"]["frac_of_ceiling"] = round(out["roofline"]["achieved"] / ceil["GBs"], 4)
            for st, r in out["roofline_large"].items():
                r["frac_of_ceiling"] = round(r["achieved"] / ceil["GBs"], 4)
            if not args.no_serving:
                log(f"bench: serving streams, {args.requests} requests, {serve_storages}")
                out["serving"] = bench_serving(torch, tclbm, n_requests=args.requests, storages=serve_storages,
                                               time_units=args.time_units)
        if not args.no_cpu_baseline:
            from paper_1610_07114_amd import workloads as W
            specs = W.batched_rb_specs(256, seed=0)[:8]
            out["cpu_baseline"] = cpu_baseline([W.rb_from_spec(s) for s in specs],
                                               label="the first 8 lattices of the batched RB workload "
                                                     f"({sum(s['nx'] * s['ny'] for s in specs)} nodes)")
            if not args.no_extras:
                log("bench: FP64 oracle on one and on all host threads, configs 1-3")
                out["cpu_baseline_detail"] = cpu_baseline_detail()
        print(json.dumps(out), flush=True)
        return

    case, wname = workload_case(args.workload)
    log(f"bench: {wname} {args.storage}, warmup {args.warmup}, steps {args.steps}")
    r = bench_single(torch, tclbm, case, args.storage, args.steps, args.warmup, args.reduce_every,
                     args.strip_rows, args.graph_chunk)
    mlups = r["nodes"] * args.steps / r["wall"] / 1e6
    bpl = bytes_per_lup(args.storage, case.thermal)
    out = {
        "metric": "TCLBM MLUPS",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["wall"] * 1e3 / args.steps, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.storage == "f64" else "f32",
        "data": "synthetic (seeded)",
        "config": {"workload": wname, "nx": case.nx, "ny": case.ny, "storage": args.storage,
                   "steps_per_reduction": args.reduce_every, "device_ms": round(r["dev_ms"], 3)},
        "roofline": roofline(bpl, r["nodes"], r["avg_launch_s"],
                             load_traffic(args.traffic_json, f"{wname}_{args.storage}"), kernel=r["kernel"]),
        "nu": None,
    }
    if case.name == "rayleigh_benard":
        m = case.meta
        out["nu"] = 1.0 + r["sums"].nu_num / r["nodes"] * m["H"] / (m["kappa"] * m["dT"])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline([case])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
