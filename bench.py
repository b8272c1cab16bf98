#!/usr/bin/env python3
"""Benchmark of the fused TCLBM step on one MI355X.

One "step" is one time step of the whole hot path over the lattice: pull
streaming, wall treatment, macroscopic variables, correction gradients,
cascaded collision of f with force and correction sources, energy-DF collision
with the coupling source, store (one fused kernel), plus the FP64 Nusselt/mass
reduction every `--reduce-every` steps.  Inputs are seeded and synthetic and
resident in HBM before timing starts.

Prints one JSON line on stdout.  `value` is the MLUPS of the selected workload
(whole job, wall clock); `roofline` is the HBM roofline of its step kernel
(algorithmic bytes per launch / average launch time from HIP events on the
library's stream); `cpu_baseline` is the FP64 CPU reference timed on a bounded
sample of the same workload on the host cores.  With the default workload the
line also carries, measured in the same run:
  roofline_large  the step kernel on an 8192x4096 lattice (HBM-resident state)
  batch           256 seeded uneven Rayleigh-Benard lattices advanced by one
                  launch per step, autotuned, aggregate MLUPS and roofline
  serving         a seeded Poisson stream of RB/Couette solve requests served
                  with continuous batching and 16-bit storage (solves/s,
                  p50/p99 latency, Nu error against stored FP64 values), and the
                  same stream through the plain one-lattice-at-a-time FP32 path
  hbm_ceiling     a plain chunked 2 GiB copy on the same GPU; roofline_large
                  and batch also state their fraction of it
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
    """Achievable HBM bandwidth of a plain streaming copy (read + write bytes per
    launch / launch time; each block copies one contiguous 16 KiB chunk), the
    measured ceiling beside the 8 TB/s peak."""
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
def bench_batch(torch, tclbm, n=256, seed=0, storage="f32", steps=1000, warmup=200, strip_rows=0, graph_chunk=None,
                traffic_json=None):
    """The batched workload: n seeded 2N x N Rayleigh-Benard lattices (N
    log-uniform on [32, 512], Ra log-uniform on [1e4, 1e6], Pr uniform on
    [0.5, 7]) advanced together, one launch per step, HIP-graph chunks.  The
    autotuner's trial steps (strip height x graph chunk) are part of the
    warm-up; a given strip height (and graph chunk) replaces the autotuner.
    `traffic` is the stored counter measurement for the strip height in use."""
    from paper_1610_07114_amd import serving as S
    from paper_1610_07114_amd import workloads as W
    specs = W.batched_rb_specs(n, seed=seed)
    t0 = time.perf_counter()
    cases = [W.rb_from_spec(s) for s in specs]
    nodes = sum(c.nx * c.ny for c in cases)
    stream = torch.cuda.Stream(torch.device("cuda:0"))
    lats = [tclbm.Lattice(c, storage=storage, stream=stream) for c in cases]
    del cases
    log(f"batch: {n} seeded lattices resident ({time.perf_counter() - t0:.1f} s)")
    b = tclbm.Batch(lats)
    tune = None
    if strip_rows > 0:
        b.set_strip_rows(strip_rows)
        if graph_chunk is not None:
            b.set_graph_chunk(graph_chunk)
    else:
        tune = S.autotune_batch(b, log=log)
        log(f"batch autotune: {tune}")
    rows_in_use = b.strip_rows
    b.step(warmup)
    stream.synchronize()
    t0 = time.perf_counter()
    ms = b.step_timed(steps)
    wall = time.perf_counter() - t0
    waves = b.waves
    b.close()
    unstable = 0
    for lat in lats:
        _, _, _, _, _, st = tclbm.tclbm_moments(lat.h, lat.case.nx, lat.case.ny, fields=False, check=False)
        unstable += st != tclbm.OK
        lat.close()
    avg = ms / 1e3 / steps
    bpl = bytes_per_lup(storage)
    return {"workload": f"batched_rayleigh_benard_{n}x(2N x N, N log-uniform 32..512, seed {seed})",
            "instances": n, "nodes": nodes, "storage": storage, "steps": steps, "warmup": warmup,
            "mlups": round(nodes * steps / wall / 1e6, 1), "ms_per_step": round(wall * 1e3 / steps, 4),
            "autotune": tune, "waves_per_step": waves, "unstable_instances": int(unstable),
            "strip_rows": rows_in_use,
            "roofline": roofline(bpl, nodes, avg,
                                 load_traffic(traffic_json, f"batched_rayleigh_benard_{n}_{storage}_rows{rows_in_use}")
                                 if traffic_json else None, kernel="batch_step_kernel")}


# ------------------------------------------------------------------ serving ---
def golden_requests(S, start_id, rate_span, seed=7):
    """Requests for the instances whose FP64 Nusselt history is stored, at
    seeded arrival times inside the stream; their run lengths equal the stored
    schedule so the final Nu can be compared with the FP64 value."""
    import numpy as np
    try:
        g = json.load(open(GOLDEN_BATCH_NU))
    except Exception:
        return [], {}
    rng = np.random.default_rng(seed)
    out, ref = [], {}
    for k, inst in enumerate(g["instances"]):
        # only histories that ended steady: their final value is the steady Nu
        if not (inst["steps"] and inst["steps"][-1] == inst["total"] and math.isfinite(inst["nu_mean"])
                and inst["unsteadiness"] < 2e-3):
            continue
        s = inst["spec"]
        rid = start_id + k
        out.append(S.Request(rid, "rb", s["nx"], s["ny"], s["Ra"], s["Pr"], inst["total"],
                             float(rng.uniform(0, rate_span)), s["seed"]))
        ref[rid] = inst["nu"][-1]
    return out, ref


def bench_serving(torch, tclbm, n_requests=500, storage="f16", seed=0, load=0.8, time_units=1.0,
                  sequential_fp32=True):
    from paper_1610_07114_amd import serving as S
    import numpy as np
    # capacity: the aggregate lattice-update rate of a closed-loop run
    # (everything queued at t = 0) of a calibration stream from the same
    # distribution, divided by the mean work of the stream's own requests
    # (the work per request is heavy-tailed, ~N^3, so counting solves of a
    # different sample would misjudge it)
    calib = S.make_requests(max(40, n_requests // 8), rate=1.0, seed=seed + 1000, time_units=time_units)
    for r in calib:
        r.arrival = 0.0
    srv = S.Server(storage=storage)
    t0 = time.perf_counter()
    res = srv.run(calib, realtime=False)
    cap_wall = time.perf_counter() - t0
    cal_lups = sum(r.nx * r.ny * r.steps for r in res) / cap_wall
    reqs = S.make_requests(n_requests, rate=1.0, seed=seed, time_units=time_units)
    mean_work = sum(r.nx * r.ny * r.steps for r in reqs) / len(reqs)
    capacity = cal_lups / mean_work
    rate = load * capacity
    reqs = S.make_requests(n_requests, rate=rate, seed=seed, time_units=time_units)
    span = reqs[-1].arrival
    gold, ref = golden_requests(S, n_requests, span)
    reqs = sorted(reqs + gold, key=lambda r: r.arrival)
    log(f"serving: closed loop {cal_lups / 1e6:.0f} MLUPS ({len(calib)} calibration requests, {cap_wall:.1f} s), "
        f"mean work {mean_work:.3g} LUP -> capacity {capacity:.2f} solves/s; "
        f"stream of {len(reqs)} requests at {rate:.2f}/s over {span:.1f} s")
    t0 = time.perf_counter()
    res = srv.run(reqs, realtime=True)
    wall = time.perf_counter() - t0
    # latency and throughput of the stream itself; the long Nu-check requests
    # ride along and are reported by their error only
    summ = S.summarize([r for r in res if r.rid not in ref], wall)
    errs = [abs(r.nu - ref[r.rid]) / abs(ref[r.rid]) for r in res if r.rid in ref]
    out = {"storage": storage, "arrival_rate_per_s": round(rate, 3), "load_vs_capacity": load,
           "capacity_solves_per_s": round(capacity, 3), "closed_loop_mlups": round(cal_lups / 1e6, 1),
           "mean_work_lup": round(mean_work), **summ,
           "run_length": f"{time_units} H/u_c per request (u_c = 0.08 RB, u0 = 0.05 Couette); "
                         f"{len(gold)} more requests with a stored steady FP64 Nu run their stored length "
                         f"(120 H/u_c) and are excluded from the latency figures",
           "phases_s": {k: round(v, 2) for k, v in srv.phase_s.items()}, "rebatches": srv.rebatches,
           "nu_rel_err_vs_fp64": {"max": max(errs) if errs else None, "n": len(errs),
                                  "median": float(np.median(errs)) if errs else None}}
    if sequential_fp32:
        # the plain path: one FP32 lattice at a time, first come first served
        seq = sorted(reqs, key=lambda r: r.arrival)
        srv1 = S.Server(storage="f32", max_slots=1)
        t0 = time.perf_counter()
        res1 = srv1.run(seq, realtime=True)
        wall1 = time.perf_counter() - t0
        errs1 = [abs(r.nu - ref[r.rid]) / abs(ref[r.rid]) for r in res1 if r.rid in ref]
        out["single_lattice_fp32"] = {**S.summarize([r for r in res1 if r.rid not in ref], wall1),
                                      "nu_rel_err_vs_fp64": {"max": max(errs1) if errs1 else None,
                                                             "n": len(errs1)}}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--workload", default="rb", choices=["rb", "shock", "couette", "large", "batch", "serve"])
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16", "f64"])
    ap.add_argument("--reduce-every", type=int, default=1000)
    ap.add_argument("--strip-rows", type=int, default=0)
    ap.add_argument("--batch-strip-rows", type=int, default=0,
                    help="batch workload: fixed strip height (with --graph-chunk) instead of the autotuner")
    ap.add_argument("--graph-chunk", type=int, default=32)
    ap.add_argument("--requests", type=int, default=500, help="serving stream length")
    ap.add_argument("--serve-storage", default="f16", choices=["f16", "bf16", "f32"])
    ap.add_argument("--no-extras", action="store_true",
                    help="only the selected workload (no large-lattice roofline, batch or serving figures)")
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

    if args.workload == "batch":
        log("bench: batched RB workload, 256 instances")
        b = bench_batch(torch, tclbm, storage=args.storage, steps=min(args.steps, 2000),
                        warmup=min(args.warmup, 400), strip_rows=args.batch_strip_rows,
                        graph_chunk=args.graph_chunk if args.batch_strip_rows > 0 else None,
                        traffic_json=args.traffic_json)
        out = {"metric": "TCLBM MLUPS", "value": b["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": b["steps"],
               "warmup": b["warmup"], "ms_per_step": b["ms_per_step"], "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded)",
               "config": {"workload": b["workload"], "storage": args.storage, "instances": b["instances"],
                          "nodes": b["nodes"], "unstable_instances": b["unstable_instances"],
                          "autotune": b["autotune"]},
               "roofline": b["roofline"]}
        if not args.no_cpu_baseline:
            from paper_1610_07114_amd import workloads as W
            specs = W.batched_rb_specs(256, seed=0)[:8]
            out["cpu_baseline"] = cpu_baseline([W.rb_from_spec(s) for s in specs],
                                               label="first 8 lattices of the batched RB workload")
        print(json.dumps(out), flush=True)
        return

    if args.workload == "serve":
        s = bench_serving(torch, tclbm, n_requests=args.requests, storage=args.serve_storage)
        out = {"metric": "batched serving solves/s", "value": s["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
               "steps": s["requests"], "warmup": 0, "ms_per_step": round(1e3 / max(s["solves_per_s"], 1e-9), 3),
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
               "data": "synthetic (seeded)", "config": {"workload": "serving stream", **s}}
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

    if args.workload == "rb" and not args.no_extras:
        big, bname = workload_case("large")
        log(f"bench: {bname} f32 roofline, 200 warmup + 1000 timed steps")
        rl = bench_single(torch, tclbm, big, "f32", 1000, 200, 1000, 0, 32)
        out["roofline_large"] = {"workload": bname, "mlups": round(rl["nodes"] * 1000 / rl["wall"] / 1e6, 1),
                                 **roofline(144, rl["nodes"], rl["avg_launch_s"],
                                            load_traffic(args.traffic_json, f"{bname}_f32"), kernel=rl["kernel"])}
        del big
        log("bench: batched RB, 256 instances, f32")
        out["batch"] = bench_batch(torch, tclbm, storage="f32", traffic_json=args.traffic_json)
        # the measured ceiling beside the specification: a plain chunked copy
        log("bench: HBM copy ceiling, 2 GiB -> 2 GiB")
        ceil = copy_probe(torch, tclbm)
        out["hbm_ceiling"] = ceil
        out["roofline_large"]["frac_of_ceiling"] = round(out["roofline_large"]["achieved"] / ceil["GBs"], 4)
        out["batch"]["roofline"]["frac_of_ceiling"] = round(out["batch"]["roofline"]["achieved"] / ceil["GBs"], 4)
        log(f"bench: serving stream, {args.requests} requests, {args.serve_storage}")
        out["serving"] = bench_serving(torch, tclbm, n_requests=args.requests, storage=args.serve_storage)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline([case])
        if args.workload == "rb" and not args.no_extras:
            log("bench: FP64 oracle on one and on all host threads, configs 1-3")
            out["cpu_baseline_detail"] = cpu_baseline_detail()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
