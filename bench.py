#!/usr/bin/env python3
"""Benchmark of the fused TCLBM step on one MI355X.

One "step" is one time step of the whole hot path over the lattice: pull
streaming, macroscopic variables, correction gradients, cascaded collision of
f with force and correction sources, energy-DF collision with the coupling
source, store (one fused kernel), plus the FP64 Nusselt/mass reduction every
`--reduce-every` steps.  Inputs are seeded and synthetic and resident in HBM
before timing starts.

Prints one JSON line on stdout: MLUPS of the workload (whole job), the HBM
roofline of the step kernel (algorithmic bytes per launch / average launch
time from HIP events on the library's stream), and the FP64 CPU reference
timed on a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


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


def cpu_baseline(case, seconds_target: float = 12.0):
    """The FP64 oracle as it stands, on the host cores, over a bounded number of
    steps of the same workload."""
    import numpy as np  # noqa: F401
    import oracle as O
    p = O.Params(nx=case.nx, ny=case.ny, R=case.R, T0=case.T0, gamma=case.gamma, Pr=case.Pr, tau_f=case.tau_f,
                 w2=case.w2, w3=case.w3, w4=case.w4, ax=case.ax, ay=case.ay, thermal=case.thermal,
                 correction=case.correction, bc=case.bc, wall_ux=case.wall_ux, wall_uy=case.wall_uy,
                 wall_T=case.wall_T)
    L = O.Lattice(p, case.rho, case.ux, case.uy, case.T)
    t0 = time.perf_counter()
    L.step(2)
    dt = max(time.perf_counter() - t0, 1e-6)
    n = max(2, min(5000, int(seconds_target / (dt / 2))))
    t0 = time.perf_counter()
    L.step(n)
    dt = time.perf_counter() - t0
    return {"value": round(case.nx * case.ny * n / dt / 1e6, 3), "unit": "MLUPS", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{case.name} {case.nx}x{case.ny}, {n} steps from the seeded initial state, FP64, "
                      f"{dt:.1f} s"}


def copy_probe(torch, tclbm, nbytes: int = 2 << 30, reps: int = 20):
    """Achievable HBM bandwidth of a plain streaming copy (read + write bytes per
    launch / launch time), the measured ceiling beside the 8 TB/s peak."""
    dev = torch.device("cuda:0")
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    a.fill_(1)
    s = torch.cuda.Stream(dev)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--workload", default="rb", choices=["rb", "shock", "couette", "large"])
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16", "f64"])
    ap.add_argument("--reduce-every", type=int, default=1000)
    ap.add_argument("--strip-rows", type=int, default=0)
    ap.add_argument("--graph-chunk", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="time the plain HBM copy kernel (2 x 2 GiB) instead and exit")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="per-launch HBM traffic from rocprofv3 counters (if measured for this kernel)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (the batched and single-lattice paths shard by "
              "instance or slab across GPUs by design, but no multi-GPU path is built); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1610_07114_amd import tclbm

    if args.copy_probe:
        print(json.dumps(copy_probe(torch, tclbm)), flush=True)
        return

    case, wname = workload_case(args.workload)
    dev = torch.device("cuda:0")
    lat = tclbm.Lattice(case, storage=args.storage, device="cuda:0")
    lat.set_tuning(args.strip_rows, args.graph_chunk)
    nodes = case.nx * case.ny

    def run(nsteps):
        done = 0
        while done < nsteps:
            k = min(args.reduce_every, nsteps - done)
            lat.step(k)
            done += k
            if done % args.reduce_every == 0:
                lat.moments(fields=False)   # FP64 sums (mass, energy, Nusselt numerator)

    log(f"bench: {wname} {args.storage}, warmup {args.warmup}, steps {args.steps}")
    run(args.warmup)
    torch.cuda.synchronize(dev)

    # timed region: wall clock around K steps, device events on the library's stream
    stream = lat.stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    ev0.record(stream)
    run(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    dev_ms = ev0.elapsed_time(ev1)

    # kernel-only average: a separate pass of pure steps timed with HIP events
    kern_ms = lat.step_timed(args.steps)
    avg_launch_s = kern_ms / 1e3 / args.steps
    _, _, _, _, sums = lat.moments(fields=False)
    lat.close()

    mlups = nodes * args.steps / wall / 1e6
    bpl = bytes_per_lup(args.storage, case.thermal)
    achieved = bpl * nodes / avg_launch_s / 1e9
    traffic = None
    try:
        tj = json.load(open(args.traffic_json))
        key = f"{wname}_{args.storage}"
        if key in tj:
            traffic = tj[key]["bytes_per_launch"]
    except Exception:
        pass

    out = {
        "metric": "TCLBM MLUPS",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.storage == "f64" else "f32",
        "data": "synthetic (seeded)",
        "config": {"workload": wname, "nx": case.nx, "ny": case.ny, "storage": args.storage,
                   "steps_per_reduction": args.reduce_every, "device_ms": round(dev_ms, 3)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "step_kernel", "bytes_per_lup": bpl,
                     "avg_launch_us": round(avg_launch_s * 1e6, 3)},
        "nu_num": sums.nu_num,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
