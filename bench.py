"""Benchmark: Gcell-steps/s of the explicit-implicit stepper on one MI355X.

Workload: the single-device cell, 1024 x 4096 (r, z) nodes, 8 layers, FP64,
dt = 0.2 us, 2 ms / 20 ms pulse at 5e8 W/m^3.  A "step" is one time step of
the whole grid (source schedule, coefficient evaluation, explicit z half,
implicit radial line solves, boundary completion).  Inputs are seeded
synthetic problems with the workload's shapes and value ranges; the field is
resident in HBM before timing starts.

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL_STEP = {"f64": 16, "f32": 8}   # read T, write T^


def cpu_baseline(cell, seconds):
    """The oracle as it stands on the host cores, on a bounded sample: the
    full radial grid, 16 interior lines, as many steps as fit in `seconds`."""
    import cellgen
    import oracle
    oracle.build(force=False)
    sample = cellgen.with_nz(cell, 18)
    cores = os.cpu_count() or 1
    n = 20
    oracle.forward(sample, nsteps=2, nthreads=cores)         # warm
    while True:
        t0 = time.perf_counter()
        oracle.forward(sample, nsteps=n, nthreads=cores)
        dt = time.perf_counter() - t0
        if dt > seconds / 4 or n > 10_000_000:
            break
        n *= 4
    cells = sample["nr"] * sample["nz"] * n
    return {"value": cells / dt / 1e9, "unit": "Gcell-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": "%d x %d nodes (full radial grid, 16 interior lines), %d steps, "
                      "%.1f s on %d threads" % (sample["nr"], sample["nz"], n, dt, cores)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20_000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on exactly one GPU; --gpus %d is not supported"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import cellgen
    import paper_1408_5853_amd as P

    cell = cellgen.config2(0)
    plan = P.Plan(cell, args.dtype)
    T = plan.init()
    ws = plan.workspace(max(args.steps, args.warmup))
    stream = torch.cuda.current_stream()
    if args.warmup:
        plan.forward(T, 0, args.warmup, ws=ws)
    plan.poll(ws)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    plan.forward(T, args.warmup, args.steps, ws=ws)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    plan.poll(ws)
    cells = cell["nr"] * cell["nz"]
    value = cells * args.steps / (ms * 1e-3) / 1e9
    per_step_ms = ms / args.steps
    bytes_per_launch = BYTES_PER_CELL_STEP[args.dtype] * cells
    achieved = bytes_per_launch / (per_step_ms * 1e-3) / 1e9
    out = {
        "metric": "Gcell-steps/s & % HBM roofline (fwd, batched, adjoint) vs CPU oracle, 1 GPU",
        "value": round(value, 3),
        "unit": "Gcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(per_step_ms, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "single-device cell 1024x4096 (r,z) nodes, 8 layers, "
                               "dt=2e-7 s, 2 ms/20 ms pulse at 5e8 W/m^3",
                   "nr": cell["nr"], "nz": cell["nz"], "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None,
                     "kernel": "k_step (one launch per step)",
                     "bytes_per_launch": bytes_per_launch},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cell, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
