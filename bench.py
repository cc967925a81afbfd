"""Benchmark: Gcell-steps/s of the explicit-implicit stepper on one MI355X.

Headline workload: the single-device cell, 1024 x 4096 (r, z) nodes, 8
layers, FP64, dt = 0.2 us, 2 ms / 20 ms pulse at 5e8 W/m^3, 100,000 steps
(one full period).  A "step" is one time step of the whole grid: pulse
schedule, lagged coefficient evaluation, explicit z half, implicit radial
line solves, boundary completion.  Inputs are seeded synthetic cells with
the workload's shapes and value ranges; the field is resident in HBM before
timing starts.

Extra measurements in the same JSON line (not part of `value`): the FP32
(compensated pair) rate on the same cell, the batched design sweep (256
uneven cells) against the same cells stepped one at a time, the cost of a
gradient (forward + checkpointed adjoint) relative to a forward on the
adjoint workload (512 x 2048, 50,000 steps), with checkpoints only and with
the states of the last steps kept in up to 200 GiB of HBM, and gradients per
second of the
batched-adjoint design loop (64 designs of 512 x 1024, 20 Adam iterations
over a prefix of 1,000 of the 100,000 steps, the final J of all 64 designs
checked against the oracle).

Prints one JSON line.  --gpus above 1 is refused: the stepper runs on one GPU.
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
FP64_VECTOR_TFLOPS = 78.6
BYTES_PER_CELL_STEP = 16          # FP64: read T, write T^
F32_BYTES_PER_CELL_STEP = 8       # FP32: read T, write T^ (algorithmic)
F32_PAIR_BYTES_PER_CELL_STEP = 16  # what the compensated pair storage moves
GRAD_BYTES_PER_CELL_STEP = 64     # forward 16 + recompute 16 + adjoint 32 (FP64)
GRAD_STORE_GIB = 200              # device memory the stored-tail gradient may take

# The headline kernel's HBM traffic comes from the committed rocprofv3
# counter summary, and only when that summary was taken on the kernel
# sources of this tree (their hash is written in it); otherwise null.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_step_f64_1024x4096.md")
KERNEL_SOURCES = ["paper_1408_5853_amd/csrc/forward.hip", "paper_1408_5853_amd/csrc/device_common.h",
                  "paper_1408_5853_amd/csrc/internal.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """sha256 (first 16 hex digits) of the stepping kernel's source files."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(path=TRAFFIC_PROFILE):
    """HBM bytes per launch of the headline kernel from its counter summary,
    if the summary names this tree's kernel source hash; else None."""
    import re
    try:
        text = open(path).read()
    except OSError:
        return None
    m = re.search(r"kernel source sha256\[:16\]: `?([0-9a-f]{16})", text)
    t = re.search(r"HBM bytes per launch: `?([0-9,]+)", text)
    if not m or not t or m.group(1) != kernel_source_hash():
        return None
    return int(t.group(1).replace(",", ""))


def measured_valu_busy(path=TRAFFIC_PROFILE):
    """Fraction of the headline kernel's cycles its SIMDs issue VALU work,
    from the same counter summary (its kernel source hash must match)."""
    import re
    try:
        text = open(path).read()
    except OSError:
        return None
    m = re.search(r"kernel source sha256\[:16\]: `?([0-9a-f]{16})", text)
    t = re.search(r"VALU busy per launch[^`]*`([0-9.]+)`", text)
    if not m or not t or m.group(1) != kernel_source_hash():
        return None
    return float(t.group(1))


def timed(stream, fn):
    """Seconds between two HIP events on `stream` around the work `fn`
    enqueues.  A spin kernel (about a millisecond) goes first, before the
    start event, so that the host has enqueued the first launches by the
    time the start event is reached: a short timed region then measures the
    kernels, not the host's latency to its first launch."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        torch.cuda._sleep(2_000_000)
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3


def host_threads():
    """Threads the host offers this process (its CPU affinity; at most 16,
    one GPU's share of the host's cores on an eight-GPU node)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_rate(sample, lines, threads, seconds):
    import oracle
    n = 10
    oracle.forward(sample, nsteps=2, nthreads=threads)         # warm
    while True:
        t0 = time.perf_counter()
        oracle.forward(sample, nsteps=n, nthreads=threads)
        dt = time.perf_counter() - t0
        if dt > seconds / 3 or n > 10_000_000:
            break
        n *= 3
    return sample["nr"] * lines * n / dt / 1e9, n, dt


def cpu_baseline(cell, seconds):
    """The oracle as it stands on the host cores, on a bounded sample of the
    workload: its full grid over a prefix of steps (as many as fit in about
    `seconds`; the rate does not depend on the step), counting the interior
    lines only (the two z-boundary lines are copies), on every thread and on
    one."""
    import oracle
    oracle.build(force=False)
    cores = host_threads()
    lines = cell["nz"] - 2
    v, n, dt = _oracle_rate(cell, lines, cores, 0.7 * seconds)
    v1, n1, dt1 = _oracle_rate(cell, lines, 1, 0.3 * seconds)
    return {"value": round(v, 5), "unit": "Gcell-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": "the workload's full grid, %d radial nodes x %d interior lines (counted "
                      "cells are the solved interior lines only), the first %d of its %d "
                      "steps in %.1f s on %d threads" % (cell["nr"], lines, n, cell["nsteps"],
                                                         dt, cores),
            "one_core": {"value": round(v1, 5), "steps": n1, "seconds": round(dt1, 2)}}


# Steps run on a new resident state before it is reset to the initial field:
# the GPU's clocks ramp up over the first tens of milliseconds of work after
# an idle spell (measured on the 1024 x 4096 cell: about 32 us per step for
# the first steps, 28.4-28.6 us after some 500), so a short timed region
# right after a few warm-up steps would report the ramp, not the kernel.
SETTLE_STEPS = 4000


def rate(P, cell, dtype, steps, warmup, stream):
    """Seconds for `steps` steps of `cell` with the field resident in the
    kernels' layout (cryo_state_*), after `warmup` untimed steps: steps
    warmup .. warmup + steps - 1 of the cell from its initial field (the
    state is first settled with SETTLE_STEPS steps and reloaded with the
    initial field)."""
    plan = P.Plan(cell, dtype)
    T0 = plan.init()
    st = P.State(plan, T0)
    st.forward(0, SETTLE_STEPS)
    st.poll()
    st.load(T0)
    if warmup:
        st.forward(0, warmup)
    secs = timed(stream, lambda: st.forward(warmup, steps))
    st.poll()
    return secs, plan


def batch_extra(P, steps, stream, tune_cache=None):
    """The design sweep (256 uneven cells, FP32 pairs) as one batch with the
    batch autotuner's launch shapes, against the same cells stepped one at a
    time with tuned launches (each shape group's representative tuned by
    cryo_autotune, its shape given to the group).  `tune_cache` (a text file
    of the tuner) lets a profiled run take the shapes an unprofiled run
    picked."""
    import collections

    import cellgen
    cells = cellgen.sweep_cells(0)
    total = sum(c["nr"] * c["nz"] for c in cells)
    t0 = time.perf_counter()
    shapes = P.tune_batch(cells, "f32", cache=tune_cache)
    tune_s = time.perf_counter() - t0
    b = P.Batch(cells, "f32", shapes=shapes)
    T = b.init()
    ws = b.workspace()
    b.forward(T, 0, 64, ws)                                   # capture + warm
    secs_b = timed(stream, lambda: b.forward(T, 64, steps, ws))
    b.poll(ws)
    # one at a time: every cell its own launches, fields resident in the
    # kernels' layout; shapes tuned per group of equal default shape
    groups = collections.defaultdict(list)
    for i, c in enumerate(cells):
        groups[P.Plan(c, "f32").shape()[:2]].append(i)
    single = [None] * len(cells)
    for idx in groups.values():
        rep = max(idx, key=lambda i: cells[i]["nr"] * cells[i]["nz"])
        sh, _ = P.autotune(cells[rep], "f32", steps=20)
        for i in idx:
            single[i] = (sh[0], sh[1], max(1, min(sh[2], cells[i]["nz"] - 2)))
    plans = []
    for c, sh in zip(cells, single):
        p = P.Plan(c, "f32")
        p.set_shape(*sh)
        plans.append(p)
    states = [P.State(p, p.init()) for p in plans]
    for st in states:
        st.forward(0, 4)

    def one_by_one():
        for st in states:
            st.forward(4, steps)

    secs_1 = timed(stream, one_by_one)
    rate_b = total * steps / secs_b
    return {"workload": "design sweep: 256 cells, nr 128-512, nz 256-2048, 4-8 layers, FP32 pairs",
            "steps": steps, "cells": total,
            "batch_shapes": sorted(set(shapes)), "batch_tune_s": round(tune_s, 2),
            "batched_gcell_steps_s": round(rate_b / 1e9, 2),
            # algorithmic FP32 traffic: read T, write T^ (8 B per node and step)
            "batched_hbm_frac": round(rate_b * F32_BYTES_PER_CELL_STEP / 1e9 / HBM_PEAK_GBS, 4),
            # what the compensated pairs move (16 B per node and step)
            "batched_pair_storage_frac": round(rate_b * F32_PAIR_BYTES_PER_CELL_STEP / 1e9
                                               / HBM_PEAK_GBS, 4),
            "one_at_a_time_shapes": sorted(set(single)),
            "one_at_a_time_gcell_steps_s": round(total * steps / secs_1 / 1e9, 2),
            "speedup": round(secs_1 / secs_b, 2)}


def gradient_extra(P, steps, stream, store_gib=GRAD_STORE_GIB):
    """A forward and a gradient of `steps` steps on the adjoint workload,
    both timed with HIP events on the stream (the gradient enqueued with
    cryo_gradient_async, its workspace made beforehand): with checkpoints
    only (reported under "checkpoints_only"), then with a gradient store that
    fits in `store_gib` GiB (at most 85 % of the free device memory), whose
    figures are the top-level ones, with its bitwise check against the
    first."""
    import cellgen
    import numpy as np
    import torch
    c = cellgen.adjoint_cell(0)
    tgt = cellgen.tracking_target(c, steps)
    td = torch.tensor(tgt, dtype=torch.float64, device="cuda")
    plan = P.Plan(c, "f64")
    sh = P._gradient_shape(c)
    plan.set_shape(*sh)
    T = plan.init()
    ws = plan.workspace(steps)
    plan.forward(T, 0, 10, ws=ws)
    T = plan.init()
    t_fwd = timed(stream, lambda: plan.forward(T, 0, steps, ws=ws))
    T0 = plan.init()
    torch.cuda.synchronize()
    gws = torch.empty(plan.gradient_workspace_bytes(steps), dtype=torch.uint8, device="cuda")
    res = {}
    t_grad = timed(stream, lambda: res.update(
        out=plan.gradient_async(td, T0, nsteps=steps, ws=gws)))
    plan.poll(gws)
    J = float(res["out"][0].item())
    g = res["out"][1].cpu().numpy()
    cells = c["nr"] * c["nz"]
    # checkpoints only: algorithmic bytes of a gradient step are forward and
    # recompute 16 B each, the adjoint 32 B (read T^n, T^{n+1}, lam^{n+1};
    # write lam^n)
    ck = {"workload": "adjoint: 512x2048, 6 layers, FP64, checkpoint stride ceil(sqrt(N))",
          "workspace_gib": round(gws.numel() / 2**30, 2), "gradient_s": round(t_grad, 3),
          "gradient_over_forward": round(t_grad / t_fwd, 2),
          "gradient_gcell_steps_s": round(cells * steps / t_grad / 1e9, 2),
          "gradient_hbm_frac": round(cells * steps / t_grad * GRAD_BYTES_PER_CELL_STEP / 1e9
                                     / HBM_PEAK_GBS, 4)}
    out = {"steps": steps, "forward_s": round(t_fwd, 3), "J": J,
           "grad_finite": bool(np.all(np.isfinite(g)))}
    del res, gws
    torch.cuda.empty_cache()
    d = 0
    if store_gib > 0:
        free, _ = torch.cuda.mem_get_info()
        budget = int(min(store_gib * 2**30, 0.85 * free))
        d = plan.gradient_store_for(steps, budget)
    if d > 0:
        # the states of the last d steps kept from the forward (no recompute
        # for them): the recompute's 16 B only for the other steps
        plan.set_gradient_store(d)
        gws = torch.empty(plan.gradient_workspace_bytes(steps), dtype=torch.uint8, device="cuda")
        res = {}
        t_st = timed(stream, lambda: res.update(
            out=plan.gradient_async(td, T0, nsteps=steps, ws=gws)))
        plan.poll(gws)
        Js = float(res["out"][0].item())
        gs = res["out"][1].cpu().numpy()
        recomputed = (steps - d) / steps
        out.update({
            "workload": "adjoint: 512x2048, 6 layers, FP64, the last %d of %d steps' states kept "
                        "from the forward (gradient store), checkpoints every "
                        "ceil(sqrt(%d)) steps before them" % (d, steps, steps - d),
            "stored_steps": d, "workspace_gib": round(gws.numel() / 2**30, 2),
            "gradient_s": round(t_st, 3), "gradient_over_forward": round(t_st / t_fwd, 2),
            "gradient_gcell_steps_s": round(cells * steps / t_st / 1e9, 2),
            "gradient_hbm_frac": round(cells * steps / t_st * (48 + 16 * recomputed) / 1e9
                                       / HBM_PEAK_GBS, 4),
            "equal_bitwise_to_checkpoints_only": bool(Js == J and np.array_equal(gs, g))})
        plan.set_gradient_store(0)
        del res, gws
        torch.cuda.empty_cache()
    else:
        out.update(ck)
    out["checkpoints_only"] = ck
    return out


def design_extra(P, steps, iters, stream):
    """The batched-adjoint design loop: all 64 designs of 512 x 1024 nodes,
    `iters` Adam iterations (iters + 1 gradient_many calls of 64 gradients)
    over a prefix of `steps` steps of their 100,000, run twice: with a
    checkpointed workspace per design (reported under
    "checkpointed_per_design"), then on two shared workspaces that keep
    every state (the top-level figures; the J history must be bitwise the
    same).  The final J of every design is checked against the oracle on
    its exact z-invariant reduction (4 axial nodes; host threads over the
    designs), four of them listed."""
    import cellgen
    import numpy as np
    import oracle
    from paper_1408_5853_amd.design import design_adam
    cells = cellgen.design_cells(0, nsteps=steps)
    tg = [cellgen.tracking_target(c, steps) for c in cells]
    P.gradient_many(cells[:2], tg[:2], streams=2)                # warm
    t0 = time.perf_counter()
    final, hist = design_adam(cells, tg, iters=iters, lr=0.05)
    secs = time.perf_counter() - t0
    ngrad = len(cells) * (iters + 1)
    cell_steps = sum(c["nr"] * c["nz"] for c in cells) * steps * (iters + 1)
    from concurrent.futures import ThreadPoolExecutor

    def oracle_J(i):
        _, S = oracle.forward(cellgen.with_nz(final[i], 4), nsteps=steps, surf=True, nthreads=1)
        return float(np.sum((S - tg[i]) ** 2))

    with ThreadPoolExecutor(host_threads()) as ex:
        Jo_all = list(ex.map(oracle_J, range(len(cells))))
    rel = [abs(float(hist[-1][i]) - Jo_all[i]) / abs(Jo_all[i]) for i in range(len(cells))]
    check = [{"design": i, "J_gpu": float(hist[-1][i]), "J_oracle": Jo_all[i],
              "rel_diff": rel[i]} for i in (0, 21, 42, 63)]
    # the same loop on two shared workspaces (one per stream) that keep every
    # state of the run (gradient store): no recompute, a few GiB in all
    import torch
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    _, hist_s = design_adam(cells, tg, iters=iters, lr=0.05, store=steps, shared=2)
    secs_s = time.perf_counter() - t0
    torch.cuda.empty_cache()
    return {"workload": "design loop: 64 designs of 512x1024, FP64 adjoint, Adam lr 0.05 in "
                        "log(amplitude, width, thicknesses), prefix of %d of 100,000 steps; "
                        "two shared workspaces keeping every state (gradient store)" % steps,
            "steps": steps, "adam_iterations": iters, "gradients": ngrad,
            "workspaces": 2, "stored_steps": steps,
            "seconds": round(secs_s, 3), "gradients_per_s": round(ngrad / secs_s, 2),
            "forward_equivalent_gcell_steps_s": round(cell_steps / secs_s / 1e9, 2),
            "J_history_equal_bitwise_to_checkpointed": bool(np.array_equal(hist_s, hist)),
            "mean_J_first": float(hist[0].mean()), "mean_J_last": float(hist[-1].mean()),
            "designs_improved": int(np.sum(hist[-1] < hist[0])),
            "final_J_vs_oracle": check,
            "final_J_vs_oracle_all": {"designs": len(cells), "max_rel_diff": max(rel)},
            "checkpointed_per_design": {"workspaces": len(cells), "seconds": round(secs, 3),
                                        "gradients_per_s": round(ngrad / secs, 2)}}


def paper_shape_extra(P, steps, stream):
    """The paper's largest timed grid (631 x 1201 nodes, 100,000 steps in its
    Table 4) on a bounded sample of steps, beside the paper's figure for its
    OpenCL code (context only: other hardware, other laws and domain)."""
    import cellgen
    c = cellgen.paper_shape(0)
    secs, plan = rate(P, c, "f64", steps, 200, stream)
    cells = c["nr"] * c["nz"]
    return {"workload": "paper-shape cell 631x1201, FP64", "steps": steps,
            "kernel_shape": list(plan.shape()),
            "gcell_steps_s": round(cells * steps / secs / 1e9, 2),
            "projected_s_for_100000_steps": round(secs / steps * 1e5, 2),
            "paper_table4_context": "631x1201, 100,000 steps: 12.9 min on its GPU "
                                    "(0.098 Gcell-steps/s), 64.0 min on its CPU"}


def turn_on_extra(P, steps, stream):
    """The transient turn-on model (eq. (22)) on the device cell: a run that
    starts on a pulse start (its first step as 100 sub-steps of dt/100) timed
    with and without the model; one pulse start per 100,000 steps at this
    cell's period and dt."""
    import cellgen
    c = cellgen.device_cell(0)
    per_period = int(round(c["period"] / c["dt"]))
    out = {"workload": "device cell 1024x4096, FP64, %d steps from a pulse start" % steps}
    for on in (False, True):
        plan = P.Plan(dict(c, turn_on=on), "f64")
        T = plan.init()
        ws = plan.workspace(steps)
        plan.forward(T, 0, steps, ws=ws)                  # warm (device tables)
        T = plan.init()
        secs = timed(stream, lambda: plan.forward(T, 0, steps, ws=ws))
        plan.poll(ws)
        out["with_model_s" if on else "without_model_s"] = round(secs, 5)
    extra = out["with_model_s"] - out["without_model_s"]
    plain = out["without_model_s"] / steps
    out["turn_on_step_ms"] = round(1e3 * (plain + extra), 4)
    out["plain_step_ms"] = round(1e3 * plain, 4)
    out["overhead_per_period_pct"] = round(100 * extra / (per_period * plain), 4)
    return out


def poly_extra(P, steps, stream):
    """The polynomial laws (eqs. (23), (24)) with the Joule source (eq. (25))
    on the device cell (seeded coefficients around its power laws)."""
    import cellgen
    c = cellgen.poly_variant(cellgen.device_cell(0), 0, joule_tref=30.0)
    secs, plan = rate(P, c, "f64", steps, 200, stream)
    r = c["nr"] * c["nz"] * steps / secs / 1e9
    return {"workload": "device cell 1024x4096, FP64, polynomial laws + Joule source",
            "steps": steps, "kernel_shape": list(plan.shape()),
            "gcell_steps_s": round(r, 2),
            "hbm_frac": round(r * BYTES_PER_CELL_STEP / HBM_PEAK_GBS, 4)}


def stepped_extra(P, steps, stream):
    """The stepped domain of eq. (9) on the device cell: a layered section
    over the lower 80 % of the axis, a terminal of the inner 256 radial nodes
    above it."""
    import cellgen
    c = cellgen.device_cell(0)
    zf, nt = int(0.8 * (c["nz"] - 1)), 256
    c["stepped"] = dict(z_full=zf, nr_top=nt)
    secs, plan = rate(P, c, "f64", steps, 200, stream)
    nodes = c["nr"] * c["nz"]
    inside = c["nr"] * (zf + 1) + nt * (c["nz"] - 1 - zf)
    return {"workload": "device cell 1024x4096, FP64, terminal of 256 radial nodes above "
                        "line %d" % zf, "steps": steps, "kernel_shape": list(plan.shape()),
            "grid_gcell_steps_s": round(nodes * steps / secs / 1e9, 2),
            "domain_gcell_steps_s": round(inside * steps / secs / 1e9, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100_000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the timed region, copy this many MiB device to device once "
                         "(a kernel of known traffic that calibrates the HBM byte counters)")
    ap.add_argument("--gradient-only", type=int, default=0, metavar="N",
                    help="profiling aid: time only a forward and a gradient of N steps on the "
                         "adjoint cell and print that result")
    ap.add_argument("--grad-store-gib", type=float, default=GRAD_STORE_GIB, metavar="GIB",
                    help="device memory the stored-tail gradient may take (0: skip it)")
    ap.add_argument("--batch-only", type=int, default=0, metavar="N",
                    help="profiling aid: time only the batched sweep (and the same cells one "
                         "at a time) over N steps and print that result")
    ap.add_argument("--tune-cache", default=None, metavar="PATH",
                    help="text cache of the batch autotuner (reused when it holds this batch)")
    ap.add_argument("--design-only", type=int, default=0, metavar="N",
                    help="time only the design loop (20 Adam iterations over N steps) and print "
                         "that result")
    ap.add_argument("--poly-only", type=int, default=0, metavar="N",
                    help="profiling aid: time only N steps of the polynomial-law path on the "
                         "device cell and print that result")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the stepper runs on exactly one GPU; --gpus %d is not supported"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import cellgen
    import paper_1408_5853_amd as P

    stream = torch.cuda.current_stream()
    if args.gradient_only:
        gradient_extra(P, 50, stream, args.grad_store_gib)  # warm
        print(json.dumps({"gradient": gradient_extra(P, args.gradient_only, stream,
                                                     args.grad_store_gib)}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batch": batch_extra(P, args.batch_only, stream, args.tune_cache)}),
              flush=True)
        return
    if args.design_only:
        print(json.dumps({"design_loop": design_extra(P, args.design_only, 20, stream)}),
              flush=True)
        return
    if args.poly_only:
        print(json.dumps({"poly_laws": poly_extra(P, args.poly_only, stream)}), flush=True)
        return
    cell = cellgen.device_cell(0)
    cells = cell["nr"] * cell["nz"]
    log("bench: device cell 1024x4096 FP64, %d steps after %d warmup" % (args.steps, args.warmup))
    secs, plan = rate(P, cell, "f64", args.steps, args.warmup, stream)
    value = cells * args.steps / secs / 1e9
    ms_step = 1e3 * secs / args.steps
    # the timed region holds exactly one k_step launch per step on this
    # stream (the field is resident: no layout conversion, no other kernel),
    # so region / steps is the kernel's average launch duration plus the gap
    # between launches
    achieved = BYTES_PER_CELL_STEP * cells / (secs / args.steps) / 1e9
    out = {
        "metric": "Gcell-steps/s & % HBM roofline (fwd, batched, adjoint) vs CPU oracle, 1 GPU",
        "value": round(value, 3),
        "unit": "Gcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "single-device cell 1024x4096 (r,z) nodes, 8 layers, dt=2e-7 s, "
                               "2 ms/20 ms pulse at 5e8 W/m^3",
                   "nr": cell["nr"], "nz": cell["nz"], "kernel_shape": list(plan.shape())},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(),
                     # FP64 sits near the VALU ridge: the profile's VALU busy
                     # fraction of the same kernel sources (null if changed)
                     "valu_busy": measured_valu_busy(),
                     "kernel": "k_step",
                     "bytes_per_launch": BYTES_PER_CELL_STEP * cells,
                     "kernel_source_sha256_16": kernel_source_hash(),
                     "note": "algorithmic 16 B/cell-step over the HIP-event time of the timed "
                             "steps; traffic = rocprofv3 FETCH_SIZE and WRITE_SIZE per launch "
                             "scaled by a plain copy, from the committed profile of these "
                             "kernel sources (null if they changed since)"},
    }
    if args.copy_mib:
        n = args.copy_mib * (1 << 20) // 8
        src = torch.rand(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": 8 * n, "written": 8 * n}
    extra = None
    if not args.no_extra:
        log("bench: FP32 pair rate")
        s32, _ = rate(P, cell, "f32", 20_000, 500, stream)
        r32 = cells * 20_000 / s32 / 1e9
        extra = {"f32_pair_gcell_steps_s": round(r32, 3),
                 # algorithmic FP32 bytes (8 B per cell-step)
                 "f32_hbm_frac": round(r32 * F32_BYTES_PER_CELL_STEP / HBM_PEAK_GBS, 4),
                 # bytes the compensated pairs move (16 B per cell-step)
                 "f32_pair_storage_frac": round(r32 * F32_PAIR_BYTES_PER_CELL_STEP
                                                / HBM_PEAK_GBS, 4)}
        log("bench: batched sweep")
        extra["batch"] = batch_extra(P, 2000, stream, args.tune_cache)
        log("bench: gradient")
        extra["gradient"] = gradient_extra(P, 50_000, stream, args.grad_store_gib)
        log("bench: paper shape")
        extra["paper_shape"] = paper_shape_extra(P, 10_000, stream)
        log("bench: turn-on model")
        extra["turn_on"] = turn_on_extra(P, 1000, stream)
        log("bench: polynomial laws")
        extra["poly_laws"] = poly_extra(P, 5000, stream)
        log("bench: stepped domain")
        extra["stepped_domain"] = stepped_extra(P, 5000, stream)
        log("bench: design loop")
        extra["design_loop"] = design_extra(P, 1000, 20, stream)
    if extra is not None:
        out["extra"] = extra
    if not args.no_cpu:
        log("bench: CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(cell, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
