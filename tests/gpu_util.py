"""Helpers for the GPU tests: run the HIP stepper through the C ABI."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(cell, nsteps, T0=None, dtype="f64", k0=0, surf=True, ws=None):
    import torch

    import paper_1408_5853_amd as P
    plan = P.Plan(cell, dtype)
    T = plan.init() if T0 is None else plan.field_from(T0)
    if ws is None:
        ws = plan.workspace(nsteps)
    S = torch.zeros(max(nsteps, 1), dtype=torch.float64, device="cuda") if surf else None
    plan.forward(T, k0, nsteps, ws=ws, surf=S)
    plan.poll(ws)
    torch.cuda.synchronize()
    return plan.field_values(T), (S.cpu().numpy()[:nsteps] if surf else None)


def rel_err(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))
