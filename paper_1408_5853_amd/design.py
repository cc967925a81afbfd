"""Batched design loop (the batched-adjoint workload): Adam in
log-parameter space over each design's pulse amplitude, pulse width and layer
thicknesses, one gradient_many call (all designs' forward and adjoint sweeps
on the GPU) per iteration.  The update itself is a handful of host-side
numbers per design."""
from __future__ import annotations

import copy

import numpy as np

from . import gradient_many, params_of, with_params


def design_params(cell):
    """Design variables of the batched design loop: [amplitude, width,
    thickness_0..L-1] (the layer conductivity scales stay fixed)."""
    return params_of(cell)[:2 + len(cell["layers"])]


def design_adam(cells, targets, iters, lr=0.05, nsteps=None, ckpt=0, streams=0,
                betas=(0.9, 0.999), eps=1e-8, store=0, shared=0):
    """Adam in log-parameter space over design_params of every design, with
    one gradient_many call per iteration (`store` and `shared` as there: k
    shared workspaces with a gradient store each trade recompute for
    memory).  Returns (final cells, J history [iters + 1][n]): the last row
    is J at the final designs.  The pulse width is kept below its period."""
    cells = [copy.deepcopy(c) for c in cells]
    n = len(cells)
    m = [None] * n
    v = [None] * n
    hist = []
    for it in range(iters + 1):
        J, grads, _ = gradient_many(cells, targets, nsteps=nsteps, ckpt=ckpt, streams=streams,
                                    store=store, shared=shared)
        hist.append(J.copy())
        if it == iters:
            break
        for i, c in enumerate(cells):
            L = len(c["layers"])
            th = design_params(c)
            gl = th * grads[i][:2 + L]                  # dJ/dlog(theta)
            m[i] = gl * (1 - betas[0]) if m[i] is None else betas[0] * m[i] + (1 - betas[0]) * gl
            v[i] = gl * gl * (1 - betas[1]) if v[i] is None else betas[1] * v[i] + (1 - betas[1]) * gl * gl
            mh = m[i] / (1 - betas[0] ** (it + 1))
            vh = v[i] / (1 - betas[1] ** (it + 1))
            new = th * np.exp(-lr * mh / (np.sqrt(vh) + eps))
            new[1] = min(new[1], 0.999 * c["period"])
            full = params_of(c)
            full[:2 + L] = new
            cells[i] = with_params(c, full)
    return cells, np.array(hist)
