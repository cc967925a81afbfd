"""Write the stored oracle results of the full-size z-active cells under
tests/golden/ (twin_*.npz).

The as-written device and adjoint cells are exactly z-invariant, so their
explicit axial half (eq. (11)) does nothing; their z-active twins hold the
top line z = z_max at the initial temperature (eq. (6)), so the axial
fluxes near it are active.  The oracle takes minutes on these full grids, so
its results over a 10,000-step prefix are stored rather than recomputed in
the tests: the surface-mean trace every 10th step, and whole radial lines
at the bottom, in the middle and in the layers below the held top line.
Only the oracle (and the seeded input generator) is called here, with
every host thread.  Each file records the sha256 of the oracle's sources
and the problem dictionary it was run on; a CPU test checks that the oracle
is unchanged and that the generator still draws that problem.  Run from the
repository root:

    python tests/golden/make_twins.py
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import cellgen  # noqa: E402
import oracle  # noqa: E402

STEPS = 10_000
TRACE_EVERY = 10
SOURCES = ["oracle/oracle.c", "oracle/__init__.py"]


def sources_hash():
    h = hashlib.sha256()
    for f in SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def sample_lines(nz):
    """Lines stored whole: the bottom, the middle, and a widening ladder of
    lines below the held top line nz - 1."""
    top = [nz - 2 - k for k in (0, 1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144, 233)]
    return sorted(set([1, 2, nz // 2] + top))


def cases():
    """(name, cell) of every stored run."""
    return [("twin_device_cell", cellgen.device_cell(0, z_active=True)),
            ("twin_adjoint_cell", cellgen.adjoint_cell(0, z_active=True))]


def path_of(name):
    return os.path.join(HERE, name + "_10k.npz")


def main():
    for name, cell in cases():
        t0 = time.time()
        T, S = oracle.forward(cell, nsteps=STEPS, surf=True)
        lines = np.array(sample_lines(cell["nz"]), dtype=np.int64)
        steps = np.arange(TRACE_EVERY, STEPS + 1, TRACE_EVERY, dtype=np.int64)
        np.savez(path_of(name), steps=steps, surface=S[steps - 1], lines=lines,
                 field=T[lines], nsteps=np.int64(STEPS),
                 sources_sha256=np.array(sources_hash()),
                 problem_json=np.array(json.dumps(cell, sort_keys=True)))
        print("wrote %s (%.0f s)" % (path_of(name), time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
