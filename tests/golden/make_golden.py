"""Write the stored expected values under tests/golden/ from the CPU oracle.

Only the oracle (and the seeded input generator) is called here.  Each
fixture is a run of the scheme of Sec. 3 (eqs. (8)-(20)) on a seeded cell:
the surface-mean trace at a few steps and sampled node temperatures, at full
precision (repr of the double).  Run from the repository root:

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import cellgen  # noqa: E402
import oracle  # noqa: E402

SAMPLE_STEPS = [1, 10, 100, 1000, 3000]


def cases():
    """(name, citation, cell, steps) of every fixture."""
    c0 = cellgen.with_nz(cellgen.small_cell(0), 4)
    c1 = cellgen.small_cell(1, z_active=True)
    c1 = cellgen.with_nz(c1, 12)
    c2 = cellgen.with_nz(cellgen.small_cell(2), 4)
    dt = c2["dt"]
    c2.update(t_on=3 * dt, width=5 * dt, period=20 * dt, turn_on=True)
    c3 = cellgen.poly_variant(cellgen.with_nz(cellgen.small_cell(3, z_active=True), 10), 3,
                              joule_tref=30.0)
    c4 = cellgen.with_nz(cellgen.small_cell(4, z_active=True), 12)
    c4["stepped"] = dict(z_full=6, nr_top=30)
    return [
        ("small_cell0_nz4", "eqs. (8)-(20), as-written cell (z-invariant)", c0, 3000),
        ("small_cell3_poly_joule", "eqs. (8)-(20) with the polynomial laws of eqs. (23), (24) "
                                   "and the Joule source of eq. (25)", c3, 1500),
        ("small_cell4_stepped", "eqs. (8)-(20) on the stepped domain of eq. (9)", c4, 1500),
        ("small_cell1_z_active_nz12", "eqs. (8)-(20) with the explicit z half (eq. (11)) active",
         c1, 3000),
        ("small_cell2_turn_on", "eqs. (8)-(20) with the turn-on model of eq. (22), "
                                "pulses every 20 steps", c2, 100),
    ]


def record(cell, n):
    T, S = oracle.forward(cell, nsteps=n, surf=True, nthreads=1)
    rng = np.random.default_rng(12345)
    nz, nr = T.shape
    idx = [(int(j), int(i)) for j, i in zip(rng.integers(0, nz, 16), rng.integers(0, nr, 16))]
    idx += [(1, nr - 1), (nz - 2, 0)]
    return {
        "surface": {str(k): repr(float(S[k - 1])) for k in SAMPLE_STEPS if k <= n},
        "field": [[j, i, repr(float(T[j, i]))] for j, i in idx],
    }


def main():
    out = {}
    for name, cite, cell, n in cases():
        rec = record(cell, n)
        rec.update(citation=cite, steps=n)
        out[name] = rec
    path = os.path.join(HERE, "oracle_runs.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
