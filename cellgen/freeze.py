"""Write the measured workloads' problem dictionaries as frozen JSON files
(cellgen/frozen/*.json): the files, not the random number generator, are the
record of the inputs the tests and the benchmark use; a CPU test checks that
the generator still produces them exactly.  Run from the repository root:

    python cellgen/freeze.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import cellgen  # noqa: E402


def workloads():
    """(name, what, problem dictionaries) of every frozen workload."""
    return [
        ("small_cell", "64x128 cell, 4 layers, 10,000 steps (seed 0)", [cellgen.small_cell(0)]),
        ("small_cell_z_active", "the same with the top line held (seed 0)",
         [cellgen.small_cell(0, z_active=True)]),
        ("device_cell", "1024x4096 cell, 8 layers, 100,000 steps (seed 0): the headline workload",
         [cellgen.device_cell(0)]),
        ("device_cell_z_active", "the same with the top line held (seed 0)",
         [cellgen.device_cell(0, z_active=True)]),
        ("sweep_cells", "design sweep: 256 uneven cells, 20,000 steps each (seed 0)",
         cellgen.sweep_cells(0)),
        ("adjoint_cell", "512x2048 cell, 6 layers, 50,000 steps (seed 0)", [cellgen.adjoint_cell(0)]),
        ("design_cells", "design loop: 64 designs of 512x1024, 100,000 steps (seed 0)",
         cellgen.design_cells(0)),
        ("paper_shape", "631x1201 cell, 100,000 steps (seed 0)", [cellgen.paper_shape(0)]),
    ]


def path_of(name):
    return os.path.join(HERE, "frozen", name + ".json")


def main():
    for name, what, cells in workloads():
        with open(path_of(name), "w") as f:
            json.dump({"workload": what, "problems": cells}, f, indent=0, sort_keys=True)
            f.write("\n")
        print("wrote", path_of(name))


if __name__ == "__main__":
    main()
