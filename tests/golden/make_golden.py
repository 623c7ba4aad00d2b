"""Write the oracle regression fixtures in this folder.

Calls only ``oracle/`` (and the seeded generator); run from the repo root:
``python tests/golden/make_golden.py``.  The fixture freezes the oracle's
output for the 256x256 full-span-line workload (seed 0, T=40, depth 8,
both passes), so a later change to the oracle's arithmetic shows up here.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    w = synth.workload("line256", 0)
    x, y = oracle.edge_points(w.image)
    res = oracle.detect(x, y, w.width, w.height, w.threshold, w.max_depth)
    out = {
        "what": "oracle output for line256 seed 0 (256x256, 8 full-span lines, 1% noise), "
                "T=40, depth 8, code variant, both passes",
        "E": int(len(x)),
        "n_cells": int(len(res.cells)),
        "members_sum": int(res.members.astype(np.int64).sum()),
        "stats_columns": list(oracle.STAT_NAMES),
        "stats": {str(p): s.tolist() for p, s in res.stats.items()},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "line256_seed0.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
