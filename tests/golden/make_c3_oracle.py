"""Writes c3_oracle.json: expected values for the GPU tests of the 3D 24^3 x 6
tets problem (delta = 3h, eps = delta/16, L_max = 4, constant kernel), computed
by the FP64 CPU oracle alone (too slow to recompute inside a GPU test):

  * leaf integrations per level of Algorithm 1 over the whole mesh (counted
    without evaluating them);
  * four whole rows of the matrix (all pairs touching the row's node, each pair
    by Algorithm 1), at an interior node, a node next to the constrained layer,
    a node of that layer and a node near an edge of the free region.

Run from the repository root:  python tests/golden/make_c3_oracle.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2101_08825_amd import workloads as W  # noqa: E402


def node(n, ii):
    return int(sum(ii[d] * (n + 1) ** d for d in range(3)))


def main():
    wl = W.WORKLOADS["c3_3d24"]
    mesh = wl.mesh()
    n, k = mesh.n, mesh.k_gamma
    om = oracle.OracleMesh(mesh.coords, mesh.conn)
    prm = oracle.params(wl.delta, wl.eps, wl.lmax)
    t = time.time()
    leaves = oracle.leaf_counts(om, prm, np.arange(mesh.n_elems))
    print(f"leaf counts {list(leaves[:wl.lmax + 1])} ({time.time() - t:.1f} s)", flush=True)
    picks = {"interior": [n // 2] * 3, "next_to_layer": [k + 1] * 3, "layer": [k] * 3,
             "near_edge": [k + 1, n // 2, n - k - 1]}
    rows = {}
    for name, ii in picks.items():
        r = node(n, ii)
        t = time.time()
        cols, vals = oracle.rows(om, prm, wl.delta + wl.eps, [r])[0]
        print(f"row {name} {r}: {len(cols)} entries ({time.time() - t:.1f} s)", flush=True)
        rows[name] = {"node": r, "index": ii, "cols": [int(c) for c in cols],
                      "vals": [float(v).hex() for v in vals]}
    out = {
        "source": "FP64 CPU oracle (oracle/), written by tests/golden/make_c3_oracle.py",
        "workload": "3D [0,1]^3, 24^3 cubes x 6 Kuhn tets, delta = 3h, eps = delta/16, L_max = 4, "
                    "15-point rule, constant kernel C_{delta,eps}, four-term form",
        "leaves_per_level": [int(x) for x in leaves[:wl.lmax + 1]],
        "rows": rows,
    }
    with open(os.path.join(HERE, "c3_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
