"""Writes colourings_workloads.json: the oracle's torus colouring (n_c, sigma)
for the lattice shapes of the benchmark workloads.  Calls only the oracle.

    python tests/golden/make_colourings.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import colouring  # noqa: E402

CASES = [((16, 16, 16, 32), 2), ((24, 24, 24, 48), 4), ((16, 16, 16, 32), 1),
         ((16, 16, 16, 32), 3), ((24, 24, 24, 48), 2), ((8, 8, 8, 8), 2),
         ((4, 4, 4, 4), 1), ((32, 32, 32), 4), ((24, 24, 24), 4)]

if __name__ == "__main__":
    out = []
    for dims, d in CASES:
        nc, sig = colouring.search(dims, d)
        out.append(dict(dims=list(dims), d=d, n_c=nc, sigma=list(sig)))
        print(dims, d, nc, sig, flush=True)
    json.dump(dict(source="oracle.colouring.search (exhaustive, first valid sigma in "
                          "lexicographic order)", cases=out),
              open(os.path.join(HERE, "colourings_workloads.json"), "w"), indent=1)
