"""Writes oracle_c1_trajectory.json.  Calls only the oracle and the instance
generator; run from the repository root: python tests/golden/make_golden.py"""
import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2501_17996_amd import instances as I  # noqa: E402

KEEP = {1, 2, 3, 10, 50, 99, 100, 101, 150, 200, 300, 400, 500, 561}


def main():
    s = oracle.OracleSolver(I.config1(0))
    rows = []
    for k in range(1, max(KEEP) + 1):
        M = s.step(check=True)
        if k in KEEP:
            rows.append({key: (M[key] if math.isfinite(M[key]) else None)
                         for key in ("k", "omega", "dF", "dY", "rel_kkt", "infeasible_frac")})
            rows[-1]["k"] = k
    out = {"instance": "config1 seed 0 (ring 10 + 30 chords, log utility)",
           "written_by": "tests/golden/make_golden.py (oracle only)", "rows": rows}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_c1_trajectory.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
