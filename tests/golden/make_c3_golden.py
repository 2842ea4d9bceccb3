"""Writes oracle_c3_golden.json: the FP64 oracle on config3 seed 0 (n = 1000 ring + chords of
out-degree 10, lognormal capacities, power utility gamma = 1/2).

* Sampled iterates at k = 100, 200 and 300: 1000 entries of F^{k-1/2} and 1000 of Y^k at seeded
  random positions, with omega, the step norms, the check metrics of iteration k and the largest
  magnitudes of F and Y (the scale of the 1e-10 relative comparison).
* The solve from the cold start to rel_kkt <= 1e-4 with the residual checked every 50
  iterations: the stop iteration and the objective p = -U(T^), the FP64 reference of the FP32
  solve at the same tolerance.

Calls only the oracle and the instance generator (about half an hour on 8 cores); run from the
repository root: python tests/golden/make_c3_golden.py [threads]"""
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2501_17996_amd import instances as I  # noqa: E402

CHECKPOINTS = (100, 200, 300)
SAMPLES = 1000
TOL, CHECK_EVERY = 1e-4, 50
METRICS = ("omega", "dF", "dY", "r", "rel_primal", "rel_dual", "rel_gap", "rel_kkt", "primal_obj", "dual_obj",
           "infeasible_frac")


def fin(x):
    return x if math.isfinite(x) else None


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    inst = I.config3(0)
    n, m = inst.n, inst.m
    rng = np.random.default_rng(2024)
    f_idx = rng.integers(0, n * m, SAMPLES)        # flat F[l*n + i]
    y_idx = rng.integers(0, n * n, SAMPLES)        # flat Y[j*n + i]
    s = oracle.OracleSolver(inst, threads=threads)
    t0 = time.time()
    rows, k = [], 0
    for kc in CHECKPOINTS:
        s.run(kc - k - 1, check=False)
        M = s.step(check=True)
        k = kc
        F, Y, sc = s.get_state()
        rows.append({"k": kc, **{key: fin(M[key]) for key in METRICS},
                     "F_max_abs": float(np.max(np.abs(F))), "Y_max_abs": float(np.max(np.abs(Y))),
                     "F": [float(F[x]) for x in f_idx], "Y": [float(Y[x]) for x in y_idx]})
        print(f"k={kc} omega {M['omega']:.6g} rel_kkt {M['rel_kkt']:.3g} ({time.time() - t0:.0f} s)", flush=True)
    # the solve to the tolerance continues the same trajectory (checks only observe)
    state = s.solve(TOL, stop_rule=0, max_iter=100000, check_every=CHECK_EVERY)
    M = s.metrics()
    out = {"instance": "config3 seed 0: n=1000 ring+chords out-degree 10, c~lognormal(0,0.5), power gamma=0.5",
           "written_by": "tests/golden/make_c3_golden.py (oracle only)",
           "f_index": [int(x) for x in f_idx], "y_index": [int(x) for x in y_idx], "checkpoints": rows,
           "solve": {"tol": TOL, "check_every": CHECK_EVERY, "state": state, "iters": int(M["k"]),
                     **{key: fin(M[key]) for key in METRICS}},
           "seconds": time.time() - t0, "threads": threads}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_c3_golden.json"), "w") as f:
        json.dump(out, f)
    print(json.dumps(out["solve"]), flush=True)


if __name__ == "__main__":
    main()
