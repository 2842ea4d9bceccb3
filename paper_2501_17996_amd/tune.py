"""Launch-shape tuner for the two-phase iteration.

Times every compiled edge shape (``mcf_edge_shapes``) whose columns hold n entries, with each
node-phase block (64 and 256 threads), on a ring + chords instance of out-degree 10 (the shape
of the larger workloads) at a ladder of sizes n, for FP32 and FP64 iterates, and writes the
fastest pair per size into ``csrc/tuned_shapes.inc``.  That table is compiled into libmcf.so:
an entry covers every n up to its size above the previous entry's, so the shape is a function of
(n, precision) alone and a solve never depends on timing.  Entries of sizes not measured in a run
are kept from the existing table.  Rebuild the library after running.

A candidate's time is the mean duration of its regular iterations (edge and node launches),
from the events the dispatches record (``mcf_enable_kernel_timing``), after warm-up iterations.

    python -m paper_2501_17996_amd.tune [--sizes 128,256,...] [--summary FILE]
"""
from __future__ import annotations

import argparse
import os
import re
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
INC = os.path.join(HERE, "csrc", "tuned_shapes.inc")
LADDER = [128, 256, 512, 1024, 2048, 4096, 8192, 12288, 16384]
NODE_BLOCKS = (64, 256)
WARMUP, TIMED = 20, 63   # sampled iterations k = 21, 28, ..., 77: regular ones only


def covers(waves: int, vectors: int, n: int, precision: int) -> bool:
    vec = 4 if precision == 1 else 2
    return n <= 64 * waves * vectors * vec


def time_candidate(mcf, inst, precision, waves, vectors, node_block):
    S = mcf.Solver(inst, precision=precision, tol=1e-12, check_every=1000, max_iter=10**6,
                   kernel_mode=mcf.MCF_KERNELS_TWO_PHASE, edge_waves=waves, edge_vectors=vectors,
                   node_block=node_block)
    try:
        S.run(WARMUP)
        mcf.mcf_enable_kernel_timing(S.h, True)
        S.run(TIMED)
        ms, cnt = mcf.mcf_kernel_time(S.h)
        mcf.mcf_enable_kernel_timing(S.h, False)
        return ms / max(cnt, 1)
    finally:
        S.close()


def tune(sizes, log=print):
    import torch
    from . import instances as I
    from . import mcf
    torch.cuda.set_device(0)
    results = {}   # (precision, n) -> list of (ms, waves, vectors, node_block)
    for precision in (1, 0):
        shapes = mcf.mcf_edge_shapes(precision)
        for n in sizes:
            inst = I.ring_instance(n, 10, seed=n)
            rows = []
            for waves, vectors in shapes:
                if not covers(waves, vectors, n, precision):
                    continue
                for nb in NODE_BLOCKS:
                    t0 = time.perf_counter()
                    ms = time_candidate(mcf, inst, precision, waves, vectors, nb)
                    rows.append((ms, waves, vectors, nb))
                    log(f"{'fp32' if precision else 'fp64'} n={n:5d} waves={waves:2d} vectors={vectors} "
                        f"node_block={nb:3d}: {ms * 1e3:9.2f} us/iteration ({time.perf_counter() - t0:.1f} s)")
            rows.sort()
            results[(precision, n)] = rows
    return results


ENTRY = re.compile(r"^\s*\{(\d+), (\d+), \{(\d+), (\d+), (\d+)\}, (\d+)\},\s*//\s*([0-9.]+) us")


def read_inc(path=INC):
    """The entries of an existing table: {(bytes, n_max): (waves, vectors, par, node_block, us)}."""
    out = {}
    if os.path.exists(path):
        for line in open(path):
            m = ENTRY.match(line)
            if m:
                b, n, w, v, par, nb = (int(m.group(k)) for k in range(1, 7))
                out[(b, n)] = (w, v, par, nb, float(m.group(7)))
    return out


def write_inc(results, sizes, path=INC):
    entries = read_inc(path)
    for precision in (1, 0):
        for n in sizes:
            rows = results.get((precision, n))
            if rows:
                ms, waves, vectors, nb = rows[0]
                entries[(4 if precision else 8, n)] = (waves, vectors, 1 if waves == 1 else 0, nb, ms * 1e3)
    lines = ["// Two-phase launch shapes by measurement, written by paper_2501_17996_amd/tune.py on one",
             "// MI355X (ring + chords instances of out-degree 10; mean regular-iteration time of the",
             "// edge and node launches).  Entries ascend in n_max per iterate size.",
             "static const TunedEntry TUNED_SHAPES[] = {"]
    for b in (4, 8):
        for n in sorted(k[1] for k in entries if k[0] == b):
            w, v, par, nb, us = entries[(b, n)]
            lines.append(f"    {{{b}, {n}, {{{w}, {v}, {par}}}, {nb}}},  // {us:.2f} us")
    lines.append("};")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def write_summary(results, sizes, path):
    with open(path, "w") as f:
        f.write("# Two-phase launch shapes measured by `paper_2501_17996_amd/tune.py`\n\n")
        f.write("Ring + chords instances of out-degree 10 (m = 10 n), mean time of a regular iteration "
                "(edge and node launches) from dispatch-recorded events, after "
                f"{WARMUP} warm-up iterations. The first row of each size is the one the table takes.\n\n")
        f.write("```\npython -m paper_2501_17996_amd.tune --summary profiles/tuning_two_phase_shapes.md\n```\n\n")
        for precision in (1, 0):
            f.write(f"## {'FP32' if precision else 'FP64'} iterates\n\n")
            f.write("| n | edge waves | edge vectors | node block | us per iteration | vs best |\n|---|---|---|---|---|---|\n")
            for n in sizes:
                rows = results.get((precision, n), [])
                if not rows:
                    continue
                best = rows[0][0]
                for ms, waves, vectors, nb in rows:
                    f.write(f"| {n} | {waves} | {vectors} | {nb} | {ms * 1e3:.2f} | {ms / best:.2f} |\n")
            f.write("\n")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--sizes", default=",".join(str(x) for x in LADDER))
    ap.add_argument("--summary", default=None, help="also write a markdown table of every measurement")
    ap.add_argument("--no-write", action="store_true", help="measure only; leave the table as it is")
    ap.add_argument("--out", default=INC, help="where to write the table (default: the compiled-in one)")
    args = ap.parse_args(argv)
    sizes = [int(x) for x in args.sizes.split(",")]
    res = tune(sizes, log=lambda s: print(s, flush=True))
    if not args.no_write:
        write_inc(res, sizes, args.out)
        print(f"wrote {args.out}", flush=True)
    if args.summary:
        write_summary(res, sizes, args.summary)
        print(f"wrote {args.summary}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
