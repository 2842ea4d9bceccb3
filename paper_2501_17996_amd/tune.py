"""Launch-shape tuner for the two-phase iteration and the batching pool.

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

With ``--pool`` it tunes the batching pool instead: for each bucket b of the largest n a pool
admits (64, 128, 256, 512) it fills a pool with 64 instances of n uniform in (b/2, b],
out-degree uniform in 4..16, half log and half power(1/2) utility (the shape of the serving
stream), and times a pool iteration over all of them (events on the pool's stream, after
warm-up steps) with each compiled number of waves per node workgroup, and with every instance
in the two-phase iteration instead (flat edge items, then node items); the fastest goes into
``csrc/tuned_pool.inc``: a pool takes the waves of the entry for its n_max, and an instance of n
nodes the organisation of the entry for n (``mcf_pool_instance_options``).  The choice is a
function of (n, precision) alone.

    python -m paper_2501_17996_amd.tune --pool [--summary FILE]
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
    return n <= 64 * abs(waves) * vectors * vec   # waves -1: the flat form, one wave per column


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


POOL_INC = os.path.join(HERE, "csrc", "tuned_pool.inc")
POOL_BUCKETS = (64, 128, 256, 512)
POOL_WAVES = {1: (1, 2, 4, 8), 0: (8,)}  # compiled waves per node workgroup, per precision


def pool_instances(b: int, slots: int = 64):
    import numpy as np
    from . import instances as I
    rng = np.random.default_rng(b)
    out = []
    for q in range(slots):
        n = int(rng.integers(max(20, b // 2 + 1), b + 1))
        deg = int(rng.integers(4, 17))
        out.append(I.ring_instance(n, min(deg, n - 1), seed=5000 + b + q, utility=q % 2, gamma=0.5))
    return out


def two_phase_options(mcf, n, precision):
    """The two-phase form a pool runs: flat edge phase, 64-thread node blocks."""
    vec = 4 if precision == 1 else 2
    nv = 1 if n <= 64 * vec else 2 if n <= 128 * vec else 4
    return dict(kernel_mode=mcf.MCF_KERNELS_TWO_PHASE, edge_waves=-1, edge_vectors=nv, node_block=64)


def time_pool(mcf, torch, insts, precision, b, waves, org=0, steps=8, K=20):
    """Microseconds per pool iteration over every instance (tolerance out of reach).  org: 0 every
    instance fused, 1 every instance in the two-phase iteration, or a predicate on n choosing
    the two-phase iteration for some."""
    stream = torch.cuda.Stream()
    pool = mcf.Pool(precision, 0, len(insts), K, stream=stream.cuda_stream, n_max=b, waves=waves)
    two = org if callable(org) else (lambda n: bool(org))
    hs = [mcf.Solver(i, precision=precision, tol=1e-14, check_every=K, max_iter=10 ** 8,
                     **(two_phase_options(mcf, i.n, precision) if two(i.n) else {})) for i in insts]
    try:
        for h in hs:
            pool.admit(h)
        for _ in range(3):
            pool.step(K)
            pool.sync()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            pool.step(K)
        e1.record(stream)
        pool.sync()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / (steps * K)
    finally:
        pool.close()
        for h in hs:
            h.close()


def tune_pool(log=print):
    import torch
    from . import instances as I
    from . import mcf
    torch.cuda.set_device(0)
    results = {}   # (precision, b) -> sorted [(us, waves, org)]
    orgs = {}      # (precision, b) -> organisation of that bucket's instances in a mixed pool
    mix = [I.serving_request(r) for r in range(64)]
    for precision in (1, 0):
        for b in POOL_BUCKETS:
            insts = pool_instances(b)
            rows = []
            for waves in POOL_WAVES[precision]:
                us = time_pool(mcf, torch, insts, precision, b, waves)
                rows.append((us, waves, 0))
                log(f"pool {'fp32' if precision else 'fp64'} n_max={b:3d} fused waves={waves}: {us:8.2f} us/iteration "
                    f"({sum(i.n for i in insts)} nodes)")
            us = time_pool(mcf, torch, insts, precision, b, POOL_WAVES[precision][-1], org=1)
            rows.append((us, 0, 1))
            log(f"pool {'fp32' if precision else 'fp64'} n_max={b:3d} two-phase: {us:8.2f} us/iteration")
            rows.sort()
            results[(precision, b)] = rows
        # The organisation of an instance is decided in a mixed pool (the first 64 requests of the
        # serving stream, with the waves measured best for n_max = 512): a bucket's instances go
        # two-phase only if the pool is faster with them so than with every instance fused, since
        # the two-phase launches cost their latency whatever the number of instances in them.
        waves = sorted(r for r in results[(precision, 512)] if r[2] == 0)[0][1]
        base = time_pool(mcf, torch, mix, precision, 512, waves, org=0)
        log(f"pool {'fp32' if precision else 'fp64'} serving mix, all fused: {base:8.2f} us/iteration")
        orgs[(precision, 0)] = base
        lo = 0
        for b in POOL_BUCKETS:
            us = time_pool(mcf, torch, mix, precision, 512, waves, org=lambda n, lo=lo, b=b: lo < n <= b)
            orgs[(precision, b)] = 1 if us < 0.99 * base else 0
            log(f"pool {'fp32' if precision else 'fp64'} serving mix, n in ({lo}, {b}] two-phase: {us:8.2f} "
                f"us/iteration -> {'two-phase' if orgs[(precision, b)] else 'fused'}")
            results[(precision, b)].append((us, -b, 2))   # a mixed-pool row (listed, not a shape)
            lo = b
    results["orgs"] = orgs
    return results


def write_pool_inc(results, path=POOL_INC):
    lines = ["// Batching-pool launch shapes by measurement, written by paper_2501_17996_amd/tune.py (--pool)",
             "// on one MI355X: 64 instances of n in (n_max/2, n_max], out-degree 4..16, log and power(1/2);",
             "// mean time of a pool iteration over all of them.  Entries ascend in n_max per iterate size:",
             "// {bytes, largest n, waves per node workgroup of the fused items, organisation of an instance of",
             "// that size: 0 fused, 1 two-phase}.  The organisation is decided in a mixed pool (64 requests of",
             "// the serving stream): two-phase only where moving that size's instances there made it faster.",
             "static const TunedPool TUNED_POOL[] = {"]
    for precision in (1, 0):
        for b in POOL_BUCKETS:
            rows = results.get((precision, b))
            if rows:
                fused = sorted(r for r in rows if r[2] == 0)
                org = results["orgs"][(precision, b)]
                lines.append(f"    {{{4 if precision else 8}, {b}, {fused[0][1]}, {org}}},  // {fused[0][0]:.2f} us")
    lines.append("};")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def write_pool_summary(results, path):
    with open(path, "w") as f:
        f.write("# Batching-pool shapes measured by `paper_2501_17996_amd/tune.py --pool`\n\n")
        f.write("64 instances per pool, n uniform in (n_max/2, n_max], out-degree uniform in 4..16, half log "
                "and half power(1/2) utility; mean time of one pool iteration over all of them (the "
                "check every 20 iterations included), events on the pool's stream after 3 warm-up steps. The "
                "first row of each bucket is the one the table takes.\n\n")
        f.write("```\npython -m paper_2501_17996_amd.tune --pool --summary profiles/tuning_pool_shapes.md\n```\n\n")
        f.write("| precision | n_max | organisation | waves per node | us per pool iteration | vs best |\n"
                "|---|---|---|---|---|---|\n")
        for precision in (1, 0):
            for b in POOL_BUCKETS:
                rows = [r for r in results.get((precision, b), []) if r[2] < 2]
                for us, waves, org in rows:
                    f.write(f"| {'FP32' if precision else 'FP64'} | {b} | {'two-phase' if org else 'fused'} | "
                            f"{waves if not org else '-'} | {us:.2f} | {us / rows[0][0]:.3f} |\n")
        f.write("\nThe organisation of an instance is decided in a mixed pool: the first 64 requests of the serving "
                "stream, with the bucket's instances in the two-phase iteration and the others fused, against all "
                "fused (the two-phase launches cost their latency whatever the number of instances in them).\n\n")
        f.write("| precision | two-phase instances | us per pool iteration | table |\n|---|---|---|---|\n")
        for precision in (1, 0):
            if (precision, 0) in results["orgs"]:
                f.write(f"| {'FP32' if precision else 'FP64'} | none | {results['orgs'][(precision, 0)]:.2f} | |\n")
            lo = 0
            for b in POOL_BUCKETS:
                mixed = [r for r in results.get((precision, b), []) if r[2] == 2]
                if mixed:
                    org = results["orgs"][(precision, b)]
                    f.write(f"| {'FP32' if precision else 'FP64'} | n in ({lo}, {b}] | {mixed[0][0]:.2f} | "
                            f"{'two-phase' if org else 'fused'} |\n")
                lo = b


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
                # waves -1 (flat) is the compiled shape {1, vectors, 2}; 1 (concurrent) is {1, vectors, 1}
                w, par = (1, 2) if waves == -1 else (waves, 1 if waves == 1 else 0)
                entries[(4 if precision else 8, n)] = (w, vectors, par, nb, ms * 1e3)
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
    ap.add_argument("--out", default=None, help="where to write the table (default: the compiled-in one)")
    ap.add_argument("--pool", action="store_true", help="tune the batching pool's shapes instead")
    args = ap.parse_args(argv)
    if args.pool:
        res = tune_pool(log=lambda s: print(s, flush=True))
        if not args.no_write:
            write_pool_inc(res, args.out or POOL_INC)
            print(f"wrote {args.out or POOL_INC}", flush=True)
        if args.summary:
            write_pool_summary(res, args.summary)
            print(f"wrote {args.summary}", flush=True)
        return 0
    args.out = args.out or INC
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
