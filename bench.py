"""Benchmark of the PDMCF hot path on one MI355X.

Default workload: config4, the largest single-GPU configuration: n = 10000 nodes, ring +
chords with out-degree 10 (m = 100000), capacities U[0.5, 2], log utility with
w ~ U[0.5, 1.5], FP32 iterates (1e9 flow variables, 4 GB per iterate array) with FP64
reductions, relative KKT tolerance 1e-3, instance resident in HBM.  A step is one block of 50
whole PDHG iterations of the running solve (edge phase, node phase and FP64 control in every
iteration; the residual/KKT check, its residual pass and the stop test at the block's last
iteration), replayed from the block's captured HIP graph.  The same run also reports the
time to the tolerance of a full config4 solve from the cold start, the full solves of config2
and config3, a short serving stream (p50/p99) and the saturated batching pool.

Prints one JSON line with the throughput in edge-dest updates per second
(n * m * iterations / second), the roofline of the iteration measured with HIP events on the
solver's stream inside the timed region, and the CPU oracle timed on a bounded sample of the
same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def measured_traffic(workload: str):
    """HBM bytes per launch of the dominant kernel from the committed counter runs, or None
    when the kernel source changed after the counters were taken."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    except OSError:
        return None
    if kernels_sha256() != rec.get("kernels_sha256") or workload not in rec:
        return None
    return rec[workload]["bytes_per_launch"]


def kernels_sha256() -> str:
    """Hash of the kernel source and the launch-shape table the traffic figures belong to."""
    import hashlib
    h = hashlib.sha256()
    for f in ("mcf_kernels.hip", "tuned_shapes.inc", "tuned_pool.inc"):
        h.update(open(os.path.join(ROOT, "paper_2501_17996_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def workload(name: str):
    from paper_2501_17996_amd import instances as I
    if name == "c2":
        return I.config2(0), 1e-4, ("n=200 ring+chords out-degree 10 (m=2000), c~U[0.5,2], log utility "
                                    "w~U[0.5,1.5], solve to rel KKT 1e-4")
    if name == "c3":
        return I.config3(0), 1e-4, ("n=1000 ring+chords out-degree 10 (m=10000), c~lognormal(0,0.5), "
                                    "power utility gamma=0.5, solve to rel KKT 1e-4")
    if name == "c4":
        return I.config4(0), 1e-3, ("n=10000 ring+chords out-degree 10 (m=100000), c~U[0.5,2], log utility, "
                                    "solve to rel KKT 1e-3")
    raise SystemExit(f"unknown workload {name}")


def alg_bytes(n: int, m: int, s: int, fused: bool, check: bool) -> float:
    """Algorithmic bytes of one timed unit: one whole PDHG iteration, the single fused launch
    or the edge and node launches of the two-phase organisation.

    The per-iteration model s (4 n m + 3 n^2): F read and written, Fbar written and read,
    Y read and written, W read.  Neither organisation stores Fbar (the fused one recomputes
    the projection at both end nodes, the two-phase one carries P = F A^T), but both are
    credited with the model's bytes, which is what a plain implementation of the iteration
    moves.  A check iteration also writes Fhat and D (2 s n m) and T and U' (16 n^2)."""
    b = s * (4.0 * n * m + 3.0 * n * n)
    if check:
        b += 2.0 * s * n * m + 16.0 * n * n
    return b


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_solve(inst, tol, check_every, budget_s: float):
    """The FP64 oracle on the host cores, on the same instance from the cold start, in blocks of
    check_every iterations (the last one checked) until the relative KKT residual reaches tol or
    the time budget runs out.  When it converges, its primal objective is the FP64 reference the
    GPU result is compared with."""
    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    O = oracle.OracleSolver(inst, threads=threads)
    iters, t0 = 0, time.perf_counter()
    converged = False
    while time.perf_counter() - t0 < budget_s:
        for _ in range(check_every):
            mo = O.step(check=(_ == check_every - 1))
        iters += check_every
        if mo["rel_kkt"] <= tol:
            converged = True
            break
    dt = time.perf_counter() - t0
    what = (f"FP64 solve of the same instance from the cold start to rel KKT {tol:g} (residual every "
            f"{check_every}): {iters} iterations" if converged else
            f"{iters} PDHG iterations of the same instance from the cold start (residual every {check_every}), "
            f"FP64, stopped at the time budget before reaching rel KKT {tol:g}")
    return {"value": inst.n * inst.m * iters / dt, "unit": "edge-dest updates/s", "cores": threads,
            "kind": "oracle", "sample": f"{what}, {dt:.1f} s on {threads} threads of {cpu_model()}",
            "converged": converged, "iters": iters, "primal_obj": mo["primal_obj"] if converged else None}


def cpu_baseline_iterations(inst, iters: int, threads: int):
    """The FP64 oracle's per-iteration time on the host: `iters` iterations from the cold start
    (the first also touches the oracle's arrays for the first time), each timed; the median."""
    import oracle
    O = oracle.OracleSolver(inst, threads=threads)
    times = []
    for _ in range(iters):
        t0 = time.perf_counter()
        O.step(check=False)
        times.append(time.perf_counter() - t0)
    O.close()
    times.sort()
    return times[len(times) // 2], times


def timed_solves(mcf, torch, name, reps, check_every):
    """`reps` full solves of a configuration from the cold start (setup and upload done once):
    wall time to the tolerance, iterations, throughput."""
    inst, tol, desc = workload(name)
    S = mcf.Solver(inst, precision=mcf.MCF_FP32, tol=tol, check_every=check_every, max_iter=200000,
                   stream=torch.cuda.current_stream().cuda_stream)
    try:
        S.solve()          # warm-up: captures the block graphs
        S.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters = 0
        for _ in range(reps):
            S.reset()
            st = S.solve()
            iters += st["iters"]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
    finally:
        S.close()
    return {"workload": desc + f", FP32 iterates, residual every {check_every}", "time_to_tol_ms": dt * 1e3,
            "iters": iters // reps, "state": st["state_name"], "rel_kkt": st["rel_kkt"],
            "primal_obj": st["primal_obj"], "edge_dest_updates_per_s": inst.n * inst.m * (iters / reps) / dt}


def pool_leg(mcf, torch, slots: int, steps: int, K: int):
    """The batching pool saturated: the first `slots` requests of the serving stream (seed 1000+r,
    n ~ U{20..500}, out-degree ~ U{4..16}, log/power(0.5)) admitted together, FP32, run for
    `steps` steps of K iterations (tolerance out of reach, so every slot iterates throughout).
    The timed unit is one pool iteration over every slot (the persistent iteration launch, plus
    the amortised check, residual, control and gather), timed with events on the pool's stream."""
    from paper_2501_17996_amd import instances as I
    stream = torch.cuda.Stream()     # a stream of its own (default priority): the events bracket its work
    insts = [I.serving_request(r) for r in range(slots)]
    pool = mcf.Pool(mcf.MCF_FP32, 0, slots, K, stream=stream.cuda_stream)
    # each instance in the organisation the pool runs fastest for its size
    hs = [mcf.Solver(i, tol=1e-14, check_every=K, max_iter=10 ** 8, **pool.instance_options(i.n)) for i in insts]
    for h in hs:
        pool.admit(h)
    for _ in range(3):
        pool.step(K)
        pool.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        pool.step(K)
    e1.record(stream)
    pool.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    shape = pool.shape()
    two_phase = sum(h.layout()["kernel_mode"] == "two_phase" for h in hs)
    pool.close()
    for h in hs:
        h.close()
    per_it = ev_ms * 1e-3 / (steps * K)
    alg = sum(alg_bytes(i.n, i.m, 4, True, False) * (K - 1) / K + alg_bytes(i.n, i.m, 4, True, True) / K
              for i in insts)
    upd = sum(i.n * i.m for i in insts)
    return {"workload": f"{slots} requests of the serving stream in one pool, FP32, steps of {K} iterations",
            "n_total": sum(i.n for i in insts), "nm_total": upd, "shape": shape,
            "two_phase_instances": two_phase,
            "us_per_iteration": per_it * 1e6, "edge_dest_updates_per_s": upd / per_it,
            "wall_updates_per_s": upd * steps * K / wall,
            "roofline": {"bound": "hbm", "achieved": alg / per_it / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": alg / per_it / 1e9 / HBM_PEAK_GBS, "traffic": measured_traffic("pool"),
                         "alg_bytes_per_iteration": alg,
                         "working_set_bytes": sum(mcf.mcf_workspace_bytes(i.n, i.m, 1) for i in insts)}}


def serve_bench(args):
    print(json.dumps(serve_run(args)), flush=True)


def serve_run(args):
    """Serving stream: requests r = 0.. (seed 1000+r; n ~ U{20..500}, out-degree ~ U{4..16},
    log or power(0.5) utility), FP32 iterates batched in one pool, Poisson arrivals at
    `load` x the throughput of a saturated calibration run.  Reports p50/p99 latency and
    throughput, beside the FP64 single-instance solve of the first requests one at a time."""
    import torch
    from paper_2501_17996_amd import instances as I
    from paper_2501_17996_amd import mcf
    from paper_2501_17996_amd.serve import GpuBackend, Request, serve

    torch.cuda.set_device(0)
    tol, K = 1e-4, args.check_every

    def stream(count, rate, offset=0):
        times = I.poisson_arrivals(count, rate, seed=7) if rate > 0 else [0.0] * count
        return [Request(r, float(t), (lambda r=r: I.serving_request(r))) for r, t in zip(range(offset, offset + count), times)]

    budget = int(args.serve_budget_gb * 2 ** 30)
    be = GpuBackend(mcf.MCF_FP32, budget, args.slots, K, tol, max_iter=args.serve_max_iter,
                    adapt_until=args.adapt_until)
    _, calib = serve(stream(args.calib, 0.0, offset=args.requests), be)
    rate = args.load * calib["instances_per_s"]
    records, summ = serve(stream(args.requests, rate), be)
    be.close()
    # the plain FP64 single-instance solve, one request after another
    n_single = min(args.single, args.requests)
    t0, upd = time.perf_counter(), 0.0
    for r in range(n_single):
        inst = I.serving_request(r)
        S = mcf.Solver(inst, precision=mcf.MCF_FP64, tol=tol, check_every=K, max_iter=args.serve_max_iter,
                       adapt_until=args.adapt_until)
        st = S.solve()
        upd += inst.n * inst.m * st["iters"]
        S.close()
    t_single = time.perf_counter() - t0
    out = {
        "metric": "served MCF instances/s (FP32 batched pool, rel KKT 1e-4)",
        "value": summ["instances_per_s"], "unit": "instances/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.requests} requests seed 1000+r, n~U{{20..500}}, out-degree~U{{4..16}}, "
                               f"log/power(0.5), Poisson arrivals at {args.load} x saturated throughput",
                   "slots": args.slots, "check_every": K, "hbm_budget_gb": args.serve_budget_gb,
                   "adapt_until": args.adapt_until,
                   "arrival_rate_per_s": rate, "calibration": calib},
        "latency_p50_s": summ["latency_p50_s"], "latency_p99_s": summ["latency_p99_s"],
        "service_p50_s": summ["service_p50_s"], "service_p99_s": summ["service_p99_s"],
        "edge_dest_updates_per_s": summ["edge_dest_updates_per_s"], "converged": summ["converged"],
        "requests": summ["requests"], "rejected": summ["rejected"], "makespan_s": summ["makespan_s"],
        "single_fp64": {"requests": n_single, "instances_per_s": n_single / t_single,
                        "edge_dest_updates_per_s": upd / t_single},
    }
    return out


def warmstart_bench(args):
    """Section 3.1 warm start: the perturbed problem (weights (1 +/- nu) w) is solved until its
    iterate is feasible; the original problem then starts from that (F, Y, omega).  Reports
    iterations of the original solve, cold and warm, for several tolerances: how much a warm
    start saves depends on how far past first feasibility the stopping rule lies."""
    import torch
    from paper_2501_17996_amd import instances as I
    from paper_2501_17996_amd import mcf, warmstart

    torch.cuda.set_device(0)
    inst = I.ring_instance(1000, 10, seed=11)
    prec = mcf.MCF_FP32 if args.precision == "fp32" else mcf.MCF_FP64
    rows = []
    for tol in (1e-2, 1e-3, 1e-4):
        def make(i, tol=tol):
            return mcf.Solver(i, precision=prec, tol=tol, check_every=10, max_iter=200000)
        cold = make(inst).solve()
        rows.append({"tol": tol, "nu": 0.0, "iters": cold["iters"], "state": cold["state_name"]})
        for nu in (0.1, 0.3):
            for keep in (True, False):
                warm, spent = warmstart.warm_started(make, inst, nu, seed=int(nu * 1000), keep_omega=keep)
                st = warm.solve()
                rows.append({"tol": tol, "nu": nu, "keep_omega": keep, "perturbed_iters": spent,
                             "iters": st["iters"], "state": st["state_name"],
                             "saving": 1.0 - st["iters"] / max(1, cold["iters"])})
                warm.close()
                print(json.dumps(rows[-1]), flush=True)
    print(json.dumps({"workload": "warm start, n=1000 ring+chords out-degree 10, log utility",
                      "precision": args.precision, "rows": rows}), flush=True)


def knn_bench(args):
    """The paper's own workload (Section 3.1): q-nearest-neighbour bidirected geometric graphs,
    log utility with log w ~ U[log .3, log 3], log c ~ U[log .5, log 5].  Section 3.1 states the
    accuracy of its solutions as a normalized (per pair) utility within about 0.01 of the
    optimum.  Here each instance runs in blocks of 10 iterations until the certified per-pair gap
    (p - d) / (n (n-1)) is at most 0.01 (p - d bounds the suboptimality of -U, since d is the dual
    function of (e-L) at a feasible dual), and reports that iteration count beside Table 1's, with
    the first feasible iteration, the first with relative gap <= 1e-3, the first within 0.01 per
    pair of the optimum p* of a long FP64 solve (the paper's own measure, against an interior-point
    optimum), and the paper's residual r^k / (n m) against its threshold 0.01 / (n (n-1))."""
    import torch
    from paper_2501_17996_amd import instances as I
    from paper_2501_17996_amd import mcf

    torch.cuda.set_device(0)
    # (n, q): (m, iterations, GPU seconds) of Table 1, or with --table2 of Table 2 (sizes 3000 to
    # 10000, whose long FP64 reference solves are skipped: only the certified gap is reported)
    paper = {(100, 10): (1178, 490, 0.5), (200, 10): (2316, 690, 0.7), (300, 10): (3472, 840, 0.8),
             (500, 10): (5738, 950, 1.1), (500, 20): (11176, 790, 1.4), (1000, 10): (11424, 7220, 19.5),
             (1000, 20): (22286, 1040, 5.1)}
    if args.table2:
        paper = {(3000, 10): (34424, 4140, 96.0), (5000, 10): (57338, 3970, 395.0),
                 (10000, 10): (114054, 4380, 1908.0)}
    prec = mcf.MCF_FP32 if args.precision == "fp32" else mcf.MCF_FP64
    limit = args.iters if args.iters > 0 else 20000
    rows = []
    for (n, q), (pm, pit, pt) in paper.items():
        for seed in range(args.seeds):
            inst = I.knn_geometric(n, q, seed)
            eps = 0.01 / (n * (n - 1))
            S = mcf.Solver(inst, precision=prec, tol=eps, stop_rule=mcf.MCF_STOP_PAPER, check_every=10,
                           max_iter=limit, adapt_until=-1 if args.adapt_until is None else args.adapt_until)
            first = {"feasible": None, "pair_gap_0.01": None, "rel_gap_1e-3": None, "paper_rule": None}
            hist = []
            t0 = time.perf_counter()
            best_r = math.inf
            while True:
                st = S.run(10)
                k, el = st["iters"], time.perf_counter() - t0
                gap = st["primal_obj"] - st["dual_obj"]
                best_r = min(best_r, st["r_paper"])
                hist.append((k, el, st["primal_obj"]))
                hits = {"feasible": st["infeasible_frac"] == 0.0,
                        "pair_gap_0.01": math.isfinite(gap) and gap <= 0.01 * n * (n - 1),
                        "rel_gap_1e-3": st["rel_gap"] <= 1e-3,
                        "paper_rule": st["r_paper"] < eps}
                for key, hit in hits.items():
                    if hit and first[key] is None:
                        first[key] = (k, el)
                if first["pair_gap_0.01"] is not None or k >= limit or st["state_name"] != "running":
                    break
            per_it = el / max(1, k)
            S.close()
            # The optimum p* from a long FP64 solve, with the primal weight frozen after iteration
            # 2000 (Section 2.4): adapted indefinitely, omega drifts down on these instances and the
            # iterate loses feasibility again.  p* - d* bounds the reference's own error.
            if args.table2:
                rst = {"primal_obj": math.nan, "dual_obj": math.nan, "iters": 0, "state_name": "skipped"}
            else:
                R = mcf.Solver(inst, precision=mcf.MCF_FP64, tol=1e-6, check_every=100, max_iter=args.ref_iters,
                               adapt_until=2000)
                rst = R.solve()
                R.close()
            p_star, d_star = rst["primal_obj"], rst["dual_obj"]
            within = None
            if math.isfinite(p_star):
                within = next(((k_, el_) for k_, el_, p_ in hist
                               if math.isfinite(p_) and p_ - p_star <= 0.01 * n * (n - 1)), None)
            rows.append({"n": n, "q": q, "seed": seed, "m": inst.m,
                         **{f"iters_{key}": (v[0] if v else None) for key, v in first.items()},
                         "iters_within_0.01_of_opt": within[0] if within else None,
                         "seconds_within_0.01_of_opt": within[1] if within else None,
                         "seconds_pair_gap_0.01": first["pair_gap_0.01"][1] if first["pair_gap_0.01"] else None,
                         "ms_per_iter": per_it * 1e3, "min_r_over_nm": best_r, "eps": eps,
                         "opt_per_pair": p_star / (n * (n - 1)), "opt_gap_per_pair": (p_star - d_star) / (n * (n - 1)),
                         "opt_iters": rst["iters"], "opt_state": rst["state_name"],
                         "paper_m": pm, "paper_iters": pit, "paper_seconds": pt})
            print(json.dumps(rows[-1]), flush=True)
    print(json.dumps({"workload": "kNN geometric graphs (Section 3.1 recipe) to the paper's stated accuracy",
                      "precision": args.precision, "rows": rows}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c4",
                    help="c4 (default; steps are blocks of iterations of one solve), c2 or c3 (steps are full "
                         "solves), pool, serve, warmstart, knn")
    ap.add_argument("--block", type=int, default=50, help="c4: iterations per step (the last one checked)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--check-every", type=int, default=None,
                    help="residual check interval: default 50 for single solves (a check costs about two "
                         "iterations; a solve overshoots by fewer than K), 20 for the serving loop and the pool")
    ap.add_argument("--cpu-budget", type=float, default=30.0,
                    help="seconds of host time for the oracle's solve legs (they stop earlier once converged)")
    ap.add_argument("--cpu-iters", type=int, default=3, help="c4: oracle iterations timed for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-full-solve", action="store_true", help="c4: skip the time-to-tolerance solve")
    ap.add_argument("--no-extras", action="store_true",
                    help="c4: skip the config2/config3 solves, the pool and the serving legs")
    ap.add_argument("--kernel-mode", type=int, default=0, help="0 auto, 1 two-phase, 2 fused")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 256 MiB device copy first (a counter reference of known size)")
    ap.add_argument("--iters", type=int, default=0,
                    help="c2/c3: run this many iterations per step instead of a full solve")
    ap.add_argument("--requests", type=int, default=2000, help="serving workload: stream length")
    ap.add_argument("--calib", type=int, default=200, help="serving workload: saturated calibration requests")
    ap.add_argument("--load", type=float, default=0.8, help="serving workload: arrival rate / saturated rate")
    ap.add_argument("--slots", type=int, default=64, help="serving workload and pool: pool slots")
    ap.add_argument("--single", type=int, default=50, help="serving workload: FP64 single-instance comparison size")
    ap.add_argument("--serve-budget-gb", type=float, default=16.0)
    ap.add_argument("--serve-max-iter", type=int, default=60000)
    ap.add_argument("--seeds", type=int, default=1, help="knn workload: seeds per size")
    ap.add_argument("--ref-iters", type=int, default=60000, help="knn workload: iteration cap of the FP64 optimum")
    ap.add_argument("--table2", action="store_true", help="knn workload: the sizes of Table 2 (n = 3000 to 10000)")
    ap.add_argument("--adapt-until", type=int, default=None,
                    help="freeze omega from this iteration on (Section 2.4); default: never for the solve "
                         "workloads, 1000 for the serving stream")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU (the single-instance path and the pool); "
                                   "--gpus must be 1"}))
        raise SystemExit(2)

    if args.workload == "warmstart":
        warmstart_bench(args)
        return
    if args.workload == "knn":
        knn_bench(args)
        return
    if args.check_every is None:
        args.check_every = 20 if args.workload in ("serve", "pool") else 50
    if args.workload == "serve":
        if args.adapt_until is None:
            args.adapt_until = 1000
        serve_bench(args)
        return
    if args.adapt_until is None:
        args.adapt_until = -1

    import torch
    from paper_2501_17996_amd import mcf

    torch.cuda.set_device(0)
    if args.copy_calibration:
        # kernels of known size for the counter runs: a 256 MiB fill (writes) and copy (reads and writes)
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "pool":
        print(json.dumps(pool_leg(mcf, torch, args.slots, args.steps, args.check_every)), flush=True)
        return
    inst, tol, desc = workload(args.workload)
    prec = mcf.MCF_FP32 if args.precision == "fp32" else mcf.MCF_FP64
    s = 4 if prec == mcf.MCF_FP32 else 8
    stream = torch.cuda.current_stream()
    blocks = args.workload == "c4"
    K = args.block if blocks else args.check_every
    S = mcf.Solver(inst, precision=prec, tol=tol, check_every=K, max_iter=200000,
                   stream=stream.cuda_stream, kernel_mode=args.kernel_mode, adapt_until=args.adapt_until)

    def step():
        if blocks:
            return S.run(K)          # K more iterations of the running solve, the last one checked
        S.reset()
        return S.run(args.iters) if args.iters > 0 else S.solve()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # a pair of stream events spans each timed step (kernel roofline)
    mcf.mcf_enable_kernel_timing(S.h, True)
    iters = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = step()
        iters += K if blocks else st["iters"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    edge_ms, launches = mcf.mcf_kernel_time(S.h)
    mcf.mcf_enable_kernel_timing(S.h, False)
    n, m = inst.n, inst.m
    fused = S.layout()["kernel_mode"] == "fused"
    # the timed iterations keep the check / regular mix of the whole run
    checks = launches / K
    alg = alg_bytes(n, m, s, fused, False) * (launches - checks) + alg_bytes(n, m, s, fused, True) * checks
    achieved = alg / (edge_ms * 1e-3) / 1e9 if edge_ms > 0 else 0.0
    value = n * m * iters / dt
    out = {
        "metric": "PDHG edge-dest updates/s (n*m*iters/s)",
        "value": value,
        "unit": "edge-dest updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == mcf.MCF_FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "m": m, "precision": args.precision, "adapt_until": args.adapt_until,
                   "reductions": "f64", "check_every": K, "tol": tol,
                   "step": (f"{K} iterations of one solve (the last checked), replayed from the block's graph"
                            if blocks else f"{args.iters} iterations from the cold start" if args.iters > 0
                            else "full solve from the cold start"),
                   "iters_per_step": iters / args.steps, "k_after_timing": st["iters"],
                   "rel_kkt_after_timing": st["rel_kkt"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload) if args.kernel_mode == 0 else None,
                     "alg_bytes_per_launch": alg / max(1, launches),
                     "kernel": "fused iteration" if fused else "edge + node phases (one iteration)",
                     "avg_launch_us": edge_ms * 1e3 / max(1, launches),
                     "launches": launches,
                     "events": "one pair of HIP events on the solver's stream around each timed step: every "
                               "launch of its iterations, the check, residual pass and control included"},
    }
    if not blocks:
        out["config"]["time_to_tol_ms"] = dt / args.steps * 1e3
        out["config"]["final_rel_kkt"] = st["rel_kkt"]
    if blocks and not args.no_full_solve:
        # time to the tolerance: one full solve from the cold start, instance resident in HBM
        print(f"[bench] full solve of {args.workload} to rel KKT {tol:g}", file=sys.stderr, flush=True)
        S.reset()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        fs = S.solve()
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - t1
        out["time_to_tol"] = {"seconds": t_solve, "iters": fs["iters"], "state": fs["state_name"],
                              "rel_kkt": fs["rel_kkt"], "primal_obj": fs["primal_obj"], "tol": tol,
                              "check_every": K, "edge_dest_updates_per_s": n * m * fs["iters"] / t_solve}
    S.close()
    p_c2 = None
    if blocks and not args.no_extras:
        print("[bench] config2 / config3 solves, pool, serving", file=sys.stderr, flush=True)
        extras = {"c2": timed_solves(mcf, torch, "c2", 5, 50), "c3": timed_solves(mcf, torch, "c3", 3, 50)}
        gold = os.path.join(ROOT, "tests", "golden", "oracle_c3_golden.json")
        if os.path.exists(gold):
            p_ref = json.load(open(gold))["solve"]["primal_obj"]
            extras["c3"]["fp64_oracle_objective"] = p_ref
            extras["c3"]["fp64_oracle_objective_relerr"] = (abs(extras["c3"]["primal_obj"] - p_ref)
                                                             / max(1.0, abs(p_ref)))
        extras["pool"] = pool_leg(mcf, torch, args.slots, 20, 20)
        sargs = argparse.Namespace(**vars(args))
        sargs.requests, sargs.calib, sargs.single, sargs.check_every = 300, 64, 20, 20
        sargs.adapt_until = 1000
        extras["serving"] = serve_run(sargs)
        out["extras"] = extras
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        if blocks:
            threads = max(1, min(16, os.cpu_count() or 1))
            med, times = cpu_baseline_iterations(inst, args.cpu_iters, threads)
            out["cpu_baseline"] = {
                "value": n * m / med, "unit": "edge-dest updates/s", "cores": threads, "kind": "oracle",
                "sample": f"median of {args.cpu_iters} FP64 PDHG iterations of the same instance from the cold "
                          f"start (edge and node phases, no check) on {threads} threads of {cpu_model()}: "
                          + ", ".join(f"{t:.2f}" for t in times) + " s",
                "s_per_iteration": med}
            if "extras" in out:
                cb = cpu_baseline_solve(workload("c2")[0], 1e-4, 50, args.cpu_budget)
                p_c2 = cb.pop("primal_obj")
                # one host thread, per iteration (a config4 iteration takes over a minute on one thread)
                c2 = workload("c2")[0]
                med1, _ = cpu_baseline_iterations(c2, 5, 1)
                cb["one_thread"] = {"value": c2.n * c2.m / med1, "s_per_iteration": med1,
                                    "sample": "median of 5 FP64 iterations from the cold start on 1 thread"}
                out["extras"]["c2"]["cpu_baseline"] = cb
        else:
            cb = cpu_baseline_solve(inst, tol, args.check_every, args.cpu_budget)
            p_c2 = cb.pop("primal_obj")
            out["cpu_baseline"] = cb
        if p_c2 is not None:
            tgt = out["extras"]["c2"] if blocks else out
            gpu_p = tgt["primal_obj"] if blocks else st["primal_obj"]
            if blocks or args.iters == 0:
                # the GPU result against the FP64 oracle at the same KKT tolerance
                tgt["fp64_oracle_objective_relerr"] = abs(gpu_p - p_c2) / max(1.0, abs(p_c2))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
