"""Batching pool on the GPU: every instance gets the same result alone and in
a mix (bitwise, the work of one instance never depends on another), continuous
batching reproduces it, it agrees with the single-instance solver, and
admission respects slots and the HBM budget."""
import math
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2501_17996_amd import instances as I
from tests.test_gpu_parity import assert_infeasible_count_exact

pytestmark = pytest.mark.gpu

K = 20
THREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def M():
    from paper_2501_17996_amd import mcf
    mcf.lib()
    return mcf


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu-case] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield


def _mix():
    """Uneven instances: n from 12 to 500, out-degree 3 to 12, log and power utilities."""
    spec = [(12, 3, 0), (70, 5, 1), (150, 8, 0), (260, 6, 1), (400, 6, 0), (500, 12, 1), (33, 4, 1), (128, 7, 0)]
    return [I.ring_instance(n, d, seed=40 + q, utility=u, gamma=0.5) for q, (n, d, u) in enumerate(spec)]


def _drain(M, pool, handles, slots, limit=4000):
    """Steps the pool until every slot is done; returns {slot: (status, F, Y, T)} at retirement."""
    out = {}
    live = dict(zip(slots, handles))
    steps = 0
    while live and steps < limit:
        pool.step(K)
        pool.sync()
        steps += 1
        for sl in list(live):
            st = pool.poll(sl)
            if st["state_name"] != "running":
                pool.retire(sl)
                h = live.pop(sl)
                F, Y, _ = h.get_state()
                _, T, _ = h.solution()
                out[sl] = (st, F, Y, T)
    assert not live, "pool did not finish"
    return out


def _solver(M, inst, precision, tol):
    return M.Solver(inst, precision=precision, tol=tol, check_every=K, max_iter=60000)


@pytest.mark.parametrize("precision", [1, 0])
def test_pool_alone_equals_mix_bitwise(M, precision):
    insts = _mix()
    tol = 1e-4
    alone = []
    for inst in insts:
        pool = M.Pool(precision, max_slots=1, check_every=K)
        h = _solver(M, inst, precision, tol)
        sl = pool.admit(h)
        alone.append(_drain(M, pool, [h], [sl])[sl])
        pool.close()
    pool = M.Pool(precision, max_slots=len(insts), check_every=K)
    hs = [_solver(M, inst, precision, tol) for inst in insts]
    sls = [pool.admit(h) for h in hs]
    mix = _drain(M, pool, hs, sls)
    for q, sl in enumerate(sls):
        a, b = alone[q], mix[sl]
        assert a[0]["state_name"] == b[0]["state_name"]
        assert a[0]["iters"] == b[0]["iters"]
        np.testing.assert_array_equal(a[1], b[1])
        np.testing.assert_array_equal(a[2], b[2])
        np.testing.assert_array_equal(a[3], b[3])
        print(f"instance {q}: n={insts[q].n} iters {a[0]['iters']} rel_kkt {a[0]['rel_kkt']:.2e}", flush=True)


def test_continuous_batching_equals_alone(M):
    """Three slots for eight requests: each later request enters a slot freed by a
    converged one while the others keep iterating."""
    insts = _mix()
    tol = 1e-4
    ref = {}
    for q, inst in enumerate(insts):
        pool = M.Pool(1, max_slots=1, check_every=K)
        h = _solver(M, inst, 1, tol)
        sl = pool.admit(h)
        ref[q] = _drain(M, pool, [h], [sl])[sl]
        pool.close()
    pool = M.Pool(1, max_slots=3, check_every=K)
    queue = list(range(len(insts)))
    live = {}
    done = {}
    admitted_late = 0
    while queue or live:
        while queue and len(live) < 3:
            q = queue.pop(0)
            h = _solver(M, insts[q], 1, tol)
            live[pool.admit(h)] = (q, h)
            admitted_late += pool.info()["iterations"] > 0
        pool.step(K)
        pool.sync()
        for sl in list(live):
            st = pool.poll(sl)
            if st["state_name"] != "running":
                pool.retire(sl)
                q, h = live.pop(sl)
                F, Y, _ = h.get_state()
                done[q] = (st, F, Y)
    assert admitted_late >= len(insts) - 3
    for q in range(len(insts)):
        assert done[q][0]["iters"] == ref[q][0]["iters"]
        np.testing.assert_array_equal(done[q][1], ref[q][1])
        np.testing.assert_array_equal(done[q][2], ref[q][2])


def test_pool_agrees_with_single_instance_solver(M):
    """The pool (8 waves per node) and the single-instance fused iteration (16 waves)
    add the same terms in different orders: same iterations, objectives within 1e-9."""
    insts = _mix()[:4]
    pool = M.Pool(0, max_slots=4, check_every=K)
    hs = [_solver(M, inst, 0, 1e-5) for inst in insts]
    sls = [pool.admit(h) for h in hs]
    res = _drain(M, pool, hs, sls)
    for q, inst in enumerate(insts):
        st = _solver(M, inst, 0, 1e-5).solve()
        pst = res[sls[q]][0]
        assert abs(pst["iters"] - st["iters"]) <= K
        assert pst["primal_obj"] == pytest.approx(st["primal_obj"], rel=1e-9)


def test_pool_alpha_fair_alone_equals_mix_and_single(M):
    """An alpha-fair instance (alpha = 2) in the pool: bitwise the same alone and beside log and
    power instances, and the single-instance solver's objective (FP64, 1e-9)."""
    a = I.ring_instance(90, 5, seed=77, utility=I.UTIL_ALPHA, gamma=2.0)
    insts = [a] + _mix()[:3]
    tol = 1e-4
    pool = M.Pool(0, max_slots=1, check_every=K)
    h = _solver(M, a, 0, tol)
    sl = pool.admit(h)
    alone = _drain(M, pool, [h], [sl])[sl]
    pool.close()
    pool = M.Pool(0, max_slots=len(insts), check_every=K)
    hs = [_solver(M, inst, 0, tol) for inst in insts]
    sls = [pool.admit(h) for h in hs]
    mix = _drain(M, pool, hs, sls)[sls[0]]
    assert alone[0]["state_name"] == mix[0]["state_name"] == "converged"
    assert alone[0]["iters"] == mix[0]["iters"]
    for x, y in zip(alone[1:], mix[1:]):
        np.testing.assert_array_equal(x, y)
    st = _solver(M, a, 0, tol).solve()
    assert abs(st["iters"] - alone[0]["iters"]) <= K
    assert alone[0]["primal_obj"] == pytest.approx(st["primal_obj"], rel=1e-9)
    print(f"alpha-fair in the pool: iters {alone[0]['iters']} single {st['iters']}", flush=True)


def test_pool_fp32_objective_matches_fp64(M):
    insts = _mix()
    out = {}
    for precision in (0, 1):
        pool = M.Pool(precision, max_slots=len(insts), check_every=K)
        hs = [_solver(M, inst, precision, 1e-4) for inst in insts]
        sls = [pool.admit(h) for h in hs]
        res = _drain(M, pool, hs, sls)
        out[precision] = [res[sl][0] for sl in sls]
    for a, b in zip(out[0], out[1]):
        rel = abs(a["primal_obj"] - b["primal_obj"]) / max(1.0, abs(a["primal_obj"]))
        assert rel <= 1e-5, (a["primal_obj"], b["primal_obj"])


def test_pool_admission_limits(M):
    insts = _mix()
    small = _solver(M, insts[0], 1, 1e-4)
    big = _solver(M, insts[5], 1, 1e-4)
    fp = M.mcf_workspace_bytes(insts[0].n, insts[0].m, 1)
    pool = M.Pool(1, hbm_budget=fp + 1024, max_slots=2, check_every=K)
    pool.admit(small)
    with pytest.raises(M.MCFError) as ei:
        pool.admit(big)                       # over the budget
    assert ei.value.code == M.MCF_E_NOMEM
    with pytest.raises(M.MCFError) as ei:
        pool.admit(small)                     # already admitted
    assert ei.value.code == M.MCF_E_ARG
    with pytest.raises(M.MCFError) as ei:
        small.solve()                         # pooled handles answer only status
    assert ei.value.code == M.MCF_E_STATE
    other = _solver(M, insts[1], 0, 1e-4)     # other precision
    with pytest.raises(M.MCFError) as ei:
        pool.admit(other)
    assert ei.value.code == M.MCF_E_ARG
    info = pool.info()
    assert info["active"] == 1 and info["used_bytes"] == fp
    pool.close()
    small.solve()                             # a standalone handle again after the pool is gone


def test_pool_max_iter_and_slot_reuse(M):
    inst = _mix()[2]
    pool = M.Pool(1, max_slots=1, check_every=K)
    h = M.Solver(inst, precision=1, tol=1e-12, check_every=K, max_iter=3 * K)
    sl = pool.admit(h)
    for _ in range(5):
        pool.step(K)
        pool.sync()
    st = pool.poll(sl)
    assert st["state_name"] == "max_iter" and st["iters"] == 3 * K
    pool.retire(sl)
    h2 = _solver(M, _mix()[0], 1, 1e-4)
    assert pool.admit(h2) == sl
    res = _drain(M, pool, [h2], [sl])
    assert res[sl][0]["state_name"] == "converged"


def _relerr(a, b):
    scale = max(float(np.max(np.abs(b))), 1e-300)
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) / scale


def test_pool_fp64_matches_oracle_at_checkpoints(M):
    """The eight-instance mix in one FP64 pool against the oracle: at pool checkpoints
    k = 20, 100 and 200 every instance's F^{k-1/2}, Y^k and omega match the oracle's to 1e-10
    relative, and so do the metrics of the check that ends the step (objectives, gap,
    residuals; the infeasible count exactly).  At each checkpoint the instances are retired,
    read and admitted again, which must continue the same trajectories."""
    insts = _mix()
    pool = M.Pool(0, max_slots=len(insts), check_every=K)
    hs = [_solver(M, inst, 0, 1e-13) for inst in insts]     # nothing stops before k = 200
    live = {pool.admit(h): q for q, h in enumerate(hs)}
    orcs = [oracle.OracleSolver(inst, threads=THREADS) for inst in insts]
    done = 0
    for k in (20, 100, 200):
        while done < k:
            pool.step(K)
            pool.sync()
            done += K
        recs = {q: pool.poll(sl) for sl, q in live.items()}
        for sl in list(live):
            pool.retire(sl)
        for q, inst in enumerate(insts):
            O = orcs[q]
            kk = int(O.get_state()[2]["k"])
            O.run(k - kk - 1, check=False)
            mo = O.step(check=True)
            Fg, Yg, sg = hs[q].get_state()
            Fo, Yo, so = O.get_state()
            assert sg["k"] == so["k"] == k
            ef, ey = _relerr(Fg, Fo), _relerr(Yg, Yo)
            assert ef <= 1e-10 and ey <= 1e-10, (q, k, ef, ey)
            assert sg["omega"] == pytest.approx(so["omega"], rel=1e-10)
            g = recs[q]
            assert g["iters"] == k and g["checked"] == 1
            for key in ("primal_obj", "dual_obj"):
                if math.isfinite(mo[key]):
                    assert g[key] == pytest.approx(mo[key], rel=1e-10, abs=1e-12), (q, k, key)
                else:
                    assert g[key] == mo[key]
            assert_infeasible_count_exact(g, mo, hs[q], O, what=f"pool instance {q} k {k}")
            if math.isfinite(mo["rel_kkt"]):
                assert abs(g["rel_kkt"] ** 2 - mo["rel_kkt"] ** 2) <= 1e-8 * mo["rel_kkt"] ** 2 + 1e-14
            print(f"pool vs oracle: instance {q} n={inst.n} k={k} F {ef:.1e} Y {ey:.1e}", flush=True)
        live = {pool.admit(h): q for q, h in enumerate(hs)}
    pool.close()


@pytest.mark.parametrize("step,waves", [(K, 8), (7, 8), (K, 4), (7, 2), (7, 1)])
def test_pool_graphs_equal_direct_launches(M, step, waves):
    """Steps replayed from captured graphs (keyed by the step length and the iterations where
    some instance adapts omega) give bitwise the results of launching every kernel directly.
    Steps of 7 iterations put the adaptations at several offsets within a step; instances
    admitted at different pool iterations shift them further."""
    insts = _mix()
    out = []
    for graphs in (1, 0):
        pool = M.Pool(1, max_slots=len(insts), check_every=step, waves=waves, graphs=graphs)
        assert pool.shape()["waves"] == waves
        hs = [M.Solver(inst, precision=1, tol=1e-4, check_every=step, max_iter=60000) for inst in insts]
        live, res, queue = {}, {}, list(range(len(insts)))
        while queue or live:
            if queue:                        # one admission per step: different G0 for each
                q = queue.pop(0)
                live[pool.admit(hs[q])] = q
            pool.step(step)
            pool.sync()
            for sl in list(live):
                st = pool.poll(sl)
                if st["state_name"] != "running":
                    pool.retire(sl)
                    q = live.pop(sl)
                    F, Y, _ = hs[q].get_state()
                    res[q] = (st["iters"], st["primal_obj"], F, Y)
        out.append(res)
        pool.close()
    for q in range(len(insts)):
        a, b = out[0][q], out[1][q]
        assert a[0] == b[0] and a[1] == b[1]
        np.testing.assert_array_equal(a[2], b[2])
        np.testing.assert_array_equal(a[3], b[3])


@pytest.mark.parametrize("small", [4, 2, 1])
def test_pool_fewer_waves_alone_equals_mix(M, small):
    """The 4-, 2- and 1-wave node workgroups (FP32): alone and in the mix bitwise, and the same
    solution as the 8-wave shape up to the order of its sums."""
    insts = _mix()
    res = {}
    for waves in (small, 8):
        pool = M.Pool(1, max_slots=len(insts), check_every=K, waves=waves)
        hs = [_solver(M, inst, 1, 1e-4) for inst in insts]
        sls = [pool.admit(h) for h in hs]
        mix = _drain(M, pool, hs, sls)
        res[waves] = [mix[sl] for sl in sls]
        pool.close()
    for q in (0, 5):
        pool = M.Pool(1, max_slots=1, check_every=K, waves=small)
        h = _solver(M, insts[q], 1, 1e-4)
        sl = pool.admit(h)
        alone = _drain(M, pool, [h], [sl])[sl]
        pool.close()
        assert alone[0]["iters"] == res[small][q][0]["iters"]
        np.testing.assert_array_equal(alone[1], res[small][q][1])
        np.testing.assert_array_equal(alone[2], res[small][q][2])
    for a, b in zip(res[small], res[8]):
        assert a[0]["state_name"] == b[0]["state_name"] == "converged"
        rel = abs(a[0]["primal_obj"] - b[0]["primal_obj"]) / max(1.0, abs(b[0]["primal_obj"]))
        assert rel <= 1e-5


def test_pool_n_max_limits_admission_and_shape(M):
    pool = M.Pool(1, max_slots=2, check_every=K, n_max=128)
    assert pool.shape()["max_ept"] == 2
    big = _solver(M, _mix()[2], 1, 1e-4)         # n = 150
    with pytest.raises(M.MCFError) as ei:
        pool.admit(big)
    assert ei.value.code == M.MCF_E_ARG
    small = _solver(M, _mix()[1], 1, 1e-4)       # n = 70
    sl = pool.admit(small)
    res = _drain(M, pool, [small], [sl])
    assert res[sl][0]["state_name"] == "converged"


def test_serve_loop_on_the_gpu_equals_alone(M):
    """serve() through the GPU backend: twelve requests of the serving stream on three slots,
    admitted as slots free up, each in the organisation the pool gives its size.  Each request's
    result equals that instance run alone in a one-slot pool of the same shape (iterations and
    objective exactly), and every arena block is returned."""
    from paper_2501_17996_amd.serve import GpuBackend, Request, serve
    reqs = [I.serving_request(r) for r in range(12)]
    budget = 3 * max(M.mcf_workspace_bytes(i.n, i.m, 1) for i in reqs) + (1 << 20)
    be = GpuBackend(M.MCF_FP32, budget, 3, K, 1e-4, max_iter=60000, adapt_until=1000)
    stream = [Request(r, 0.002 * r, reqs[r]) for r in range(12)]
    records, summary = serve(stream, be)
    assert summary["requests"] == 12 and summary["rejected"] == 0
    assert be.arena.free == [(0, be.arena.size)]
    be.close()
    for rec in records:
        inst = I.serving_request(rec.rid)
        pool = M.Pool(1, max_slots=1, check_every=K)
        h = M.Solver(inst, tol=1e-4, check_every=K, max_iter=60000, adapt_until=1000,
                     **pool.instance_options(inst.n))    # the organisation serve() gives it
        sl = pool.admit(h)
        st = _drain(M, pool, [h], [sl], limit=4000)[sl][0]
        pool.close()
        assert rec.state == st["state_name"] == "converged"
        assert rec.iters == st["iters"] and rec.primal_obj == st["primal_obj"], rec.rid
    print(f"serve on the GPU: {summary['requests']} requests, p50 {summary['latency_p50_s']:.3f} s", flush=True)


def test_pool_graph_cache_eviction(M):
    """Steps of every length from 1 to 40 make more step shapes than the graph cache holds: the
    least recently used graphs are dropped and captured again, and the results stay bitwise
    those of direct launches."""
    insts = _mix()[:3]
    out = []
    for graphs in (1, 0):
        pool = M.Pool(1, max_slots=3, check_every=K, graphs=graphs)
        hs = [M.Solver(inst, precision=1, tol=1e-12, check_every=K, max_iter=10 ** 6) for inst in insts]
        sls = [pool.admit(h) for h in hs]
        for rep in range(2):
            for L in range(1, 41):
                pool.step(L)
                pool.sync()
        for sl in sls:
            pool.retire(sl)
        out.append([h.get_state()[:2] for h in hs])
        pool.close()
    for (Fa, Ya), (Fb, Yb) in zip(out[0], out[1]):
        np.testing.assert_array_equal(Fa, Fb)
        np.testing.assert_array_equal(Ya, Yb)


def test_slow_instance_in_the_pool_tracks_the_oracle(M):
    """The ring of 400 nodes with out-degree 4 (log utility, seed 44) does not reach rel_kkt 1e-4
    with omega adapted throughout: in the FP64 oracle omega rises to about 9500, falls back near
    300 (rel_kkt 3e-3 at iteration 9000), then drifts down to 9e-5 by iteration 65000 while the
    dual residual stays at rel_kkt 0.024 -- the drift of the adaptive primal weight seen on the
    paper's kNN instances.  With omega frozen from iteration 1000 (Section 2.4) the oracle
    converges at iteration 13000.  An earlier pool test that required every instance of its mix
    to converge within 60000 iterations failed on this one.  Here the FP64 pool and the oracle
    agree on its first 1000 iterations (state to 1e-10, omega, rel_kkt), both still far from the
    tolerance: the behaviour is the method's on this instance, not the pool's."""
    inst = I.ring_instance(400, 4, seed=44, utility=0, gamma=0.5)
    pool = M.Pool(0, max_slots=1, check_every=K)
    h = M.Solver(inst, precision=0, tol=1e-4, check_every=K, max_iter=60000)
    sl = pool.admit(h)
    for _ in range(1000 // K):
        pool.step(K)
        pool.sync()
    st = pool.poll(sl)
    pool.retire(sl)
    O = oracle.OracleSolver(inst, threads=THREADS)
    O.run(999, check=False)
    mo = O.step(check=True)
    Fg, Yg, sg = h.get_state()
    Fo, Yo, so = O.get_state()
    assert sg["k"] == so["k"] == 1000 and st["iters"] == 1000
    assert _relerr(Fg, Fo) <= 1e-10 and _relerr(Yg, Yo) <= 1e-10
    assert sg["omega"] == pytest.approx(so["omega"], rel=1e-10)
    assert abs(st["rel_kkt"] ** 2 - mo["rel_kkt"] ** 2) <= 1e-8 * mo["rel_kkt"] ** 2 + 1e-14
    assert st["rel_kkt"] > 1e-2 and mo["rel_kkt"] > 1e-2
    print(f"slow instance at k=1000: rel_kkt {st['rel_kkt']:.3e} (oracle {mo['rel_kkt']:.3e}), "
          f"omega {sg['omega']:.4g}", flush=True)


def _two_phase_kw(M, n, precision):
    """The two-phase form the pool runs: flat edge phase with the fewest vectors per lane that hold
    n, 64-thread node blocks."""
    vec = 4 if precision == 1 else 2
    nv = 1 if n <= 64 * vec else 2 if n <= 128 * vec else 4
    return dict(kernel_mode=M.MCF_KERNELS_TWO_PHASE, edge_waves=-1, edge_vectors=nv, node_block=64)


def _mixed_solvers(M, insts, precision, tol, max_iter=60000):
    """Even-indexed instances in the two-phase iteration, odd ones fused."""
    return [M.Solver(inst, precision=precision, tol=tol, check_every=K, max_iter=max_iter,
                     **(_two_phase_kw(M, inst.n, precision) if q % 2 == 0 else {}))
            for q, inst in enumerate(insts)]


def test_pool_two_phase_slots_match_oracle(M):
    """Two-phase instances in the pool (flat edge items, then node items, each launch covering
    every two-phase slot) beside fused ones, FP64: at pool checkpoints k = 20, 100 and 200 each
    instance's F, Y and omega match the oracle's to 1e-10 and its check metrics match too."""
    insts = _mix()
    pool = M.Pool(0, max_slots=len(insts), check_every=K)
    hs = _mixed_solvers(M, insts, 0, 1e-13)
    assert [h.layout()["kernel_mode"] for h in hs[:2]] == ["two_phase", "fused"]
    live = {pool.admit(h): q for q, h in enumerate(hs)}
    orcs = [oracle.OracleSolver(inst, threads=THREADS) for inst in insts]
    done = 0
    for k in (20, 100, 200):
        while done < k:
            pool.step(K)
            pool.sync()
            done += K
        recs = {q: pool.poll(sl) for sl, q in live.items()}
        for sl in list(live):
            pool.retire(sl)
        for q, inst in enumerate(insts):
            O = orcs[q]
            O.run(k - int(O.get_state()[2]["k"]) - 1, check=False)
            mo = O.step(check=True)
            Fg, Yg, sg = hs[q].get_state()
            Fo, Yo, so = O.get_state()
            assert sg["k"] == so["k"] == k
            ef, ey = _relerr(Fg, Fo), _relerr(Yg, Yo)
            assert ef <= 1e-10 and ey <= 1e-10, (q, k, ef, ey)
            assert sg["omega"] == pytest.approx(so["omega"], rel=1e-10)
            g = recs[q]
            for key in ("primal_obj", "dual_obj"):
                if math.isfinite(mo[key]):
                    assert g[key] == pytest.approx(mo[key], rel=1e-10, abs=1e-12), (q, k, key)
                else:
                    assert g[key] == mo[key]
            assert_infeasible_count_exact(g, mo, hs[q], O, what=f"pool instance {q} k {k}")
        live = {pool.admit(h): q for q, h in enumerate(hs)}
    pool.close()


@pytest.mark.parametrize("graphs", [1, 0])
def test_pool_mixed_organisations_alone_equals_mix(M, graphs):
    """FP32: each instance gives bitwise the same result alone in a one-slot pool and in the mix of
    both organisations, with steps replayed from graphs or launched directly."""
    insts = _mix()
    pool = M.Pool(1, max_slots=len(insts), check_every=K, graphs=graphs)
    hs = _mixed_solvers(M, insts, 1, 1e-4)
    sls = [pool.admit(h) for h in hs]
    mix = _drain(M, pool, hs, sls)
    pool.close()
    for q in (0, 2, 5):
        pool = M.Pool(1, max_slots=1, check_every=K, graphs=1)
        h = _mixed_solvers(M, [insts[q]] * (q % 2 + 1), 1, 1e-4)[q % 2]
        sl = pool.admit(h)
        alone = _drain(M, pool, [h], [sl])[sl]
        pool.close()
        b = mix[sls[q]]
        assert alone[0]["state_name"] == b[0]["state_name"] == "converged"
        assert alone[0]["iters"] == b[0]["iters"]
        for x, y in zip(alone[1:], b[1:]):
            np.testing.assert_array_equal(x, y)


def test_pool_two_phase_admission(M):
    """A two-phase instance is admitted only in the form the pool runs; instance_options gives it."""
    pool = M.Pool(1, max_slots=2, check_every=K)
    inst = _mix()[2]                                        # n = 150
    other = M.Solver(inst, precision=1, tol=1e-4, kernel_mode=M.MCF_KERNELS_TWO_PHASE, edge_waves=1,
                     edge_vectors=1, node_block=64)         # the concurrent edge phase
    with pytest.raises(M.MCFError) as ei:
        pool.admit(other)
    assert ei.value.code == M.MCF_E_ARG
    kw = pool.instance_options(inst.n)
    assert kw["precision"] == 1 and kw["kernel_mode"] in (M.MCF_KERNELS_FUSED, M.MCF_KERNELS_TWO_PHASE)
    pool.admit(M.Solver(inst, tol=1e-4, **kw))
    pool.admit(M.Solver(inst, precision=1, tol=1e-4, **_two_phase_kw(M, inst.n, 1)))
    with pytest.raises(M.MCFError):
        pool.instance_options(600)


def test_pool_edge_list_growth_keeps_graphs_valid(M):
    """Two-phase slots admitted one at a time, with a step between admissions, so that the pool's
    list of flat edge items grows while graphs of earlier steps are cached (the first growth keeps
    the same launch grid, so the same step key comes back): the graphs captured before a growth
    are dropped with the old list, and every instance's result equals that of the same sequence
    launched without graphs."""
    insts = [_mix()[q] for q in (0, 2, 4)]                  # n = 12, 150, 400: 5, 150, 300 edge items

    def run(graphs):
        pool = M.Pool(1, max_slots=3, check_every=K, graphs=graphs)
        hs = [M.Solver(inst, precision=1, tol=1e-4, check_every=K, max_iter=60000, **_two_phase_kw(M, inst.n, 1))
              for inst in insts]
        sls = []
        for h in hs:
            sls.append(pool.admit(h))
            pool.step(K)
            pool.sync()
        out = _drain(M, pool, hs, sls)
        pool.close()
        return [out[sl] for sl in sls]

    with_graphs, direct = run(1), run(0)
    for q, (x, y) in enumerate(zip(with_graphs, direct)):
        assert x[0]["state_name"] == y[0]["state_name"] == "converged", q
        assert x[0]["iters"] == y[0]["iters"], q
        for u, v in zip(x[1:], y[1:]):
            np.testing.assert_array_equal(u, v)
