"""Batching pool on the GPU: every instance gets the same result alone and in
a mix (bitwise, the work of one instance never depends on another), continuous
batching reproduces it, it agrees with the single-instance solver, and
admission respects slots and the HBM budget."""
import sys

import numpy as np
import pytest

from paper_2501_17996_amd import instances as I

pytestmark = pytest.mark.gpu

K = 20


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
