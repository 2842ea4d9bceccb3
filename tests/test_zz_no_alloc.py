"""The entry point that allocates nothing (mcf_solve_static, a static device workspace per GPU)
against the handle API on the same instances: the same kernels in the same order, so the same
bits.  Three calls in a row, each smaller than the one before (two-phase n = 600, fused n = 200,
n = 10), so every call runs on what the previous one left in the static array."""
import sys

import numpy as np
import pytest

from paper_2501_17996_amd import instances as I

pytestmark = pytest.mark.gpu


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


def _cases():
    return [(I.ring_instance(600, 4, seed=61), 1e-4), (I.config2(0), 1e-4), (I.config1(0), 1e-6)]


@pytest.mark.parametrize("precision", [0, 1])
def test_static_solve_equals_handle_solve(M, precision):
    for inst, tol in _cases():
        need = M.mcf_workspace_bytes(inst.n, inst.m, precision)
        assert need <= M.MCF_STATIC_BYTES
        o = M.mcf_options_default()
        o.precision, o.tol, o.check_every, o.max_iter = precision, tol, 10, 40000
        F, T, Y, st = M.mcf_solve_static(inst.n, inst.tail, inst.head, inst.cap, inst.utility, inst.gamma, inst.w, o)
        S = M.Solver(inst, precision=precision, tol=tol, check_every=10, max_iter=40000)
        sr = S.solve()
        Fr, Tr, Yr = S.solution()
        S.close()
        print(f"static n={inst.n} prec {precision}: {st['state_name']} at {st['iters']}, "
              f"handle {sr['state_name']} at {sr['iters']}", flush=True)
        assert st["state_name"] == sr["state_name"] == "converged"
        assert st["iters"] == sr["iters"]
        for key in ("primal_obj", "dual_obj", "rel_kkt", "omega", "infeasible_frac"):
            assert st[key] == sr[key], key
        np.testing.assert_array_equal(F, Fr)
        np.testing.assert_array_equal(T, Tr)
        np.testing.assert_array_equal(Y, Yr)


def test_static_solve_refuses_what_does_not_fit(M):
    inst = I.config3(0)
    assert M.mcf_workspace_bytes(inst.n, inst.m, 1) > M.MCF_STATIC_BYTES
    o = M.mcf_options_default()
    o.precision = 1
    with pytest.raises(M.MCFError) as ei:
        M.mcf_solve_static(inst.n, inst.tail, inst.head, inst.cap, inst.utility, inst.gamma, inst.w, o)
    assert ei.value.code == M.MCF_E_ARG
