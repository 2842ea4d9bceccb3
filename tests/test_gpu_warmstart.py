"""Warm start of Section 3.1 through mcf_set_state."""
import sys

import numpy as np
import pytest

from paper_2501_17996_amd import instances as I

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu-case] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield


def test_warm_start_from_perturbed_problem_is_faster():
    from paper_2501_17996_amd import mcf, warmstart
    inst = I.config2(4)

    def make(i):
        return mcf.Solver(i, precision=mcf.MCF_FP32, tol=1e-4, check_every=10, max_iter=100000)

    cold = make(inst).solve()
    warm, spent = warmstart.warm_started(make, inst, 0.1, seed=3)
    assert 0 < spent < cold["iters"]
    st = warm.solve()
    print(f"cold {cold['iters']} iterations; warm {st['iters']} after {spent} on the perturbed problem")
    assert st["state_name"] == "converged"
    assert st["iters"] < cold["iters"]
    assert st["primal_obj"] == pytest.approx(cold["primal_obj"], rel=1e-4)


def test_restart_from_converged_state_converges_at_first_check():
    from paper_2501_17996_amd import mcf
    inst = I.config1(2)
    S = mcf.Solver(inst, precision=mcf.MCF_FP64, tol=1e-6)
    st = S.solve()
    F, Y, sc = S.get_state()
    T = mcf.Solver(inst, precision=mcf.MCF_FP64, tol=1e-6)
    T.set_state(F, Y, k=0, omega=sc["omega"])
    st2 = T.solve()
    assert st2["state_name"] == "converged" and st2["iters"] <= 5
    assert st2["primal_obj"] == pytest.approx(st["primal_obj"], rel=1e-7)
