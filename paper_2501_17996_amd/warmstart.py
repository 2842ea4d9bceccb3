"""Warm start of Section 3.1 ("Warm start"): solve a problem whose utility weights
are perturbed to (1 +/- nu) w, each sign with probability 1/2, only until the
iterate is feasible (every off-diagonal traffic positive), then start the
original problem from that flow, dual and primal weight.  The paper notes that
carrying the primal weight over matters: with omega reset to 1 a warm start
needs about as many iterations as a cold one.
"""
from __future__ import annotations

import numpy as np

from . import instances as I


def perturbed(inst, nu: float, seed: int):
    """A copy of `inst` with w_ij replaced by (1 + nu) w_ij or (1 - nu) w_ij, each with probability 1/2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sign = np.where(rng.random(inst.w.shape[0]) < 0.5, 1.0, -1.0)
    w = inst.w * (1.0 + nu * sign)
    return I.Instance(inst.n, inst.tail, inst.head, inst.cap, inst.utility, inst.gamma, w,
                      name=f"{inst.name}+pert{nu}", seed=seed)


def first_feasible_state(solver, block: int = 10, max_iter: int = 100000):
    """Runs `solver` in blocks of `block` iterations until its checked traffic is positive
    off the diagonal; returns (F, Y, omega, iterations)."""
    while True:
        st = solver.run(block)
        if st["infeasible_frac"] == 0.0 or st["iters"] >= max_iter:
            F, Y, sc = solver.get_state()
            return F, Y, sc["omega"], st["iters"]


def warm_started(make_solver, inst, nu: float, seed: int, keep_omega: bool = True, block: int = 10):
    """Returns (warm solver positioned at the warm start, iterations spent on the perturbed
    problem).  `make_solver(instance)` builds an mcf.Solver."""
    pert = make_solver(perturbed(inst, nu, seed))
    F, Y, omega, spent = first_feasible_state(pert, block=block)
    pert.close()
    warm = make_solver(inst)
    warm.set_state(F, Y, k=0, omega=omega if keep_omega else 1.0)
    return warm, spent
