"""Pins of the oracle's PDMCF iteration (Algorithm 2.1) against closed forms,
dense restatements through the incidence matrix, library solvers and
invariants.  CPU only."""
import math

import numpy as np
import pytest
from scipy import optimize
from scipy.sparse import csgraph, csr_matrix

from paper_2501_17996_amd import instances as I
from tests import mathref as R


# the utility parameter each test uses: power gamma = 1/2, alpha-fair alpha = 2
GAMMA = {0: 0.0, 1: 0.5, 2: 2.0}


def _inst(n, tail, head, cap, w_math, utility=0, gamma=0.0, name="tiny"):
    """Build an Instance from a weight matrix given as (i, j) -> w_ij."""
    w = np.ascontiguousarray(np.asarray(w_math, dtype=np.float64).T).reshape(-1)
    return I.Instance(n, np.asarray(tail, np.int32), np.asarray(head, np.int32), np.asarray(cap, np.float64),
                      utility, gamma, w, name=name)


def _state_math(orc_solver, inst):
    F, Y, sc = orc_solver.get_state()
    import oracle
    return oracle.as_math_F(F, inst.n, inst.m), oracle.as_math_sq(Y, inst.n), sc


def _last_math(orc_solver, inst):
    import oracle
    Fh, Th, Q = orc_solver.get_last()
    n, m = inst.n, inst.m
    return oracle.as_math_F(Fh, n, m), oracle.as_math_sq(Th, n), oracle.as_math_F(Q, n, m)


# ----------------------------------------------------- worked first iteration
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_worked_first_iteration(orc, seed):
    """From F^{-1/2} = 0, Y^0 = I - 1 1^T every quantity of iteration 0 has a
    closed form (Section 2.5 initialization with (e-pdhg-step)):
    Y^0 A = A, Q^0 = eta A, Fhat has min(eta, c_l) in row head(l) only, ..."""
    inst = I.config1(seed)
    n, m = inst.n, inst.m
    s = orc.OracleSolver(inst)
    eta = s.eta
    M = s.step(check=True)
    F1, Y1, sc = _state_math(s, inst)
    Fh, Th, Q = _last_math(s, inst)
    A = R.incidence(n, inst.tail, inst.head)
    W = R.weights_matrix(inst)
    mins = np.minimum(eta, inst.cap)
    # (2) Q^0 = eta A
    np.testing.assert_allclose(Q, eta * A, rtol=0, atol=1e-15)
    # (3) Fhat: a single nonzero min(eta, c_l) at row head(l)
    expect = np.zeros((n, m))
    expect[inst.head, np.arange(m)] = mins
    np.testing.assert_allclose(Fh, expect, rtol=1e-15, atol=1e-16)
    # (4) F^{1/2} = 1.9 Fhat
    np.testing.assert_allclose(F1, 1.9 * expect, rtol=1e-15, atol=1e-16)
    # (5)-(7) Yhat^1_ij = prox(-1 + 2 eta sum_{l: j->i} min(eta, c_l)), Y^1 = 1.9 Yhat + 0.9 off-diagonal
    S = np.zeros((n, n))
    for l in range(m):
        S[inst.head[l], inst.tail[l]] += mins[l]
    yarg = -1.0 + 2.0 * eta * S
    yhat = (yarg - np.sqrt(yarg ** 2 + 4 * eta * W)) / 2.0   # quadratic root z^2 - y z - beta w = 0, z < 0
    off = R.offdiag_mask(n)
    np.testing.assert_allclose(Y1[off], (1.9 * yhat + 0.9)[off], rtol=1e-13)
    assert (np.diag(Y1) == 0).all()
    # (8),(9) step norms
    assert M["dF"] == pytest.approx(1.9 * math.sqrt(np.sum(mins ** 2)), rel=1e-14)
    assert M["dY"] == pytest.approx(1.9 * np.linalg.norm((yhat + 1.0)[off]), rel=1e-13)
    # (10) k = 0 is a multiple of k_adapt: omega^1 = (dY/dF)^(1/2) (omega^0)^(1/2)
    assert sc["omega"] == pytest.approx(math.sqrt(M["dY"] / M["dF"]), rel=1e-14)
    assert sc["alpha"] == pytest.approx(eta / sc["omega"], rel=1e-15)
    assert sc["beta"] == pytest.approx(eta * sc["omega"], rel=1e-15)
    # (11) ||D^0||^2 = sum_l eta^2 + (eta - c_l)_+^2
    assert M["e"] == pytest.approx(np.sum(eta ** 2 + np.maximum(eta - inst.cap, 0) ** 2), rel=1e-14)
    # dual objective at Y^0: -sum_{i!=j} (w - w log w) ... with sign: (-u)^*(-1) = -w + w log w
    Wo = W[off]
    d0 = -np.sum(-Wo + Wo * np.log(Wo)) - np.sum(inst.cap)
    assert M["dual_obj"] == pytest.approx(d0, rel=1e-13)
    # (13) T^_{ij} = sum of min(eta,c) over direct edges j->i; infeasible unless every pair has an edge
    np.testing.assert_allclose(Th[off], S[off], rtol=1e-15, atol=1e-16)
    pairs = len(set(zip(inst.tail.tolist(), inst.head.tolist())))
    assert M["infeasible_frac"] == pytest.approx(1 - pairs / (n * (n - 1)))
    assert math.isinf(M["r"]) and math.isinf(M["rel_kkt"])
    # second step: k = 1 is not a multiple of 100, omega is unchanged
    s.step(check=False)
    _, _, sc2 = _state_math(s, inst)
    assert sc2["omega"] == sc["omega"]


# ------------------------------------------------ one step vs dense restatement
def _dense_step(inst, F, Y, alpha, beta, rho=1.9):
    """(e-pdhg-step) written with the dense incidence matrix, a brute-force
    projection and the polynomial/quadratic prox roots."""
    from tests.test_oracle_pins import _project_bruteforce
    n, m = inst.n, inst.m
    A = R.incidence(n, inst.tail, inst.head)
    W = R.weights_matrix(inst)
    Q = F + alpha * (Y @ A)
    Fh = np.zeros_like(Q)
    for l in range(m):
        Fh[:, l] = _project_bruteforce(Q[:, l], inst.cap[l])[0]
    Fb = 2 * Fh - F
    V = Fb @ A.T
    Yh = np.zeros_like(Y)
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            y = Y[i, j] - beta * V[i, j]
            if inst.utility == 0:
                Yh[i, j] = (y - math.sqrt(y * y + 4 * beta * W[i, j])) / 2
            elif inst.utility == 2:
                # alpha = 2: r = sqrt(-z) is the positive root of r^3 + y r - beta sqrt(w)
                assert inst.gamma == 2.0
                roots = np.roots([1.0, 0.0, y, -beta * math.sqrt(W[i, j])])
                r = max(q.real for q in roots if abs(q.imag) < 1e-9)
                Yh[i, j] = -r * r
            else:
                g = inst.gamma
                c1 = g / (1 - g)
                c2 = beta * (1 / g - 1) * (W[i, j] * g) ** (1 / (1 - g))
                assert abs(c1 - 1) < 1e-15
                roots = np.roots([1.0, y, 0.0, -c1 * c2])
                t = max(r.real for r in roots if abs(r.imag) < 1e-9)
                Yh[i, j] = -t
    return rho * Fh + (1 - rho) * F, rho * Yh + (1 - rho) * Y, Fh, Q


@pytest.mark.parametrize("utility", [0, 1, 2])
def test_step_matches_dense_restatement(orc, utility):
    rng = np.random.default_rng(11 + utility)
    n = 4
    tail = [0, 1, 2, 3, 0, 2]
    head = [1, 2, 3, 0, 2, 1]
    cap = rng.uniform(0.5, 1.5, len(tail))
    W = rng.uniform(0.5, 1.5, (n, n))
    np.fill_diagonal(W, 0)
    inst = _inst(n, tail, head, cap, W, utility=utility, gamma=GAMMA[utility])
    import oracle
    s = orc.OracleSolver(inst)
    F = np.abs(rng.normal(0, 0.5, (n, len(tail))))
    Y = -np.abs(rng.normal(1, 0.5, (n, n)))
    np.fill_diagonal(Y, 0)
    omega = 1.7
    s.set_state(F.T.reshape(-1), Y.T.reshape(-1), k=5, omega=omega)
    alpha, beta = s.eta / omega, s.eta * omega
    s.step(check=True)
    F1, Y1, _ = _state_math(s, inst)
    Fh, _, Q = _last_math(s, inst)
    F1d, Y1d, Fhd, Qd = _dense_step(inst, F, Y, alpha, beta)
    np.testing.assert_allclose(Q, Qd, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(Fh, Fhd, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(F1, F1d, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(Y1, Y1d, rtol=1e-10, atol=1e-13)
    # the column primitives give the same as the full step
    fh, fb, fn, mu = oracle.edge_column(F[:, 2], Y[:, head[2]], Y[:, tail[2]], alpha, cap[2], 1.9)
    np.testing.assert_allclose(fn, F1d[:, 2], rtol=1e-12, atol=1e-14)
    Fb = 2 * Fhd - F
    j = 2
    fin = np.stack([Fb[:, l] for l in range(len(tail)) if head[l] == j])
    fout = np.stack([Fb[:, l] for l in range(len(tail)) if tail[l] == j])
    v, yh, yn = oracle.node_column(j, fin, fout, Y[:, j], W[:, j], beta, 1.9, utility, inst.gamma)
    A = R.incidence(n, inst.tail, inst.head)
    np.testing.assert_allclose(v, (Fb @ A.T)[:, j], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(yn, Y1d[:, j], rtol=1e-10, atol=1e-13)


# ------------------------------------------------------------- closed forms
def _solve_tight(orc, inst, tol=1e-9, max_iter=400000):
    s = orc.OracleSolver(inst)
    st = s.solve(tol, max_iter=max_iter)
    assert st == "converged", s.metrics()
    return s


@pytest.mark.parametrize("utility", [0, 1, 2])
def test_cf1_two_nodes(orc, utility):
    """n = 2, e1 = 2->1, e2 = 1->2: each pair has exactly one edge, so the
    optimum fills it: T_12 = c_1, T_21 = c_2, and Y_ij = -u'(T_ij)."""
    c = np.array([0.7, 1.3])
    W = np.array([[0.0, 0.9], [1.2, 0.0]])
    inst = _inst(2, [1, 0], [0, 1], c, W, utility=utility, gamma=GAMMA[utility])
    s = _solve_tight(orc, inst)
    Fh, Th, _ = _last_math(s, inst)
    assert Th[0, 1] == pytest.approx(c[0], rel=1e-7)
    assert Th[1, 0] == pytest.approx(c[1], rel=1e-7)
    np.testing.assert_allclose(Fh, [[c[0], 0], [0, c[1]]], rtol=1e-7, atol=1e-8)
    M = s.metrics()
    assert abs(M["primal_obj"] - M["dual_obj"]) < 1e-6 * (1 + abs(M["primal_obj"]))


@pytest.mark.parametrize("utility,n,gamma", [(0, 5, 0.0), (0, 7, 0.0), (1, 5, 0.5), (1, 6, 0.5), (1, 6, 0.3),
                                             (2, 5, 2.0), (2, 6, 2.0)])
def test_cf2_ring(orc, utility, n, gamma):
    """Directed ring, uniform c and w: with hop distance d = (i - j) mod n,
    log: T_ij = c / ((n-1) d);  power(gamma): T_ij = c d^(-1/(1-gamma)) / sum_d d^(-gamma/(1-gamma)),
    c / (H_{n-1} d^2) at gamma = 1/2;  alpha-fair: T_ij = c d^(-1/a) / sum_d d^(1-1/a)
    (in every case u'(T_d) is proportional to d and sum_d d T_d = c)."""
    c, w = 1.3, 0.8
    tail = np.arange(n)
    head = (tail + 1) % n
    W = np.full((n, n), w)
    np.fill_diagonal(W, 0)
    inst = _inst(n, tail, head, np.full(n, c), W, utility=utility, gamma=gamma)
    s = _solve_tight(orc, inst)
    _, Th, _ = _last_math(s, inst)
    H = sum(1.0 / d for d in range(1, n))
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            d = (i - j) % n
            if utility == 0:
                expect = c / ((n - 1) * d)
            elif utility == 1 and gamma == 0.5:
                expect = c / (H * d * d)
            elif utility == 1:
                expect = c * d ** (-1 / (1 - gamma)) / sum(e ** (-gamma / (1 - gamma)) for e in range(1, n))
            else:
                expect = c * d ** (-1 / gamma) / sum(e ** (1 - 1 / gamma) for e in range(1, n))
            assert Th[i, j] == pytest.approx(expect, rel=1e-6)


def _ring_optimum(n, c, w, utility):
    H = sum(1.0 / d for d in range(1, n))
    if utility == 2:
        a = GAMMA[2]
        S = sum(e ** (1 - 1 / a) for e in range(1, n))
        t = {d: c * d ** (-1 / a) / S for d in range(1, n)}
    else:
        t = {d: (c / ((n - 1) * d) if utility == 0 else c / (H * d * d)) for d in range(1, n)}
    F = np.zeros((n, n))   # edge k is k -> k+1
    for i in range(n):
        for k in range(n):
            D = (i - k) % n
            if D != 0:
                F[i, k] = sum(t[d] for d in range(D, n))
    T = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                T[i, j] = t[(i - j) % n]
    return F, T


@pytest.mark.parametrize("utility", [0, 1, 2])
def test_fixed_point_at_ring_optimum(orc, utility):
    """Started at the optimal (F*, Y*) with Y*_ij = -u'(T*_ij), one PDHG step
    stays there and the residual vanishes (a saddle point is a fixed point)."""
    n, c, w = 6, 1.1, 0.9
    tail = np.arange(n)
    head = (tail + 1) % n
    W = np.full((n, n), w)
    np.fill_diagonal(W, 0)
    inst = _inst(n, tail, head, np.full(n, c), W, utility=utility, gamma=GAMMA[utility])
    F, T = _ring_optimum(n, c, w, utility)
    A = R.incidence(n, tail, head)
    np.testing.assert_allclose(-F @ A.T, T + np.diag(np.diag(-F @ A.T)), atol=1e-14)
    Y = np.zeros((n, n))
    off = R.offdiag_mask(n)
    Y[off] = -R.dutil(inst, T[off], W[off])
    s = orc.OracleSolver(inst)
    s.set_state(F.T.reshape(-1), Y.T.reshape(-1), k=1, omega=1.0)
    M = s.step(check=True)
    # rounding scales with the prices (|Y| is about 20 at alpha = 2, 1-3 for log and power)
    scale = max(1.0, np.abs(Y).max())
    assert M["dF"] < 1e-13 * scale and M["dY"] < 1e-13 * scale
    # (e-res) evaluates r = a - b^2/e, which cancels to rounding level (~1e-16 a)
    assert M["r"] < 1e-13 * max(1.0, M["a"])
    assert M["rel_kkt"] < 1e-6
    assert M["rel_primal"] < 1e-12 and abs(M["rel_gap"]) < 1e-12


@pytest.mark.parametrize("n", [3, 4])
def test_cf3_complete_bidirected(orc, n):
    """Complete bidirected graph with w_ij = kappa c_{j->i}: direct routing at
    full capacity is optimal, T_ij = c_{j->i}."""
    rng = np.random.default_rng(n)
    tail, head = zip(*[(j, i) for i in range(n) for j in range(n) if i != j])
    cap = rng.uniform(0.5, 2.0, len(tail))
    kappa = 0.7
    W = np.zeros((n, n))
    for l, (j, i) in enumerate(zip(tail, head)):
        W[i, j] = kappa * cap[l]
    inst = _inst(n, tail, head, cap, W)
    s = _solve_tight(orc, inst)
    _, Th, _ = _last_math(s, inst)
    for l, (j, i) in enumerate(zip(tail, head)):
        assert Th[i, j] == pytest.approx(cap[l], rel=1e-7)


# ------------------------------------------------- library optimum, tiny cases
def _shortest_path_feasible(n, tail, head, cap):
    """alpha F^sp of Section 1.1 ("Existence and uniqueness"): unit flow from every
    source to every destination on a fewest-edges path, scaled to capacity."""
    m = len(tail)
    G = csr_matrix((np.ones(m), (tail, head)), shape=(n, n))
    _, pred = csgraph.shortest_path(G, unweighted=True, return_predecessors=True)
    eid = {(int(t), int(h)): l for l, (t, h) in enumerate(zip(tail, head))}
    F = np.zeros((n, m))
    for j in range(n):
        for i in range(n):
            if i == j:
                continue
            v = i
            while v != j:
                u = pred[j, v]
                F[i, eid[(int(u), int(v))]] += 1.0
                v = u
    a = 1.0 / np.max(F.sum(0) / cap)
    return a * F


@pytest.mark.parametrize("case", range(6))
def test_optimum_against_slsqp(orc, case):
    rng = np.random.default_rng(100 + case)
    if case in (0, 1, 4):
        n = 3
        tail, head = zip(*[(j, i) for i in range(n) for j in range(n) if i != j])
    else:
        n = 4
        tail, head = [0, 1, 2, 3, 0, 2], [1, 2, 3, 0, 2, 1]
    tail, head = np.array(tail), np.array(head)
    m = len(tail)
    cap = rng.uniform(0.5, 2.0, m)
    W = rng.uniform(0.5, 1.5, (n, n))
    np.fill_diagonal(W, 0)
    utility = case % 2 if case < 4 else 2
    inst = _inst(n, tail, head, cap, W, utility=utility, gamma=GAMMA[utility])
    A = R.incidence(n, tail, head)
    off = R.offdiag_mask(n)

    def negU(x):
        T = -(x.reshape(n, m) @ A.T)
        return -np.sum(R.util(inst, T[off], W[off]))

    def grad(x):
        T = -(x.reshape(n, m) @ A.T)
        Up = np.zeros((n, n))
        Up[off] = R.dutil(inst, T[off], W[off])
        return (Up @ A).reshape(-1)      # d(-U)/dF = U' A

    x0 = _shortest_path_feasible(n, tail, head, cap).reshape(-1)
    # the alpha-fair objective is infinite at T = 0: keep SLSQP's iterates off it (the bound is
    # far below the optimal traffic, so it is inactive at the optimum)
    floor = 1e-3 if utility == 2 else 1e-9
    cons = [{"type": "ineq", "fun": lambda x: cap - x.reshape(n, m).sum(0)},
            {"type": "ineq", "fun": lambda x: (-(x.reshape(n, m) @ A.T))[off] - floor}]
    res = optimize.minimize(negU, x0, jac=grad, bounds=[(0, None)] * (n * m), constraints=cons,
                            method="SLSQP", options={"ftol": 1e-15, "maxiter": 2000})
    assert res.status in (0, 8), res.message  # 8: the line search stalls at rounding level
    Tref = -(res.x.reshape(n, m) @ A.T)
    s = _solve_tight(orc, inst)
    _, Th, _ = _last_math(s, inst)
    np.testing.assert_allclose(Th[off], Tref[off], rtol=2e-4, atol=1e-6)
    assert Tref[off].min() > 10 * floor
    # U* >= U^sp (the shortest-path point is feasible)
    assert -s.metrics()["primal_obj"] >= -negU(x0) - 1e-9


# ------------------------------------------------------ residual and duality
def _conj_numeric(inst, y, w):
    """(-u)^*(y) = sup_s (y s + u(s)) by scalar maximization."""
    f = lambda s: -(y * s + R.util(inst, s, w))
    res = optimize.minimize_scalar(f, bounds=(1e-9, 1e4), method="bounded", options={"xatol": 1e-12})
    return -res.fun


def _support_lp(yacol, c):
    """sup { <g, f> : f >= 0, 1^T f <= c } as a linear program."""
    n = len(yacol)
    res = optimize.linprog(-yacol, A_ub=np.ones((1, n)), b_ub=[c], bounds=[(0, None)] * n, method="highs")
    return -res.fun


@pytest.mark.parametrize("utility", [0, 1, 2])
def test_residual_and_gap_against_definitions(orc, utility):
    """r(Q) of (e-res) against a brute-force minimization over gamma >= 0, with
    G = U'A from dense algebra; the dual objective against numeric conjugates
    and a per-edge LP (the reduced Lagrangian (e-L) minimized over F)."""
    rng = np.random.default_rng(5 + utility)
    n = 4
    tail, head = zip(*[(j, i) for i in range(n) for j in range(n) if i != j])
    tail, head = np.array(tail), np.array(head)
    m = len(tail)
    cap = rng.uniform(0.5, 2.0, m)
    W = rng.uniform(0.5, 1.5, (n, n))
    np.fill_diagonal(W, 0)
    inst = _inst(n, tail, head, cap, W, utility=utility, gamma=GAMMA[utility])
    import oracle
    s = orc.OracleSolver(inst)
    A = R.incidence(n, tail, head)
    off = R.offdiag_mask(n)
    Fstar = np.zeros((n, m))
    Fstar[head, np.arange(m)] = cap
    Q = Fstar + rng.normal(0, 0.3, (n, m))
    Fh = np.stack([oracle.project(Q[:, l], cap[l])[0] for l in range(m)], axis=1)
    Y = -rng.uniform(0.3, 2.0, (n, n))
    np.fill_diagonal(Y, 0)
    M = s.eval_residual(Q.T.reshape(-1), Fh.T.reshape(-1), Y.T.reshape(-1))
    T = -(Fh @ A.T)
    assert (T[off] > 0).all()
    Up = np.zeros((n, n))
    Up[off] = R.dutil(inst, T[off], W[off])
    G = Up @ A
    D = Fh - Q
    assert M["a"] == pytest.approx(np.sum(G * G), rel=1e-12)
    assert M["b"] == pytest.approx(np.sum(G * D), rel=1e-12, abs=1e-12)
    assert M["e"] == pytest.approx(np.sum(D * D), rel=1e-12)
    res = optimize.minimize_scalar(lambda g: np.sum((G - g * D) ** 2), bounds=(0, 1e3), method="bounded",
                                   options={"xatol": 1e-12})
    rb = min(res.fun, np.sum(G * G))
    assert M["r"] == pytest.approx(rb, rel=1e-7, abs=1e-12)
    assert M["rel_dual"] == pytest.approx(math.sqrt(rb / np.sum(G * G)), rel=1e-6, abs=1e-9)
    p = -np.sum(R.util(inst, T[off], W[off]))
    assert M["primal_obj"] == pytest.approx(p, rel=1e-12)
    YA = Y @ A
    d = -sum(_conj_numeric(inst, Y[i, j], W[i, j]) for i in range(n) for j in range(n) if i != j) \
        - sum(_support_lp(YA[:, l], cap[l]) for l in range(m))
    assert M["dual_obj"] == pytest.approx(d, rel=1e-7, abs=1e-8)
    assert M["primal_obj"] >= M["dual_obj"] - 1e-9
    Tdual = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                Tdual[i, j] = optimize.minimize_scalar(
                    lambda s_: -(Y[i, j] * s_ + R.util(inst, s_, W[i, j])), bounds=(1e-9, 1e4),
                    method="bounded", options={"xatol": 1e-12}).x
    relp = np.linalg.norm((Tdual - T)[off]) / np.linalg.norm(T[off])
    assert M["rel_primal"] == pytest.approx(relp, rel=1e-5)
    # an infeasible T gives r = infinity (e-res, third case)
    Fh2 = Fh.copy()
    Fh2[:, :] = 0
    M2 = s.eval_residual(Q.T.reshape(-1), Fh2.T.reshape(-1), Y.T.reshape(-1))
    assert math.isinf(M2["r"]) and math.isinf(M2["rel_kkt"]) and M2["infeasible_frac"] == 1.0


def test_invariants_along_trajectory(orc):
    inst = I.config1(2)
    n, m = inst.n, inst.m
    s = orc.OracleSolver(inst)
    A = R.incidence(n, inst.tail, inst.head)
    for k in range(300):
        M = s.step(check=True)
        Fh, Th, _ = _last_math(s, inst)
        F, Y, _ = _state_math(s, inst)
        assert (Fh >= 0).all()
        assert (Fh.sum(0) <= inst.cap * (1 + n * 2.0 ** -52)).all()
        np.testing.assert_allclose(Th.sum(1), 0.0, atol=1e-12)                 # T 1 = 0
        Td = -(Fh @ A.T)
        np.testing.assert_allclose(Th, Td, atol=1e-13)                          # T + F A^T = 0
        assert (np.diag(Y) == 0).all()
        if math.isfinite(M["primal_obj"]) and math.isfinite(M["dual_obj"]):
            assert M["primal_obj"] - M["dual_obj"] >= -1e-9 * (1 + abs(M["primal_obj"]))


def test_stop_rules_and_states(orc):
    inst = I.config1(0)
    s = orc.OracleSolver(inst)
    assert s.solve(1e-6, max_iter=5) == "max_iter"
    assert s.metrics()["k"] == 5
    # the paper's rule r^k < n m eps
    s2 = orc.OracleSolver(inst)
    eps = 0.01 / (inst.n * (inst.n - 1))
    assert s2.solve(eps, stop_rule=1, max_iter=100000) == "converged"
    M = s2.metrics()
    assert M["r"] < inst.n * inst.m * eps
    # one iteration earlier the rule did not hold
    s3 = orc.OracleSolver(inst)
    s3.run(int(M["k"]) - 1)
    assert not (s3.metrics()["r"] < inst.n * inst.m * eps)
    # a NaN planted in F is reported as divergence
    s4 = orc.OracleSolver(inst)
    s4.run(3)
    s4.poison("F", 7)
    assert s4.solve(1e-6, max_iter=100) == "diverged"


def test_check_interval_does_not_change_trajectory(orc):
    inst = I.config1(1)
    a, b = orc.OracleSolver(inst), orc.OracleSolver(inst)
    a.run(137, check=True)
    b.run(137, check=False)
    Fa, Ya, sa = a.get_state()
    Fb, Yb, sb = b.get_state()
    np.testing.assert_array_equal(Fa, Fb)
    np.testing.assert_array_equal(Ya, Yb)
    assert sa == sb


def test_threads_do_not_change_results(orc):
    inst = I.config2(0)
    a, b = orc.OracleSolver(inst, threads=1), orc.OracleSolver(inst, threads=4)
    a.run(20)
    b.run(20)
    Fa, Ya, _ = a.get_state()
    Fb, Yb, _ = b.get_state()
    np.testing.assert_array_equal(Fa, Fb)
    np.testing.assert_array_equal(Ya, Yb)
    assert a.metrics() == b.metrics() or all(
        (x == y) or (math.isnan(x) and math.isnan(y)) for x, y in zip(a.metrics().values(), b.metrics().values()))


def test_adapt_period_and_threshold(orc):
    """Algorithm 2.1 step 3: omega changes only after iterations k that are
    multiples of k_adapt, and only when both step norms exceed tau."""
    inst = I.config1(0)
    s = orc.OracleSolver(inst, k_adapt=3)
    omegas = [s.step(check=False)["omega"] for _ in range(8)]
    changed = [k for k in range(1, 8) if omegas[k] != omegas[k - 1]]
    assert omegas[0] != 1.0 and changed == [3, 6]
    frozen = orc.OracleSolver(inst, tau=1e9)
    assert all(frozen.step(check=False)["omega"] == 1.0 for _ in range(5))
    # the freeze of Section 2.4: no change at or after adapt_until
    fz = orc.OracleSolver(inst, k_adapt=3, adapt_until=6)
    om = [fz.step(check=False)["omega"] for _ in range(12)]
    assert [k for k in range(1, 12) if om[k] != om[k - 1]] == [3]


def test_paper_parameters_golden(orc):
    """Defaults equal the values the paper prints (tests/golden/paper_parameters.json)."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")))
    inst = I.config1(0)
    s = orc.OracleSolver(inst)          # defaults of the binding
    M = s.step(check=False)
    a = orc.OracleSolver(inst, rho=g["rho"]["value"], theta=g["theta"]["value"], tau=g["tau"]["value"],
                         omega0=g["omega0"]["value"], k_adapt=g["k_adapt"]["value"])
    Ma = a.step(check=False)
    assert all(x == y or (math.isnan(x) and math.isnan(y)) for x, y in zip(Ma.values(), M.values()))


def test_trajectory_regression_golden(orc):
    """The C1 seed-0 trajectory written by tests/golden/make_golden.py (oracle only)."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_c1_trajectory.json")))
    s = orc.OracleSolver(I.config1(0))
    rows = {r["k"]: r for r in g["rows"]}
    for k in range(1, max(rows) + 1):
        M = s.step(check=True)
        if k in rows:
            for key in ("omega", "dF", "dY", "rel_kkt", "infeasible_frac"):
                exp = rows[k][key]
                if exp is None:
                    assert not math.isfinite(M[key])
                else:
                    assert M[key] == pytest.approx(exp, rel=1e-12, abs=1e-300)


# ------------------------------------------------------------- parallel edges
def test_parallel_edges_equal_merged_capacity(orc):
    """Two parallel edges with capacities c1, c2 carry exactly the flows one edge of capacity
    c1 + c2 could (the projection acts per column, the constraint sets add), so the optimal
    traffic of (e-prob), which is unique, must be the same for both graphs.  The two runs have
    different incidence matrices, d_max and eta, hence different trajectories."""
    base = I.ring_instance(8, 3, seed=21)
    dup = I.with_parallel_edges(base, 6, seed=4)
    picks = dup.meta["parallel_of"]
    merged_cap = base.cap.copy()
    for q, l in enumerate(picks):
        merged_cap[l] += dup.cap[base.m + q]
    merged = I.Instance(base.n, base.tail, base.head, merged_cap, base.utility, base.gamma, base.w,
                        name="merged")
    out = []
    for inst in (dup, merged):
        s = orc.OracleSolver(inst)
        assert s.solve(1e-9, max_iter=200000, check_every=10) == "converged"
        _, T, _ = _last_math(s, inst)
        out.append((T, s.metrics()["primal_obj"]))
    np.testing.assert_allclose(out[0][0], out[1][0], rtol=1e-6, atol=1e-8)
    assert out[0][1] == pytest.approx(out[1][1], rel=1e-9)


# ------------------------------------------- adaptive primal weight away from 1
@pytest.mark.parametrize("theta,omega0", [(0.5, 1.0), (0.3, 1.0), (0.3, 3.0)])
def test_primal_weight_update_away_from_one(orc, theta, omega0):
    """(e-primal_weight) at iterations where omega^k != 1: omega^{k+1} =
    (Delta_Y / Delta_F)^theta (omega^k)^(1 - theta), with the step norms
    Delta_F = ||F^{k+1/2} - F^{k-1/2}||_F and Delta_Y = ||Y^{k+1} - Y^k||_F formed here
    from the states read before and after the step (Section 2.4), and alpha = eta/omega,
    beta = eta omega with eta = 1/sqrt(2 d_max) from the degrees (e-eta).  The runs pass
    k = 100 and k = 200, so omega^k is the one an earlier adaptation left, away from 1 (and with
    omega^0 = 3 also at k = 0): dropping the (omega^k)^(1 - theta) factor, or using the wrong
    exponent, fails here."""
    inst = I.config1(0)
    n = inst.n
    deg = np.bincount(inst.tail, minlength=n) + np.bincount(inst.head, minlength=n)
    eta = 1.0 / math.sqrt(2.0 * deg.max())
    s = orc.OracleSolver(inst, theta=theta, k_adapt=100, omega0=omega0)
    checked = 0
    for k in range(0, 201):
        F0, Y0, sc0 = s.get_state()
        assert sc0["k"] == k
        s.step(check=False)
        F1, Y1, sc1 = s.get_state()
        dF = float(np.linalg.norm(F1 - F0))
        dY = float(np.linalg.norm(Y1 - Y0))
        if k % 100 == 0:
            assert dF > 1e-5 and dY > 1e-5
            want = (dY / dF) ** theta * sc0["omega"] ** (1.0 - theta)
            assert sc1["omega"] == pytest.approx(want, rel=1e-12)
            if k > 0 or omega0 != 1.0:
                # the pin only bites where omega^k is away from 1 and the new value differs from
                # both (dY/dF)^theta and the theta = 1/2 update by far more than the tolerance
                assert abs(math.log(sc0["omega"])) > 0.01
                assert abs(sc1["omega"] / (dY / dF) ** theta - 1.0) > 1e-3
                if theta != 0.5:
                    assert abs(sc1["omega"] / math.sqrt(dY / dF * sc0["omega"]) - 1.0) > 1e-3
                checked += 1
        else:
            assert sc1["omega"] == sc0["omega"]
        assert sc1["alpha"] == pytest.approx(eta / sc1["omega"], rel=1e-15)
        assert sc1["beta"] == pytest.approx(eta * sc1["omega"], rel=1e-15)
    assert checked == (3 if omega0 != 1.0 else 2)


# --------------------------------------------- relative KKT from its three parts
def _kkt_parts_by_definition(inst, Q, Fh, Y):
    """p, d, rel_primal, rel_dual and rel_gap of a (Q, Fhat, Y) triple from dense algebra,
    scalar minimizations and per-edge LPs: none of them from the oracle."""
    n, m = inst.n, inst.m
    A = R.incidence(n, inst.tail, inst.head)
    W = R.weights_matrix(inst)
    off = R.offdiag_mask(n)
    T = -(Fh @ A.T)
    assert (T[off] > 0).all()
    Up = np.zeros((n, n))
    Up[off] = R.dutil(inst, T[off], W[off])
    G = Up @ A
    D = Fh - Q
    res = optimize.minimize_scalar(lambda g: np.sum((G - g * D) ** 2), bounds=(0, 1e4), method="bounded",
                                   options={"xatol": 1e-13})
    r = min(res.fun, np.sum(G * G))
    reld = math.sqrt(max(r, 0.0) / np.sum(G * G))
    p = -np.sum(R.util(inst, T[off], W[off]))
    YA = Y @ A
    d = -sum(_conj_numeric(inst, Y[i, j], W[i, j]) for i in range(n) for j in range(n) if i != j) \
        - sum(_support_lp(YA[:, l], inst.cap[l]) for l in range(m))
    Tdual = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                Tdual[i, j] = optimize.minimize_scalar(
                    lambda s_: -(Y[i, j] * s_ + R.util(inst, s_, W[i, j])), bounds=(1e-9, 1e4),
                    method="bounded", options={"xatol": 1e-13}).x
    relp = np.linalg.norm((Tdual - T)[off]) / np.linalg.norm(T[off])
    relg = (p - d) / (1.0 + abs(p) + abs(d))
    return {"p": p, "d": d, "rel_primal": relp, "rel_dual": reld, "rel_gap": relg, "Up": Up, "G": G}


def test_relative_kkt_composition(orc):
    """The relative KKT residual (the reading of the configurations' tolerances):
    rel_gap = (p - d)/(1 + |p| + |d|) and rel_kkt = max(rel_primal, rel_dual, rel_gap), each
    part computed here by definition.  Three triples make each part the strict maximum in
    turn, so a rel_kkt that leaves a part out fails one of them; a fourth with one
    off-diagonal Y_ij >= 0 (outside the conjugates' domain) must give rel_kkt = +inf."""
    rng = np.random.default_rng(41)
    n = 4
    tail, head = zip(*[(j, i) for i in range(n) for j in range(n) if i != j])
    tail, head = np.array(tail), np.array(head)
    m = len(tail)
    cap = rng.uniform(0.5, 2.0, m)
    W = rng.uniform(0.5, 1.5, (n, n))
    np.fill_diagonal(W, 0)
    inst = _inst(n, tail, head, cap, W)
    import oracle
    s = orc.OracleSolver(inst)
    # a feasible projected flow with T > 0 off the diagonal
    Q0 = np.zeros((n, m))
    Q0[head, np.arange(m)] = cap
    Q0 += rng.normal(0, 0.2, (n, m))
    Fh = np.stack([oracle.project(Q0[:, l], cap[l])[0] for l in range(m)], axis=1)
    A = R.incidence(n, tail, head)
    T = -(Fh @ A.T)
    off = R.offdiag_mask(n)
    Ystar = np.zeros((n, n))
    Ystar[off] = -R.dutil(inst, T[off], W[off])        # prices that ask for exactly T: rel_primal = 0
    base = _kkt_parts_by_definition(inst, Fh, Fh, Ystar)
    G = base["G"]
    cases = {
        # D = 0: r = ||G||^2, rel_dual = 1 > rel_gap, rel_primal = 0
        "rel_dual": (Fh, Ystar),
        # prices a tenth of those asking for T: T(Y) = 10 T, rel_primal = 9
        "rel_primal": (Q0, Ystar / 10.0),
        # D parallel to G: r = 0, rel_dual = 0; rel_primal = 0; only the support gap is left
        "rel_gap": (Fh - 0.05 * G, Ystar),
    }
    flat = lambda X: np.ascontiguousarray(X.T).reshape(-1)
    for want, (Q, Y) in cases.items():
        ref = _kkt_parts_by_definition(inst, Q, Fh, Y)
        M = s.eval_residual(flat(Q), flat(Fh), flat(Y))
        parts = {k: ref[k] for k in ("rel_primal", "rel_dual", "rel_gap")}
        top = max(parts, key=parts.get)
        assert top == want, (want, parts)
        others = sorted(parts.values())
        assert others[-1] > 1.5 * others[-2] + 1e-6, (want, parts)
        assert M["primal_obj"] == pytest.approx(ref["p"], rel=1e-12)
        assert M["dual_obj"] == pytest.approx(ref["d"], rel=1e-7)
        assert M["rel_gap"] == pytest.approx(ref["rel_gap"], rel=1e-6, abs=1e-9)
        assert M["rel_primal"] == pytest.approx(ref["rel_primal"], rel=1e-5, abs=1e-7)
        assert M["rel_dual"] == pytest.approx(ref["rel_dual"], rel=1e-5, abs=1e-6)
        assert M["rel_kkt"] == pytest.approx(max(parts.values()), rel=1e-5, abs=1e-6)
    # one off-diagonal price >= 0: the dual function is -inf, the gap and rel_kkt +inf,
    # while T stays feasible (r finite)
    for bad in (0.0, 0.25):
        Y = Ystar.copy()
        Y[2, 1] = bad
        M = s.eval_residual(flat(Q0), flat(Fh), flat(Y))
        assert math.isfinite(M["r"]) and M["infeasible_frac"] == 0.0
        assert M["dual_obj"] == -math.inf
        assert math.isinf(M["rel_gap"]) and math.isinf(M["rel_kkt"])
