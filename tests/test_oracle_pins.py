"""Pins of the CPU oracle against the paper and against mathematics that does
not go through the oracle itself: brute force, closed forms, library solvers,
invariants.  CPU only."""
import itertools
import math

import numpy as np
import pytest
from scipy import optimize

from paper_2501_17996_amd import instances as I
from tests import mathref as R


# ------------------------------------------------------------------ projection
def _project_bruteforce(q, c):
    """Projection onto {x >= 0, 1^T x <= c} by enumerating the support: for each
    candidate support S, solve the KKT system and keep the feasible one.
    (Section 2.3, first proximal operator.)"""
    n = len(q)
    if np.maximum(q, 0).sum() <= c:
        return np.maximum(q, 0), 0.0
    best = None
    for r in range(1, n + 1):
        for S in itertools.combinations(range(n), r):
            S = list(S)
            mu = (q[S].sum() - c) / len(S)
            if mu <= 0:
                continue
            inside = all(q[i] > mu for i in S)
            outside = all(q[i] <= mu for i in range(n) if i not in S)
            if inside and outside:
                x = np.zeros(n)
                x[S] = q[S] - mu
                best = (x, mu)
    assert best is not None
    return best


@pytest.mark.parametrize("seed", range(40))
def test_projection_matches_bruteforce(orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 8))
    q = rng.normal(0, 1, n) * rng.choice([0.1, 1, 5])
    c = float(rng.uniform(0.05, 2.0))
    x, mu = orc.project(q, c)
    xb, mub = _project_bruteforce(q, c)
    np.testing.assert_allclose(x, xb, rtol=1e-12, atol=1e-14)
    assert mu == pytest.approx(mub, rel=1e-12, abs=1e-15)


def test_projection_against_qp_solver(orc):
    """A generic constrained least-squares solve (SLSQP) agrees with the projection."""
    rng = np.random.default_rng(3)
    for _ in range(5):
        q = rng.normal(0, 1, 12)
        c = 0.7
        x, _ = orc.project(q, c)
        res = optimize.minimize(lambda z: 0.5 * np.sum((z - q) ** 2), np.zeros(12), jac=lambda z: z - q,
                                bounds=[(0, None)] * 12,
                                constraints=[{"type": "ineq", "fun": lambda z: c - z.sum(),
                                              "jac": lambda z: -np.ones_like(z)}],
                                method="SLSQP", options={"ftol": 1e-14, "maxiter": 500})
        np.testing.assert_allclose(x, res.x, atol=1e-7)


@pytest.mark.parametrize("n", [1, 2, 17, 200, 1000])
def test_projection_kkt(orc, n):
    rng = np.random.default_rng(n)
    for scale in (0.01, 1.0, 30.0):
        q = rng.normal(0.2, 1.0, n) * scale
        c = 1.3
        x, mu = orc.project(q, c)
        assert (x >= 0).all()
        assert x.sum() <= c * (1 + n * 2.0 ** -52) + 1e-15
        if np.maximum(q, 0).sum() <= c:
            assert mu == 0.0
            np.testing.assert_array_equal(x, np.maximum(q, 0))
        else:
            assert mu > 0
            assert x.sum() == pytest.approx(c, rel=1e-12)
            pos = x > 0
            np.testing.assert_allclose(q[pos] - x[pos], mu, rtol=1e-10, atol=1e-12 * scale)
            assert (q[~pos] <= mu + 1e-12 * scale).all()


def test_projection_special_cases(orc):
    # all nonpositive -> zero, mu = 0
    x, mu = orc.project(np.array([-1.0, -2.0, 0.0]), 1.0)
    assert mu == 0 and (x == 0).all()
    # single entry above capacity -> clipped to c
    x, mu = orc.project(np.array([5.0]), 2.0)
    assert x[0] == pytest.approx(2.0) and mu == pytest.approx(3.0)
    # equal entries: mass shared equally
    x, mu = orc.project(np.full(4, 1.0), 2.0)
    np.testing.assert_allclose(x, 0.5)


# --------------------------------------------------------------- dual proxes
def _prox_conj_by_moreau(y, beta, w, inst_util, gamma):
    """prox_{beta f*}(y) = y - beta prox_{f/beta}(y/beta) (Moreau), with f = -u and
    prox_{f/beta} found by a bounded scalar minimization over s > 0."""
    v = y / beta

    def obj(s):
        if inst_util == 0:
            u = w * math.log(s)
        elif inst_util == 1:
            u = w * s ** gamma
        else:
            u = w * s ** (1.0 - gamma) / (1.0 - gamma)
        return -u / beta + 0.5 * (s - v) ** 2

    hi = 4.0 * (abs(v) + math.sqrt(w / beta) + w / beta) + 10.0   # above the minimizer
    res = optimize.minimize_scalar(obj, bounds=(1e-12, hi), method="bounded",
                                   options={"xatol": 1e-13, "maxiter": 5000})
    return y - beta * res.x


@pytest.mark.parametrize("y", [-5.0, -1.0, -0.01, 0.0, 0.3, 2.0, 40.0])
@pytest.mark.parametrize("beta,w", [(0.2, 1.0), (3.0, 0.6), (0.01, 1.4)])
def test_prox_log(orc, y, beta, w):
    z = orc.prox_log(y, beta, w)
    assert z < 0
    # z is the negative root of z^2 - y z - beta w = 0 (optimality of the prox)
    assert z * z - y * z - beta * w == pytest.approx(0.0, abs=1e-13 * max(1.0, y * y, beta * w))
    # the Moreau route cancels (z = y - beta s*), so its accuracy scales with |y|
    assert z == pytest.approx(_prox_conj_by_moreau(y, beta, w, 0, 0.0), rel=1e-6, abs=1e-8 * max(1.0, abs(y)))


@pytest.mark.parametrize("y", [-5.0, -1.0, -0.01, 0.0, 0.3, 2.0, 40.0])
@pytest.mark.parametrize("beta,w", [(0.2, 1.0), (3.0, 0.6), (0.01, 1.4)])
def test_prox_power_half_cubic(orc, y, beta, w):
    z = orc.prox_power(y, beta, w, 0.5)
    assert z < 0
    # gamma = 1/2: t = -z is the positive root of t^3 + y t^2 - beta w^2 / 4
    roots = np.roots([1.0, y, 0.0, -beta * w * w / 4.0])
    real = [r.real for r in roots if abs(r.imag) < 1e-9 * max(1, abs(r)) and r.real > 0]
    assert len(real) == 1
    assert -z == pytest.approx(real[0], rel=1e-9)
    assert z == pytest.approx(_prox_conj_by_moreau(y, beta, w, 1, 0.5), rel=1e-6, abs=1e-8 * max(1.0, abs(y)))


@pytest.mark.parametrize("gamma", [0.1, 0.2, 0.35, 0.7, 0.9])
@pytest.mark.parametrize("y", [-3.0, -0.1, 0.0, 1.5])
def test_prox_power_general_gamma(orc, gamma, y):
    beta, w = 0.4, 1.2
    z = orc.prox_power(y, beta, w, gamma)
    assert z < 0
    assert z == pytest.approx(_prox_conj_by_moreau(y, beta, w, 1, gamma), rel=1e-6, abs=1e-8 * max(1.0, abs(y)))


# alpha-fair utility u(s) = w s^(1-a)/(1-a): the general strictly concave increasing u of
# Section 1.1, whose scalar prox Section 2.3 leaves to the general case
@pytest.mark.parametrize("y", [-5.0, -1.0, -0.01, 0.0, 0.3, 2.0, 40.0])
@pytest.mark.parametrize("beta,w", [(0.2, 1.0), (3.0, 0.6), (0.01, 1.4)])
def test_prox_alpha_two_cardano(orc, y, beta, w):
    """a = 2 (u = -w/s, traffic s(z) = sqrt(w/-z)): with r = sqrt(-z) the optimality condition
    z + beta s(z) = y is the depressed cubic r^3 + y r - beta sqrt(w) = 0, solved by Cardano's
    formula (one real root when the discriminant is positive, else the largest of three)."""
    z = orc.prox_alpha(y, beta, w, 2.0)
    assert z < 0
    P, Q = y, -beta * math.sqrt(w)
    disc = (Q / 2) ** 2 + (P / 3) ** 3
    if disc >= 0:
        sq = math.sqrt(disc)
        r = float(np.cbrt(-Q / 2 + sq) + np.cbrt(-Q / 2 - sq))
    else:
        r = 2 * math.sqrt(-P / 3) * math.cos(math.acos((3 * Q / (2 * P)) * math.sqrt(-3 / P)) / 3)
    assert -z == pytest.approx(r * r, rel=1e-9)


@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.8])
@pytest.mark.parametrize("y", [-3.0, -0.1, 0.0, 1.5])
def test_prox_alpha_below_one_is_power(orc, alpha, y):
    """For a < 1, w s^(1-a)/(1-a) is the power utility with gamma = 1 - a and weight w/(1-a)."""
    beta, w = 0.4, 1.2
    z = orc.prox_alpha(y, beta, w, alpha)
    assert z == pytest.approx(orc.prox_power(y, beta, w / (1 - alpha), 1 - alpha), rel=1e-12)


@pytest.mark.parametrize("y", [-3.0, -0.1, 0.0, 1.5, 30.0])
def test_prox_alpha_near_one_is_log(orc, y):
    """w s^(1-a)/(1-a) = w/(1-a) + w log s + O(1-a); the constant does not move the prox."""
    for a in (1 - 1e-7, 1 + 1e-7):
        assert orc.prox_alpha(y, 0.4, 1.2, a) == pytest.approx(orc.prox_log(y, 0.4, 1.2), rel=1e-5)


@pytest.mark.parametrize("alpha", [1.5, 2.5, 4.0, 8.0, 16.0])
@pytest.mark.parametrize("y", [-4.0, -0.2, 0.0, 0.7, 25.0])
def test_prox_alpha_general(orc, alpha, y):
    beta, w = 0.3, 0.9
    z = orc.prox_alpha(y, beta, w, alpha)
    assert z < 0
    # optimality: z + beta s(z) = y, s(z) = (w/-z)^(1/a) the traffic that price z asks for
    assert z + beta * (w / -z) ** (1 / alpha) == pytest.approx(y, abs=1e-12 * max(1.0, abs(y)))
    assert z == pytest.approx(_prox_conj_by_moreau(y, beta, w, 2, alpha), rel=1e-6, abs=1e-8 * max(1.0, abs(y)))


# ----------------------------------------------------------------------- eta
@pytest.mark.parametrize("maker", [lambda: I.config1(0), lambda: I.config1(3), lambda: I.config2(1),
                                   lambda: I.knn_geometric(40, 4, 0)])
def test_eta_bound(orc, maker):
    inst = maker()
    A = R.incidence(inst.n, inst.tail, inst.head)
    L = A @ A.T
    eta = orc.eta(inst.n, inst.tail, inst.head)
    dmax = np.max(np.diag(L))
    assert eta == pytest.approx(1.0 / math.sqrt(2 * dmax), rel=1e-15)
    # Appendix A: lambda_max(A A^T) <= 2 d_max, so eta <= 1/||A||_2
    assert np.linalg.eigvalsh(L).max() <= 2 * dmax + 1e-9
    assert eta <= 1.0 / np.linalg.norm(A, 2) + 1e-15


def test_laplacian_structure():
    inst = I.config1(1)
    A = R.incidence(inst.n, inst.tail, inst.head)
    L = A @ A.T
    for i in range(inst.n):
        for j in range(inst.n):
            if i != j:
                cnt = np.sum((inst.tail == i) & (inst.head == j)) + np.sum((inst.tail == j) & (inst.head == i))
                assert L[i, j] == -cnt
