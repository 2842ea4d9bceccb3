"""Seeded synthetic MCF instances.

This module only draws problem data (graph, capacities, utility weights).  It
holds none of the solver's arithmetic, so the CPU oracle and the HIP path can
both take their inputs from here without sharing any of the method.

Conventions (Section 1.1 of the paper, "Network" and "Traffic matrix"):

* edge ``l`` goes from ``tail[l]`` to ``head[l]``; the incidence matrix has
  ``A[head[l], l] = +1`` and ``A[tail[l], l] = -1``;
* ``w`` is a flat ``n*n`` float64 array with ``w[j*n + i]`` the weight of the
  traffic that starts at node ``j`` and ends at node ``i`` (the utility of the
  entry ``T_ij``).  The diagonal is unused and set to zero.

All draws come from ``numpy.random.Generator(PCG64(seed))`` in a fixed order:
topology, then capacities, then weights.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

UTIL_LOG = 0
UTIL_POWER = 1
UTIL_ALPHA = 2   # alpha-fair: u(s) = w s^(1-alpha) / (1-alpha), alpha > 0, alpha != 1


@dataclass
class Instance:
    n: int
    tail: np.ndarray          # int32[m]
    head: np.ndarray          # int32[m]
    cap: np.ndarray           # float64[m]
    utility: int              # UTIL_LOG, UTIL_POWER or UTIL_ALPHA
    gamma: float              # gamma of the power utility, alpha of the alpha-fair one (ignored for log)
    w: np.ndarray             # float64[n*n], w[j*n+i]
    name: str = ""
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.tail.shape[0])

    @property
    def nm(self) -> int:
        return self.n * self.m


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _ring(n: int):
    t = np.arange(n, dtype=np.int64)
    return t, (t + 1) % n


def ring_plus_random_chords(n: int, n_chords: int, rng) -> tuple[np.ndarray, np.ndarray]:
    """Directed ring i -> i+1 (mod n), then ``n_chords`` distinct chords drawn
    uniformly among ordered pairs that are neither self-loops nor ring edges."""
    rt, rh = _ring(n)
    used = set(zip(rt.tolist(), rh.tolist()))
    if n_chords > n * (n - 1) - n:
        raise ValueError("too many chords for this n")
    ct, ch = [], []
    while len(ct) < n_chords:
        u = int(rng.integers(0, n))
        v = int(rng.integers(0, n))
        if u == v or (u, v) in used:
            continue
        used.add((u, v))
        ct.append(u)
        ch.append(v)
    tail = np.concatenate([rt, np.asarray(ct, dtype=np.int64)])
    head = np.concatenate([rh, np.asarray(ch, dtype=np.int64)])
    return tail.astype(np.int32), head.astype(np.int32)


def ring_plus_outdegree(n: int, deg: int, rng) -> tuple[np.ndarray, np.ndarray]:
    """Directed ring plus, for every node u, ``deg-1`` chord targets drawn
    without replacement from all nodes except u and u+1: out-degree ``deg``."""
    if not (1 <= deg <= n - 1):
        raise ValueError("out-degree must be in [1, n-1]")
    rt, rh = _ring(n)
    k = deg - 1
    ct = np.empty(n * k, dtype=np.int64)
    ch = np.empty(n * k, dtype=np.int64)
    for u in range(n):
        x = rng.choice(n - 2, size=k, replace=False).astype(np.int64) if k else np.empty(0, np.int64)
        a, b = sorted((u, (u + 1) % n))
        x = x + (x >= a)
        x = x + (x >= b)
        ct[u * k:(u + 1) * k] = u
        ch[u * k:(u + 1) * k] = x
    tail = np.concatenate([rt, ct]).astype(np.int32)
    head = np.concatenate([rh, ch]).astype(np.int32)
    return tail, head


def _weights(n: int, lo: float, hi: float, rng) -> np.ndarray:
    w = rng.uniform(lo, hi, size=(n, n))
    np.fill_diagonal(w, 0.0)
    return np.ascontiguousarray(w).reshape(-1)


def config1(seed: int = 0) -> Instance:
    """n=10, ring + 30 random chords (m=40), c ~ U[0.5,1.5], log utility, w ~ U[0.5,1.5]."""
    rng = _rng(seed)
    n = 10
    tail, head = ring_plus_random_chords(n, 30, rng)
    cap = rng.uniform(0.5, 1.5, size=tail.shape[0])
    w = _weights(n, 0.5, 1.5, rng)
    return Instance(n, tail, head, cap, UTIL_LOG, 0.0, w, name="ring10+30chords/log", seed=seed)


def config2(seed: int = 0) -> Instance:
    """n=200, ring + chords to out-degree 10 (m=2000), c ~ U[0.5,2], log utility, w ~ U[0.5,1.5]."""
    rng = _rng(seed)
    n = 200
    tail, head = ring_plus_outdegree(n, 10, rng)
    cap = rng.uniform(0.5, 2.0, size=tail.shape[0])
    w = _weights(n, 0.5, 1.5, rng)
    return Instance(n, tail, head, cap, UTIL_LOG, 0.0, w, name="ring200-deg10/log", seed=seed)


def config3(seed: int = 0) -> Instance:
    """n=1000, out-degree 10 (m=1e4), c ~ lognormal(0,0.5), power utility w*s^0.5, w ~ U[0.5,1.5]."""
    rng = _rng(seed)
    n = 1000
    tail, head = ring_plus_outdegree(n, 10, rng)
    cap = rng.lognormal(0.0, 0.5, size=tail.shape[0])
    w = _weights(n, 0.5, 1.5, rng)
    return Instance(n, tail, head, cap, UTIL_POWER, 0.5, w, name="ring1000-deg10/power0.5", seed=seed)


def config4(seed: int = 0) -> Instance:
    """n=1e4, out-degree 10 (m=1e5), c ~ U[0.5,2], log utility, w ~ U[0.5,1.5]."""
    rng = _rng(seed)
    n = 10000
    tail, head = ring_plus_outdegree(n, 10, rng)
    cap = rng.uniform(0.5, 2.0, size=tail.shape[0])
    w = _weights(n, 0.5, 1.5, rng)
    return Instance(n, tail, head, cap, UTIL_LOG, 0.0, w, name="ring10000-deg10/log", seed=seed)


def ring_instance(n: int, deg: int, seed: int, utility: int = UTIL_LOG, gamma: float = 0.5,
                  cap_range=(0.5, 2.0), w_range=(0.5, 1.5)) -> Instance:
    """Generic ring + out-degree instance (the shape of the serving requests)."""
    rng = _rng(seed)
    tail, head = ring_plus_outdegree(n, deg, rng)
    cap = rng.uniform(cap_range[0], cap_range[1], size=tail.shape[0])
    w = _weights(n, w_range[0], w_range[1], rng)
    g = gamma if utility in (UTIL_POWER, UTIL_ALPHA) else 0.0
    return Instance(n, tail, head, cap, utility, g, w, name=f"ring{n}-deg{deg}", seed=seed)


def serving_request(r: int) -> Instance:
    """Request ``r`` of the serving stream: seed 1000+r, n ~ U{20..500},
    out-degree ~ U{4..16}, log or power(0.5) utility with probability 1/2 each,
    c ~ U[0.5,2], w ~ U[0.5,1.5]."""
    seed = 1000 + r
    rng = _rng(seed)
    n = int(rng.integers(20, 501))
    deg = int(rng.integers(4, 17))
    utility = UTIL_LOG if rng.random() < 0.5 else UTIL_POWER
    tail, head = ring_plus_outdegree(n, deg, rng)
    cap = rng.uniform(0.5, 2.0, size=tail.shape[0])
    w = _weights(n, 0.5, 1.5, rng)
    g = 0.5 if utility == UTIL_POWER else 0.0
    return Instance(n, tail, head, cap, utility, g, w, name=f"req{r}", seed=seed,
                    meta={"request": r, "deg": deg})


def poisson_arrivals(count: int, rate: float, seed: int = 7) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process with the given rate."""
    rng = _rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def knn_geometric(n: int, q: int, seed: int) -> Instance:
    """The paper's experimental workload (Section 3.1, "Data and parameters"):
    n points uniform in the unit square, both directions of an edge between two
    points when either is among the q nearest neighbours of the other,
    log c ~ U[log 0.5, log 5], log utility with log w ~ U[log 0.3, log 3]."""
    rng = _rng(seed)
    xi = rng.uniform(0.0, 1.0, size=(n, 2))
    d2 = ((xi[:, None, :] - xi[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d2, np.inf)
    nbr = np.argsort(d2, axis=1, kind="stable")[:, :q]
    adj = np.zeros((n, n), dtype=bool)
    rows = np.repeat(np.arange(n), q)
    adj[rows, nbr.reshape(-1)] = True
    adj = adj | adj.T
    t, h = np.nonzero(adj)
    cap = np.exp(rng.uniform(np.log(0.5), np.log(5.0), size=t.shape[0]))
    w = np.exp(rng.uniform(np.log(0.3), np.log(3.0), size=(n, n)))
    np.fill_diagonal(w, 0.0)
    return Instance(n, t.astype(np.int32), h.astype(np.int32), cap, UTIL_LOG, 0.0,
                    np.ascontiguousarray(w).reshape(-1), name=f"knn{n}-q{q}", seed=seed)


CONFIGS = {"c1": config1, "c2": config2, "c3": config3, "c4": config4}


def with_parallel_edges(inst: Instance, count: int, seed: int) -> Instance:
    """A copy of `inst` with `count` of its edges duplicated (same tail and head), each copy with
    a capacity of its own drawn from U[0.5, 2]; the copies are appended after the edges of `inst`."""
    rng = _rng(seed)
    pick = rng.choice(inst.m, size=count, replace=False)
    tail = np.concatenate([inst.tail, inst.tail[pick]]).astype(np.int32)
    head = np.concatenate([inst.head, inst.head[pick]]).astype(np.int32)
    cap = np.concatenate([inst.cap, rng.uniform(0.5, 2.0, size=count)])
    return Instance(inst.n, tail, head, cap, inst.utility, inst.gamma, inst.w.copy(),
                    name=f"{inst.name}+par{count}", seed=seed, meta={"parallel_of": pick.tolist()})


def hub_instance(n: int, seed: int, utility: int = UTIL_LOG, gamma: float = 0.5) -> Instance:
    """Ring over nodes 1..n-1 plus a hub, node 0, joined to every other node in both directions:
    the hub has 2(n-1) incident edges (a skewed degree distribution), every other node four."""
    rng = _rng(seed)
    others = np.arange(1, n, dtype=np.int32)
    ring_t = others
    ring_h = np.concatenate([others[1:], others[:1]])
    hub = np.zeros(n - 1, dtype=np.int32)
    tail = np.concatenate([ring_t, hub, others]).astype(np.int32)
    head = np.concatenate([ring_h, others, hub]).astype(np.int32)
    cap = rng.uniform(0.5, 2.0, size=tail.shape[0])
    w = _weights(n, 0.5, 1.5, rng)
    g = gamma if utility in (UTIL_POWER, UTIL_ALPHA) else 0.0
    return Instance(n, tail, head, cap, utility, g, w, name=f"hub{n}", seed=seed)
