"""Serving-loop bookkeeping on a CPU stand-in backend: admission by slots and
memory footprint, continuous batching, retirement, latency percentiles."""
import numpy as np

from paper_2501_17996_amd import instances as I
from paper_2501_17996_amd.serve import Arena, Request, percentile, serve
from tests.fake_backend import OracleBackend


def test_arena_first_fit_and_coalescing():
    a = Arena(4096)
    x = a.alloc(1000)
    y = a.alloc(1000)
    z = a.alloc(1000)
    assert x == (0, 1024) and y == (1024, 1024) and z == (2048, 1024)
    assert a.alloc(2000) is None
    a.release(*y)
    assert a.alloc(2000) is None          # fragmented: 1024 + 1024 not adjacent
    a.release(*x)
    assert a.alloc(2000) == (0, 2048)     # x and y coalesced
    a.release(0, 2048)
    a.release(*z)
    assert a.free == [(0, 4096)]


def test_percentile():
    xs = list(range(1, 101))
    assert percentile(xs, 50) == 50.5
    assert percentile(xs, 99) == 99.01
    assert np.isnan(percentile([], 50))


def _stream(count, seed=3):
    rng = np.random.default_rng(seed)
    reqs, t = [], 0.0
    for r in range(count):
        t += rng.exponential(0.002)
        n = int(rng.integers(8, 24))
        inst = I.ring_instance(n, int(rng.integers(3, 6)), seed=100 + r,
                               utility=int(rng.integers(0, 2)), gamma=0.5)
        reqs.append(Request(r, t, inst))
    return reqs


def test_serving_loop_admission_and_completion():
    reqs = _stream(24)
    biggest = max(r.inst.n * r.inst.m * 32 for r in reqs)
    be = OracleBackend(budget=3 * biggest, max_slots=4, check_every=10, tol=1e-4)
    records, summary = serve(reqs, be)
    assert summary["requests"] == 24 and summary["converged"] == 24
    assert be.peak_slots <= 4
    assert be.peak_bytes <= 3 * biggest
    assert be.arena.free == [(0, be.arena.size)]     # every block returned
    assert sorted(r.rid for r in records) == list(range(24))
    for r in records:
        assert r.arrival <= r.admitted <= r.done
        assert r.iters % 10 == 0 and r.rel_kkt <= 1e-4
    assert summary["latency_p50_s"] <= summary["latency_p99_s"]
    assert summary["service_p50_s"] <= summary["latency_p99_s"]


def test_serving_results_do_not_depend_on_the_mix():
    """Each request gets the same result whatever else is batched with it."""
    out = {}
    for slots in (1, 5):
        reqs = _stream(10, seed=5)      # the loop releases each instance once it is served
        be = OracleBackend(budget=1 << 40, max_slots=slots, check_every=10, tol=1e-5)
        records, _ = serve(reqs, be)
        out[slots] = {r.rid: (r.iters, r.primal_obj) for r in records}
    assert out[1] == out[5]
