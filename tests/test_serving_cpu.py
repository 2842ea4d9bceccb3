"""Serving-loop bookkeeping on a CPU stand-in backend: admission by slots and
memory footprint, continuous batching, retirement, latency percentiles."""
import numpy as np
from hypothesis import given, settings
from hypothesis import strategies as hst

from paper_2501_17996_amd import instances as I
from paper_2501_17996_amd.serve import ALIGN, Arena, Request, percentile, serve
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


def test_requests_that_cannot_be_served_are_rejected_not_waited_on():
    """A request larger than the whole arena, one the backend cannot batch, and one whose
    admission fails each get a record in state "rejected"; the loop serves the rest and
    returns (it must not wait forever on the head of the queue), and every arena block and
    handle is released."""
    reqs = _stream(12, seed=9)
    sizes = [r.inst.n for r in reqs]
    big = I.ring_instance(60, 4, seed=77)
    huge = Request(100, 0.0005, big)                       # footprint above the arena
    odd = Request(101, 0.001, I.ring_instance(30, 3, seed=78))   # refused by accepts()
    bad = Request(102, 0.0015, I.ring_instance(29, 3, seed=79))  # admit() raises
    budget = 4 * max(r.inst.n * r.inst.m * 32 for r in reqs)
    assert big.n * big.m * 32 > budget
    be = OracleBackend(budget=budget, max_slots=3, check_every=10, tol=1e-4, max_n=max(sizes),
                       refuse_admit={29})
    assert 29 not in sizes and 30 > max(sizes)
    records, summary = serve(reqs + [huge, odd, bad], be)
    by = {r.rid: r for r in records}
    for rid in (100, 101, 102):
        assert by[rid].state == "rejected" and "reason" in by[rid].extra
    assert summary["rejected"] == 3 and summary["requests"] == 12 and summary["converged"] == 12
    assert be.arena.free == [(0, be.arena.size)] and be.live == 0


def test_serving_loop_keeps_one_step_in_flight_while_host_works():
    """Handles of queued requests are created while a step is in flight, and finished
    instances are destroyed after the next step is enqueued."""
    events = []

    class Traced(OracleBackend):
        in_flight = False

        def step(self):
            assert not self.in_flight
            self.in_flight = True
            events.append("step")
            super().step()

        def sync(self):
            self.in_flight = False
            events.append("sync")

        def create(self, inst):
            h = super().create(inst)
            if h is not None:
                events.append("create:busy" if self.in_flight else "create:idle")
            return h

        def destroy(self, h):
            events.append("destroy:busy" if self.in_flight else "destroy:idle")
            super().destroy(h)

    reqs = [Request(r, 0.0, I.ring_instance(10, 3, seed=200 + r)) for r in range(8)]
    be = Traced(budget=1 << 30, max_slots=2, check_every=10, tol=1e-4)
    records, summary = serve(reqs, be)
    assert summary["requests"] == 8
    creates = [e for e in events if e.startswith("create")]
    destroys = [e for e in events if e.startswith("destroy")]
    # the first two handles are built before any step; every later one during a step
    assert creates[:2] == ["create:idle", "create:idle"] and set(creates[2:]) == {"create:busy"}
    # every destroy but those after the last step overlaps a step
    assert destroys.count("destroy:busy") >= len(destroys) - 2


@settings(max_examples=30, deadline=None)
@given(sizes=hst.lists(hst.tuples(hst.integers(3, 12), hst.floats(0.0, 0.005)), min_size=1, max_size=10),
       slots=hst.integers(1, 4), budget=hst.integers(1500, 30000), refuse=hst.sets(hst.integers(3, 12), max_size=2),
       max_n=hst.integers(3, 12))
def test_serving_invariants_on_random_streams(sizes, slots, budget, refuse, max_n):
    """Random streams (sizes, arrival gaps), slot counts, arena sizes, sizes the backend cannot batch
    and sizes whose admission fails: every request is answered exactly once, rejected exactly when
    its footprint exceeds the arena, its size is not batched or its admission fails, and otherwise
    solved; slots and memory are never oversubscribed, and every block and handle is returned."""
    reqs, t = [], 0.0
    for r, (n, gap) in enumerate(sizes):
        t += gap
        reqs.append(Request(r, t, I.ring_instance(n, min(2, n - 1), seed=500 + r)))
    be = OracleBackend(budget=budget, max_slots=slots, check_every=10, tol=1e-3, max_iter=300, max_n=max_n,
                       refuse_admit=refuse)
    fp = {q.rid: q.inst.n * q.inst.m * be.bpv for q in reqs}
    nn = {q.rid: q.inst.n for q in reqs}
    records, summary = serve(reqs, be)
    assert sorted(r.rid for r in records) == list(range(len(reqs)))
    for r in records:
        too_big = (fp[r.rid] + ALIGN - 1) // ALIGN * ALIGN > budget
        should_reject = too_big or nn[r.rid] > max_n or nn[r.rid] in refuse
        assert (r.state == "rejected") == should_reject, (r.rid, r.state, too_big, nn[r.rid])
        if r.state != "rejected":
            assert r.state in ("converged", "max_iter")
            assert r.arrival <= r.admitted <= r.done
    assert summary["requests"] + summary["rejected"] == len(reqs)
    assert be.peak_slots <= slots and be.peak_bytes <= budget
    assert be.arena.free == [(0, be.arena.size)] and be.live == 0
