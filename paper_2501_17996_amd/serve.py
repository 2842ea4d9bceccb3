"""Continuous-batching serving loop for MCF requests on one GPU.

Requests (an instance and an arrival time) are admitted into a batching pool
(``mcf_pool_*``) as slots and device memory free up.  Every pool step advances
all admitted instances together -- one kernel launch per iteration for all of
them -- and ends with a residual check of each.  Converged instances are retired
at once, their memory is returned, and queued requests take their place while
the others keep iterating.

Device memory comes from one arena (a torch allocation) that the loop
sub-allocates first-fit: admission is by HBM footprint (``mcf_workspace_bytes``),
and no device allocation happens while serving.

The loop is written against a small backend interface (footprint, create,
admit, step, sync, poll, retire, destroy) so that its bookkeeping can be tested
with a CPU stand-in.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

ALIGN = 256


@dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the run
    inst: object            # instances.Instance, or a callable that builds it on first use

    def instance(self):
        if callable(self.inst):
            self.inst = self.inst()
        return self.inst


@dataclass
class Record:
    rid: int
    n: int
    m: int
    arrival: float
    admitted: float = math.nan
    done: float = math.nan
    iters: int = 0
    state: str = ""
    rel_kkt: float = math.nan
    primal_obj: float = math.nan
    slot: int = -1
    extra: dict = field(default_factory=dict)

    @property
    def latency(self) -> float:
        return self.done - self.arrival

    @property
    def service(self) -> float:
        return self.done - self.admitted


class Arena:
    """First-fit allocator of byte ranges inside one device allocation."""

    def __init__(self, nbytes: int):
        self.size = int(nbytes)
        self.free = [(0, self.size)]   # sorted, disjoint (offset, length)

    def alloc(self, nbytes: int):
        need = (int(nbytes) + ALIGN - 1) // ALIGN * ALIGN
        for k, (off, ln) in enumerate(self.free):
            if ln >= need:
                if ln == need:
                    self.free.pop(k)
                else:
                    self.free[k] = (off + need, ln - need)
                return off, need
        return None

    def release(self, off: int, ln: int):
        self.free.append((off, ln))
        self.free.sort()
        merged = []
        for o, l in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + l)
            else:
                merged.append((o, l))
        self.free = merged

    def free_bytes(self) -> int:
        return sum(l for _, l in self.free)


class GpuBackend:
    """libmcf batching pool with instance workspaces carved from one torch allocation."""

    def __init__(self, precision: int, hbm_budget: int, max_slots: int, check_every: int, tol: float,
                 max_iter: int = 200000, adapt_until: int = -1):
        import torch

        from . import mcf
        self.mcf = mcf
        self.torch = torch
        self.precision, self.tol, self.max_iter, self.adapt_until = precision, tol, max_iter, adapt_until
        self.check_every = check_every
        self.buf = torch.empty(int(hbm_budget), dtype=torch.uint8, device="cuda")
        self.base = self.buf.data_ptr()
        self.arena = Arena(hbm_budget)
        self.setup_stream = torch.cuda.Stream()
        self.pool = mcf.Pool(precision, hbm_budget, max_slots, check_every)
        self.max_slots = max_slots
        self.capacity = int(hbm_budget)

    def accepts(self, inst) -> bool:
        """The pool batches instances that take the single-launch iteration (n <= 512)."""
        return inst.n <= self.mcf.FUSED_MAX_N

    def footprint(self, inst) -> int:
        # the workspace of the organisation the pool will run (mcf_workspace_bytes gives AUTO's;
        # the two-phase one needs no second copy of F, so this bound holds for both)
        return self.mcf.mcf_workspace_bytes(inst.n, inst.m, self.precision)

    def create(self, inst):
        got = self.arena.alloc(self.footprint(inst))
        if got is None:
            return None
        off, ln = got
        # the organisation and launch shape the pool runs fastest for this size
        shape = self.pool.instance_options(inst.n)
        s = self.mcf.Solver(inst, tol=self.tol, max_iter=self.max_iter, check_every=self.check_every,
                            stream=self.setup_stream.cuda_stream, workspace=self.base + off, workspace_bytes=ln,
                            adapt_until=self.adapt_until, **shape)
        s.arena_block = got
        return s

    def admit(self, h) -> int:
        return self.pool.admit(h)

    def step(self):
        self.pool.step(self.check_every)

    def sync(self):
        self.pool.sync()

    def poll(self, slot: int) -> dict:
        return self.pool.poll(slot)

    def retire(self, slot: int):
        self.pool.retire(slot)

    def destroy(self, h):
        block = h.arena_block
        h.close()
        self.arena.release(*block)

    def close(self):
        self.pool.close()


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return math.nan
    k = (len(xs) - 1) * q / 100.0
    lo, hi = int(math.floor(k)), int(math.ceil(k))
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def serve(requests, backend, clock=time.perf_counter, keep=None, idle_wait=1e-4):
    """Runs the request stream to completion.  ``requests`` are sorted by arrival.
    ``keep(record, handle)`` may read a finished instance (its solution) before it is
    destroyed.  Returns (records, summary).

    The device is kept busy while the host works: once the step in flight has ended, the
    loop retires finished instances, admits the handles it created meanwhile, and enqueues
    the next step at once; only then does it destroy retired handles, hand results to
    ``keep`` and build the handles of queued requests (instance, CSR, upload on a stream of
    its own), all of which overlaps the step now running.

    A request whose footprint exceeds the whole arena, or that the backend cannot batch
    (``backend.accepts``), or whose creation or admission fails, is answered at once with
    a record in state "rejected" instead of waiting forever at the head of the queue."""
    pending = deque(sorted(requests, key=lambda r: r.arrival))
    queue = deque()
    ready = deque()                  # (request, handle, record) created, not yet admitted
    active = {}                      # slot -> (request, handle, record)
    retired = []                     # (request, handle, record) to destroy after the next enqueue
    records = []
    capacity = getattr(backend, "capacity", None)
    accepts = getattr(backend, "accepts", None)
    t0 = clock()
    steps = 0
    updates = 0.0
    in_flight = False

    def reject(req, inst, why):
        rec = Record(req.rid, inst.n, inst.m, req.arrival, admitted=clock() - t0, state="rejected")
        rec.done = rec.admitted
        rec.extra["reason"] = why
        records.append(rec)
        req.inst = None

    def prepare():
        # arrivals, then handles for queued requests while slots and memory allow
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            queue.append(pending.popleft())
        while queue and len(active) + len(ready) < backend.max_slots:
            req = queue[0]
            inst = req.instance()
            fp = backend.footprint(inst)
            if capacity is not None and (fp + ALIGN - 1) // ALIGN * ALIGN > capacity:
                queue.popleft()
                reject(req, inst, f"footprint {fp} B exceeds the arena ({capacity} B)")
                continue
            if accepts is not None and not accepts(inst):
                queue.popleft()
                reject(req, inst, "the backend cannot batch this instance")
                continue
            try:
                h = backend.create(inst)
            except Exception as e:  # invalid instance: answer it, keep serving the others
                queue.popleft()
                reject(req, inst, f"create failed: {e}")
                continue
            if h is None:
                break                # no room in the arena now: wait for a retirement
            queue.popleft()
            ready.append((req, h, Record(req.rid, inst.n, inst.m, req.arrival)))

    def finish(req, h, rec):
        if keep is not None:
            keep(rec, h)
        backend.destroy(h)
        req.inst = None              # the library holds its own copy; free the host arrays
        records.append(rec)

    prepare()
    while pending or queue or ready or active or in_flight:
        if in_flight:
            backend.sync()
            in_flight = False
            t_done = clock() - t0
            for slot in list(active):
                req, h, rec = active[slot]
                st = backend.poll(slot)
                updates += float(rec.n) * rec.m * (st["iters"] - rec.iters)
                rec.iters = st["iters"]
                if st["state_name"] == "running":
                    continue
                backend.retire(slot)
                rec.done = t_done
                rec.state = st["state_name"]
                rec.rel_kkt = st["rel_kkt"]
                rec.primal_obj = st["primal_obj"]
                retired.append((req, h, rec))
                del active[slot]
        # admission: FIFO, into free slots
        while ready and len(active) < backend.max_slots:
            req, h, rec = ready.popleft()
            try:
                slot = backend.admit(h)
            except Exception as e:
                backend.destroy(h)
                rec.admitted = rec.done = clock() - t0
                rec.state = "rejected"
                rec.extra["reason"] = f"admit failed: {e}"
                req.inst = None
                records.append(rec)
                continue
            st = backend.poll(slot)
            rec.iters = st["iters"]
            rec.admitted = clock() - t0
            rec.slot = slot
            active[slot] = (req, h, rec)
        if active:
            backend.step()
            in_flight = True
            steps += 1
        # host work while the step runs
        for item in retired:
            finish(*item)
        retired.clear()
        prepare()
        if not in_flight and not ready and not active and pending:
            wait = pending[0].arrival - (clock() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.01) if wait > idle_wait else 0)
    makespan = clock() - t0
    served = [r for r in records if r.state != "rejected"]
    lat = [r.latency for r in served]
    svc = [r.service for r in served]
    summary = {
        "requests": len(served),
        "rejected": len(records) - len(served),
        "makespan_s": makespan,
        "instances_per_s": len(served) / makespan if makespan > 0 else math.nan,
        "edge_dest_updates_per_s": updates / makespan if makespan > 0 else math.nan,
        "latency_p50_s": percentile(lat, 50),
        "latency_p99_s": percentile(lat, 99),
        "service_p50_s": percentile(svc, 50),
        "service_p99_s": percentile(svc, 99),
        "steps": steps,
        "converged": sum(r.state == "converged" for r in served),
    }
    return records, summary
