"""A CPU stand-in for the serving backend: each admitted instance is advanced by
the oracle, check_every iterations per step, so the serving loop's admission,
slot and retirement bookkeeping can be tested without a GPU."""
import oracle
from paper_2501_17996_amd.serve import Arena


class OracleBackend:
    def __init__(self, budget, max_slots, check_every, tol, max_iter=100000, bytes_per_var=32, max_n=None,
                 refuse_admit=()):
        self.arena = Arena(budget)
        self.capacity = int(budget)
        self.max_n = max_n                  # accepts(): instances up to this size (None: all)
        self.refuse_admit = set(refuse_admit)  # admit() raises for instances of these sizes
        self.live = 0                       # handles created and not yet destroyed
        self.max_slots, self.check_every, self.tol, self.max_iter = max_slots, check_every, tol, max_iter
        self.bpv = bytes_per_var
        self.slots = {}
        self.peak_slots = 0
        self.peak_bytes = 0
        self.steps = 0

    def footprint(self, inst):
        return inst.n * inst.m * self.bpv

    def create(self, inst):
        got = self.arena.alloc(self.footprint(inst))
        if got is None:
            return None
        h = oracle.OracleSolver(inst)
        h.n_nodes = inst.n
        self.live += 1
        h.block = got
        h.status = {"iters": 0, "state_name": "running", "rel_kkt": float("inf"), "primal_obj": float("inf")}
        self.peak_bytes = max(self.peak_bytes, self.arena.size - self.arena.free_bytes())
        return h

    def accepts(self, inst):
        return self.max_n is None or inst.n <= self.max_n

    def admit(self, h):
        if h.n_nodes in self.refuse_admit:
            raise ValueError("refused by the pool")
        slot = min(set(range(self.max_slots)) - set(self.slots))
        self.slots[slot] = h
        self.peak_slots = max(self.peak_slots, len(self.slots))
        return slot

    def step(self):
        self.steps += 1
        for h in self.slots.values():
            if h.status["state_name"] != "running":
                continue
            k = h.status["iters"]
            st = h.solve(self.tol, max_iter=min(k + self.check_every, self.max_iter), check_every=self.check_every)
            M = h.metrics()
            k = int(M["k"])
            state = "converged" if st == "converged" else ("max_iter" if k >= self.max_iter else "running")
            h.status = {"iters": k, "state_name": state, "rel_kkt": M["rel_kkt"], "primal_obj": M["primal_obj"]}

    def sync(self):
        pass

    def poll(self, slot):
        return dict(self.slots[slot].status)

    def retire(self, slot):
        del self.slots[slot]

    def destroy(self, h):
        self.arena.release(*h.block)
        self.live -= 1
        h.close()
