"""Scheduling logic of the continuous-batching server, on the CPU with a fake engine.

The fake engine stands in for the GPU: a solve of a w-node box takes a fixed number of
rounds, footprints scale with the box, and a simulated clock advances per round, so
admission, the HBM budget, the hierarchy cache and retirement are checked exactly.
"""
import dataclasses

import pytest

import workloads as W
from paper_0907_4863_amd import capi
from paper_0907_4863_amd.serve import Record, ServeConfig, Server, summarize


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class FakeEngine:
    def __init__(self, clock, round_s=0.01):
        self.clock = clock
        self.round_s = round_s
        self.hier = {}
        self.live_states = 0
        self.max_live = 0
        self.setups = 0
        self.starts = []
        self.warm_live = 0

    def key(self, w):
        return (w.shape.kind, w.nx, w.ny, w.nz)

    def footprint(self, w, precision):
        n = w.nx * w.ny * w.nz
        return 10 * n, 60 * n

    def setup(self, w, precision):
        self.setups += 1
        H = object()
        self.hier[id(H)] = H
        self.clock.t += 0.002
        return H, 10 * w.nx * w.ny * w.nz, w.nx * w.ny * w.nz

    def release_hierarchy(self, H):
        del self.hier[id(H)]

    def start(self, H, b, tol, max_iter, x0=None):
        self.live_states += 1
        self.max_live = max(self.max_live, self.live_states)
        self.starts.append(x0)
        # a warm start saves one round
        left = max(int(b) - (1 if x0 is not None else 0), 1)
        return {"left": left, "it": 0}

    def step(self, hs):
        self.clock.t += self.round_s
        for h in hs:
            if h["left"] > 0:
                h["left"] -= 1
                h["it"] += 1

    def query(self, h):
        return h["left"] == 0, {"iterations": h["it"], "status": 0, "rel_res_true": 1e-9}

    def finish(self, h, keep_warm=False):
        self.live_states -= 1
        if keep_warm:
            self.warm_live += 1
            return None, ("x", id(h))
        return None, None

    def warm_bytes(self, w):
        return 8 * w.nx * w.ny * w.nz

    def release_warm(self, x):
        self.warm_live -= 1


@dataclasses.dataclass
class Req:
    rid: int
    arrival_s: float
    workload: object
    rounds: int


def _req(rid, t, edge, rounds, kind=W.CYLINDER):
    w = W.Workload(f"r{rid}", W.serving_shape(kind, 1), edge, edge, edge, W.VARIANT_LIN,
                   W.PREC_MIXED)
    return Req(rid, t, w, rounds)


def _serve(reqs, **cfg):
    clock = Clock()
    eng = FakeEngine(clock)
    srv = Server(ServeConfig(**cfg), eng, clock=clock, sleep=clock.sleep)
    recs = srv.run(reqs, rhs_of=lambda r: r.rounds)
    return srv, eng, {r.rid: r for r in recs}


def test_all_requests_served_with_their_iterations():
    reqs = [_req(i, 0.003 * i, 10 + i, 5 + i % 3) for i in range(12)]
    srv, eng, recs = _serve(reqs, hbm_budget_bytes=1 << 40, max_active=4)
    assert len(recs) == 12
    for r in reqs:
        assert recs[r.rid].iterations == r.rounds and recs[r.rid].status == 0
    assert srv.max_concurrent <= 4 and eng.max_live <= 4
    s = summarize(list(recs.values()))
    assert s["completed"] == 12 and s["p99_latency_ms"] >= s["p50_latency_ms"] > 0


def test_late_arrivals_join_running_batch():
    """Continuous batching: a request arriving mid-run starts before the long one ends."""
    reqs = [_req(0, 0.0, 10, 50), _req(1, 0.05, 11, 3)]
    _, _, recs = _serve(reqs, hbm_budget_bytes=1 << 40, max_active=4)
    assert recs[1].admit_s < recs[0].done_s
    assert recs[1].done_s < recs[0].done_s


def test_budget_limits_concurrency():
    reqs = [_req(i, 0.0, 10, 4) for i in range(6)]
    per = 60 * 1000 + 10 * 1000  # state + hierarchy of one 10^3 box
    srv, eng, recs = _serve(reqs, hbm_budget_bytes=2 * per + 10, max_active=16,
                            cache_hierarchies=False)
    assert len(recs) == 6 and all(r.status == 0 for r in recs.values())
    assert eng.max_live == 2
    assert srv.peak_used <= 2 * per + 10


def test_oversized_request_rejected_not_deadlocked():
    reqs = [_req(0, 0.0, 40, 3), _req(1, 0.0, 10, 3)]
    srv, _, recs = _serve(reqs, hbm_budget_bytes=100 * 1000, max_active=4)
    assert recs[0].status == capi.NOMEM and recs[1].status == 0
    assert srv.rejected == [0]


def test_hierarchy_cache_reuse_and_eviction():
    same = [_req(i, 0.001 * i, 12, 3) for i in range(4)]
    srv, eng, recs = _serve(same, hbm_budget_bytes=1 << 40, max_active=1)
    assert eng.setups == 1 and sum(r.cache_hit for r in recs.values()) == 3
    # a budget that holds one hierarchy + state at a time forces eviction between shapes
    mixed = [_req(0, 0.0, 12, 3), _req(1, 0.0, 13, 3), _req(2, 0.0, 12, 3)]
    per13 = 70 * 13 ** 3
    srv2, eng2, recs2 = _serve(mixed, hbm_budget_bytes=per13 + 10, max_active=1)
    assert all(r.status == 0 for r in recs2.values())
    # the 12^3 hierarchy had to be evicted to admit the 13^3 request, then rebuilt
    assert eng2.setups == 3 and srv2.peak_used <= per13 + 10
    assert not recs2[2].cache_hit


# ---------------------------------------------------------------------------------------
# Hierarchies built on a worker thread (engines with concurrent_setup), as GpuEngine does.


class ThreadedFakeEngine(FakeEngine):
    concurrent_setup = True

    def __init__(self, clock, round_s=0.01):
        super().__init__(clock, round_s)
        import threading
        self.lock = threading.Lock()
        self.setup_threads = set()

    def setup(self, w, precision):
        import threading
        with self.lock:
            self.setup_threads.add(threading.get_ident())
            return super().setup(w, precision)


def _serve_threaded(reqs, **cfg):
    import threading
    clock = Clock()
    eng = ThreadedFakeEngine(clock)
    srv = Server(ServeConfig(**cfg), eng, clock=clock, sleep=clock.sleep)
    recs = srv.run(reqs, rhs_of=lambda r: r.rounds)
    return srv, eng, {r.rid: r for r in recs}, threading.get_ident()


def test_worker_setup_serves_every_request_once_per_geometry():
    """Hierarchies built off the main thread: every request finishes with its own
    iterations, one build per geometry (requests of a geometry whose build is running wait
    on it), the budget holds, and all memory but the cached hierarchies is returned."""
    reqs = [_req(i, 0.0, 10 + i % 3, 4 + i % 5) for i in range(12)]
    srv, eng, recs, main = _serve_threaded(reqs, hbm_budget_bytes=1 << 40, max_active=5,
                                           warm_start=False)
    assert len(recs) == 12 and all(r.status == 0 for r in recs.values())
    for r in reqs:
        assert recs[r.rid].iterations == r.rounds
    assert eng.setups == 3 and main not in eng.setup_threads
    assert srv.max_concurrent <= 5 and eng.max_live <= 5 and eng.live_states == 0
    assert srv.used == sum(e["bytes"] for e in srv.cache.values())
    assert sum(r.setup_ms > 0 or r.cache_hit for r in recs.values()) >= 3


def test_worker_setup_respects_budget_and_rejects_oversized():
    reqs = [_req(i, 0.0, 10, 4) for i in range(6)] + [_req(6, 0.0, 40, 3)]
    per = 60 * 1000 + 10 * 1000
    srv, eng, recs, _ = _serve_threaded(reqs, hbm_budget_bytes=2 * per + 10, max_active=16,
                                        cache_hierarchies=False)
    assert recs[6].status == capi.NOMEM and srv.rejected == [6]
    assert all(recs[i].status == 0 for i in range(6))
    assert srv.peak_used <= 2 * per + 10 and eng.max_live <= 2
    assert srv.used == 0 and not srv.cache


def test_repeat_geometry_starts_from_the_resident_solution():
    """Section 4's warm start in the server: the second and third requests of a geometry
    start from the solution of the one before; other geometries start from zero."""
    reqs = [_req(0, 0.0, 20, 5), _req(1, 1.0, 20, 5), _req(2, 2.0, 24, 5), _req(3, 3.0, 20, 5)]
    srv, eng, recs = _serve(reqs, hbm_budget_bytes=10 ** 9)
    assert [recs[i].warm_from for i in range(4)] == [-1, 0, -1, 1]
    assert recs[1].iterations == recs[0].iterations - 1
    assert summarize(list(recs.values()))["warm_starts"] == 2
    srv.close()
    assert eng.warm_live == 0 and srv.used == 0


def test_resident_solutions_count_in_the_budget_and_go_with_eviction():
    reqs = [_req(0, 0.0, 20, 3), _req(1, 1.0, 30, 3), _req(2, 2.0, 20, 3)]
    n20, n30 = 20 ** 3, 30 ** 3
    # room for the 30^3 geometry's hierarchy and state, but not beside the 20^3 one's
    # hierarchy and resident solution
    budget = 10 * n30 + 60 * n30 + 1000
    assert budget < 10 * n20 + 8 * n20 + 10 * n30 + 60 * n30
    srv, eng, recs = _serve(reqs, hbm_budget_bytes=budget)
    assert all(r.status == 0 for r in recs.values())
    assert recs[2].warm_from == -1  # geometry 20 was evicted for geometry 30
    assert srv.peak_used <= budget
    srv.close()
    assert eng.warm_live == 0


def test_warm_start_off():
    reqs = [_req(0, 0.0, 20, 5), _req(1, 1.0, 20, 5)]
    srv, eng, recs = _serve(reqs, warm_start=False)
    assert recs[1].warm_from == -1 and eng.starts == [None, None] and eng.warm_live == 0
