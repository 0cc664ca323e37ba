"""Scheduling logic of the request server on the CPU, with a stand-in backend:
admission never exceeds the memory budget or the slot limit, every request is
served, later arrivals are admitted while earlier batches run, and a failing
batch does not poison the others."""
import threading
import time

import numpy as np
import pytest

from paper_1606_08150_amd import serve


class FakeGraph:
    def __init__(self, n, m):
        self.n, self.m = n, m


class FakeBackend:
    """Each batch 'runs' for a fixed time; results are the request ids.  A
    batch's workspace is the sum of its requests' (ws_of), every worker starts
    with a pool of pool0 bytes."""

    def __init__(self, graphs, run_s=0.002, fail_graph=None, pool0=1 << 30, ws_of=None):
        self.graphs = graphs
        self.run_s = run_s
        self.fail_graph = fail_graph
        self.pool0 = pool0
        self.ws_of = ws_of or (lambda r: 1000)
        self.lock = threading.Lock()
        self.concurrent = 0
        self.max_concurrent = 0
        self.batches = []
        self.grown = []

    def free_bytes(self):
        return 1 << 40

    def worker_state(self):
        return {"pool": self.pool0}

    def close_state(self, state):
        pass

    def pool_bytes(self, state):
        return state["pool"]

    def grow(self, state, nbytes):
        with self.lock:
            self.grown.append(nbytes)
        state["pool"] = max(state["pool"], nbytes)

    def workspace(self, batch):
        return sum(self.ws_of(r) for r in batch)

    def allocate(self, r):
        r.out = None

    def execute(self, state, batch):
        with self.lock:
            self.concurrent += 1
            self.max_concurrent = max(self.max_concurrent, self.concurrent)
            self.batches.append([r.rid for r in batch])
        time.sleep(self.run_s)
        with self.lock:
            self.concurrent -= 1
        if self.fail_graph is not None and any(r.graph == self.fail_graph for r in batch):
            raise RuntimeError("injected failure")
        for r in batch:
            r.out = r.rid * 10 + r.kind


def make(count=400, rate=20000.0, graphs=8):
    gs = [FakeGraph(1000 * (i + 1), 16000 * (i + 1)) for i in range(graphs)]
    srcs = [np.arange(10) for _ in gs]
    reqs = serve.poisson_requests(count, rate, srcs, n_x=4, seed=3)
    return gs, reqs


def test_poisson_stream_is_seeded_and_has_the_rate():
    _, a = make(count=20000, rate=5000.0)
    _, b = make(count=20000, rate=5000.0)
    assert [(r.kind, r.graph, r.arg, r.t_arrive) for r in a] == [(r.kind, r.graph, r.arg, r.t_arrive) for r in b]
    span = a[-1].t_arrive - a[0].t_arrive
    assert abs(len(a) / span - 5000.0) / 5000.0 < 0.05
    frac = np.mean([r.kind == serve.SSSP for r in a])
    assert abs(frac - 0.5) < 0.02


def test_admission_budget_and_slots():
    adm = serve.Admission(100, 3)
    assert adm.try_admit(40) and adm.try_admit(40)
    assert not adm.try_admit(40)  # bytes
    assert adm.try_admit(20)
    assert not adm.try_admit(0)   # slots
    adm.release(40)
    assert adm.try_admit(30) and adm.peak_used == 100 and adm.peak_slots == 3
    assert not adm.fits_ever(101) and adm.fits_ever(100)


def test_every_request_served_within_budget_with_overlap():
    gs, reqs = make()
    be = FakeBackend(gs)
    budget = 4 * max(serve.request_bytes(k, g.n, g.m) for g in gs for k in (0, 1))
    srv = serve.Server(be, workers=4, budget_bytes=budget, max_slots=16, max_batch=8, keep_outputs=True)
    try:
        out = srv.run(reqs, time_limit=30)
    finally:
        srv.close()
    assert all(r.out == r.rid * 10 + r.kind for r in out)
    assert srv.admission.peak_used <= budget and srv.admission.peak_slots <= 16
    assert srv.admission.used == 0 and srv.admission.slots == 0
    assert be.max_concurrent >= 2  # batches overlapped
    assert all(r.t_arrive <= r.t_admit <= r.t_start <= r.t_done for r in out)
    assert sorted(i for b in be.batches for i in b) == list(range(len(reqs)))
    s = serve.summarize(out)
    assert s["requests"] == len(reqs) and s["failed"] == 0 and s["p99_ms"] >= s["p50_ms"]


def test_a_failed_batch_does_not_poison_the_others():
    gs, reqs = make(count=200)
    be = FakeBackend(gs, fail_graph=3)
    srv = serve.Server(be, workers=2, budget_bytes=1 << 40, max_slots=64, max_batch=1, keep_outputs=True)
    try:
        out = srv.run(reqs, time_limit=30)
    finally:
        srv.close()
    for r in out:
        if r.graph == 3:
            assert r.error is not None
        else:
            assert r.error is None and r.out == r.rid * 10 + r.kind


def test_oversized_request_is_rejected():
    gs, reqs = make(count=10)
    srv = serve.Server(FakeBackend(gs), workers=1, budget_bytes=10, max_slots=4)
    try:
        with pytest.raises(ValueError):
            srv.run(reqs)
    finally:
        srv.close()


class FakeTree:
    def __init__(self, n):
        self.n = n


def test_tree_requests_join_the_stream_without_changing_the_rest():
    gs = [FakeGraph(1000, 16000) for _ in range(4)]
    srcs = [np.arange(10) for _ in gs]
    base = serve.poisson_requests(5000, 5000.0, srcs, n_x=4, seed=5)
    mixed = serve.poisson_requests(5000, 5000.0, srcs, n_x=4, seed=5, tree_fraction=0.3, n_trees=3)
    assert [r.t_arrive for r in base] == [r.t_arrive for r in mixed]
    trees = [r for r in mixed if r.kind in serve.TREE_KINDS]
    assert abs(len(trees) / len(mixed) - 0.3) < 0.03
    assert {r.kind for r in trees} == set(serve.TREE_KINDS) and {r.graph for r in trees} == {0, 1, 2}
    for a, b in zip(base, mixed):
        if b.kind not in serve.TREE_KINDS:
            assert (a.kind, a.graph, a.arg) == (b.kind, b.graph, b.arg)
    with pytest.raises(ValueError):
        serve.poisson_requests(10, 100.0, srcs, n_x=4, seed=5, tree_fraction=0.5)


def test_tree_requests_are_admitted_by_their_own_size():
    gs, _ = make(count=1)
    be = FakeBackend(gs)
    be.trees = [FakeTree(5000), FakeTree(200000)]
    srcs = [np.arange(10) for _ in gs]
    reqs = serve.poisson_requests(300, 20000.0, srcs, n_x=4, seed=8, tree_fraction=0.5, n_trees=2)
    srv = serve.Server(be, workers=3, budget_bytes=1 << 40, max_slots=32, max_batch=8, keep_outputs=True)
    try:
        out = srv.run(reqs, time_limit=30)
    finally:
        srv.close()
    assert all(r.out == r.rid * 10 + r.kind for r in out)
    for r in out:
        if r.kind in serve.TREE_KINDS:
            assert r.nbytes == serve.request_bytes(r.kind, be.trees[r.graph].n, 0)
    assert srv.admission.used == 0 and srv.admission.slots == 0


def test_a_request_that_would_grow_a_pool_waits_for_memory():
    """Budget 800 bytes; one worker whose pool holds 100.  r0 (output 300,
    workspace 50) runs first; r1 (output 100) needs a 700-byte workspace, so
    its worker must grow to 700, charged whole (the replaced pool stays
    allocated): with r0's output still held that would be 300 + 100 + 700 >
    800, so r1 stays queued until r0 is done, then the growth is charged for
    good and r1 runs."""
    gs = [FakeGraph(75, 10), FakeGraph(25, 10)]
    reqs = [serve.Request(0, serve.SPMV, 0, 0, 0.0), serve.Request(1, serve.SPMV, 1, 0, 0.0)]
    be = FakeBackend(gs, run_s=0.05, pool0=100, ws_of=lambda r: 50 if r.graph == 0 else 700)
    srv = serve.Server(be, workers=1, budget_bytes=800, max_slots=8, max_batch=8, keep_outputs=True)
    try:
        out = srv.run(reqs, time_limit=30)
    finally:
        srv.close()
    r0, r1 = out
    assert r0.nbytes == 300 and r1.nbytes == 100
    assert be.batches == [[0], [1]]          # cut to what the pool holds, then r1 alone
    assert r1.t_start >= r0.t_done            # queued, not over-admitted
    assert be.grown == [700] and srv.grows == 1
    assert srv.admission.peak_used <= 800 and srv.admission.pool_growth == 700
    assert srv.admission.used == 700          # the growth stays charged; outputs are released


def test_a_growth_that_can_never_fit_is_refused_up_front():
    gs = [FakeGraph(10, 10)]
    reqs = [serve.Request(0, serve.SPMV, 0, 0, 0.0)]
    be = FakeBackend(gs, pool0=100, ws_of=lambda r: 10_000)
    srv = serve.Server(be, workers=2, budget_bytes=1000, max_slots=8)
    try:
        with pytest.raises(ValueError):
            srv.run(reqs)
    finally:
        srv.close()


def test_admitted_requests_give_memory_back_when_a_growth_could_never_run():
    """Budget 1000, one worker with a 100-byte pool.  r0 needs a 700-byte
    workspace (a growth charged 700); r1..r3 (output 200 each) arrive with it and are
    admitted too, leaving no room for the growth while nothing runs.  The
    later requests give their outputs back and wait, r0 grows the pool and
    runs, then the others run in the grown pool."""
    gs = [FakeGraph(25, 10), FakeGraph(50, 10)]
    reqs = [serve.Request(0, serve.SPMV, 0, 0, 0.0)] + [serve.Request(i, serve.SPMV, 1, 0, 0.0) for i in (1, 2, 3)]
    be = FakeBackend(gs, run_s=0.01, pool0=100, ws_of=lambda r: 700 if r.graph == 0 else 50)
    srv = serve.Server(be, workers=1, budget_bytes=1000, max_slots=8, max_batch=8, keep_outputs=True)
    try:
        out = srv.run(reqs, time_limit=30)
    finally:
        srv.close()
    assert all(r.error is None for r in out)
    assert be.batches[0] == [0] and sorted(i for b in be.batches[1:] for i in b) == [1, 2, 3]
    assert be.grown == [700] and srv.admission.peak_used <= 1000
