"""Continuous-batching request server over resident graphs and trees.

Requests (SSSP from a source, SpMV with one of the graph's resident x vectors,
or tree descendants / heights of a resident tree) arrive over time.  The scheduler admits a waiting request as soon as
the device-memory budget and the slot limit allow it, and hands each batch of
admitted requests to an idle worker.  Every worker owns a libwc context and its
own HIP stream, so batches launched while others are still on the device run
concurrently; SSSP requests of one batch go through one wc_sssp_batch call
(their work is consolidated across requests), SpMV requests through wc_spmv,
tree requests through wc_tree_descendants / wc_tree_height.
Each result is the same as the request run alone (bit-identical distances;
SpMV results bit-identical for a fixed mode and tune).

Device memory is budgeted exactly.  A request holds its output from admission
to completion; a batch also needs its worker's consolidation workspace (the
context pool), which the backend computes with the library's plan-only mode (the
bytes the calls would carve, nothing enqueued).  A batch whose workspace exceeds
its worker's pool is cut down; a single request that still needs a larger pool
is dispatched only when the growth fits the remaining budget, otherwise it waits
for memory to free.  A growth is charged its whole new pool, for good: the
library keeps the replaced pool (calls in flight may still use it) for as long
as the worker's context lives, and pools never shrink.
The budget is measured after the workers' contexts (and their pools) exist.

Only the scheduling lives here; every request's arithmetic runs in libwc.  The
device side is a backend object, so the scheduling can be exercised on the
CPU with a stand-in backend.
"""
from __future__ import annotations

import collections
import queue
import threading
import time
from dataclasses import dataclass, field

import numpy as np

SSSP, SPMV, TREE_DESC, TREE_HEIGHT = 0, 1, 2, 3
TREE_KINDS = (TREE_DESC, TREE_HEIGHT)


@dataclass
class Request:
    rid: int
    kind: int          # SSSP, SPMV, TREE_DESC or TREE_HEIGHT
    graph: int         # index of a resident graph (SSSP, SpMV) or tree (tree kinds)
    arg: int           # SSSP source vertex, SpMV x-vector index; unused for trees
    t_arrive: float    # seconds from the start of the run
    nbytes: int = 0
    t_admit: float = -1.0
    t_start: float = -1.0
    t_done: float = -1.0
    out: object = None
    error: object = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrive


class Admission:
    """Admits a request while its bytes fit the remaining budget and a slot is
    free; a request larger than the whole budget is rejected outright."""

    def __init__(self, budget_bytes: int, max_slots: int):
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.used = 0
        self.slots = 0
        self.peak_used = 0
        self.peak_slots = 0
        self.pool_growth = 0  # bytes of pool growth charged so far (never released)

    def fits_ever(self, nbytes: int) -> bool:
        return nbytes <= self.budget

    def try_admit(self, nbytes: int) -> bool:
        if self.slots >= self.max_slots or self.used + nbytes > self.budget:
            return False
        self.used += nbytes
        self.slots += 1
        self.peak_used = max(self.peak_used, self.used)
        self.peak_slots = max(self.peak_slots, self.slots)
        return True

    def release(self, nbytes: int):
        self.used -= nbytes
        self.slots -= 1
        assert self.used >= 0 and self.slots >= 0

    def try_grow(self, nbytes: int) -> bool:
        """Charges a pool growth for good (pools are never released while the
        context lives), if it fits."""
        if self.used + nbytes > self.budget:
            return False
        self.used += nbytes
        self.pool_growth += nbytes
        self.peak_used = max(self.peak_used, self.used)
        return True


def request_bytes(kind: int, n: int, m: int) -> int:
    """Device bytes a request holds from admission to completion: its output
    (n 32-bit distances, values or tree results; m unused).  The consolidation
    workspace lives in the worker's pool and is budgeted per batch."""
    return 4 * n


def poisson_requests(count: int, rate: float, sources_per_graph, n_x: int, seed: int, sssp_fraction: float = 0.5,
                     tree_fraction: float = 0.0, n_trees: int = 0):
    """Seeded request stream: exponential inter-arrival times at `rate` per
    second, kind SSSP with probability sssp_fraction (else SpMV), graph uniform,
    SSSP source uniform over the graph's vertices with out-edges, SpMV x uniform
    over n_x.  With tree_fraction > 0, that share of the requests (drawn after
    the others, so the rest of the stream is unchanged) become tree descendants
    or heights (even odds) of a uniform one of n_trees resident trees."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    kinds = np.where(rng.random(count) < sssp_fraction, SSSP, SPMV)
    graphs = rng.integers(0, len(sources_per_graph), size=count)
    reqs = []
    for i in range(count):
        g = int(graphs[i])
        if kinds[i] == SSSP:
            cand = sources_per_graph[g]
            arg = int(cand[rng.integers(0, len(cand))])
        else:
            arg = int(rng.integers(0, n_x))
        reqs.append(Request(i, int(kinds[i]), g, arg, float(t[i])))
    if tree_fraction > 0:
        if n_trees < 1:
            raise ValueError("tree requests need at least one resident tree")
        tree_rng = np.random.default_rng([seed, 7])
        is_tree = tree_rng.random(count) < tree_fraction
        tree_kind = np.where(tree_rng.random(count) < 0.5, TREE_DESC, TREE_HEIGHT)
        tree_idx = tree_rng.integers(0, n_trees, size=count)
        for i in np.flatnonzero(is_tree).tolist():
            reqs[i].kind, reqs[i].graph, reqs[i].arg = int(tree_kind[i]), int(tree_idx[i]), 0
    return reqs


@dataclass
class ResidentGraph:
    csr: object                # wc.DeviceCSR
    w: object                  # int32 view of uint32 weights (device)
    val: object                # fp32 values (device)
    xs: list = field(default_factory=list)  # fp32 x vectors (device)

    @property
    def n(self):
        return self.csr.n

    @property
    def m(self):
        return self.csr.m


class GpuBackend:
    """libwc on one device: one context and one stream per worker, and one
    plan-only context that computes the workspace of a batch."""

    def __init__(self, graphs, device: int = 0, sssp_mode="grid", spmv_mode="grid", trees=(), tree_mode="grid",
                 pool_bytes: int = 256 << 20):
        self.graphs = graphs
        self.trees = list(trees)  # wc.DeviceTree
        self.device = device
        self.sssp_mode, self.spmv_mode, self.tree_mode = sssp_mode, spmv_mode, tree_mode
        self.pool_bytes0 = pool_bytes
        self._planner = None

    def free_bytes(self) -> int:
        import torch
        return int(torch.cuda.mem_get_info(self.device)[0])

    def worker_state(self):
        import torch
        from . import wc
        return wc.Context(self.device, pool_bytes=self.pool_bytes0), torch.cuda.Stream(device=self.device)

    def close_state(self, state):
        state[0].close()

    def close(self):
        if self._planner is not None:
            self._planner.close()
            self._planner = None

    def pool_bytes(self, state) -> int:
        return state[0].pool_info()[0]

    def pool_grows(self, state) -> int:
        return state[0].pool_info()[1]

    def grow(self, state, nbytes: int):
        state[0].reserve(nbytes)

    def workspace(self, batch) -> int:
        """Pool bytes the batch's calls carve on a worker (the library's own
        plan; the calls run one after another, so the largest one counts)."""
        from . import wc
        import torch
        if self._planner is None:
            self._planner = wc.Context(self.device, pool_bytes=1 << 20)
            # stands in for outputs not allocated yet: a plan-only call writes nothing
            self._placeholder = torch.empty(1, dtype=torch.int32, device=f"cuda:{self.device}")
        return self._planner.workspace_bytes(lambda c: self._issue(c, batch, None, plan=True))

    def allocate(self, r):
        import torch
        if r.kind in TREE_KINDS:
            r.out = torch.empty(self.trees[r.graph].n, dtype=torch.int32, device=f"cuda:{self.device}")
            return
        g = self.graphs[r.graph]
        dt = torch.int32 if r.kind == SSSP else torch.float32
        r.out = torch.empty(g.n, dtype=dt, device=f"cuda:{self.device}")

    def _issue(self, ctx, batch, stream, plan=False):
        def out(r):
            return r.out if not plan or r.out is not None else self._placeholder
        sssp = [r for r in batch if r.kind == SSSP]
        if sssp:
            gs = [self.graphs[r.graph] for r in sssp]
            ctx.sssp_batch([g.csr for g in gs], [g.w for g in gs], [r.arg for r in sssp],
                           modes=[self.sssp_mode] * len(sssp), outs=[out(r) for r in sssp], stream=stream)
        for r in batch:
            if r.kind == SPMV:
                g = self.graphs[r.graph]
                ctx.spmv(g.csr, g.val, g.xs[r.arg], mode=self.spmv_mode, out=out(r), stream=stream)
            elif r.kind in TREE_KINDS:
                fn = ctx.tree_descendants if r.kind == TREE_DESC else ctx.tree_height
                fn(self.trees[r.graph], mode=self.tree_mode, out=out(r), stream=stream)

    def execute(self, state, batch):
        """Runs one batch on the worker's stream and waits for it."""
        import torch
        ctx, stream = state
        with torch.cuda.stream(stream):
            self._issue(ctx, batch, stream)
        stream.synchronize()


class _Worker(threading.Thread):
    def __init__(self, server, index):
        super().__init__(daemon=True)
        self.server = server
        self.index = index
        self.state = server.backend.worker_state()
        self.inbox: queue.Queue = queue.Queue()

    def run(self):
        be = self.server.backend
        while True:
            item = self.inbox.get()
            if item is None:
                break
            batch, grow_to = item
            now = self.server.clock()
            for r in batch:
                r.t_start = now
            try:
                if grow_to:
                    be.grow(self.state, grow_to)  # charged to the budget by the scheduler
                be.execute(self.state, batch)
            except Exception as e:  # a failed batch must not poison the others
                for r in batch:
                    r.error = e
            now = self.server.clock()
            for r in batch:
                r.t_done = now
            self.server._done.put((self.index, batch))

    def close(self):
        self.inbox.put(None)
        self.join()
        self.server.backend.close_state(self.state)


class Server:
    def __init__(self, backend, workers: int = 4, budget_bytes: int | None = None, max_slots: int = 512,
                 max_batch: int = 64, keep_outputs: bool = False):
        self.backend = backend
        self.max_batch = max_batch
        self.keep_outputs = keep_outputs
        self._done: queue.Queue = queue.Queue()
        self._t0 = time.perf_counter()
        # the workers' contexts (and their pools) exist before the budget is measured
        self.workers = [_Worker(self, i) for i in range(workers)]
        self.pool = [int(backend.pool_bytes(w.state)) for w in self.workers]
        if budget_bytes is None:
            budget_bytes = backend.free_bytes() // 2
        self.admission = Admission(budget_bytes, max_slots)
        self.grows = 0
        self._ws_cache = {}
        for w in self.workers:
            w.start()

    def clock(self) -> float:
        return time.perf_counter() - self._t0

    def close(self):
        for w in self.workers:
            w.close()
        if hasattr(self.backend, "close"):
            self.backend.close()

    def _single_workspace(self, r) -> int:
        key = (r.kind, r.graph)
        if key not in self._ws_cache:
            self._ws_cache[key] = int(self.backend.workspace([r]))
        return self._ws_cache[key]

    def _fit_batch(self, wi, batch, ready):
        """Cuts `batch` until its workspace fits worker wi's pool (the cut
        requests go back to the front of `ready`).  Returns the pool size the
        worker must grow to first (0: none), or -1 when even the first request
        needs a growth the budget cannot take now (everything goes back)."""
        need = int(self.backend.workspace(batch))
        while need > self.pool[wi] and len(batch) > 1:
            ready.appendleft(batch.pop())
            need = int(self.backend.workspace(batch))
        if need <= self.pool[wi]:
            return 0
        if not self.admission.try_grow(need):  # the replaced pool stays allocated
            ready.appendleft(batch.pop())
            return -1
        self.pool[wi] = need
        self.grows += 1
        return need

    def _complete(self, wi, batch, idle):
        idle.add(wi)
        for r in batch:
            self.admission.release(r.nbytes)
            if not self.keep_outputs:
                r.out = None
        return len(batch)

    def run(self, requests, time_limit: float = 120.0):
        """Serves `requests` (sorted by t_arrive) in real time and returns them with
        admission, start and completion times filled in."""
        largest_pool = max(self.pool)
        for r in requests:
            if r.kind in TREE_KINDS:
                r.nbytes = request_bytes(r.kind, self.backend.trees[r.graph].n, 0)
            else:
                g = self.backend.graphs[r.graph]
                r.nbytes = request_bytes(r.kind, g.n, g.m)
            ws = self._single_workspace(r)
            growth = ws if ws > largest_pool else 0  # a growth holds the whole new pool
            if not self.admission.fits_ever(r.nbytes + growth):
                raise ValueError(f"request {r.rid} needs {r.nbytes + growth} bytes, more than the whole budget")
        self._t0 = time.perf_counter()
        waiting: collections.deque = collections.deque()
        ready: collections.deque = collections.deque()
        nxt, done, total = 0, 0, len(requests)
        idle = set(range(len(self.workers)))
        while done < total:
            now = self.clock()
            if now > time_limit:
                raise TimeoutError(f"served {done} of {total} requests within {time_limit} s")
            while nxt < total and requests[nxt].t_arrive <= now:
                waiting.append(requests[nxt])
                nxt += 1
            # admission, in arrival order, while memory and slots allow
            while waiting and self.admission.try_admit(waiting[0].nbytes):
                r = waiting.popleft()
                r.t_admit = now
                self.backend.allocate(r)
                ready.append(r)
            # batched on arrival: every idle worker takes what is ready now, as
            # much as its pool holds (a growth only when the budget takes it)
            while ready and idle:
                wi = max(idle, key=lambda i: self.pool[i])
                batch = [ready.popleft() for _ in range(min(self.max_batch, len(ready)))]
                grow_to = self._fit_batch(wi, batch, ready)
                if grow_to < 0:
                    if len(idle) < len(self.workers):
                        break  # waits for completions to free memory
                    # nothing runs, so nothing will free memory: the requests
                    # admitted after the first one give their outputs back
                    # (they wait again) until its pool growth fits
                    need = int(self.backend.workspace([ready[0]])) - self.pool[wi]
                    while len(ready) > 1 and self.admission.used + need > self.admission.budget:
                        r = ready.pop()
                        self.admission.release(r.nbytes)
                        r.out, r.t_admit = None, -1.0
                        waiting.appendleft(r)
                    if self.admission.used + need > self.admission.budget:
                        r = ready.popleft()  # the budget left can never take it
                        self.admission.release(r.nbytes)
                        r.out, r.error = None, MemoryError(f"request {r.rid} needs a pool growth of {need} bytes, "
                                                          "more than the budget left")
                        r.t_start = r.t_done = self.clock()
                        done += 1
                    continue
                idle.discard(wi)
                self.workers[wi].inbox.put((batch, grow_to))
            # completions free memory and slots for the next admissions
            progressed = False
            while True:
                try:
                    wi, batch = self._done.get_nowait()
                except queue.Empty:
                    break
                done += self._complete(wi, batch, idle)
                progressed = True
            if not progressed and not (ready and idle):
                wait = 0.0005
                if nxt < total:
                    wait = min(wait, max(0.0, requests[nxt].t_arrive - self.clock()))
                try:
                    wi, batch = self._done.get(timeout=wait) if wait > 0 else self._done.get_nowait()
                    done += self._complete(wi, batch, idle)
                except queue.Empty:
                    pass
        return requests


def summarize(requests, reached_edges: int | None = None) -> dict:
    lat = np.array([r.latency for r in requests]) * 1e3
    span = max(r.t_done for r in requests) - min(r.t_arrive for r in requests)
    out = {"requests": len(requests), "p50_ms": round(float(np.percentile(lat, 50)), 3),
           "p99_ms": round(float(np.percentile(lat, 99)), 3), "mean_ms": round(float(lat.mean()), 3),
           "throughput_rps": round(len(requests) / span, 1), "span_s": round(span, 3),
           "failed": sum(1 for r in requests if r.error is not None)}
    if reached_edges is not None:
        out["sssp_gteps"] = round(reached_edges / span / 1e9, 4)
    return out
