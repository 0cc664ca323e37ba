"""Continuous batching on the GPU: every request's result is the same alone and
in the mix (SSSP and tree results bit-identical and equal to the oracle; SpMV
bit-identical to the same call alone and within the 1e-5 bound of the
oracle)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import say
from paper_1606_08150_amd import serve, wc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def resident():
    sizes = synth.serving_graph_sizes(6, 10, 13)
    host, dev = [], []
    for k, n in enumerate(sizes):
        g, w, val, xs = synth.serving_graph(k, n, n_x=2)
        host.append((g, w, val, xs))
        dev.append(serve.ResidentGraph(wc.DeviceCSR.from_host(g.row_ptr, g.col),
                                       torch.from_numpy(w.view(np.int32)).cuda(), torch.from_numpy(val).cuda(),
                                       [torch.from_numpy(x).cuda() for x in xs]))
    trees = [synth.random_tree(3000, seed=31), synth.random_tree(20000, seed=32)]
    dtrees = [wc.DeviceTree.from_host(t.parent, t.child_ptr, t.child) for t in trees]
    return host, dev, trees, dtrees


def test_results_same_alone_and_in_the_mix(ctx, resident):
    host, dev, trees, dtrees = resident
    srcs = [np.flatnonzero(np.diff(g.row_ptr) > 0) for g, _, _, _ in host]
    reqs = serve.poisson_requests(240, 20000.0, srcs, n_x=2, seed=9, tree_fraction=0.25, n_trees=len(trees))
    assert any(r.kind in serve.TREE_KINDS for r in reqs)
    say(f"serving {len(reqs)} requests")
    be = serve.GpuBackend(dev, trees=dtrees, pool_bytes=64 << 10)
    srv = serve.Server(be, workers=3, budget_bytes=64 << 20, max_slots=48, max_batch=16, keep_outputs=True)
    try:
        out = srv.run(reqs, time_limit=60)
        # every pool growth went through admission (64 KiB pools: single requests need more)
        assert sum(be.pool_grows(w.state) for w in srv.workers) == srv.grows >= 1
    finally:
        srv.close()
    assert all(r.error is None for r in out)
    assert srv.admission.peak_used <= 64 << 20
    for r in out:
        if r.kind in serve.TREE_KINDS:
            t = trees[r.graph]
            fn = ctx.tree_descendants if r.kind == serve.TREE_DESC else ctx.tree_height
            alone = fn(dtrees[r.graph], mode="grid")
            torch.cuda.synchronize()
            mixed = r.out.cpu().numpy()
            assert np.array_equal(mixed, alone.cpu().numpy()), r.rid
            ref = (oracle.tree_descendants if r.kind == serve.TREE_DESC else oracle.tree_height)(t.child_ptr, t.child)
            assert np.array_equal(mixed, ref), r.rid
            continue
        g, w, val, xs = host[r.graph]
        d = dev[r.graph]
        if r.kind == serve.SSSP:
            alone = ctx.sssp(d.csr, d.w, r.arg, mode="grid")
            torch.cuda.synchronize()
            mixed = r.out.cpu().numpy().view(np.uint32)
            assert np.array_equal(mixed, alone.cpu().numpy().view(np.uint32)), r.rid
            assert np.array_equal(mixed, oracle.sssp_dijkstra(g.row_ptr, g.col, w, r.arg)), r.rid
        else:
            alone = ctx.spmv(d.csr, d.val, d.xs[r.arg], mode="grid")
            torch.cuda.synchronize()
            mixed = r.out.cpu().numpy()
            assert np.array_equal(mixed.view(np.uint32), alone.cpu().numpy().view(np.uint32)), r.rid
            y_ref, b = oracle.spmv_f64(g.row_ptr, g.col, val, xs[r.arg])
            assert oracle.spmv_check(y_ref, b, mixed) == (0, -1), r.rid
    s = serve.summarize(out)
    say(f"serving summary {s}")
    assert s["failed"] == 0


def test_full_resident_set_under_load(ctx):
    """The full serving configuration (64 resident graphs of 2^14..2^20 vertices,
    4 x vectors each) at a rate above saturation: every SSSP result passes the
    shortest-path certificate and every SpMV result the 1e-5 bound."""
    sizes = synth.serving_graph_sizes(64, 14, 20)
    say(f"generating 64 resident graphs ({sum(sizes)} vertices)")
    host, dev = [], []
    for k, n in enumerate(sizes):
        g, w, val, xs = synth.serving_graph(k, n, n_x=4)
        host.append((g, w, val, xs))
        dev.append(serve.ResidentGraph(wc.DeviceCSR.from_host(g.row_ptr, g.col),
                                       torch.from_numpy(w.view(np.int32)).cuda(), torch.from_numpy(val).cuda(),
                                       [torch.from_numpy(x).cuda() for x in xs]))
    srcs = [np.flatnonzero(np.diff(g.row_ptr) > 0) for g, _, _, _ in host]
    reqs = serve.poisson_requests(300, 20000.0, srcs, n_x=4, seed=21)
    say(f"serving {len(reqs)} requests on the full resident set")
    be = serve.GpuBackend(dev)
    srv = serve.Server(be, workers=4, max_slots=512, max_batch=64, keep_outputs=True)
    try:
        out = srv.run(reqs, time_limit=120)
        assert sum(be.pool_grows(w.state) for w in srv.workers) == srv.grows
        assert srv.admission.peak_used <= srv.admission.budget
    finally:
        srv.close()
    assert all(r.error is None for r in out)
    for r in out:
        g, w, val, xs = host[r.graph]
        if r.kind == serve.SSSP:
            d = r.out.cpu().numpy().view(np.uint32)
            assert oracle.sssp_certify(g.row_ptr, g.col, w, r.arg, d) == (0, -1), r.rid
        else:
            y_ref, b = oracle.spmv_f64(g.row_ptr, g.col, val, xs[r.arg])
            assert oracle.spmv_check(y_ref, b, r.out.cpu().numpy()) == (0, -1), r.rid
    del dev
    torch.cuda.empty_cache()
