"""Plan-only mode (the workspace query a serving loop budgets with): a call on
a plan-only context enqueues nothing and records the pool bytes it would carve;
a context whose pool has exactly that size runs the real call without growing,
and a smaller one has to grow."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import say
from paper_1606_08150_amd import wc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def data(c1_graph):
    g, w = c1_graph
    dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    dw = torch.from_numpy(w.view(np.int32)).cuda()
    val = torch.from_numpy(synth.values(g.m)).cuda()
    x = torch.from_numpy(synth.vector_x(g.n)).cuda()
    t = synth.random_tree(1 << 14)
    dt = wc.DeviceTree.from_host(t.parent, t.child_ptr, t.child)
    trees = [wc.DeviceTree.from_host(s.parent, s.child_ptr, s.child) for s in synth.batch_trees(8, 4.0, 12.0)]
    return g, dg, dw, val, x, dt, trees


def calls(data):
    g, dg, dw, val, x, dt, trees = data
    out = torch.full((g.n,), -5, dtype=torch.int32, device="cuda")
    yout = torch.full((g.n,), -5.0, dtype=torch.float32, device="cuda")
    tout = torch.full((dt.n,), -5, dtype=torch.int32, device="cuda")
    cases = []
    for mode in ("flat", "wave", "block", "grid"):
        cases.append((f"sssp-{mode}", out, lambda c, m=mode: c.sssp(dg, dw, 0, mode=m, out=out)))
        cases.append((f"bfs-{mode}", out, lambda c, m=mode: c.bfs(dg, 0, mode=m, out=out)))
        cases.append((f"spmv-{mode}", yout, lambda c, m=mode: c.spmv(dg, val, x, mode=m, out=yout)))
        cases.append((f"tree-{mode}", tout, lambda c, m=mode: c.tree_descendants(dt, mode=m, out=tout)))
    out2 = torch.full((g.n,), -5, dtype=torch.int32, device="cuda")
    cases.append(("sssp-batch", out2, lambda c: c.sssp_batch([dg, dg], [dw, dw], [0, 5], outs=[out, out2])))
    cases.append(("tree-batch", tout, lambda c: c.tree_height_batch(trees, mode="grid")))
    return cases


def test_plan_only_enqueues_nothing_and_the_plan_is_exact(data):
    probe = wc.Context(0, pool_bytes=1 << 20)
    try:
        for name, sentinel, fn in calls(data):
            sentinel.fill_(-5)  # the previous case's real call wrote its output
            torch.cuda.synchronize()
            need = probe.workspace_bytes(fn)
            torch.cuda.synchronize()
            say(f"plan {name}: {need} bytes")
            assert need > 0, name
            # nothing ran: the output still holds its fill value
            assert (sentinel.cpu().numpy() == -5).all(), name
            exact = wc.Context(0, pool_bytes=need)
            try:
                fn(exact)
                torch.cuda.synchronize()
                assert exact.pool_info() == (need, 0), name
            finally:
                exact.close()
            if need > 8192:
                small = wc.Context(0, pool_bytes=need - 4096)
                try:
                    fn(small)
                    torch.cuda.synchronize()
                    assert small.pool_info()[1] == 1, name
                finally:
                    small.close()
    finally:
        probe.close()


def test_reserve_grows_once(data):
    c = wc.Context(0, pool_bytes=1 << 20)
    try:
        assert c.pool_info() == (1 << 20, 0)
        c.reserve(1 << 10)
        assert c.pool_info() == (1 << 20, 0)
        c.reserve(3 << 20)
        assert c.pool_info() == (3 << 20, 1)
    finally:
        c.close()


def test_growth_while_calls_are_in_flight_on_other_streams():
    """A growth does not wait for the device: calls still in flight keep the
    replaced pool, which the context retires and releases when it next drains
    the device.  One context with a 64 KiB pool; products and SSSP calls on
    graphs of increasing size issued alternately on two side streams, each
    stream ordered after the other's work (calls sharing a context must be
    serialized) but with no host synchronization, so a call can grow the pool
    while the one before still runs; every result matches the oracle."""
    import oracle
    from gpu_util import dev_to_u32, f32_to_dev, u32_to_dev
    cases = []
    for k, scale in enumerate((9, 11, 13, 15)):
        g = synth.rmat_csr(scale, 16 << scale, seed=700 + k)
        w = synth.weights(g.m, seed=710 + k)
        val, x = synth.values(g.m, seed=720 + k), synth.vector_x(g.n, seed=730 + k)
        y_ref, b = oracle.spmv_f64(g.row_ptr, g.col, val, x)
        d_ref = oracle.sssp_dijkstra(g.row_ptr, g.col, w, 0)
        dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
        cases.append(dict(dg=dg, dw=u32_to_dev(w), dv=f32_to_dev(val), dx=f32_to_dev(x),
                          y=torch.full((g.n,), -5.0, dtype=torch.float32, device="cuda"),
                          d=torch.full((g.n,), -5, dtype=torch.int32, device="cuda"), y_ref=y_ref, b=b, d_ref=d_ref))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    c = wc.Context(0, pool_bytes=1 << 16)
    try:
        say("growth: 4 products and 4 SSSP calls of growing size on two streams, no sync between them")
        cur = 0
        for k, cs in enumerate(cases):
            for call in (lambda s: c.spmv(cs["dg"], cs["dv"], cs["dx"], mode="grid", out=cs["y"], stream=s),
                         lambda s: c.sssp(cs["dg"], cs["dw"], 0, mode="wave", out=cs["d"], stream=s)):
                nxt = 1 - cur
                streams[nxt].wait_stream(streams[cur])  # serialized on the device, not on the host
                call(streams[nxt])
                cur = nxt
        torch.cuda.synchronize()
        for k, cs in enumerate(cases):
            assert oracle.spmv_check(cs["y_ref"], cs["b"], cs["y"].cpu().numpy()) == (0, -1), k
            assert np.array_equal(dev_to_u32(cs["d"]), cs["d_ref"]), k
        assert c.pool_info()[1] >= 3
    finally:
        c.close()
