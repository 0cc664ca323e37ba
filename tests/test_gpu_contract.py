"""GPU tests of the status contract of include/wc.h.

* Back-to-back calls on one context with no synchronization in between: the
  rounds a call enqueues past its last one with work publish their (empty)
  round counts after the next call has started; those values carry the earlier
  call's epoch and must never end the next call early.
* A device-side wait that gives up is reported as WC_ETIMEOUT with or without
  stats: the wait bound is shortened from the host (wc_ctx_set_wait_limit) so
  that the packet-queue waves give up, and every kernel still exits normally.
* Refused calls enqueue nothing: with per-kernel timing on, a refused call
  leaves no kernel record.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev_to_u32, say, u32_to_dev
from paper_1606_08150_amd import wc

pytestmark = pytest.mark.gpu
MODES = ["flat", "wave", "block", "grid"]


def dev_tree(t):
    return wc.DeviceTree.from_host(t.parent, t.child_ptr, t.child)


@pytest.mark.parametrize("mode", MODES)
def test_back_to_back_calls_without_sync(ctx, c1_graph, mode):
    g, w = c1_graph
    dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    dw = u32_to_dev(w)
    deg = np.diff(g.row_ptr)
    sink = int(np.flatnonzero(deg == 0)[0])  # a source without out-edges: one round with work
    ref_sink = oracle.sssp_dijkstra(g.row_ptr, g.col, w, sink)
    ref_0 = oracle.sssp_dijkstra(g.row_ptr, g.col, w, 0)
    star = synth.star_tree(3000)
    rt = synth.random_tree(1 << 14, seed=7)
    dstar, drt = dev_tree(star), dev_tree(rt)
    ref_star = oracle.tree_height(star.child_ptr, star.child)
    ref_rt = oracle.tree_height(rt.child_ptr, rt.child)
    sg = synth.symmetrize(g)
    pr = synth.priorities(sg.n)
    dsg = wc.DeviceCSR.from_host(sg.row_ptr, sg.col)
    dpr = u32_to_dev(pr)
    ref_col = oracle.color_jp(sg.row_ptr, sg.col, pr)[0]
    say(f"back-to-back calls without synchronization, mode={mode}")
    torch.cuda.synchronize()
    outs = []
    for rep in range(3):
        a = ctx.sssp(dg, dw, sink, mode=mode)
        b = ctx.sssp(dg, dw, 0, mode=mode)
        c = ctx.tree_height(dstar, mode=mode)
        d = ctx.tree_height(drt, mode=mode)
        e = ctx.color(dsg, dpr, mode=mode)
        f = ctx.bfs(dg, sink, mode=mode)
        h = ctx.sssp(dg, dw, 0, mode=mode)
        outs.append((a, b, c, d, e, f, h))
    torch.cuda.synchronize()
    ref_bfs = oracle.bfs(g.row_ptr, g.col, sink)
    for a, b, c, d, e, f, h in outs:
        assert np.array_equal(dev_to_u32(a), ref_sink)
        assert np.array_equal(dev_to_u32(b), ref_0)
        assert np.array_equal(c.cpu().numpy(), ref_star)
        assert np.array_equal(d.cpu().numpy(), ref_rt)
        assert np.array_equal(e.cpu().numpy(), ref_col)
        assert np.array_equal(dev_to_u32(f), ref_bfs)
        assert np.array_equal(dev_to_u32(h), ref_0)


def test_back_to_back_batches_without_sync(ctx):
    inst = synth.batch_instances(24, lo_log2=8, hi_log2=12)
    graphs, weights = [g for g, _ in inst], [w for _, w in inst]
    dgs = [wc.DeviceCSR.from_host(g.row_ptr, g.col) for g in graphs]
    dws = [u32_to_dev(w) for w in weights]
    sinks = [int(np.flatnonzero(np.diff(g.row_ptr) == 0)[0]) if np.any(np.diff(g.row_ptr) == 0) else 0
             for g in graphs]
    refs_sink = [oracle.sssp_dijkstra(g.row_ptr, g.col, w, s) for g, w, s in zip(graphs, weights, sinks)]
    refs_0 = [oracle.sssp_dijkstra(g.row_ptr, g.col, w, 0) for g, w in zip(graphs, weights)]
    say("batched SSSP back to back without synchronization")
    torch.cuda.synchronize()
    runs = []
    for graph_rounds in (0, 3, 0):
        runs.append((ctx.sssp_batch(dgs, dws, sinks, graph_rounds=graph_rounds),
                     ctx.sssp_batch(dgs, dws, [0] * len(dgs), graph_rounds=graph_rounds)))
    torch.cuda.synchronize()
    for a, b in runs:
        for i in range(len(graphs)):
            assert np.array_equal(dev_to_u32(a[i]), refs_sink[i]), i
            assert np.array_equal(dev_to_u32(b[i]), refs_0[i]), i


def chain(n):
    return synth.chain_tree(n)


@pytest.mark.parametrize("mode", ["wave", "block"])
@pytest.mark.parametrize("stats", [False, True])
def test_queue_wait_timeout_is_reported(mode, stats):
    """With a 1 microsecond bound, waves that take a ticket before its packet is
    published give up at once; a chain tree publishes its packets one after
    another, so some wave does.  The call must say so, without stats too."""
    c = wc.Context(0)
    t = chain(3000)
    dt = dev_tree(t)
    ref = oracle.tree_descendants(t.child_ptr, t.child)
    try:
        c.set_wait_limit(1)
        say(f"tree queue with a 1 us wait bound, mode={mode} stats={stats}")
        with pytest.raises(wc.WcError) as ei:
            c.tree_descendants(dt, mode=mode, stats=stats)
        assert ei.value.status == -4
        torch.cuda.synchronize()
        c.set_wait_limit(0)  # back to the default bound: the same call completes
        got = c.tree_descendants(dt, mode=mode, stats=stats)
        torch.cuda.synchronize()
        got = got[0] if stats else got
        assert np.array_equal(got.cpu().numpy(), ref)
    finally:
        c.close()


def test_refused_calls_enqueue_nothing(c1_graph):
    g, w = c1_graph
    c = wc.Context(0)
    dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    dw = u32_to_dev(w)
    x = torch.zeros(g.n, dtype=torch.float32, device="cuda")
    val = torch.ones(g.m, dtype=torch.float32, device="cuda")
    t = synth.random_tree(1 << 12, seed=3)
    dt = dev_tree(t)
    od = torch.from_numpy(synth.out_degree(g)).cuda()
    sg = synth.symmetrize(g)
    dsg = wc.DeviceCSR.from_host(sg.row_ptr, sg.col)
    dpr = u32_to_dev(synth.priorities(sg.n))
    calls = []
    for mode in MODES:
        calls += [
            (f"sssp {mode} driver 1", lambda m=mode: c.sssp(dg, dw, 0, mode=m, tune=wc.make_tune(driver=1))),
            (f"bfs {mode} driver 1", lambda m=mode: c.bfs(dg, 0, mode=m, tune=wc.make_tune(driver=1))),
            (f"spmv {mode} driver 1", lambda m=mode: c.spmv(dg, val, x, mode=m, tune=wc.make_tune(driver=1))),
            (f"pagerank {mode} driver 1", lambda m=mode: c.pagerank(dg, od, 2, mode=m, tune=wc.make_tune(driver=1))),
            (f"color {mode} driver 1", lambda m=mode: c.color(dsg, dpr, mode=m, tune=wc.make_tune(driver=1))),
            (f"td {mode} driver 1", lambda m=mode: c.tree_descendants(dt, mode=m, tune=wc.make_tune(driver=1))),
            (f"th {mode} driver 1", lambda m=mode: c.tree_height(dt, mode=m, tune=wc.make_tune(driver=1))),
            (f"sssp batch {mode} driver 1", lambda m=mode: c.sssp_batch([dg], [dw], [0], modes=[m],
                                                                        tunes=[wc.make_tune(driver=1)])),
        ]
        if mode != "grid":
            calls += [
                (f"sssp {mode} driver 2", lambda m=mode: c.sssp(dg, dw, 0, mode=m, tune=wc.make_tune(driver=2))),
                (f"spmv {mode} driver 2", lambda m=mode: c.spmv(dg, val, x, mode=m, tune=wc.make_tune(driver=2))),
                (f"td {mode} driver 2", lambda m=mode: c.tree_descendants(dt, mode=m, tune=wc.make_tune(driver=2))),
            ]
    calls += [("sssp bad source", lambda: c.sssp(dg, dw, g.n, mode="grid")),
              ("td driver 3", lambda: c.tree_descendants(dt, mode="grid", tune=wc.make_tune(driver=3)))]
    try:
        c.set_timing(True)
        for name, call in calls:
            say(f"refused: {name}")
            with pytest.raises(wc.WcError) as ei:
                call()
            assert ei.value.status == -1, name
            assert c.kernel_records() == [], name
        torch.cuda.synchronize()
    finally:
        c.set_timing(False)
        c.close()
