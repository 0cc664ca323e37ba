"""Repeat runs that would expose races: 100 calls per mode issued back to back
on one stream, with no host synchronization between them and each into its own
output, all compared afterwards: SSSP against the oracle's distances, SpMV
bitwise against its first result (and that one within the tolerance of the
binary64 product), recursive BFS against the oracle's levels, and tree
descendants in the packet-queue modes against the oracle.  Coloring (whose
calls wait for each round's count, but not for the call's last kernels) runs
25 calls per mode the same way."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev_to_u32, f32_to_dev, say, u32_to_dev
from paper_1606_08150_amd import wc

pytestmark = pytest.mark.gpu
MODES = ["flat", "wave", "block", "grid"]
REPS = 100


@pytest.mark.parametrize("mode", MODES)
def test_sssp_and_spmv_back_to_back(ctx, c1_graph, mode):
    g, w = c1_graph
    dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    dw = u32_to_dev(np.asarray(w, np.uint32))
    ref = oracle.sssp_dijkstra(g.row_ptr, g.col, np.asarray(w, np.uint32), 0)
    val, x = synth.values(g.m), synth.vector_x(g.n)
    y_ref, b = oracle.spmv_f64(g.row_ptr, g.col, val, x)
    dv, dx = f32_to_dev(val), f32_to_dev(x)
    say(f"races: {REPS} SSSP and {REPS} SpMV calls back to back, mode={mode}")
    dists = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in range(REPS)]
    ys = [torch.empty(g.n, dtype=torch.float32, device="cuda") for _ in range(REPS)]
    for k in range(REPS):
        ctx.sssp(dg, dw, 0, mode=mode, out=dists[k])
        ctx.spmv(dg, dv, dx, mode=mode, out=ys[k])
    torch.cuda.synchronize()
    for k in range(REPS):
        assert np.array_equal(dev_to_u32(dists[k]), ref), k
    y0 = ys[0].cpu().numpy()
    assert oracle.spmv_check(y_ref, b, y0)[0] == 0
    for k in range(1, REPS):
        assert np.array_equal(ys[k].cpu().numpy().view(np.uint32), y0.view(np.uint32)), k


@pytest.mark.parametrize("mode", ["wave", "block"])
def test_queue_modes_back_to_back(ctx, c1_graph, mode):
    g, _ = c1_graph
    dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    ref = oracle.bfs(g.row_ptr, g.col, 0)
    t = synth.random_tree(1 << 14, seed=12)
    dt = wc.DeviceTree.from_host(t.parent, t.child_ptr, t.child)
    dref = oracle.tree_descendants(t.child_ptr, t.child)
    say(f"races: {REPS} recursive BFS and {REPS} tree calls back to back, mode={mode}")
    levels = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in range(REPS)]
    descs = [torch.empty(t.n, dtype=torch.int32, device="cuda") for _ in range(REPS)]
    for k in range(REPS):
        ctx.bfs(dg, 0, mode=mode, out=levels[k])
        ctx.tree_descendants(dt, mode=mode, out=descs[k])
    torch.cuda.synchronize()
    for k in range(REPS):
        assert np.array_equal(dev_to_u32(levels[k]), ref), k
        assert np.array_equal(descs[k].cpu().numpy(), dref), k


@pytest.mark.parametrize("mode", MODES)
def test_coloring_back_to_back(ctx, c1_graph, mode):
    g = synth.symmetrize(c1_graph[0])
    p = synth.priorities(g.n)
    ref, _ = oracle.color_jp(g.row_ptr, g.col, p)
    dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    dp = u32_to_dev(p)
    say(f"races: {REPS // 4} coloring calls back to back, mode={mode}")
    outs = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in range(REPS // 4)]
    for o in outs:
        ctx.color(dg, dp, mode=mode, out=o)
    torch.cuda.synchronize()
    for k, o in enumerate(outs):
        assert np.array_equal(o.cpu().numpy(), ref), k
