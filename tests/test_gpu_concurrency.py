"""Two libwc contexts driven from two host threads on two streams at once
(coloring and PageRank, SSSP and tree heights): every result equals the
oracle's, as when the calls run alone.  Each context owns its pool and its
host-published round counts, so concurrent calls must not interfere."""
import threading

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev_to_u32, say, u32_to_dev
from paper_1606_08150_amd import wc
from tolerance import pagerank_rtol

pytestmark = pytest.mark.gpu


def run_pair(job_a, job_b):
    errors = []

    def wrap(job):
        try:
            job()
        except Exception as e:  # reported on the main thread
            errors.append(e)
    ts = [threading.Thread(target=wrap, args=(j,)) for j in (job_a, job_b)]
    for t in ts:
        t.start()
    for t in ts:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in ts), "a concurrent call did not finish"
    if errors:
        raise errors[0]


def test_coloring_and_pagerank_concurrently(c1_graph):
    g, _ = c1_graph
    sg = synth.symmetrize(g)
    prio = synth.priorities(sg.n)
    ref_c, _ = oracle.color_jp(sg.row_ptr, sg.col, prio)
    tg = synth.transpose(g)
    od = synth.out_degree(g)
    ref_r = oracle.pagerank_f64(tg.row_ptr, tg.col, od, 20)
    dsg = wc.DeviceCSR.from_host(sg.row_ptr, sg.col)
    dp = u32_to_dev(prio)
    dtg = wc.DeviceCSR.from_host(tg.row_ptr, tg.col)
    dod = torch.from_numpy(od).cuda()
    ctx_a, ctx_b = wc.Context(0), wc.Context(0)
    s_a, s_b = torch.cuda.Stream(), torch.cuda.Stream()
    out = {}

    def color_job():
        with torch.cuda.stream(s_a):
            for mode in ("grid", "block", "wave", "grid"):
                c = ctx_a.color(dsg, dp, mode=mode, stream=s_a)
                s_a.synchronize()
                out.setdefault("color", []).append(c.cpu().numpy())

    def pagerank_job():
        with torch.cuda.stream(s_b):
            for mode in ("grid", "flat", "grid"):
                r = ctx_b.pagerank(dtg, dod, 20, mode=mode, stream=s_b)
                s_b.synchronize()
                out.setdefault("rank", []).append(r.cpu().numpy())

    say("coloring and PageRank on two contexts and two streams")
    run_pair(color_job, pagerank_job)
    torch.cuda.synchronize()
    for c in out["color"]:
        assert np.array_equal(c, ref_c)
    rtol = max(pagerank_rtol(20, np.diff(tg.row_ptr), mode, tg.n) for mode in ("grid", "flat"))
    for r in out["rank"]:
        assert oracle.pagerank_check(ref_r, r, rtol) == (0, -1)
    ctx_a.close()
    ctx_b.close()


def test_sssp_and_tree_heights_concurrently(c1_graph):
    g, w = c1_graph
    ref_d = oracle.sssp_dijkstra(g.row_ptr, g.col, w, 0)
    t = synth.random_tree(1 << 16)
    ref_h = oracle.tree_height(t.child_ptr, t.child)
    dg = wc.DeviceCSR.from_host(g.row_ptr, g.col)
    dw = u32_to_dev(w)
    dt = wc.DeviceTree.from_host(t.parent, t.child_ptr, t.child)
    ctx_a, ctx_b = wc.Context(0), wc.Context(0)
    s_a, s_b = torch.cuda.Stream(), torch.cuda.Stream()
    out = {}

    def sssp_job():
        with torch.cuda.stream(s_a):
            for mode in ("grid", "block", "grid", "wave"):
                d = ctx_a.sssp(dg, dw, 0, mode=mode, stream=s_a)
                s_a.synchronize()
                out.setdefault("dist", []).append(dev_to_u32(d))

    def tree_job():
        with torch.cuda.stream(s_b):
            for mode in ("grid", "grid", "block", "flat"):
                h = ctx_b.tree_height(dt, mode=mode, stream=s_b)
                s_b.synchronize()
                out.setdefault("height", []).append(h.cpu().numpy())

    say("SSSP and tree heights on two contexts and two streams")
    run_pair(sssp_job, tree_job)
    torch.cuda.synchronize()
    for d in out["dist"]:
        assert np.array_equal(d, ref_d)
    for h in out["height"]:
        assert np.array_equal(h, ref_h)
    ctx_a.close()
    ctx_b.close()
