"""GPU parity of the batched tree calls (wc_tree_descendants_batch,
wc_tree_height_batch): many trees of uneven size in one sequence of level
launches, each tree's result bit-exact against the oracle, in flat and grid
modes, with the graph replay of repeated calls, a changed batch, and the
refusals."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import say
from paper_1606_08150_amd import wc

pytestmark = pytest.mark.gpu


def dev(t):
    return wc.DeviceTree.from_host(t.parent, t.child_ptr, t.child)


@pytest.fixture(scope="module")
def forest():
    trees = synth.batch_trees(48, 4.0, 14.0)
    trees += [synth.tree_from_parent([-1]), synth.chain_tree(400), synth.star_tree(5000), synth.kary_tree(3, 7),
              synth.layered_tree(2, 32, 128, seed=9)]
    refs = [(oracle.tree_descendants(t.child_ptr, t.child), oracle.tree_height(t.child_ptr, t.child)) for t in trees]
    return trees, refs


def check(outs, refs, k):
    for i, (o, r) in enumerate(zip(outs, refs)):
        assert np.array_equal(o.cpu().numpy(), r[k]), f"tree {i}"


@pytest.mark.parametrize("mode", ["flat", "grid"])
def test_batch_equals_oracle(ctx, forest, mode):
    trees, refs = forest
    dts = [dev(t) for t in trees]
    for tune in (None, wc.make_tune(block_threads=64, items_per_lane=1), wc.make_tune(block_threads=1024),
                 wc.make_tune(grid_blocks=3)):
        say(f"tree batch of {len(trees)} mode={mode} tune={tune.as_dict() if tune else None}")
        d = ctx.tree_descendants_batch(dts, mode=mode, tune=tune)
        h = ctx.tree_height_batch(dts, mode=mode, tune=tune)
        torch.cuda.synchronize()
        check(d, refs, 0)
        check(h, refs, 1)


def test_repeated_batch_replays_and_a_changed_batch(ctx, forest):
    trees, refs = forest
    dts = [dev(t) for t in trees]
    outs = [torch.empty(t.n, dtype=torch.int32, device="cuda") for t in trees]
    for rep in range(4):
        for o in outs:
            o.fill_(-7)
        ctx.tree_descendants_batch(dts, mode="grid", outs=outs)
        torch.cuda.synchronize()
        check(outs, refs, 0)
    # the same output arrays with a deeper tree swapped in: the recorded graph
    # must not be taken for it
    deep = synth.chain_tree(trees[0].n)
    dts2 = [dev(deep)] + dts[1:]
    ctx.tree_descendants_batch(dts2, mode="grid", outs=outs)
    torch.cuda.synchronize()
    assert np.array_equal(outs[0].cpu().numpy(), oracle.tree_descendants(deep.child_ptr, deep.child))
    check(outs[1:], refs[1:], 0)


def test_stats_levels_and_dispatches(ctx, forest):
    trees, refs = forest
    dts = [dev(t) for t in trees]
    _, st = ctx.tree_height_batch(dts, mode="grid", stats=True)
    depth = max(int(r[1][0]) for r in refs)
    assert st["rounds"] == depth + 1 or st["rounds"] == depth
    assert st["dispatches"] == st["rounds"]
    assert st["edges_processed"] == sum(t.n - 1 for t in trees)


def test_refusals(ctx, forest):
    trees, _ = forest
    dts = [dev(t) for t in trees[:3]]
    for mode, tune in (("wave", None), ("block", None), ("grid", wc.make_tune(driver=2))):
        with pytest.raises(wc.WcError) as ei:
            ctx.tree_descendants_batch(dts, mode=mode, tune=tune)
        assert ei.value.status == -1
    assert ctx.tree_descendants_batch([], mode="grid") == []


def test_full_size_batch(ctx):
    """64 random trees of 2^10..2^18 nodes (about 2^22 nodes in total)."""
    trees = synth.batch_trees(64, 10.0, 18.0, seed=17)
    say(f"tree batch of 64, {sum(t.n for t in trees)} nodes")
    dts = [dev(t) for t in trees]
    d = ctx.tree_descendants_batch(dts, mode="grid")
    h = ctx.tree_height_batch(dts, mode="grid")
    torch.cuda.synchronize()
    for i, t in enumerate(trees):
        assert np.array_equal(d[i].cpu().numpy(), oracle.tree_descendants(t.child_ptr, t.child)), i
        assert np.array_equal(h[i].cpu().numpy(), oracle.tree_height(t.child_ptr, t.child)), i
