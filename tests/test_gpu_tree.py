"""GPU parity of wc_tree_descendants / wc_tree_height against the oracle
(bit-exact), every mode and driver, special shapes, and the 2^22-node tree."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import say
from paper_1606_08150_amd import wc

pytestmark = pytest.mark.gpu
MODES = ["flat", "wave", "block", "grid"]


def run(ctx, t, what, mode, stats=False, **tune):
    dt = wc.DeviceTree.from_host(t.parent, t.child_ptr, t.child)
    tt = wc.make_tune(**tune) if tune else None
    say(f"tree {what} n={t.n} mode={mode} tune={tune}")
    fn = ctx.tree_descendants if what == "desc" else ctx.tree_height
    res = fn(dt, mode=mode, tune=tt, stats=stats)
    torch.cuda.synchronize()
    if stats:
        return res[0].cpu().numpy(), res[1]
    return res.cpu().numpy()


@pytest.fixture(scope="module")
def small_tree():
    t = synth.random_tree(1 << 16, seed=5)
    return t, oracle.tree_descendants(t.child_ptr, t.child), oracle.tree_height(t.child_ptr, t.child)


@pytest.mark.parametrize("mode", MODES)
def test_random_tree_all_modes(ctx, small_tree, mode):
    t, d, h = small_tree
    assert np.array_equal(run(ctx, t, "desc", mode), d)
    assert np.array_equal(run(ctx, t, "height", mode), h)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("tune", [dict(block_threads=64), dict(block_threads=1024), dict(items_per_lane=1),
                                  dict(items_per_lane=16), dict(grid_blocks=2),
                                  dict(block_threads=128, items_per_lane=2)])
def test_tune_sweep(ctx, small_tree, mode, tune):
    t, d, h = small_tree
    assert np.array_equal(run(ctx, t, "desc", mode, **tune), d)
    assert np.array_equal(run(ctx, t, "height", mode, **tune), h)


def shapes():
    yield "root_only", synth.tree_from_parent([-1])
    yield "pair", synth.tree_from_parent([-1, 0])
    yield "chain", synth.chain_tree(300)
    yield "star", synth.star_tree(10000)
    yield "kary2", synth.kary_tree(2, 12)
    yield "kary7", synth.kary_tree(7, 4)
    yield "wide_fanout", synth.random_tree(20000, seed=77, kmax=4096, alpha=1.2)
    yield "narrow", synth.random_tree(20000, seed=78, kmax=3, alpha=0.5, max_depth=1 << 20)
    # fixed-depth trees in the manner of the paper's tree sets (Sec. V)
    yield "layered_half", synth.layered_tree(3, 8, 16, 0.5, seed=79)
    yield "layered_full", synth.layered_tree(2, 128, 256, 1.0, seed=80)


@pytest.mark.parametrize("mode", MODES)
def test_shapes(ctx, mode):
    for name, t in shapes():
        d = oracle.tree_descendants(t.child_ptr, t.child)
        h = oracle.tree_height(t.child_ptr, t.child)
        for tune in (dict(), dict(block_threads=64, items_per_lane=1)):
            assert np.array_equal(run(ctx, t, "desc", mode, **tune), d), (name, tune)
            assert np.array_equal(run(ctx, t, "height", mode, **tune), h), (name, tune)


def test_persistent_driver_is_refused(ctx, small_tree):
    t, _, _ = small_tree
    with pytest.raises(wc.WcError) as ei:
        run(ctx, t, "desc", "grid", driver=1)
    assert ei.value.status == -1
    torch.cuda.synchronize()


def test_basic_driver_emulates_per_node_children(ctx, small_tree):
    """Driver 2 (basic dynamic parallelism emulated: one host-launched child
    kernel per internal node, deepest first) gives the oracle's results with one
    launch per internal node."""
    t, d, h = small_tree
    internal = int((np.diff(t.child_ptr) > 0).sum())
    got, st = run(ctx, t, "desc", "grid", stats=True, driver=2)
    assert np.array_equal(got, d) and st["dispatches"] == internal
    assert np.array_equal(run(ctx, t, "height", "grid", driver=2), h)
    # a chain: one launch per node but the last, each after its child
    ch = synth.chain_tree(300)
    assert np.array_equal(run(ctx, ch, "desc", "grid", driver=2), oracle.tree_descendants(ch.child_ptr, ch.child))
    assert np.array_equal(run(ctx, ch, "height", "grid", driver=2), oracle.tree_height(ch.child_ptr, ch.child))
    with pytest.raises(wc.WcError):
        run(ctx, t, "desc", "block", driver=2)
    with pytest.raises(wc.WcError):
        run(ctx, t, "desc", "grid", driver=3)
    torch.cuda.synchronize()


def test_bookkeeping(ctx, small_tree):
    t, d, h = small_tree
    internal = int((np.diff(t.child_ptr) > 0).sum())
    for mode in ("wave", "block", "grid"):
        _, st = run(ctx, t, "desc", mode, stats=True)
        # every recursive call below the root is buffered exactly once
        assert st["items_buffered"] == internal - 1, mode
        assert st["edges_processed"] == t.n - 1, mode
    _, st = run(ctx, t, "desc", "grid", stats=True)
    assert st["dispatches"] == h[0] and st["rounds"] == h[0]
    _, st = run(ctx, t, "desc", "wave", stats=True)
    assert internal / 64 <= st["dispatches"] <= internal
    _, st = run(ctx, t, "desc", "flat", stats=True)
    assert st["items_buffered"] == 0


def test_flush_cuts_packets_by_children(ctx):
    """A queue-mode flush cuts the group's buffered nodes into packets of about
    work_cap children (64 * items_per_lane for a wave) published together: on a
    wide layered tree (every internal node has 128..256 children) a 64-child cap
    makes every node a packet of its own, so the dispatches are exactly the
    internal nodes, and a larger cap packs one or two nodes per packet."""
    t = synth.layered_tree(3, 128, 256, 0.5, seed=81)
    d = oracle.tree_descendants(t.child_ptr, t.child)
    h = oracle.tree_height(t.child_ptr, t.child)
    internal = int((np.diff(t.child_ptr) > 0).sum())
    for mode in ("wave", "block"):
        for tune in (dict(), dict(items_per_lane=1), dict(block_threads=1024), dict(block_threads=64, items_per_lane=64)):
            got, st = run(ctx, t, "desc", mode, stats=True, **tune)
            assert np.array_equal(got, d), (mode, tune)
            assert st["items_buffered"] == internal - 1, (mode, tune)
            assert np.array_equal(run(ctx, t, "height", mode, **tune), h), (mode, tune)
    _, st = run(ctx, t, "desc", "wave", stats=True, items_per_lane=1)
    assert st["dispatches"] == internal
    _, st = run(ctx, t, "desc", "wave", stats=True, items_per_lane=4)
    assert internal / 2 <= st["dispatches"] <= internal


def test_repeat_runs_queue_modes(ctx, small_tree):
    t, d, h = small_tree
    for _ in range(10):
        for mode in ("wave", "block"):
            assert np.array_equal(run(ctx, t, "desc", mode), d)


@pytest.fixture(scope="module")
def c3_tree():
    say("generating 2^22-node tree")
    t = synth.random_tree(1 << 22)
    return t, oracle.tree_descendants(t.child_ptr, t.child), oracle.tree_height(t.child_ptr, t.child)


@pytest.mark.parametrize("mode", MODES)
def test_2p22_tree_bit_exact(ctx, c3_tree, mode):
    t, d, h = c3_tree
    assert np.array_equal(run(ctx, t, "desc", mode), d)
    assert np.array_equal(run(ctx, t, "height", mode), h)


def deep_tree(n, depth):
    """A chain of `depth` edges from the root, every other node a child of the root."""
    parent = [-1] + list(range(depth)) + [0] * (n - depth - 1)
    return synth.tree_from_parent(parent)


@pytest.mark.parametrize("mode", ["flat", "grid"])
def test_level_graph_replays(ctx, mode):
    """Repeated calls replay a captured graph of the levels.  Different trees
    are copied into the same device buffers, so the graph recorded for one tree
    meets a deeper one (the call falls back to host-driven levels) and a
    shallower one (the extra levels are empty); eager work runs between calls."""
    n = 5000
    trees = [("random", synth.random_tree(n, seed=11)), ("deep", deep_tree(n, 700)),
             ("star", synth.star_tree(n)), ("deeper", deep_tree(n, 1500)), ("random", synth.random_tree(n, seed=11))]
    first = trees[0][1]
    dt = wc.DeviceTree.from_host(first.parent, first.child_ptr, first.child)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    other = synth.random_tree(3000, seed=12)
    other_dt = wc.DeviceTree.from_host(other.parent, other.child_ptr, other.child)
    other_ref = oracle.tree_height(other.child_ptr, other.child)
    for name, t in trees:
        dt.parent.copy_(torch.as_tensor(t.parent, dtype=torch.int32))
        dt.child_ptr.copy_(torch.as_tensor(t.child_ptr, dtype=torch.int32))
        dt.child.copy_(torch.as_tensor(t.child, dtype=torch.int32))
        d = oracle.tree_descendants(t.child_ptr, t.child)
        h = oracle.tree_height(t.child_ptr, t.child)
        for rep in range(4):
            say(f"tree graph replay mode={mode} tree={name} rep={rep}")
            res, st = ctx.tree_descendants(dt, mode=mode, out=out, stats=True)
            torch.cuda.synchronize()
            assert np.array_equal(res.cpu().numpy(), d), (name, rep)
            assert st["rounds"] == h[0], (name, rep)
            res = ctx.tree_height(dt, mode=mode, out=out)
            torch.cuda.synchronize()
            assert np.array_equal(res.cpu().numpy(), h), (name, rep)
            e = ctx.tree_height(other_dt, mode="grid")
            torch.cuda.synchronize()
            assert np.array_equal(e.cpu().numpy(), other_ref)


@pytest.fixture(scope="module")
def dataset1_like():
    say("generating the dataset1-like layered tree")
    t = synth.layered_tree(3, 128, 256, 0.5)
    return t, oracle.tree_descendants(t.child_ptr, t.child), oracle.tree_height(t.child_ptr, t.child)


@pytest.mark.parametrize("mode", MODES)
def test_dataset1_like_tree(ctx, dataset1_like, mode):
    """Depth 3 below the root, fanout 128..256, half of the inner nodes with
    children (about 1.7M nodes)."""
    t, d, h = dataset1_like
    assert np.array_equal(run(ctx, t, "desc", mode), d)
    assert np.array_equal(run(ctx, t, "height", mode), h)
