"""Pins for the tree oracle (parallel recursion of Fig. 1(c)).

Descendant counts and heights are tied to brute-force ancestor walks, to a
recursive Python definition on tiny trees, to closed forms (chain, star,
complete k-ary) and to invariants that hold at any size.
"""
import sys

import numpy as np

import oracle
import synth


def random_parent_tree(rng, n):
    parent = np.empty(n, np.int32)
    parent[0] = -1
    for v in range(1, n):
        parent[v] = rng.integers(0, v)
    relabel = np.concatenate([[0], 1 + rng.permutation(n - 1)])
    out = np.empty(n, np.int32)
    out[relabel] = np.where(parent >= 0, relabel[np.maximum(parent, 0)], -1)
    return synth.tree_from_parent(out)


def recursive_desc_height(t):
    sys.setrecursionlimit(10000)
    desc = [0] * t.n
    height = [0] * t.n

    def visit(v):
        d, h = 0, 0
        for c in t.child[t.child_ptr[v]:t.child_ptr[v + 1]]:
            visit(c)
            d += 1 + desc[c]
            h = max(h, 1 + height[c])
        desc[v], height[v] = d, h

    visit(0)
    return np.array(desc), np.array(height)


def depths(t):
    d = np.zeros(t.n, np.int64)
    for v in range(1, t.n):
        k, u = 0, v
        while u != 0:
            u = t.parent[u]
            k += 1
        d[v] = k
    return d


def test_matches_recursion_and_brute_force_on_random_tiny_trees():
    rng = np.random.default_rng(5)
    for _ in range(300):
        n = int(rng.integers(1, 60))
        t = random_parent_tree(rng, n)
        assert oracle.tree_validate(t.parent, t.child_ptr, t.child) == 0
        d, h = recursive_desc_height(t)
        assert np.array_equal(oracle.tree_descendants(t.child_ptr, t.child), d)
        assert np.array_equal(oracle.tree_height(t.child_ptr, t.child), h)
        assert np.array_equal(oracle.tree_descendants_brute(t.parent), d)
        assert np.array_equal(oracle.tree_height_brute(t.parent), h)


def test_closed_forms():
    n = 100
    t = synth.chain_tree(n)
    assert oracle.tree_descendants(t.child_ptr, t.child).tolist() == [n - 1 - i for i in range(n)]
    assert oracle.tree_height(t.child_ptr, t.child).tolist() == [n - 1 - i for i in range(n)]
    t = synth.star_tree(n)
    assert oracle.tree_descendants(t.child_ptr, t.child).tolist() == [n - 1] + [0] * (n - 1)
    assert oracle.tree_height(t.child_ptr, t.child).tolist() == [1] + [0] * (n - 1)
    t = synth.tree_from_parent([-1])
    assert oracle.tree_descendants(t.child_ptr, t.child).tolist() == [0]
    assert oracle.tree_height(t.child_ptr, t.child).tolist() == [0]
    for k, hgt in [(2, 6), (3, 4), (7, 3)]:
        t = synth.kary_tree(k, hgt)
        d = oracle.tree_descendants(t.child_ptr, t.child)
        h = oracle.tree_height(t.child_ptr, t.child)
        dep = depths(t)
        # a node at depth r roots a complete k-ary tree of height hgt - r
        expect_h = hgt - dep
        expect_d = (k ** (expect_h + 1) - 1) // (k - 1) - 1
        assert np.array_equal(h, expect_h) and np.array_equal(d, expect_d)


def test_invariants_on_generated_tree():
    t = synth.random_tree(1 << 16, with_depth=True)
    assert oracle.tree_validate(t.parent, t.child_ptr, t.child) == 0
    d = oracle.tree_descendants(t.child_ptr, t.child)
    h = oracle.tree_height(t.child_ptr, t.child)
    assert d[0] == t.n - 1
    assert d.astype(np.int64).sum() == t.depth.astype(np.int64).sum()
    assert h[0] == t.depth.max()
    leaves = np.diff(t.child_ptr) == 0
    assert (d[leaves] == 0).all() and (h[leaves] == 0).all()
    # one level of the recursion: every node folds its children
    src = np.repeat(np.arange(t.n), np.diff(t.child_ptr))
    fold_d = np.zeros(t.n, np.int64)
    np.add.at(fold_d, src, 1 + d[t.child].astype(np.int64))
    assert np.array_equal(fold_d, d)
    fold_h = np.zeros(t.n, np.int64)
    np.maximum.at(fold_h, src, 1 + h[t.child].astype(np.int64))
    assert np.array_equal(fold_h, h)
    assert np.array_equal(oracle.tree_descendants_brute(t.parent), d)
    assert np.array_equal(oracle.tree_height_brute(t.parent), h)


def test_planted_mistakes_break_the_invariants():
    t = synth.random_tree(5000, seed=9, with_depth=True)
    d = oracle.tree_descendants(t.child_ptr, t.child)
    brute = oracle.tree_descendants_brute(t.parent)
    bad = d.copy()
    bad[int(np.flatnonzero(np.diff(t.child_ptr) > 0)[3])] += 1
    assert not np.array_equal(bad, brute)
    assert bad.astype(np.int64).sum() != t.depth.astype(np.int64).sum()


# ---- the structure check rejects what is not a tree ---------------------------------------------

def _arrays(t):
    return t.parent.copy(), t.child_ptr.copy(), t.child.copy()


def test_validate_accepts_exactly_the_trees_among_tiny_parent_arrays():
    """Brute force over every parent array of 5 nodes (parent[0] = -1, parent[v]
    in 0..4): it is a tree iff following parents from every node reaches the
    root, and the check must say so for each of the 5^4 arrays, with child lists
    built from the parent array."""
    import itertools
    n = 5
    for ps in itertools.product(range(n), repeat=n - 1):
        parent = np.array((-1,) + ps, np.int32)
        reaches_root = True
        for v in range(1, n):
            u, steps = v, 0
            while u != 0 and steps <= n:
                u, steps = parent[u], steps + 1
            reaches_root = reaches_root and u == 0
        counts = np.bincount(parent[1:], minlength=n)
        child_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
        child = np.argsort(parent[1:], kind="stable").astype(np.int32) + 1
        rc = oracle.tree_validate(parent, child_ptr, child)
        assert (rc == 0) == reaches_root, (ps, rc)
        if not reaches_root:
            assert rc == 8  # a cycle among non-root nodes: not reached from the root


def test_validate_rejects_a_cycle():
    # 0 -> 1 -> 2 is a tree; make 3 and 4 each other's parent (both listed, neither reached)
    parent = np.array([-1, 0, 1, 4, 3], np.int32)
    child_ptr = np.array([0, 1, 2, 2, 3, 4], np.int32)
    child = np.array([1, 2, 4, 3], np.int32)
    assert oracle.tree_validate(parent, child_ptr, child) == 8


def test_validate_rejects_a_wrong_parent():
    t = synth.kary_tree(3, 3)
    parent, child_ptr, child = _arrays(t)
    v = int(child[-1])
    parent[v] = 0 if parent[v] != 0 else 1  # listed under one node, parent[] names another
    assert oracle.tree_validate(parent, child_ptr, child) == 6


def test_validate_rejects_a_duplicate_child():
    # a leaf listed twice in place of another leaf: the count of entries still
    # matches n - 1 and every parent[] agrees, so only the duplicate gives it away
    t = synth.star_tree(6)
    parent, child_ptr, child = _arrays(t)
    child[1] = child[0]
    assert oracle.tree_validate(parent, child_ptr, child) == 7


def test_validate_rejects_an_unreachable_node():
    # node 5 has parent 4 and is listed under 4, but 4 and 5 hang off each other
    parent = np.array([-1, 0, 0, 0, 5, 4], np.int32)
    child_ptr = np.array([0, 3, 3, 3, 3, 4, 5], np.int32)
    child = np.array([1, 2, 3, 5, 4], np.int32)
    assert oracle.tree_validate(parent, child_ptr, child) == 8


def test_validate_rejects_bad_offsets_and_entries():
    t = synth.kary_tree(2, 3)
    parent, child_ptr, child = _arrays(t)
    bad = child_ptr.copy()
    bad[-1] = t.n  # child_ptr[n] must be n - 1
    assert oracle.tree_validate(parent, bad, np.concatenate([child, [1]]).astype(np.int32)) == 3
    bad = child_ptr.copy()
    bad[1], bad[2] = bad[2], bad[1]  # decreasing offsets
    if bad[1] != bad[2]:
        assert oracle.tree_validate(parent, bad, child) == 4
    bad = child.copy()
    bad[0] = t.n  # entry out of range
    assert oracle.tree_validate(parent, child_ptr, bad) == 5
    bad = child.copy()
    bad[0] = 0  # the root listed as a child
    assert oracle.tree_validate(parent, child_ptr, bad) == 5
    p2 = parent.copy()
    p2[0] = 0
    assert oracle.tree_validate(p2, child_ptr, child) == 2
    assert oracle.tree_validate(parent, child_ptr, child) == 0
