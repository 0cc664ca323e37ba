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
