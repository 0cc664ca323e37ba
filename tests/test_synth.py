"""Determinism and statistics of the seeded input generators."""
import hashlib

import numpy as np

import oracle
import synth


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_same_seed_same_bytes_and_different_seed_differs():
    g1, g2 = synth.rmat_csr(10, 1 << 14), synth.rmat_csr(10, 1 << 14)
    assert digest(g1.row_ptr, g1.col) == digest(g2.row_ptr, g2.col)
    g3 = synth.rmat_csr(10, 1 << 14, seed=7)
    assert digest(g1.row_ptr, g1.col) != digest(g3.row_ptr, g3.col)
    t1, t2 = synth.random_tree(1 << 12), synth.random_tree(1 << 12)
    assert digest(t1.parent, t1.child_ptr, t1.child) == digest(t2.parent, t2.child_ptr, t2.child)
    assert digest(synth.weights(1000)) == digest(synth.weights(1000))


def test_rmat_shape_scale12():
    g = synth.rmat_csr(12, 1 << 16)
    assert g.n == 4096 and g.m == 1 << 16 and g.row_ptr[-1] == g.m
    deg = g.degrees()
    # expected out-degree of vertex 0 is m (a+b)^scale
    expect = (1 << 16) * 0.76 ** 12
    assert abs(deg[0] - expect) < 6 * np.sqrt(expect)
    assert deg[0] == deg.max()
    # rows sorted by target
    for r in range(0, g.n, 97):
        seg = g.col[g.row_ptr[r]:g.row_ptr[r + 1]]
        assert (np.diff(seg) >= 0).all()
    # in-degree of 0 follows (a+c)^scale as well
    indeg0 = int((g.col == 0).sum())
    assert abs(indeg0 - expect) < 6 * np.sqrt(expect)


def test_rmat_n_rejection_keeps_endpoints_in_range():
    g = synth.rmat_csr_n(1000, 16000, seed=11)
    assert g.n == 1000 and g.m == 16000 and g.col.max() < 1000


def test_weights_values_ranges():
    w = synth.weights(200000)
    assert w.min() == 1 and w.max() == 100
    counts = np.bincount(w, minlength=101)[1:]
    assert counts.min() > 0.9 * 2000 and counts.max() < 1.1 * 2000
    v = synth.values(200000)
    assert v.min() >= -1.0 and v.max() < 1.0 and abs(v.mean()) < 0.01
    assert np.array_equal(v, (np.round((v.astype(np.float64) + 1) * 2 ** 23) / 2 ** 23 - 1).astype(np.float32))


def test_random_tree_shape():
    n = 1 << 18
    t = synth.random_tree(n, with_depth=True)
    assert oracle.tree_validate(t.parent, t.child_ptr, t.child) == 0
    fan = np.diff(t.child_ptr)
    assert t.n == n and fan.sum() == n - 1 and fan.max() <= 4096
    assert t.depth.max() <= 24
    # relabelled: ids do not follow depth order
    assert not (np.diff(t.depth) >= 0).all()
    # among nodes that drew a fanout, about 61% are leaves (P(0) = 1/sum (k+1)^-2)
    p0 = 1.0 / sum((k + 1.0) ** -2 for k in range(4097))
    assert abs(p0 - 0.608) < 0.001


def test_small_shapes():
    t = synth.kary_tree(3, 2)
    assert t.n == 13 and oracle.tree_validate(t.parent, t.child_ptr, t.child) == 0
    assert oracle.tree_validate(*[getattr(synth.chain_tree(5), k) for k in ("parent", "child_ptr", "child")]) == 0


def test_layered_tree_shape():
    for levels, lo, hi, frac in ((3, 8, 16, 0.5), (2, 32, 128, 1.0), (4, 2, 3, 1.0)):
        t = synth.layered_tree(levels, lo, hi, frac, seed=9)
        u = synth.layered_tree(levels, lo, hi, frac, seed=9)
        assert np.array_equal(t.parent, u.parent)  # seeded
        fan = np.diff(t.child_ptr)
        assert fan[0] >= lo and np.all((fan == 0) | ((fan >= lo) & (fan <= hi)))
        # depth of every node, from the parent array (parents have smaller ids)
        depth = np.zeros(t.n, dtype=np.int64)
        for v in range(1, t.n):
            depth[v] = depth[t.parent[v]] + 1
        assert depth.max() == levels
        assert np.all(fan[depth == levels] == 0)
        if frac == 1.0:
            assert np.all(fan[depth < levels] > 0)
        else:
            inner = fan[(depth > 0) & (depth < levels)] > 0
            assert 0.3 < inner.mean() < 0.7
        # children of a node are consecutive ids (level-by-level numbering)
        for v in np.flatnonzero(fan)[:50]:
            ch = t.child[t.child_ptr[v]:t.child_ptr[v + 1]]
            assert np.array_equal(ch, np.arange(ch[0], ch[0] + ch.size))
