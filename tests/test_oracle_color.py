"""Pins of the oracle's Jones-Plassmann coloring (CPU): closed forms, a direct
round-by-round simulation in numpy on tiny graphs, validity, and the
certificate (the recurrence that fixes the coloring) including planted errors."""
import numpy as np
import pytest

import oracle
import synth


def sym(n, edges):
    g, _ = synth.graph_from_edges(n, edges)
    return synth.symmetrize(g)


def test_complete_graph_is_ranked_by_priority():
    n = 7
    g = sym(n, [(i, j) for i in range(n) for j in range(n) if i != j])
    prio = np.array([5, 1, 9, 3, 9, 0, 2], dtype=np.uint32)
    c, k = oracle.color_jp(g.row_ptr, g.col, prio)
    # order: (9, id 4) > (9, id 2) > 5 > 3 > 2 > 1 > 0
    assert c.tolist() == [2, 5, 1, 3, 0, 6, 4] and k == 7


def test_star_and_path():
    g = sym(6, [(0, i) for i in range(1, 6)])
    c, k = oracle.color_jp(g.row_ptr, g.col, np.array([9, 1, 2, 3, 4, 5], np.uint32))
    assert c.tolist() == [0, 1, 1, 1, 1, 1] and k == 2
    c, k = oracle.color_jp(g.row_ptr, g.col, np.array([0, 1, 2, 3, 4, 5], np.uint32))
    assert c.tolist() == [1, 0, 0, 0, 0, 0] and k == 2
    g = sym(5, [(i, i + 1) for i in range(4)])
    # priorities increasing along the path: one vertex per round, from the far end
    c, k = oracle.color_jp(g.row_ptr, g.col, np.arange(5, dtype=np.uint32))
    assert c.tolist() == [4, 3, 2, 1, 0] and k == 5
    # alternating priorities: the peaks first, then the valleys
    c, k = oracle.color_jp(g.row_ptr, g.col, np.array([1, 0, 1, 0, 1], np.uint32))
    assert c.tolist() == [0, 1, 0, 1, 0] and k == 2


def simulate(n, adj, prio):
    """Round-by-round definition on an adjacency matrix."""
    color = -np.ones(n, dtype=np.int64)
    rank = prio.astype(np.int64) * (n + 1) + np.arange(n)
    r = 0
    while (color < 0).any():
        unc = color < 0
        ready = [v for v in range(n) if unc[v] and not any(adj[v, u] and unc[u] and rank[u] > rank[v]
                                                          for u in range(n) if u != v)]
        color[ready] = r
        r += 1
    return color, r


def test_matches_simulation_and_certificate_on_tiny_graphs():
    rng = np.random.default_rng(8)
    for trial in range(300):
        n = int(rng.integers(1, 14))
        m = int(rng.integers(0, 3 * n))
        edges = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(m)]
        g = sym(n, edges)
        adj = np.zeros((n, n), bool)
        for u, v in edges:
            if u != v:
                adj[u, v] = adj[v, u] = True
        prio = rng.integers(0, 4, size=n).astype(np.uint32)  # many ties
        c, k = oracle.color_jp(g.row_ptr, g.col, prio)
        ref, rk = simulate(n, adj, prio)
        assert np.array_equal(c, ref) and k == rk, trial
        assert oracle.color_certify(g.row_ptr, g.col, prio, c) == (0, -1), trial


def test_certificate_rejects_planted_errors():
    g = synth.symmetrize(synth.rmat_csr(10, 1 << 13, seed=4))
    prio = synth.priorities(g.n, seed=4)
    c, k = oracle.color_jp(g.row_ptr, g.col, prio)
    assert oracle.color_certify(g.row_ptr, g.col, prio, c) == (0, -1)
    deg = np.diff(g.row_ptr)
    v = int(np.flatnonzero(deg > 0)[3])
    for delta in (-1, 1):
        bad = c.copy()
        bad[v] += delta
        n_bad, first = oracle.color_certify(g.row_ptr, g.col, prio, bad)
        assert n_bad >= 1


def test_symmetrize():
    g, _ = synth.graph_from_edges(4, [(0, 1), (1, 0), (0, 0), (2, 3), (2, 3)])
    s = synth.symmetrize(g)
    assert s.row_ptr.tolist() == [0, 1, 2, 3, 4] and s.col.tolist() == [1, 0, 3, 2]
