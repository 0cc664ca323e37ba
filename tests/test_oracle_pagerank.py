"""Pins of the oracle's PageRank (CPU): closed forms, the sum-to-one invariant,
a dense power iteration built independently from the out-edge list, and the
principal eigenvector of the dense Google matrix."""
import numpy as np
import pytest

import oracle
import synth

D = 0.85


def pr(g, iters, d=D):
    t = synth.transpose(g)
    return oracle.pagerank_f64(t.row_ptr, t.col, synth.out_degree(g), iters, d)


def google_dense(n, edges, d=D):
    """Column-stochastic Google matrix from the (u, v) edge list: column u holds
    u's out-edges (weighted by multiplicity) or 1/n everywhere if u has none."""
    A = np.zeros((n, n))
    outdeg = np.zeros(n)
    for u, v in edges:
        A[v, u] += 1.0
        outdeg[u] += 1
    for u in range(n):
        if outdeg[u] > 0:
            A[:, u] /= outdeg[u]
        else:
            A[:, u] = 1.0 / n
    return d * A + (1.0 - d) / n


def test_cycle_is_uniform():
    n = 7
    g, _ = synth.graph_from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    for k in (1, 5, 30):
        assert np.allclose(pr(g, k), 1.0 / n, rtol=0, atol=1e-15)


def test_two_vertices_closed_form():
    # 0 -> 1, vertex 1 has no out-edges: one sweep from (1/2, 1/2), and the fixed point
    g, _ = synth.graph_from_edges(2, [(0, 1)])
    r = pr(g, 1)
    assert abs(r[0] - ((1 - D) / 2 + D * 0.25)) < 1e-15 and abs(r[1] - ((1 - D) / 2 + D * 0.75)) < 1e-15
    r = pr(g, 400)
    assert abs(r[0] - 1 / (2 + D)) < 1e-12 and abs(r[1] - (1 + D) / (2 + D)) < 1e-12


def random_graph(rng, n, m):
    edges = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(m)]
    return synth.graph_from_edges(n, edges)[0], edges


def test_sum_is_one_and_matches_dense_power_iteration():
    rng = np.random.default_rng(3)
    for trial in range(200):
        n = int(rng.integers(1, 12))
        m = int(rng.integers(0, 3 * n))
        g, edges = random_graph(rng, n, m)  # self-loops, multi-edges, dangling vertices
        G = google_dense(n, edges)
        r = np.full(n, 1.0 / n)
        for k in range(1, 8):
            r = G @ r
            got = pr(g, k)
            assert abs(got.sum() - 1.0) < 1e-12, (trial, k)
            assert np.allclose(got, r, rtol=0, atol=1e-13), (trial, k)


def test_converges_to_the_principal_eigenvector():
    rng = np.random.default_rng(4)
    g, edges = random_graph(rng, 30, 90)
    w, V = np.linalg.eig(google_dense(30, edges))
    v = np.real(V[:, np.argmax(np.real(w))])
    v = v / v.sum()
    assert np.allclose(pr(g, 300), v, rtol=0, atol=1e-10)


def test_transpose_round_trip():
    g = synth.rmat_csr(10, 1 << 13, seed=9)
    t = synth.transpose(g)
    assert t.row_ptr[-1] == g.row_ptr[-1]
    back = synth.transpose(t)
    assert np.array_equal(back.row_ptr, g.row_ptr)
    # rows of g are sorted, so the round trip restores col exactly
    assert np.array_equal(back.col, g.col)


def test_check_flags_a_planted_error():
    g = synth.rmat_csr(8, 1 << 11, seed=2)
    r = pr(g, 10)
    assert oracle.pagerank_check(r, r.astype(np.float32)) == (0, -1)
    bad = r.astype(np.float32).copy()
    bad[17] *= 1.0 + 5 * oracle.PAGERANK_RTOL
    assert oracle.pagerank_check(r, bad) == (1, 17)
