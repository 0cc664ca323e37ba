"""Pins for the SSSP oracle (irregular loop of Fig. 1(b)).

The oracle's Dijkstra is tied to things other than itself: Bellman-Ford brute
force, Floyd-Warshall written here in numpy, scipy's csgraph Dijkstra, closed
forms on hand-built graphs, and an optimality certificate that must reject every
planted mistake.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra as scipy_dijkstra

import oracle
import synth

INF = 0xFFFFFFFF


def random_tiny_graph(rng, n_max=64):
    n = int(rng.integers(1, n_max + 1))
    m = int(rng.integers(0, 4 * n + 1))
    src = rng.integers(0, n, size=m)
    dst = rng.integers(0, n, size=m)
    # plant self-loops and multi-edges on purpose
    if m >= 4:
        dst[0] = src[0]
        src[1], dst[1] = src[2], dst[2]
    w = rng.integers(1, 101, size=m).astype(np.uint32)
    g, wc = synth.graph_from_edges(n, zip(src.tolist(), dst.tolist()), w)
    s = int(rng.integers(0, n))
    return g, wc, s


def floyd_warshall(g, w):
    n = g.n
    d = np.full((n, n), np.inf)
    np.fill_diagonal(d, 0.0)
    for u in range(n):
        for e in range(g.row_ptr[u], g.row_ptr[u + 1]):
            v = g.col[e]
            d[u, v] = min(d[u, v], float(w[e]))
    for k in range(n):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    return d


def to_u32(dist_float):
    out = np.full(dist_float.shape, INF, dtype=np.uint64)
    fin = np.isfinite(dist_float)
    out[fin] = dist_float[fin].astype(np.uint64)
    return out.astype(np.uint32)


def test_dijkstra_matches_bellman_ford_on_1000_tiny_graphs():
    rng = np.random.default_rng(12345)
    for _ in range(1000):
        g, w, s = random_tiny_graph(rng)
        a = oracle.sssp_dijkstra(g.row_ptr, g.col, w, s)
        b = oracle.sssp_bellman_ford(g.row_ptr, g.col, w, s)
        assert np.array_equal(a, b)


def test_dijkstra_matches_floyd_warshall():
    rng = np.random.default_rng(7)
    for _ in range(100):
        g, w, s = random_tiny_graph(rng, n_max=24)
        fw = floyd_warshall(g, w)
        assert np.array_equal(oracle.sssp_dijkstra(g.row_ptr, g.col, w, s), to_u32(fw[s]))


def scipy_sssp(g, w, s):
    # csgraph sums duplicate entries, so keep the minimum weight per (u, v) first
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    key = src.astype(np.int64) * g.n + g.col
    order = np.lexsort((w, key))
    key_s, w_s = key[order], w[order]
    first = np.ones(len(key_s), dtype=bool)
    first[1:] = key_s[1:] != key_s[:-1]
    u, v, ww = key_s[first] // g.n, key_s[first] % g.n, w_s[first].astype(np.float64)
    mat = sp.csr_matrix((ww, (u, v)), shape=(g.n, g.n))
    return to_u32(scipy_dijkstra(mat, directed=True, indices=s))


def test_dijkstra_matches_scipy_on_rmat_scale12(c1_graph):
    g, w = c1_graph
    ours = oracle.sssp_dijkstra(g.row_ptr, g.col, w, 0)
    assert np.array_equal(ours, scipy_sssp(g, w, 0))
    assert oracle.sssp_certify(g.row_ptr, g.col, w, 0, ours) == (0, -1)


def test_closed_forms():
    # chain 0->1->...->n-1 with weights i+1: dist[i] = i(i+1)/2
    n = 50
    g, w = synth.graph_from_edges(n, [(i, i + 1) for i in range(n - 1)], [i + 1 for i in range(n - 1)])
    d = oracle.sssp_dijkstra(g.row_ptr, g.col, w, 0)
    assert d.tolist() == [i * (i + 1) // 2 for i in range(n)]
    # from the middle of the chain the prefix is unreachable
    d = oracle.sssp_dijkstra(g.row_ptr, g.col, w, 10)
    assert (d[:10] == INF).all() and d[10] == 0 and d[11] == 11
    # star out of 0 with weight 7: 0 at the centre, 7 elsewhere
    g, w = synth.graph_from_edges(20, [(0, i) for i in range(1, 20)], [7] * 19)
    assert oracle.sssp_dijkstra(g.row_ptr, g.col, w, 0).tolist() == [0] + [7] * 19
    # star into 0: nothing reachable from 0
    g, w = synth.graph_from_edges(20, [(i, 0) for i in range(1, 20)], [7] * 19)
    assert oracle.sssp_dijkstra(g.row_ptr, g.col, w, 0).tolist() == [0] + [INF] * 19
    # shortcut beats the direct heavy edge: 0->2 (100) vs 0->1->2 (1+1)
    g, w = synth.graph_from_edges(3, [(0, 2), (0, 1), (1, 2)], [100, 1, 1])
    assert oracle.sssp_dijkstra(g.row_ptr, g.col, w, 0).tolist() == [0, 1, 2]
    # single vertex, no edges; self-loop only
    g, w = synth.graph_from_edges(1, [], [])
    assert oracle.sssp_dijkstra(g.row_ptr, g.col, w, 0).tolist() == [0]
    g, w = synth.graph_from_edges(1, [(0, 0)], [5])
    assert oracle.sssp_dijkstra(g.row_ptr, g.col, w, 0).tolist() == [0]


def test_certificate_accepts_truth_and_rejects_planted_mistakes(c1_graph):
    g, w = c1_graph
    d = oracle.sssp_dijkstra(g.row_ptr, g.col, w, 0)
    assert oracle.sssp_certify(g.row_ptr, g.col, w, 0, d)[0] == 0
    rng = np.random.default_rng(3)
    finite = np.flatnonzero((d != INF) & (np.arange(g.n) != 0))
    unreachable = np.flatnonzero(d == INF)
    assert len(finite) > 100 and len(unreachable) > 0
    for v in rng.choice(finite, 20, replace=False):
        for delta in (-1, +1):
            bad = d.copy()
            bad[v] = np.uint32(int(bad[v]) + delta)
            assert oracle.sssp_certify(g.row_ptr, g.col, w, 0, bad)[0] != 0
        bad = d.copy()
        bad[v] = INF
        assert oracle.sssp_certify(g.row_ptr, g.col, w, 0, bad)[0] != 0
    bad = d.copy()
    bad[unreachable[0]] = 12345
    assert oracle.sssp_certify(g.row_ptr, g.col, w, 0, bad)[0] != 0
    bad = d.copy()
    bad[0] = 1
    assert oracle.sssp_certify(g.row_ptr, g.col, w, 0, bad)[0] == 1


def test_certificate_uniqueness_on_tiny_graphs():
    """Any vector the certificate accepts equals brute force (checked by planting
    random perturbations on tiny graphs)."""
    rng = np.random.default_rng(99)
    for _ in range(300):
        g, w, s = random_tiny_graph(rng, n_max=16)
        truth = oracle.sssp_bellman_ford(g.row_ptr, g.col, w, s)
        cand = truth.copy()
        v = int(rng.integers(0, g.n))
        cand[v] = np.uint32(int(rng.integers(0, 300)) if rng.random() < 0.8 else INF)
        ok = oracle.sssp_certify(g.row_ptr, g.col, w, s, cand)[0] == 0
        assert ok == bool(np.array_equal(cand, truth))


def test_reached_edges_counts_out_edges_of_reached_vertices():
    g, w = synth.graph_from_edges(5, [(0, 1), (0, 2), (1, 3), (3, 1), (4, 0), (4, 4)], [1] * 6)
    d = oracle.sssp_dijkstra(g.row_ptr, g.col, w, 0)
    assert d.tolist() == [0, 1, 1, 2, INF]
    assert oracle.sssp_reached_edges(g.row_ptr, d) == 4


def test_bad_source_is_rejected():
    g, w = synth.graph_from_edges(3, [(0, 1)], [1])
    with pytest.raises(ValueError):
        oracle.sssp_dijkstra(g.row_ptr, g.col, w, 3)
