"""Pins of the oracle's breadth-first levels (CPU): closed forms, scipy's
unweighted shortest paths, brute-force Bellman-Ford with unit weights on tiny
graphs, and the level certificate."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import oracle
import synth

INF = np.uint32(0xFFFFFFFF)


def test_path_and_star():
    g, _ = synth.graph_from_edges(6, [(i, i + 1) for i in range(5)])
    assert oracle.bfs(g.row_ptr, g.col, 0).tolist() == [0, 1, 2, 3, 4, 5]
    assert oracle.bfs(g.row_ptr, g.col, 3).tolist() == [INF, INF, INF, 0, 1, 2]
    g, _ = synth.graph_from_edges(5, [(0, i) for i in range(1, 5)])
    assert oracle.bfs(g.row_ptr, g.col, 0).tolist() == [0, 1, 1, 1, 1]


def test_matches_scipy_unweighted():
    g = synth.rmat_csr(12, 1 << 16)
    A = sp.csr_matrix((np.ones(len(g.col)), g.col, g.row_ptr), shape=(g.n, g.n))
    ref = shortest_path(A, unweighted=True, indices=0)
    got = oracle.bfs(g.row_ptr, g.col, 0)
    fin = np.isfinite(ref)
    assert np.array_equal(got[fin], ref[fin].astype(np.uint32)) and np.all(got[~fin] == INF)


def test_brute_force_and_certificate():
    rng = np.random.default_rng(6)
    for trial in range(300):
        n = int(rng.integers(1, 15))
        m = int(rng.integers(0, 3 * n))
        edges = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(m)]
        g, w = synth.graph_from_edges(n, edges)  # unit weights
        src = int(rng.integers(0, n))
        got = oracle.bfs(g.row_ptr, g.col, src)
        assert np.array_equal(got, oracle.sssp_bellman_ford(g.row_ptr, g.col, w, src)), trial
        assert oracle.sssp_certify(g.row_ptr, g.col, w, src, got) == (0, -1), trial
