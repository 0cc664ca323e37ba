"""Pins for the SpMV oracle (irregular loop over CSR rows).

Binary64 y and the magnitude bound b are tied to a dense numpy matvec, to exact
special cases (identity, single-entry rows, empty rows) and to the tolerance
test rejecting planted errors just above the bound.
"""
import numpy as np

import oracle
import synth


def dense(g, val):
    a = np.zeros((g.n, g.n))
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    np.add.at(a, (src, g.col), val.astype(np.float64))
    return a


def test_matches_dense_matvec_on_tiny_matrices():
    rng = np.random.default_rng(11)
    for _ in range(200):
        n = int(rng.integers(1, 40))
        m = int(rng.integers(0, 5 * n))
        g, _ = synth.graph_from_edges(n, zip(rng.integers(0, n, m).tolist(), rng.integers(0, n, m).tolist()))
        val = synth.uniform_pm1(m, int(rng.integers(1, 1 << 30)))
        x = synth.uniform_pm1(n, int(rng.integers(1, 1 << 30)))
        y, b = oracle.spmv_f64(g.row_ptr, g.col, val, x)
        a = dense(g, val)
        np.testing.assert_allclose(y, a @ x.astype(np.float64), rtol=0, atol=1e-12)
        # b with duplicates: sum of |product| per entry, not |sum| per (row, col)
        src = np.repeat(np.arange(n), np.diff(g.row_ptr))
        bb = np.zeros(n)
        np.add.at(bb, src, np.abs(val.astype(np.float64) * x.astype(np.float64)[g.col]))
        np.testing.assert_allclose(b, bb, rtol=0, atol=1e-12)


def test_identity_and_single_entry_rows_are_exact():
    n = 1000
    x = synth.vector_x(n)
    g, _ = synth.graph_from_edges(n, [(i, i) for i in range(n)])
    y, b = oracle.spmv_f64(g.row_ptr, g.col, np.ones(n, np.float32), x)
    assert np.array_equal(y, x.astype(np.float64))
    assert np.array_equal(b, np.abs(x).astype(np.float64))
    # single entry a at column j: y = a * x_j exactly (product of two binary32 in binary64)
    val = synth.values(n)
    perm = np.random.default_rng(1).permutation(n)
    g, _ = synth.graph_from_edges(n, [(i, int(perm[i])) for i in range(n)])
    y, _ = oracle.spmv_f64(g.row_ptr, g.col, val, x)
    assert np.array_equal(y, val.astype(np.float64) * x.astype(np.float64)[perm])


def test_empty_rows_give_zero():
    g, _ = synth.graph_from_edges(5, [(1, 2), (1, 3)])
    y, b = oracle.spmv_f64(g.row_ptr, g.col, np.array([0.5, -0.25], np.float32), np.ones(5, np.float32))
    assert y.tolist() == [0, 0.25, 0, 0, 0] and b.tolist() == [0, 0.75, 0, 0, 0]
    bad, first = oracle.spmv_check(y, b, y.astype(np.float32))
    assert bad == 0 and first == -1
    # an empty row must be exactly zero: any nonzero fails (b = 0)
    yy = y.astype(np.float32)
    yy[0] = 1e-30
    assert oracle.spmv_check(y, b, yy) == (1, 0)


def test_tolerance_accepts_fp32_sums_and_rejects_planted_errors(c1_graph):
    g, _ = c1_graph
    val, x = synth.values(g.m), synth.vector_x(g.n)
    y_ref, b = oracle.spmv_f64(g.row_ptr, g.col, val, x)
    # a straightforward binary32 sequential sum per row is within the bound
    prod = (val * x[g.col]).astype(np.float32)
    y32 = np.zeros(g.n, np.float32)
    for r in range(g.n):
        s = np.float32(0)
        for p in prod[g.row_ptr[r]:g.row_ptr[r + 1]]:
            s = np.float32(s + p)
        y32[r] = s
    assert oracle.spmv_check(y_ref, b, y32) == (0, -1)
    # planting an error of 2e-5 * b in one non-empty row must be caught
    r = int(np.flatnonzero(b > 0)[17])
    bad = y32.copy()
    bad[r] = np.float32(y_ref[r] + 2e-5 * b[r])
    assert oracle.spmv_check(y_ref, b, bad) == (1, r)
    # dropping one term of a long row must be caught
    r = int(np.argmax(np.diff(g.row_ptr)))
    e = g.row_ptr[r]
    bad = y32.copy()
    bad[r] = np.float32(y_ref[r] - float(val[e]) * float(x[g.col[e]]))
    assert oracle.spmv_check(y_ref, b, bad)[0] == 1


def test_row_blocks_on_host_threads_give_the_same_result(c1_graph):
    """spmv_f64_threads (the oracle timed on all host cores) computes every row
    exactly as spmv_f64 does; only the rows run side by side."""
    g, _ = c1_graph
    val, x = synth.values(g.m), synth.vector_x(g.n)
    y1, b1 = oracle.spmv_f64(g.row_ptr, g.col, val, x)
    for threads in (1, 3, 8, 64):
        y, b = oracle.spmv_f64_threads(g.row_ptr, g.col, val, x, threads)
        assert np.array_equal(y.view(np.uint64), y1.view(np.uint64)) and np.array_equal(b, b1), threads
