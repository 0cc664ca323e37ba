"""The fp32 error bounds of SpMV and PageRank, checked on the CPU.

* The rounding-depth model of tests/tolerance.py is pinned against a direct
  simulation of the cascade sum that counts, for every term, how often it is
  rounded.
* On the scale-22 R-MAT graph every row in every mode (default tunes and the
  tunes the GPU tests sweep) stays within depth 167, so the required
  1e-5 * sum |a_ij x_j| per row is a worst-case bound there, not only a likely one.
* A replay of the first PageRank sweep at the scale-22 hub (159,737 in-edges)
  in fp32: a plain running sum in one lane (the order flat mode used before the
  cascade) is off by more than 1e-4 relative to binary64, while the cascade
  order of flat mode and the chunked order of wave mode stay within the
  derived bound.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from tolerance import (SPMV_RTOL, U, cascade_depth, gamma, max_row_depth, pagerank_rtol, row_depth)

F = np.float32


class CascadeSim:
    """The library's Cascade (four partial sums, 32 terms per level) in fp32,
    tracking the largest number of roundings of any term in each partial sum."""

    def __init__(self):
        self.s = [F(0)] * 4
        self.d = [0] * 4  # depth of the terms held by each partial sum
        self.live = [False] * 4
        self.steps = 0

    def _add_into(self, k, value, depth, live):
        # adding into an empty (exact zero) partial sum does not round
        if self.live[k] and live:
            self.s[k] = F(self.s[k] + value)
            self.d[k] = max(self.d[k], depth) + 1
        elif live:
            self.s[k] = F(value)
            self.d[k] = depth
        self.live[k] = self.live[k] or live

    def add(self, x):
        # a term entering s0 by an add is rounded once (a fused multiply-add of
        # an exact product likewise)
        self._add_into(0, F(x), 0, True)
        if not self.d[0]:
            self.d[0] = 1
        self.steps += 1
        for level, period in ((0, 32), (1, 1024), (2, 32768)):
            if self.steps % period:
                break
            self._add_into(level + 1, self.s[level], self.d[level], self.live[level])
            self.s[level], self.d[level], self.live[level] = F(0), 0, False

    def total(self):
        v, d, live = self.s[0], self.d[0], self.live[0]
        for k in (1, 2, 3):
            if self.live[k] and live:
                v, d = F(self.s[k] + v), max(d, self.d[k]) + 1
            elif self.live[k]:
                v, d = self.s[k], self.d[k]
            live = live or self.live[k]
        return v, d


@pytest.mark.parametrize("n", [1, 2, 31, 32, 33, 64, 1000, 1024, 1025, 1056, 5000, 32768, 32769, 40000, 70000])
def test_cascade_depth_bounds_the_simulated_roundings(n):
    c = CascadeSim()
    for i in range(n):
        c.add(1.0)
    total, depth = c.total()
    assert total == F(n)  # integers below 2^24 add exactly: the simulation sums every term once
    assert depth <= cascade_depth(n)
    # the model over-counts only the exact adds into empty partial sums and the final combination
    assert cascade_depth(n) - depth <= 6


def test_cascade_depth_is_small_where_a_running_sum_is_not():
    assert cascade_depth(159_772) == 32 + 32 + 32 + 5 + 3
    assert cascade_depth(1 << 20) == 131
    assert gamma(131) < 1e-5 < gamma(168)


@pytest.fixture(scope="module")
def rmat22():
    return synth.rmat_csr(22, 1 << 26)


TUNES = [dict(), dict(threshold=1), dict(threshold=100), dict(items_per_lane=1), dict(items_per_lane=16),
         dict(block_threads=64), dict(block_threads=1024)]


@pytest.mark.parametrize("mode", ["flat", "wave", "block", "grid"])
def test_spmv_bound_is_worst_case_on_the_scale22_graph(rmat22, mode):
    out_len = np.diff(rmat22.row_ptr)
    in_len = np.bincount(rmat22.col, minlength=rmat22.n)
    for tune in TUNES:
        for lengths in (out_len, in_len):
            d = max_row_depth(lengths, mode, **tune)
            assert gamma(d) <= SPMV_RTOL, (mode, tune, d)


def test_row_depth_examples():
    # the hub's 159,772 nonzeros: flat one lane; wave and block (defaults) 1,249
    # chunks of 128 (2 per lane + butterfly), partials 20 per lane + butterfly;
    # with items_per_lane 4, 625 chunks of 256 and partials 10 per lane; grid 313
    # chunks of 512 (8 per lane + butterfly), partials 5 per lane + butterfly
    assert row_depth(159_772, "flat") == cascade_depth(159_772)
    assert row_depth(159_772, "wave") == cascade_depth(2) + 6 + cascade_depth(20) + 6
    assert row_depth(159_772, "block") == cascade_depth(2) + 6 + cascade_depth(20) + 6
    assert row_depth(159_772, "wave", items_per_lane=4) == cascade_depth(4) + 6 + cascade_depth(10) + 6
    # rows a wave or a block keeps: above the threshold (8) and up to one chunk
    # (64 * 2), by the group of g lanes that covers the row at 2 nonzeros a lane
    # (40 nonzeros: 32 lanes); with items_per_lane 4, 16 lanes
    assert row_depth(8, "wave") == cascade_depth(8)
    assert row_depth(128, "wave") == cascade_depth(2) + 6 == row_depth(128, "block")
    assert row_depth(40, "wave") == cascade_depth(2) + 5 == row_depth(40, "block")
    assert row_depth(40, "wave", items_per_lane=4) == cascade_depth(3) + 4
    assert row_depth(256, "wave", items_per_lane=4, threshold=32) == cascade_depth(4) + 6
    assert row_depth(129, "wave") == cascade_depth(2) + 6 + cascade_depth(1) + 6
    assert row_depth(159_772, "grid") == cascade_depth(8) + 6 + cascade_depth(5) + 6
    assert row_depth(8, "grid") == cascade_depth(8) and row_depth(9, "grid") == cascade_depth(5) + 1
    assert row_depth(0, "wave") == 0


def _fp32_rank(sum32, spread32, n, d=0.85):
    base = F((1.0 - float(F(d))) / n)
    return F(base + F(F(d) * F(sum32 + spread32)))


def test_pagerank_first_sweep_at_the_hub(rmat22):
    g = rmat22
    n = g.n
    od = synth.out_degree(g)
    # in-edges of vertex 0 in in-CSR order (sources ascending, with multiplicity)
    e = np.flatnonzero(g.col == 0)
    src = (np.searchsorted(g.row_ptr, e, side="right") - 1).astype(np.int64)
    assert src.size == 159_737
    r0 = F(1.0 / n)
    contrib = (r0 / od[src].astype(F)).astype(F)  # rank / outdeg, rounded once
    dangling = F(r0 * F(np.count_nonzero(od == 0)))  # exact enough: only its bound matters below
    spread = F(dangling * F(1.0 / n))

    t = synth.transpose(g)
    ref = oracle.pagerank_f64(t.row_ptr, t.col, od, 1)[0]
    in_len = np.diff(t.row_ptr)

    def rel(s):
        return abs(float(_fp32_rank(s, spread, n)) - ref) / ref

    serial = np.cumsum(contrib, dtype=F)[-1]  # a running fp32 sum in one lane
    c = CascadeSim()
    for v in contrib:
        c.add(v)
    cascade, depth = c.total()
    assert depth <= cascade_depth(src.size)
    def wave_sum(vals):
        """64 lanes, lane l taking vals l, l + 64, ... (a cascade each), then the butterfly."""
        lanes = np.zeros(64, F)
        for lane in range(64):
            cl = CascadeSim()
            for v in vals[lane::64]:
                cl.add(v)
            lanes[lane] = cl.total()[0]
        for dist in (32, 16, 8, 4, 2, 1):
            lanes = (lanes + lanes[np.arange(64) ^ dist]).astype(F)
        return lanes[0]

    # wave order for a row this long: chunks of 64 * 2 terms (the default
    # items_per_lane), each a wave sum, then a wave sum of the chunk partials in
    # chunk order
    partials = np.array([wave_sum(contrib[c:c + 128]) for c in range(0, contrib.size, 128)], F)
    wave = wave_sum(partials)

    assert rel(serial) > 1e-4  # the bound 1e-4 did not hold for the plain running sum
    assert rel(cascade) <= pagerank_rtol(1, in_len, "flat", n)
    assert rel(wave) <= pagerank_rtol(1, in_len, "wave", n)
    # the derived bounds for one and ten sweeps in every mode
    for mode in ("flat", "wave", "block", "grid"):
        assert pagerank_rtol(1, in_len, mode, n) < 1e-5
        assert pagerank_rtol(10, in_len, mode, n) < 1e-4
    assert math.isclose(float(F(1.0 / n)) * n, 1.0, rel_tol=U)
