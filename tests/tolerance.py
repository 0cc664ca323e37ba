"""Rounding-depth model of the library's fp32 sums, and the error bounds the
SpMV and PageRank parity tests use (not collected: no test_ prefix).

A sum of positive or mixed-sign terms in which no term is rounded more than d
times has |computed - exact| <= gamma(d) * sum |term| with gamma(d) =
d u / (1 - d u), u = 2^-24 (Higham, Accuracy and Stability of Numerical
Algorithms, 2nd ed., Sec. 4.2); the products a_ij x_j enter exactly (fused
multiply-add).  The functions below give, for each mode of the library, the
largest number of roundings a nonzero of a row of a given length can pass
through, following the order the kernels use:

  * a lane's serial share of N terms goes through a cascade of four partial
    sums (32 terms per level): cascade_depth(N);
  * a wave butterfly adds log2(lanes) roundings; a workgroup sum adds 6 for its
    waves' butterflies plus (waves - 1) for adding the wave partials in order;
  * grid mode: rows up to the threshold are summed inline by one lane; longer
    rows up to 64 * items_per_lane by groups of g = 2^ceil(log2(len / ipl))
    lanes; still longer rows in chunks of 64 * ipl nonzeros (a cascade per lane
    plus a 64-lane butterfly), whose partials are summed lane-strided by one
    wave (a cascade plus a butterfly);
  * wave and block modes: rows above the threshold and up to 64 * ipl
    nonzeros (one chunk) by lane groups sized as in grid mode; longer rows in
    chunks as in grid mode;
  * flat mode: the row's lane alone.
"""
import math

import numpy as np

U = 2.0 ** -24
SPMV_RTOL = 1e-5  # the required per-row bound: |y - y_ref| <= 1e-5 * sum |a_ij x_j|

DEFAULTS = {  # the library's default tune per mode (wc_default_tune)
    "flat": dict(threshold=None, block_threads=256, items_per_lane=4),
    "wave": dict(threshold=8, block_threads=256, items_per_lane=2),
    "block": dict(threshold=8, block_threads=256, items_per_lane=2),
    "grid": dict(threshold=8, block_threads=512, items_per_lane=8),
}


def gamma(d: int) -> float:
    return d * U / (1.0 - d * U)


def cascade_depth(n: int) -> int:
    """Roundings a term can pass through in a Cascade sum of n terms."""
    if n <= 0:
        return 0
    d = min(n, 32)
    if n > 32:
        d += min(math.ceil(n / 32), 32)
    if n > 1024:
        d += min(math.ceil(n / 1024), 32)
    if n > 32768:
        d += math.ceil(n / 32768)
    return d + 3  # the final s3 + (s2 + (s1 + s0))


def tune_for(mode: str, **tune) -> dict:
    t = dict(DEFAULTS[mode])
    t.update({k: v for k, v in tune.items() if k in t and v})
    return t


def row_depth(length: int, mode: str, **tune) -> int:
    """Largest number of roundings of one product on its way to y for a row of
    `length` nonzeros (the in-edge sum of PageRank is the same with a_ij = 1)."""
    t = tune_for(mode, **tune)
    T, B, ipl = t["threshold"], t["block_threads"], t["items_per_lane"]
    if length <= 0:
        return 0
    if mode == "flat" or length <= T:
        return cascade_depth(length)
    chunks = math.ceil(length / (64 * ipl))
    chunked = cascade_depth(ipl) + 6 + cascade_depth(math.ceil(chunks / 64)) + 6
    # wave, block and grid: a row up to one chunk is summed by the g-lane group
    # that covers it at ipl nonzeros a lane
    if length <= 64 * ipl:
        g = 1 << max(0, math.ceil(math.log2(math.ceil(length / ipl))))
        return cascade_depth(math.ceil(length / g)) + int(math.log2(g))
    return chunked


def max_row_depth(row_lengths, mode: str, **tune) -> int:
    lengths = np.unique(np.asarray(row_lengths))
    return max([0] + [row_depth(int(k), mode, **tune) for k in lengths])


def pagerank_rtol(iterations: int, in_lengths, mode: str, n: int, num_cus: int = 256, **tune) -> float:
    """Relative bound per vertex for `iterations` fp32 sweeps against binary64.

    Each sweep: contrib = rank / outdeg (1 rounding); the in-edge sum of positive
    terms (depth D_v); the dangling sum D (per-thread cascade over the vertices
    of a grid-stride loop, a 4-wave workgroup sum, then every block sums the
    per-block parts the same way); spread = D * fl(1/n) (2); X = sum + spread
    (1); damping * X, where the fp32 damping differs from the binary64 one by at
    most u, (2); base + that (1), where base = fl((1 - d) / n) carries at most
    (1 + d / (1 - d)) u ~ 6.7 u for d = 0.85.  All terms are positive, so a
    relative error e entering a sweep leaves it at most
    (1 + e)(1 + gamma(D*)) - 1 with D* = max(D_max + 5, D_dangling + 6, 8).
    The start 1/n is rounded once.  After K sweeps: (1 + u)(1 + gamma(D*))^K - 1,
    plus 1e-12 for the binary64 oracle's own rounding."""
    d_max = max_row_depth(in_lengths, mode, **tune)
    pgrid = min((n + 255) // 256, 4 * num_cus)
    per_thread = math.ceil(n / (pgrid * 256))
    d_dang = cascade_depth(per_thread) + 6 + 3 + cascade_depth(math.ceil(pgrid / 256)) + 6 + 3
    d_star = max(d_max + 5, d_dang + 6, 8)
    return (1 + U) * (1 + gamma(d_star)) ** iterations - 1 + 1e-12
