/*
 * Seeded synthetic inputs shared by the oracle and the GPU path.
 *
 * This file holds input generation only: a counter-based random generator,
 * R-MAT edge lists, CSR assembly, random rooted trees, edge weights, matrix
 * values and dense vectors.  None of the consolidation method's arithmetic
 * (relaxation, dot products, subtree folds) lives here.
 *
 * Random numbers: the SplitMix64 finaliser of Steele, Lea & Flood (2014),
 * "Fast splittable pseudorandom number generators", applied to a key derived
 * from (seed, stream) plus a Weyl sequence over the element index.  Every
 * element is therefore addressable on its own, which lets the generators run
 * in parallel and still produce the same bytes for a given seed.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t stream)
{
    return mix64(seed * GOLDEN + mix64(stream + GOLDEN));
}

static inline uint64_t draw(uint64_t key, uint64_t idx)
{
    return mix64(key + (idx + 1) * GOLDEN);
}

/* Uniform double in [0, 1) with 53 random bits. */
static inline double unit(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

uint64_t syn_rand(uint64_t seed, uint64_t stream, uint64_t idx)
{
    return draw(stream_key(seed, stream), idx);
}

void syn_rand_fill(uint64_t seed, uint64_t stream, int64_t count, uint64_t *out)
{
    uint64_t key = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) out[i] = draw(key, (uint64_t)i);
}

/* One R-MAT endpoint pair.  Level l (0 = most significant bit) draws one
 * uniform and picks a quadrant: [0,a) top-left, [a,a+b) top-right (target bit
 * set), [a+b,a+b+c) bottom-left (source bit set), rest bottom-right (both). */
static inline void rmat_pair(const uint64_t *keys, int scale, uint64_t idx, double a, double ab,
                             double abc, int64_t *s_out, int64_t *t_out)
{
    int64_t s = 0, t = 0;
    for (int l = 0; l < scale; ++l) {
        double u = unit(draw(keys[l], idx));
        int64_t bit = (int64_t)1 << (scale - 1 - l);
        if (u < a) {
        } else if (u < ab) {
            t |= bit;
        } else if (u < abc) {
            s |= bit;
        } else {
            s |= bit;
            t |= bit;
        }
    }
    *s_out = s;
    *t_out = t;
}

/* m R-MAT edges over 2^scale vertices; edge e uses draws with index e. */
int syn_rmat_edges(int scale, int64_t m, uint64_t seed, double a, double b, double c, int32_t *src,
                   int32_t *dst)
{
    if (scale < 1 || scale > 30 || m < 0) return -1;
    uint64_t keys[64];
    for (int l = 0; l < scale; ++l) keys[l] = stream_key(seed, 100 + (uint64_t)l);
    double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        int64_t s, t;
        rmat_pair(keys, scale, (uint64_t)e, a, ab, abc, &s, &t);
        src[e] = (int32_t)s;
        dst[e] = (int32_t)t;
    }
    return 0;
}

/* m R-MAT edges over n vertices (n need not be a power of two): pairs are drawn
 * at scale ceil(log2 n) and a pair with an endpoint >= n is rejected.  Attempts
 * are numbered 0,1,2,... and accepted pairs are kept in attempt order. */
int syn_rmat_edges_n(int64_t n, int64_t m, uint64_t seed, double a, double b, double c,
                     int32_t *src, int32_t *dst)
{
    if (n < 1 || n > ((int64_t)1 << 30) || m < 0) return -1;
    int scale = 0;
    while (((int64_t)1 << scale) < n) ++scale;
    if (scale == 0) {
        for (int64_t e = 0; e < m; ++e) src[e] = dst[e] = 0;
        return 0;
    }
    uint64_t keys[64];
    for (int l = 0; l < scale; ++l) keys[l] = stream_key(seed, 100 + (uint64_t)l);
    double ab = a + b, abc = a + b + c;
    const int64_t CH = 1 << 18;
    int64_t *bs = (int64_t *)malloc(sizeof(int64_t) * CH);
    int64_t *bt = (int64_t *)malloc(sizeof(int64_t) * CH);
    if (!bs || !bt) {
        free(bs);
        free(bt);
        return -2;
    }
    int64_t got = 0;
    uint64_t base = 0;
    while (got < m) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < CH; ++i) rmat_pair(keys, scale, base + (uint64_t)i, a, ab, abc, &bs[i], &bt[i]);
        for (int64_t i = 0; i < CH && got < m; ++i) {
            if (bs[i] < n && bt[i] < n) {
                src[got] = (int32_t)bs[i];
                dst[got] = (int32_t)bt[i];
                ++got;
            }
        }
        base += CH;
    }
    free(bs);
    free(bt);
    return 0;
}

static int cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

/* CSR from an edge list: row = source, every edge kept (duplicates and
 * self-loops included), targets sorted ascending within a row. */
int syn_csr_from_edges(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t *row_ptr,
                       int32_t *col)
{
    if (n < 0 || m < 0 || m > 0x7fffffffLL) return -1;
    memset(row_ptr, 0, sizeof(int32_t) * (size_t)(n + 1));
    for (int64_t e = 0; e < m; ++e) {
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return -1;
        row_ptr[src[e] + 1]++;
    }
    for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] += row_ptr[i];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!fill) return -2;
    memcpy(fill, row_ptr, sizeof(int32_t) * (size_t)n);
    for (int64_t e = 0; e < m; ++e) col[fill[src[e]]++] = dst[e];
    free(fill);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        int32_t len = row_ptr[i + 1] - row_ptr[i];
        if (len > 1) qsort(col + row_ptr[i], (size_t)len, sizeof(int32_t), cmp_i32);
    }
    return 0;
}

/* Edge weights uniform on the integers 1..wmax, one draw per CSR position. */
void syn_weights(int64_t m, uint64_t seed, uint32_t wmax, uint32_t *w)
{
    uint64_t key = stream_key(seed, 1);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) w[k] = 1u + (uint32_t)(draw(key, (uint64_t)k) % wmax);
}

/* Floats uniform in [-1, 1) on the 2^-23 grid: r24 * 2^-23 - 1 with a 24-bit
 * draw.  Every such value is exact in binary32. */
void syn_uniform_pm1(int64_t count, uint64_t seed, uint64_t stream, float *out)
{
    uint64_t key = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < count; ++k) {
        uint64_t r24 = draw(key, (uint64_t)k) >> 40;
        out[k] = (float)((double)r24 * 0x1.0p-23 - 1.0);
    }
}

/* Random rooted tree of exactly n nodes (root 0).
 *
 * Growth is breadth first in creation order.  A node at depth d < max_depth
 * draws its fanout k in {0..kmax} with P(k) proportional to (k+1)^-alpha; a
 * node at max_depth gets k = 0.  When a node would end the growth early (it
 * is the last node waiting in the queue, fewer than n nodes exist, and it drew
 * k = 0) its fanout is redrawn from the same law restricted to k >= 1.  The
 * last fanout is truncated to the nodes still missing.  Afterwards the non-root
 * ids are relabelled by a seeded random permutation and each child list is
 * sorted by id.
 *
 * Outputs: parent[n] (parent[0] = -1), child_ptr[n+1], child[n-1], and
 * optionally depth[n] (may be NULL).  Returns 0, or -3 when the depth cap
 * stops growth before n nodes exist. */
int syn_random_tree(int64_t n, uint64_t seed, int32_t kmax, double alpha, int32_t max_depth,
                    int32_t *parent, int32_t *child_ptr, int32_t *child, int32_t *depth)
{
    if (n < 1 || n > 0x7fffffffLL || kmax < 1) return -1;
    double *cdf = (double *)malloc(sizeof(double) * (size_t)(kmax + 1));
    int32_t *oparent = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *odepth = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *ofirst = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *ocount = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!cdf || !oparent || !odepth || !ofirst || !ocount || !perm) {
        free(cdf); free(oparent); free(odepth); free(ofirst); free(ocount); free(perm);
        return -2;
    }
    double tot = 0.0;
    for (int32_t k = 0; k <= kmax; ++k) {
        tot += pow((double)k + 1.0, -alpha);
        cdf[k] = tot;
    }
    for (int32_t k = 0; k <= kmax; ++k) cdf[k] /= tot;
    cdf[kmax] = 1.0;
    const double p0 = cdf[0];

    uint64_t kf = stream_key(seed, 200), kr = stream_key(seed, 201), kp = stream_key(seed, 202);
    oparent[0] = -1;
    odepth[0] = 0;
    int64_t made = 1;
    int rc = 0;
    for (int64_t h = 0; h < n; ++h) {
        ofirst[h] = (int32_t)made;
        ocount[h] = 0;
        if (h >= made) { rc = -3; break; }
        if (made >= n) continue;
        int32_t d = odepth[h];
        int32_t k = 0;
        if (d < max_depth) {
            double u = unit(draw(kf, (uint64_t)h));
            int32_t lo = 0, hi = kmax;
            while (lo < hi) { int32_t mid = (lo + hi) / 2; if (cdf[mid] > u) hi = mid; else lo = mid + 1; }
            k = lo;
            if (k == 0 && h == made - 1) {
                double u2 = p0 + unit(draw(kr, (uint64_t)h)) * (1.0 - p0);
                lo = 1; hi = kmax;
                while (lo < hi) { int32_t mid = (lo + hi) / 2; if (cdf[mid] > u2) hi = mid; else lo = mid + 1; }
                k = lo;
            }
        }
        if ((int64_t)k > n - made) k = (int32_t)(n - made);
        ocount[h] = k;
        for (int32_t j = 0; j < k; ++j) {
            oparent[made + j] = (int32_t)h;
            odepth[made + j] = d + 1;
        }
        made += k;
    }
    if (rc == 0 && made < n) rc = -3;
    if (rc == 0) {
        for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
        for (int64_t i = n - 1; i >= 2; --i) {
            int64_t j = 1 + (int64_t)(draw(kp, (uint64_t)i) % (uint64_t)i);
            int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
        }
        memset(child_ptr, 0, sizeof(int32_t) * (size_t)(n + 1));
        for (int64_t o = 0; o < n; ++o) child_ptr[perm[o] + 1] = ocount[o];
        for (int64_t i = 0; i < n; ++i) child_ptr[i + 1] += child_ptr[i];
        parent[0] = -1;
        for (int64_t o = 1; o < n; ++o) parent[perm[o]] = perm[oparent[o]];
        if (depth)
            for (int64_t o = 0; o < n; ++o) depth[perm[o]] = odepth[o];
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t o = 0; o < n; ++o) {
            int32_t p = perm[o], k = ocount[o];
            int32_t *dst = child + child_ptr[p];
            for (int32_t j = 0; j < k; ++j) dst[j] = perm[ofirst[o] + j];
            if (k > 1) qsort(dst, (size_t)k, sizeof(int32_t), cmp_i32);
        }
    }
    free(cdf); free(oparent); free(odepth); free(ofirst); free(ocount); free(perm);
    return rc;
}
