/*
 * Oracle: plain, slow, obviously correct CPU implementations of what the
 * workload-consolidation hot path computes.  TEST INFRASTRUCTURE ONLY: only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Consolidation is an execution strategy: the consolidated child handles each
 * buffered work item exactly as the original child would (Sec. IV.C, child
 * kernel transformation).  So every mode of the GPU path must reproduce the
 * plain definition of each problem's result, which is what this file computes:
 *
 *   SSSP  - shortest-path distances from one source over a directed CSR graph
 *           with positive integer weights (the irregular loop of Fig. 1(b)).
 *           Binary-heap Dijkstra; Bellman-Ford as a brute-force cross-check;
 *           an O(m) optimality certificate usable at any size.
 *   BFS   - breadth-first levels from one source (the recursive BFS of
 *           Sec. V reaches the same levels).  A FIFO queue.
 *   GC    - Jones-Plassmann coloring rounds over a symmetric graph with
 *           given priorities, and the recurrence that certifies it.
 *   SpMV  - y = A x in binary64 plus the per-row magnitude sum
 *           b[r] = sum |a_rj x_j| used by the tolerance test (Sec. V lists
 *           SpMV among the irregular-loop benchmarks).
 *   PR    - damped PageRank iterations over the in-edges of each vertex (the
 *           same irregular loop as SpMV, with the rank contributions of the
 *           sources in place of a_ij x_j).
 *   TD/TH - per-node proper-descendant count and per-node height of a rooted
 *           tree (the recursion of Fig. 1(c): leaf work at nodes without
 *           children, post-work folding the children's results into the node).
 *           Breadth-first order plus a reverse fold; brute-force ancestor walks
 *           as cross-checks.
 *   Consolidation bookkeeping - how many child launches the basic template of
 *           Fig. 1(a) makes, how many consolidated dispatches a given buffer
 *           scope makes and how much work they carry (Sec. IV.A, Fig. 2),
 *           the per-buffer size estimate of Sec. IV.E and the KC_X
 *           configuration of Sec. IV.E.
 *
 * Every pin that ties these functions to the paper and to mathematics lives in
 * the test suite (tests/test_oracle_*.py).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORC_INF 0xFFFFFFFFu

/* ---------------------------------------------------------------- SSSP ---- */

typedef struct {
    uint64_t key;
    int32_t v;
} heap_ent;

static void heap_push(heap_ent *h, int64_t *size, uint64_t key, int32_t v)
{
    int64_t i = (*size)++;
    h[i].key = key;
    h[i].v = v;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].key <= h[i].key) break;
        heap_ent t = h[p]; h[p] = h[i]; h[i] = t;
        i = p;
    }
}

static heap_ent heap_pop(heap_ent *h, int64_t *size)
{
    heap_ent top = h[0];
    h[0] = h[--(*size)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < *size && h[l].key < h[s].key) s = l;
        if (r < *size && h[r].key < h[s].key) s = r;
        if (s == i) break;
        heap_ent t = h[s]; h[s] = h[i]; h[i] = t;
        i = s;
    }
    return top;
}

/* Shortest-path distances from src (Fig. 1(b) relaxes every out-edge of a
 * node; the fixed point of those relaxations is this).  Unreachable = ORC_INF.
 * Returns 0, -1 on bad arguments, -2 on allocation failure, -4 if a distance
 * does not fit below ORC_INF. */
int orc_sssp_dijkstra(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint32_t *w, int32_t src,
                      uint32_t *dist)
{
    if (n < 0 || (n > 0 && (src < 0 || src >= n))) return -1;
    if (n == 0) return 0;
    int64_t m = row_ptr[n];
    uint64_t *d = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    heap_ent *h = (heap_ent *)malloc(sizeof(heap_ent) * (size_t)(m + 1));
    unsigned char *done = (unsigned char *)calloc((size_t)n, 1);
    if (!d || !h || !done) { free(d); free(h); free(done); return -2; }
    for (int32_t i = 0; i < n; ++i) d[i] = UINT64_MAX;
    int64_t size = 0;
    d[src] = 0;
    heap_push(h, &size, 0, src);
    while (size > 0) {
        heap_ent t = heap_pop(h, &size);
        int32_t u = t.v;
        if (done[u] || t.key != d[u]) continue;
        done[u] = 1;
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int32_t v = col[e];
            uint64_t nd = d[u] + (uint64_t)w[e];
            if (nd < d[v]) {
                d[v] = nd;
                heap_push(h, &size, nd, v);
            }
        }
    }
    int rc = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (d[i] == UINT64_MAX) dist[i] = ORC_INF;
        else if (d[i] >= (uint64_t)ORC_INF) { dist[i] = ORC_INF; rc = -4; }
        else dist[i] = (uint32_t)d[i];
    }
    free(d); free(h); free(done);
    return rc;
}

/* Brute force: n-1 full passes of relaxing every edge (Bellman-Ford). */
int orc_sssp_bellman_ford(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
                          int32_t src, uint32_t *dist)
{
    if (n < 0 || (n > 0 && (src < 0 || src >= n))) return -1;
    if (n == 0) return 0;
    uint64_t *d = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    if (!d) return -2;
    for (int32_t i = 0; i < n; ++i) d[i] = UINT64_MAX;
    d[src] = 0;
    for (int32_t pass = 0; pass + 1 < n; ++pass) {
        for (int32_t u = 0; u < n; ++u) {
            if (d[u] == UINT64_MAX) continue;
            for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                uint64_t nd = d[u] + (uint64_t)w[e];
                if (nd < d[col[e]]) d[col[e]] = nd;
            }
        }
    }
    int rc = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (d[i] == UINT64_MAX) dist[i] = ORC_INF;
        else if (d[i] >= (uint64_t)ORC_INF) { dist[i] = ORC_INF; rc = -4; }
        else dist[i] = (uint32_t)d[i];
    }
    free(d);
    return rc;
}

/* Optimality certificate for positive weights.  dist is the shortest-path
 * vector from src iff
 *   (1) dist[src] == 0,
 *   (2) every edge u->v with finite dist[u] has dist[v] <= dist[u] + w,
 *   (3) every finite v != src has an in-edge u->v with dist[v] == dist[u] + w,
 *   (4) dist[v] is finite exactly when v is reachable from src.
 * Returns 0 when all hold, else the number of the first failed condition, and
 * stores the offending vertex (or edge for (2)) in *where. */
int orc_sssp_certify(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint32_t *w, int32_t src,
                     const uint32_t *dist, int64_t *where)
{
    *where = -1;
    if (n == 0) return 0;
    if (src < 0 || src >= n) return -1;
    if (dist[src] != 0) { *where = src; return 1; }
    unsigned char *tight = (unsigned char *)calloc((size_t)n, 1);
    unsigned char *seen = (unsigned char *)calloc((size_t)n, 1);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!tight || !seen || !queue) { free(tight); free(seen); free(queue); return -2; }
    int rc = 0;
    for (int32_t u = 0; u < n && rc == 0; ++u) {
        if (dist[u] == ORC_INF) continue;
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            uint64_t nd = (uint64_t)dist[u] + (uint64_t)w[e];
            uint32_t dv = dist[col[e]];
            if ((uint64_t)dv > nd) { *where = e; rc = 2; break; }
            if ((uint64_t)dv == nd) tight[col[e]] = 1;
        }
    }
    for (int32_t v = 0; v < n && rc == 0; ++v)
        if (v != src && dist[v] != ORC_INF && !tight[v]) { *where = v; rc = 3; }
    if (rc == 0) {
        int64_t head = 0, tail = 0;
        queue[tail++] = src;
        seen[src] = 1;
        while (head < tail) {
            int32_t u = queue[head++];
            for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
                if (!seen[col[e]]) { seen[col[e]] = 1; queue[tail++] = col[e]; }
        }
        for (int32_t v = 0; v < n; ++v)
            if ((seen[v] != 0) != (dist[v] != ORC_INF)) { *where = v; rc = 4; break; }
    }
    free(tight); free(seen); free(queue);
    return rc;
}

/* Sum of out-degrees over vertices with a finite distance: the edges an SSSP
 * must look at (the useful work behind a traversed-edges-per-second rate). */
int64_t orc_sssp_reached_edges(int32_t n, const int32_t *row_ptr, const uint32_t *dist)
{
    int64_t s = 0;
    for (int32_t v = 0; v < n; ++v)
        if (dist[v] != ORC_INF) s += row_ptr[v + 1] - row_ptr[v];
    return s;
}

/* ----------------------------------------------------------------- BFS ---- */

/* Breadth-first levels from src (the BFS-Rec benchmark of Sec. V computes the
 * same levels by recursion): level[v] = number of edges on a shortest path, or
 * ORC_INF if v is unreachable.  A FIFO queue.  Returns 0, or -1 if memory runs
 * out. */
int orc_bfs(int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t src, uint32_t *level)
{
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!queue) return -1;
    for (int32_t v = 0; v < n; ++v) level[v] = ORC_INF;
    int32_t head = 0, tail = 0;
    level[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int32_t v = col[e];
            if (level[v] == ORC_INF) {
                level[v] = level[u] + 1;
                queue[tail++] = v;
            }
        }
    }
    free(queue);
    return 0;
}

/* ------------------------------------------------------- graph coloring ---- */

/* Graph coloring, the GC benchmark of Sec. V (named, not defined there): the
 * Jones-Plassmann rounds in which every uncolored vertex that outranks all of
 * its still-uncolored neighbours takes the round's number as its color.  A
 * vertex outranks another if its priority is larger, or equal with the larger
 * id.  g must be symmetric; self-loops are ignored.  color[v] = round of v.
 * Returns the number of rounds (colors), or -1 if memory runs out. */
static int outranks(const uint32_t *prio, int32_t a, int32_t b)
{
    return prio[a] > prio[b] || (prio[a] == prio[b] && a > b);
}

int32_t orc_color_jp(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint32_t *prio, int32_t *color)
{
    int32_t *ready = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!ready) return -1;
    for (int32_t v = 0; v < n; ++v) color[v] = -1;
    int32_t left = n, round = 0;
    while (left > 0) {
        int32_t k = 0;
        for (int32_t v = 0; v < n; ++v) {
            if (color[v] >= 0) continue;
            int ok = 1;
            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1] && ok; ++e) {
                int32_t u = col[e];
                if (u != v && color[u] < 0 && outranks(prio, u, v)) ok = 0;
            }
            if (ok) ready[k++] = v;
        }
        for (int32_t i = 0; i < k; ++i) color[ready[i]] = round;
        left -= k;
        ++round;
    }
    free(ready);
    return round;
}

/* The recurrence that fixes the coloring above: color[v] = 0 if no neighbour
 * outranks v, else 1 + the largest color among the neighbours that outrank v.
 * Returns the number of vertices violating it (or a neighbour sharing the
 * color); *first gets the first one (or -1). */
int64_t orc_color_certify(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint32_t *prio,
                          const int32_t *color, int64_t *first)
{
    int64_t bad = 0;
    *first = -1;
    for (int32_t v = 0; v < n; ++v) {
        int32_t want = 0;
        int clash = 0;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int32_t u = col[e];
            if (u == v) continue;
            if (outranks(prio, u, v) && color[u] + 1 > want) want = color[u] + 1;
            if (color[u] == color[v]) clash = 1;
        }
        if (clash || color[v] != want) {
            if (bad == 0) *first = v;
            ++bad;
        }
    }
    return bad;
}

/* ---------------------------------------------------------------- SpMV ---- */

/* y[r] = sum_e val[e] * x[col[e]] and b[r] = sum_e |val[e] * x[col[e]]|, in
 * binary64 (each product of two binary32 values is exact in binary64). */
void orc_spmv_f64(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *val, const float *x,
                  double *y, double *b)
{
    for (int32_t r = 0; r < n; ++r) {
        double s = 0.0, a = 0.0;
        for (int32_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
            double p = (double)val[e] * (double)x[col[e]];
            s += p;
            a += fabs(p);
        }
        y[r] = s;
        b[r] = a;
    }
}

/* Per-row tolerance test |y - y_ref| <= rtol * b.  Returns the number of
 * failing rows; *first gets the first one (or -1). */
int64_t orc_spmv_check(int32_t n, const double *y_ref, const double *b, const float *y, double rtol,
                       int64_t *first)
{
    int64_t bad = 0;
    *first = -1;
    for (int32_t r = 0; r < n; ++r) {
        double err = fabs((double)y[r] - y_ref[r]);
        if (!(err <= rtol * b[r])) {
            if (bad == 0) *first = r;
            ++bad;
        }
    }
    return bad;
}

/* ------------------------------------------------------------ PageRank ---- */

/* PageRank, the PR benchmark of Sec. V.  The paper names it without a formula;
 * this is the usual damped iteration in which the rank held by vertices without
 * out-edges is spread evenly over all vertices, so the ranks always sum to 1.
 * From rank = 1/n, `iterations` synchronous sweeps of
 *   rank'[v] = (1 - d) / n + d * (sum over edges u -> v of rank[u] / outdeg(u) + D / n),
 *   D = sum of rank[u] over the vertices u with outdeg(u) = 0.
 * The graph comes as its in-edges: row v of (in_row_ptr, in_col) lists the
 * source of every edge into v, with multiplicity; out_degree[u] is u's number
 * of out-edges.  Binary64 throughout.  Returns 0, or -1 if memory runs out. */
int orc_pagerank_f64(int32_t n, const int32_t *in_row_ptr, const int32_t *in_col, const int32_t *out_degree,
                     int32_t iterations, double d, double *rank)
{
    double *cur = rank, *nxt = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!nxt) return -1;
    for (int32_t v = 0; v < n; ++v) cur[v] = 1.0 / n;
    for (int32_t it = 0; it < iterations; ++it) {
        double dangling = 0.0;
        for (int32_t u = 0; u < n; ++u)
            if (out_degree[u] == 0) dangling += cur[u];
        for (int32_t v = 0; v < n; ++v) {
            double s = 0.0;
            for (int32_t e = in_row_ptr[v]; e < in_row_ptr[v + 1]; ++e) {
                int32_t u = in_col[e];
                s += cur[u] / out_degree[u];
            }
            nxt[v] = (1.0 - d) / n + d * (s + dangling / n);
        }
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    if (cur != rank) {
        memcpy(rank, cur, sizeof(double) * (size_t)n);
        free(cur);
    } else {
        free(nxt);
    }
    return 0;
}

/* --------------------------------------------------------------- trees ---- */

/* Structure check of a rooted tree in the form the recursion of Fig. 1(c)
 * walks: node 0 is the root (parent -1); child_ptr[0..n] is a non-decreasing
 * offset array from 0 to n-1; every child entry names a node in [1, n) whose
 * parent[] is the node listing it; no node is listed twice; and every node is
 * reached from the root (so the parent links have no cycle).  Returns 0 for a
 * tree; otherwise a code naming the first violation:
 *   1 n < 1                      2 parent[0] != -1 or child_ptr[0] != 0
 *   3 child_ptr[n] != n - 1      4 child_ptr decreases somewhere
 *   5 child entry out of [1, n)  6 child entry whose parent[] is another node
 *   7 node listed twice          8 node not reached from the root
 *  -2 out of memory */
int orc_tree_validate(int32_t n, const int32_t *parent, const int32_t *child_ptr, const int32_t *child)
{
    if (n < 1) return 1;
    if (parent[0] != -1 || child_ptr[0] != 0) return 2;
    if (child_ptr[n] != n - 1) return 3;
    for (int32_t p = 0; p < n; ++p)
        if (child_ptr[p + 1] < child_ptr[p]) return 4;
    /* from here on every offset lies in [0, n-1], so child[] is read in bounds */
    uint8_t *listed = (uint8_t *)calloc((size_t)n, 1);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!listed || !queue) {
        free(listed);
        free(queue);
        return -2;
    }
    int rc = 0;
    for (int32_t p = 0; p < n && rc == 0; ++p)
        for (int32_t e = child_ptr[p]; e < child_ptr[p + 1] && rc == 0; ++e) {
            const int32_t c = child[e];
            if (c <= 0 || c >= n) rc = 5;
            else if (parent[c] != p) rc = 6;
            else if (listed[c]) rc = 7;
            else listed[c] = 1;
        }
    if (rc == 0) {
        /* n - 1 distinct entries in [1, n): every non-root node is listed once;
         * breadth-first from the root then visits each node at most once */
        int64_t head = 0, tail = 0;
        queue[tail++] = 0;
        while (head < tail) {
            const int32_t u = queue[head++];
            for (int32_t e = child_ptr[u]; e < child_ptr[u + 1]; ++e) queue[tail++] = child[e];
        }
        if (tail != n) rc = 8;
    }
    free(listed);
    free(queue);
    return rc;
}

/* Breadth-first order of the nodes from the root (level by level, the order
 * in which recursive launches of Fig. 1(c) would reach them). */
static int bfs_order(int32_t n, const int32_t *child_ptr, const int32_t *child, int32_t *order)
{
    int64_t head = 0, tail = 0;
    order[tail++] = 0;
    while (head < tail) {
        int32_t u = order[head++];
        for (int32_t e = child_ptr[u]; e < child_ptr[u + 1]; ++e) {
            if (tail >= n) return -1;
            order[tail++] = child[e];
        }
    }
    return tail == n ? 0 : -1;
}

/* Tree descendants: desc[v] = number of proper descendants of v.  Leaf work
 * sets 0; post-work folds each child in as 1 + desc[child].  The reverse
 * breadth-first order finishes every child before its parent. */
int orc_tree_descendants(int32_t n, const int32_t *child_ptr, const int32_t *child, int32_t *desc)
{
    if (n < 1) return -1;
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!order) return -2;
    if (bfs_order(n, child_ptr, child, order) != 0) { free(order); return -1; }
    for (int32_t i = n - 1; i >= 0; --i) {
        int32_t v = order[i];
        int64_t s = 0;
        for (int32_t e = child_ptr[v]; e < child_ptr[v + 1]; ++e) s += 1 + (int64_t)desc[child[e]];
        desc[v] = (int32_t)s;
    }
    free(order);
    return 0;
}

/* Tree heights: height[v] = edges on the longest downward path from v to a
 * leaf (leaf = 0); post-work takes 1 + the largest child height. */
int orc_tree_height(int32_t n, const int32_t *child_ptr, const int32_t *child, int32_t *height)
{
    if (n < 1) return -1;
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!order) return -2;
    if (bfs_order(n, child_ptr, child, order) != 0) { free(order); return -1; }
    for (int32_t i = n - 1; i >= 0; --i) {
        int32_t v = order[i];
        int32_t h = 0;
        for (int32_t e = child_ptr[v]; e < child_ptr[v + 1]; ++e)
            if (1 + height[child[e]] > h) h = 1 + height[child[e]];
        height[v] = h;
    }
    free(order);
    return 0;
}

/* Brute force TD: every node walks up to the root and counts itself at each
 * proper ancestor.  Uses only parent[]. */
int orc_tree_descendants_brute(int32_t n, const int32_t *parent, int32_t *desc)
{
    memset(desc, 0, sizeof(int32_t) * (size_t)n);
    for (int32_t v = 0; v < n; ++v) {
        int64_t steps = 0;
        for (int32_t u = parent[v]; u >= 0; u = parent[u]) {
            desc[u]++;
            if (++steps > n) return -1;
        }
    }
    return 0;
}

/* Brute force TH: every node walks up; an ancestor k steps above it has a
 * downward path of length k, so its height is at least k. */
int orc_tree_height_brute(int32_t n, const int32_t *parent, int32_t *height)
{
    memset(height, 0, sizeof(int32_t) * (size_t)n);
    for (int32_t v = 0; v < n; ++v) {
        int32_t k = 0;
        for (int32_t u = parent[v]; u >= 0; u = parent[u]) {
            ++k;
            if (k > height[u]) height[u] = k;
            if (k > n) return -1;
        }
    }
    return 0;
}

/* ------------------------------------------------ consolidation bookkeeping */

/* Work items above the threshold: the items that Fig. 1(a) hands to a child
 * launch and that a consolidated parent inserts into its buffer instead. */
int64_t orc_count_heavy(int64_t count, const int64_t *work, int64_t threshold)
{
    int64_t c = 0;
    for (int64_t i = 0; i < count; ++i) c += work[i] > threshold;
    return c;
}

/* Bookkeeping of Sec. IV.A / Fig. 2.  Parent threads 0..count-1 carry work[i];
 * a thread with work[i] > threshold needs a child.  The basic template
 * launches one child per such thread.  Consolidation over scopes of `scope`
 * consecutive threads (warp, block or the whole grid) buffers those threads'
 * items and issues one consolidated child per scope that buffered anything.
 * Outputs: basic launches, consolidated dispatches, buffered items, and the
 * total work the consolidated children carry. */
void orc_consolidation_plan(int64_t count, const int64_t *work, int64_t threshold, int64_t scope,
                            int64_t *basic_launches, int64_t *dispatches, int64_t *items, int64_t *total)
{
    int64_t bl = 0, ds = 0, it = 0, tw = 0;
    if (scope < 1) scope = 1;
    for (int64_t g = 0; g < count; g += scope) {
        int64_t any = 0;
        for (int64_t i = g; i < count && i < g + scope; ++i) {
            if (work[i] > threshold) {
                ++bl;
                ++it;
                tw += work[i];
                any = 1;
            }
        }
        ds += any;
    }
    *basic_launches = bl;
    *dispatches = ds;
    *items = it;
    *total = tw;
}

/* Per-buffer capacity estimate of Sec. IV.E: the number of threads whose
 * launches are consolidated, times the variables buffered per item, times the
 * expected number of items per thread (default 4). */
int64_t orc_per_buffer_size(int64_t total_thread, int64_t total_buff_var, int64_t items_per_thread)
{
    return total_thread * total_buff_var * items_per_thread;
}

/* KC_X of Sec. IV.E: the single-kernel maximum-occupancy configuration (B, T)
 * downgraded to (ceil(B / X), T) so that X kernels fit at once. */
void orc_kc_config(int64_t blocks, int64_t threads, int64_t x, int64_t *out_blocks, int64_t *out_threads)
{
    *out_blocks = (blocks + x - 1) / x;
    if (*out_blocks < 1) *out_blocks = 1;
    *out_threads = threads;
}
