// Graph coloring with workload consolidation (the GC benchmark of Sec. V, an
// irregular loop like Fig. 1(b)).
//
// Jones-Plassmann coloring of a symmetric graph: a vertex takes color r in the
// round after its last outranking neighbour was colored (r - 1), color 0 if no
// neighbour outranks it (larger priority, ties to the larger id).  This is the
// round-by-round definition (every uncolored vertex that outranks all of its
// uncolored neighbours takes the round's color) computed data-driven: wait[v]
// counts the outranking neighbours still uncolored; a vertex colored in round
// r loops over its neighbours and releases the ones it outranks, and a vertex
// whose count reaches zero joins the queue of round r + 1 with color r + 1.
// Every edge is visited once by the count pass and once by a release, instead
// of once per round.
//
// A queued vertex's release loop is the nested work; one with more than
// `threshold` neighbours is consolidated per mode:
//   wave  - the wave's ballot mask is the buffer; the wave walks each buffered
//           vertex's neighbours 64 x kUnroll at a time (no barrier).
//   block - thread-ordered LDS buffer; after the barrier the block walks the
//           concatenated neighbour ranges.
//   In both, a buffered vertex with more than one chunk (64 * items_per_lane)
//   of neighbours is handed on as chunks to a global buffer that a grid-wide
//   drain walks right after the parent, one wave per chunk (the KC_X rule of
//   Sec. IV.E: a warp's or block's child gets many blocks), in the count pass
//   and in every round.
//   grid  - global buffer of (vertex, neighbour range) chunks drained by a
//           moldable grid after the kernel boundary, one wave per chunk.  The
//           thread that readies a vertex buffers its range right away, so the
//           drain of round r is also the parent of round r + 1: one kernel
//           per round.
//   flat  - every vertex walks all of its neighbours itself.
// Outside grid mode `threshold` applies in the count pass and the rounds
// alike; in grid mode it applies to the count pass, and every readied
// vertex's range is buffered.
#include <algorithm>
#include <climits>
#include <cstring>

#include "wc_block.h"
#include "wc_device.h"
#include "wc_internal.h"
#include "wc_stats.h"

namespace wc {
namespace {

constexpr int kPad = 32;        // ring entries on separate 128-byte lines
constexpr int kUnroll = 4;      // neighbours in flight per lane
constexpr int kNoRelease = INT_MIN;  // rcol flag: nothing to release along this edge

struct ColorArgs {
    const int *row_ptr;
    const int *col;
    const uint32_t *prio;
    int *color;       // -1 while uncolored
    int *wait;        // outranking neighbours not yet colored
    int *rcol;        // col with bit 31 set where the row's vertex does not outrank the neighbour
    int *queue0;      // vertices colored in even rounds
    int *queue1;      // ... in odd rounds
    int *qtail;       // ring of 3 (stride kPad): size of the queue of round r
    int *chunk_tail;  // ring of 3 (stride kPad)
    int4 *chunks;     // (v, begin, end, count pass: prio[v]); grid: the chunks of even rounds
    int4 *chunks1;    // grid: the chunks of odd rounds
    long long chunk_cap;
    int *colored;     // grid: vertices colored so far
    int n;
    int threshold;
    int chunk;
    unsigned long long *host_ring;
    DevStats *stats;
    int want_stats;
};

__device__ __forceinline__ bool above(uint32_t pu, int u, uint32_t pv, int v)
{
    return pu > pv || (pu == pv && u > v);
}

// Where readied vertices go: the next round's vertex queue, or (grid mode)
// the next round's chunk buffer, with the queue taking vertices whose chunks
// do not fit (buffer full).
struct Next {
    int *queue;
    int *queue_tail;
    int4 *chunks;
    int *chunk_tail;
};

// Readied vertex w (priority pw) takes color_next and is queued.  Every active
// lane of the wave calls this together.
template <bool CHUNKED>
__device__ __forceinline__ void push_ready(const ColorArgs &a, bool ready, int w, int color_next, const Next &nx,
                                           int &readied)
{
    if (ready) {
        a.color[w] = color_next;
        ++readied;
    }
    if constexpr (!CHUNKED) {
        const int s = wave_reserve(ready, nx.queue_tail);
        if (ready) nx.queue[s] = w;
    } else {
        int beg = 0, end = 0;
        if (ready) {
            beg = a.row_ptr[w];
            end = a.row_ptr[w + 1];
        }
        const int nch = (end - beg + a.chunk - 1) / a.chunk;
        const bool one = ready && nch == 1;
        const int s = wave_reserve(one, nx.chunk_tail);
        bool defer = false;
        if (one) {
            if (s < a.chunk_cap) nx.chunks[s] = make_int4(w, beg, end, 0);
            else defer = true;
        } else if (ready && nch > 1) {
            const long long base = atomic_add_dev(nx.chunk_tail, nch);
            if (base + nch <= a.chunk_cap) {
                for (int c = 0; c < nch; ++c) {
                    const int cb = beg + c * a.chunk;
                    nx.chunks[base + c] = make_int4(w, cb, min(end, cb + a.chunk), 0);
                }
            } else {
                // reserved slots below the capacity get empty ranges (the drain
                // reads no stale chunk there)
                for (long long c = base; c < base + nch && c < a.chunk_cap; ++c) nx.chunks[c] = make_int4(w, 0, 0, 0);
                defer = true;
            }
        }
        if (defer) {
            // buffer full: the next round walks w with one lane (fallback)
            a.stats->overflowed = 1;
            nx.queue[atomic_add_dev(nx.queue_tail, 1)] = w;
        }
    }
}

// Wave and block modes: the lanes with nch > 0 hand their vertex's range on
// as chunks (v, begin, end, tag) of the global buffer, one reservation per
// wave on `tail`; the wave writes each vertex's chunks together.  Returns
// false on a lane whose chunks do not all fit (buffer full): its reserved
// entries are marked empty and the lane walks the range itself (fallback).
// Every lane of the wave calls this.
__device__ __forceinline__ bool spill_chunks(const ColorArgs &a, int *tail, int v, int beg, int end, int nch, int tag)
{
    const int slot = wave_reserve_n(nch, tail);
    const bool fits = nch > 0 && (long long)slot + nch <= a.chunk_cap;
    uint64_t m = __ballot(fits);
    while (m) {
        const int b = __builtin_ctzll(m);
        m &= m - 1;
        const int s0 = readlane(slot, b), n0 = readlane(nch, b), rb = readlane(beg, b), re = readlane(end, b);
        const int rv = readlane(v, b), rt = readlane(tag, b);
        for (int c = lane_id(); c < n0; c += kWave) {
            const int cb = rb + c * a.chunk;
            a.chunks[s0 + c] = make_int4(rv, cb, min(re, cb + a.chunk), rt);
        }
    }
    if (nch > 0 && !fits) {
        for (long long c = slot; c < (long long)slot + nch && c < a.chunk_cap; ++c) a.chunks[c] = make_int4(v, 0, 0, 0);
        a.stats->overflowed = 1;
    }
    return nch == 0 || fits;
}

// A vertex colored in round r releases the neighbours e = first + k * stride
// < end of its row that it outranks (the count pass flagged the others in
// rcol); a neighbour whose count reaches zero is readied with color r + 1.
// Every active lane of the wave calls this together (the appends are
// wave-aggregated); first, stride and end may differ per lane.  Returns the
// number of releases.
template <bool CHUNKED>
__device__ __forceinline__ int release_range(const ColorArgs &a, int first, int stride, int end, int color_next,
                                             const Next &nx, int &readied)
{
    int rel = 0;
    for (int e0 = first; e0 < end; e0 += kUnroll * stride) {
        int w[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            const int e = e0 + k * stride;
            w[k] = e < end ? a.rcol[e] : kNoRelease;
        }
        int old[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            old[k] = w[k] >= 0 ? atomic_add_dev(&a.wait[w[k]], -1) : 0;
            rel += w[k] >= 0 ? 1 : 0;
        }
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) push_ready<CHUNKED>(a, old[k] == 1, w[k], color_next, nx, readied);
    }
    return rel;
}

// The consolidated child of a block (G = BLOCK) over its buffer of nb
// vertices: vertex i releases along rcol[beg_i, beg_i + deg_i),
// pre_i being the exclusive prefix of the degrees (total in all).  The group
// walks the concatenated ranges, G * kUnroll edges per step, thread t taking
// flattened edges t, t + G, ...; a cursor that only moves forward finds each
// edge's vertex.  Returns the number of releases.
template <int G>
__device__ __forceinline__ int release_items(const ColorArgs &a, const int *ibeg, const int *ipre, int nb, int total,
                                             int t, int color_next, const Next &nx, int &readied)
{
    int rel = 0, it = 0;
    for (int j0 = t; j0 < total; j0 += G * kUnroll) {
        int w[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            const int j = j0 + k * G;
            w[k] = kNoRelease;
            if (j < total) {
                while (it + 1 < nb && ipre[it + 1] <= j) ++it;
                w[k] = a.rcol[ibeg[it] + (j - ipre[it])];
            }
        }
        int old[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            old[k] = w[k] >= 0 ? atomic_add_dev(&a.wait[w[k]], -1) : 0;
            rel += w[k] >= 0 ? 1 : 0;
        }
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) push_ready<false>(a, old[k] == 1, w[k], color_next, nx, readied);
    }
    return rel;
}

template <int BLOCK>
struct ColorLds {
    int beg[BLOCK];
    int pre[BLOCK + 1];
    int scan_tmp[2 * (BLOCK / kWave)];
    int base;
};

// Round r outside grid mode: thread i takes the i-th vertex of the round's
// queue (colored r).
template <int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void color_round(ColorArgs a, int r)
{
    __shared__ ColorLds<BLOCK> sb;
    const int size = a.qtail[(r % 3) * kPad];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.qtail[((r + 2) % 3) * kPad] = 0;
        a.chunk_tail[((r + 2) % 3) * kPad] = 0;
        publish_host(a.host_ring, r % kHostRing, a.stats, size);
    }
    if (size == 0) return;
    const int *q = (r & 1) ? a.queue1 : a.queue0;
    const Next nx{(r & 1) ? a.queue0 : a.queue1, &a.qtail[((r + 1) % 3) * kPad], nullptr, nullptr};
    const int lane = lane_id();
    int readied = 0;
    StatAcc acc;
    for (int base = blockIdx.x * BLOCK; base < size; base += gridDim.x * BLOCK) {
        const int i = base + threadIdx.x;
        const bool member = i < size;
        int beg = 0, end = 0;
        if (member) {
            const int v = q[i];
            beg = a.row_ptr[v];
            end = a.row_ptr[v + 1];
        }
        const int deg = end - beg;
        const bool heavy = MODE != WC_FLAT && deg > a.threshold;
        if (a.want_stats) {
            acc.edges += deg;
            acc.buffered += heavy ? deg : 0;
            acc.items += heavy ? 1 : 0;
            if (MODE == WC_WAVE && __ballot(heavy) && lane == 0) acc.dispatches += 1;
        }
        // buffered vertices with more than one chunk go to the round's drain
        bool spill = heavy && deg > a.chunk, inline_walk = member && !heavy;
        if (__ballot(spill)) {
            const int v = spill ? q[i] : 0;
            if (!spill_chunks(a, &a.chunk_tail[(r % 3) * kPad], v, beg, end, spill ? (deg + a.chunk - 1) / a.chunk : 0,
                              0))
                inline_walk = true;
        }
        const bool mine = heavy && !spill;
        if (inline_walk) acc.updates += release_range<false>(a, beg, 1, end, r + 1, nx, readied);
        if constexpr (MODE == WC_WAVE) {
            // the ballot mask is the wave's buffer; the wave walks each buffered
            // vertex's range 64 x kUnroll neighbours at a time (walking the
            // concatenated ranges measured 12% slower here)
            uint64_t mask = __ballot(mine);
            while (mask) {
                const int b = __builtin_ctzll(mask);
                mask &= mask - 1;
                acc.updates_buffered +=
                    release_range<false>(a, readlane(beg, b) + lane, kWave, readlane(end, b), r + 1, nx, readied);
            }
        } else if constexpr (MODE == WC_BLOCK) {
            int k, off, nb, total;
            block_scan2<BLOCK>(mine ? 1 : 0, mine ? deg : 0, sb.scan_tmp, k, off, nb, total);
            if (mine) {
                sb.beg[k] = beg;
                sb.pre[k] = off;
            }
            if (a.want_stats && __syncthreads_or(heavy ? 1 : 0) && threadIdx.x == 0) acc.dispatches += 1;
            if (threadIdx.x == 0) sb.pre[nb] = total;
            __syncthreads();
            acc.updates_buffered += release_items<BLOCK>(a, sb.beg, sb.pre, nb, total, threadIdx.x, r + 1, nx, readied);
            __syncthreads();  // the LDS buffer is reused by the next window
        }
    }
    if (a.want_stats) stat_flush(a.stats, acc);
}

// Wave and block modes: the chunks that round r's parent handed on, one wave
// per chunk, right after the parent; readied vertices join round r + 1's queue.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void color_round_drain(ColorArgs a, int r)
{
    const int tail = a.chunk_tail[(r % 3) * kPad];
    const int total = (long long)tail < a.chunk_cap ? tail : (int)a.chunk_cap;
    if (total == 0) return;
    const Next nx{(r & 1) ? a.queue0 : a.queue1, &a.qtail[((r + 1) % 3) * kPad], nullptr, nullptr};
    const int gw = (blockIdx.x * BLOCK + threadIdx.x) / kWave;
    const int nw = gridDim.x * (BLOCK / kWave);
    int readied = 0;
    StatAcc acc;
    for (int c = gw; c < total; c += nw) {
        const int4 d = a.chunks[c];
        const int beg = __builtin_amdgcn_readfirstlane(d.y), end = __builtin_amdgcn_readfirstlane(d.z);
        acc.updates_buffered += release_range<false>(a, beg + lane_id(), kWave, end, r + 1, nx, readied);
    }
    if (a.want_stats) stat_flush(a.stats, acc);
}

// Round r in grid mode: one wave per buffered chunk (a readied vertex's
// neighbour range, buffered while round r - 1 ran), then one lane per vertex
// the buffer could not take.  Vertices readied here buffer their ranges for
// round r + 1.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void color_round_grid(ColorArgs a, int r)
{
    const int nchunks = a.chunk_tail[(r % 3) * kPad];
    const int ndefer = a.qtail[(r % 3) * kPad];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.chunk_tail[((r + 2) % 3) * kPad] = 0;
        a.qtail[((r + 2) % 3) * kPad] = 0;
        publish_host(a.host_ring, r % kHostRing, a.stats, (nchunks != 0 || ndefer != 0) ? 1 : 0);
    }
    if (nchunks == 0 && ndefer == 0) return;
    const int total = (long long)nchunks < a.chunk_cap ? nchunks : (int)a.chunk_cap;
    const int4 *cur = (r & 1) ? a.chunks1 : a.chunks;
    const Next nx{(r & 1) ? a.queue0 : a.queue1, &a.qtail[((r + 1) % 3) * kPad], (r & 1) ? a.chunks : a.chunks1,
                  &a.chunk_tail[((r + 1) % 3) * kPad]};
    const int gw = (blockIdx.x * BLOCK + threadIdx.x) / kWave;
    const int nw = gridDim.x * (BLOCK / kWave);
    int readied = 0;
    StatAcc acc;
    if (a.want_stats && blockIdx.x == 0 && threadIdx.x == 0 && total > 0) acc.dispatches = 1;
    for (int c = gw; c < total; c += nw) {
        const int4 d = cur[c];
        const int beg = __builtin_amdgcn_readfirstlane(d.y), end = __builtin_amdgcn_readfirstlane(d.z);
        if (a.want_stats && lane_id() == 0) {
            acc.items += 1;
            acc.buffered += end - beg;
            acc.edges += end - beg;
        }
        acc.updates_buffered += release_range<true>(a, beg + lane_id(), kWave, end, r + 1, nx, readied);
    }
    const int *dq = (r & 1) ? a.queue1 : a.queue0;
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < ndefer; i += gridDim.x * BLOCK) {
        const int v = dq[i];
        const int beg = a.row_ptr[v], end = a.row_ptr[v + 1];
        if (a.want_stats) acc.edges += end - beg;
        acc.updates += release_range<true>(a, beg, 1, end, r + 1, nx, readied);
    }
    readied = wave_sum_i(readied);
    if (lane_id() == 0 && readied) (void)atomic_add_dev(a.colored, readied);
    if (a.want_stats) stat_flush(a.stats, acc);
}

// Clears the rings before the count pass appends to the first queue.
__global__ void color_reset(ColorArgs a)
{
    if (threadIdx.x < 3) {
        a.qtail[threadIdx.x * kPad] = 0;
        a.chunk_tail[threadIdx.x * kPad] = 0;
    }
    if (threadIdx.x == 0) *a.colored = 0;
}

// Grid mode: hands the number of colored vertices to the host.
__global__ void color_publish(ColorArgs a)
{
    if (threadIdx.x == 0) publish_host(a.host_ring, kHostSlotGraph, a.stats, *a.colored);
}

// Edge e of v's row toward u: does u outrank v?  Flags the edge in rcol when
// v has nothing to release along it (u outranks v, or a self-loop).
__device__ __forceinline__ bool count_edge(const ColorArgs &a, int v, uint32_t pv, int u, int e)
{
    const bool o = u != v && above(a.prio[u], u, pv, v);
    a.rcol[e] = (o || u == v) ? (u | kNoRelease) : u;
    return o;
}

// Neighbours e = first + k * stride < end of v (priority pv) that outrank v.
__device__ __forceinline__ int count_range(const ColorArgs &a, int v, uint32_t pv, int first, int stride, int end)
{
    int cnt = 0;
    for (int e0 = first; e0 < end; e0 += kUnroll * stride) {
        int u[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            const int e = e0 + k * stride;
            u[k] = e < end ? a.col[e] : v;
        }
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            const int e = e0 + k * stride;
            if (e < end) cnt += count_edge(a, v, pv, u[k], e) ? 1 : 0;
        }
    }
    return cnt;
}

template <int BLOCK>
struct CountLds {
    int v[BLOCK];
    int beg[BLOCK];
    uint32_t p[BLOCK];
    int pre[BLOCK + 1];
    int cnt[BLOCK];
    int scan_tmp[2 * (BLOCK / kWave)];
    int base;
};

// Count pass, the first irregular loop: wait[v] = neighbours that outrank v.
// A row with more than `threshold` entries is consolidated per mode (grid,
// and wave and block rows longer than one chunk: its chunks are counted by
// color_count_drain, which adds to wait[v] = 0).
template <int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void color_count(ColorArgs a)
{
    __shared__ CountLds<BLOCK> sb;
    const int lane = lane_id();
    for (int base = blockIdx.x * BLOCK; base < a.n; base += gridDim.x * BLOCK) {
        const int v = base + threadIdx.x;
        const bool member = v < a.n;
        int beg = 0, end = 0;
        uint32_t pv = 0;
        if (member) {
            beg = a.row_ptr[v];
            end = a.row_ptr[v + 1];
            pv = a.prio[v];
        }
        const int deg = end - beg;
        const bool heavy = MODE != WC_FLAT && deg > a.threshold;
        // wave and block modes: rows with more than one chunk go to the drain
        const bool spill = (MODE == WC_WAVE || MODE == WC_BLOCK) && heavy && deg > a.chunk;
        bool inline_count = member && !heavy;
        if constexpr (MODE == WC_WAVE || MODE == WC_BLOCK) {
            if (__ballot(spill) &&
                !spill_chunks(a, &a.chunk_tail[2 * kPad], v, beg, end, spill ? (deg + a.chunk - 1) / a.chunk : 0,
                              (int)pv))
                inline_count = true;
        }
        const bool mine = heavy && !spill;
        int cnt = 0;
        if (inline_count) cnt = count_range(a, v, pv, beg, 1, end);
        if constexpr (MODE == WC_WAVE) {
            uint64_t mask = __ballot(mine);
            while (mask) {
                const int b = __builtin_ctzll(mask);
                mask &= mask - 1;
                const int c = wave_sum_i(count_range(a, readlane(v, b), readlane_u(pv, b), readlane(beg, b) + lane,
                                                     kWave, readlane(end, b)));
                if (lane == b) cnt = c;
            }
        } else if constexpr (MODE == WC_BLOCK) {
            int k, off, nb, total;
            block_scan2<BLOCK>(mine ? 1 : 0, mine ? deg : 0, sb.scan_tmp, k, off, nb, total);
            if (mine) {
                sb.v[k] = v;
                sb.beg[k] = beg;
                sb.p[k] = pv;
                sb.pre[k] = off;
                sb.cnt[k] = 0;
            }
            if (threadIdx.x == 0) sb.pre[nb] = total;
            __syncthreads();
            int it = 0;
            for (int j = threadIdx.x; j < total; j += BLOCK) {
                while (it + 1 < nb && sb.pre[it + 1] <= j) ++it;
                const int e = sb.beg[it] + (j - sb.pre[it]);
                if (count_edge(a, sb.v[it], sb.p[it], a.col[e], e)) atomicAdd(&sb.cnt[it], 1);
            }
            __syncthreads();
            if (mine) cnt = sb.cnt[k];
            __syncthreads();  // the LDS buffer is reused by the next window
        } else if constexpr (MODE == WC_GRID) {
            if (__syncthreads_or(heavy ? 1 : 0)) {
                const int nch = heavy ? (deg + a.chunk - 1) / a.chunk : 0;
                int excl, unused, tot, unused2;
                block_scan2<BLOCK>(nch, 0, sb.scan_tmp, excl, unused, tot, unused2);
                if (threadIdx.x == 0) sb.base = tot ? atomic_add_dev(&a.chunk_tail[2 * kPad], tot) : 0;
                __syncthreads();
                const long long slot = (long long)sb.base + excl;
                const bool fits = slot + nch <= a.chunk_cap;
                if (heavy) {
                    if (fits) {
                        for (int c = 0; c < nch; ++c) {
                            const int cb = beg + c * a.chunk;
                            a.chunks[slot + c] = make_int4(v, cb, min(end, cb + a.chunk), (int)pv);
                        }
                    } else {
                        a.stats->overflowed = 1;
                        for (long long c = slot; c < slot + nch && c < a.chunk_cap; ++c)
                            a.chunks[c] = make_int4(v, 0, 0, 0);
                        cnt = count_range(a, v, pv, beg, 1, end);  // fallback: counted inline
                    }
                }
                __syncthreads();  // sb.base is rewritten by the next window
            }
        }
        if (member) a.wait[v] = cnt;
    }
}

// One wave per chunk of a buffered row (grid mode; wave and block modes: rows
// longer than one chunk) adds its count to wait[v].
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void color_count_drain(ColorArgs a)
{
    const int tail = a.chunk_tail[2 * kPad];
    const int total = (long long)tail < a.chunk_cap ? tail : (int)a.chunk_cap;
    const int gw = (blockIdx.x * BLOCK + threadIdx.x) / kWave;
    const int nw = gridDim.x * (BLOCK / kWave);
    for (int c = gw; c < total; c += nw) {
        const int4 d = a.chunks[c];
        const int v = __builtin_amdgcn_readfirstlane(d.x);
        const int cnt = wave_sum_i(count_range(a, v, (uint32_t)__builtin_amdgcn_readfirstlane(d.w),
                                               __builtin_amdgcn_readfirstlane(d.y) + lane_id(), kWave,
                                               __builtin_amdgcn_readfirstlane(d.z)));
        if (lane_id() == 0 && cnt) (void)atomic_add_dev(&a.wait[v], cnt);
    }
}

// Vertices that no neighbour outranks take color 0 and form round 0 (grid:
// their neighbour ranges are buffered as chunks); the others start
// uncolored.  One reservation per block step.
constexpr int kSeedBlock = 256;
template <bool CHUNKED>
__global__ __launch_bounds__(kSeedBlock) void color_seed(ColorArgs a)
{
    __shared__ int scan_tmp[2 * (kSeedBlock / kWave)];
    __shared__ int s_base;
    for (int base = blockIdx.x * kSeedBlock; base < a.n; base += gridDim.x * kSeedBlock) {
        const int v = base + threadIdx.x;
        const bool member = v < a.n;
        const bool first = member && a.wait[v] == 0;
        if (member) a.color[v] = first ? 0 : -1;
        if constexpr (!CHUNKED) {
            int k, unused, tot, unused2;
            block_scan2<kSeedBlock>(first ? 1 : 0, 0, scan_tmp, k, unused, tot, unused2);
            if (threadIdx.x == 0 && tot) s_base = atomic_add_dev(&a.qtail[0], tot);
            __syncthreads();
            if (first) a.queue0[s_base + k] = v;
        } else {
            int beg = 0, end = 0;
            if (first) {
                beg = a.row_ptr[v];
                end = a.row_ptr[v + 1];
            }
            const int nch = (end - beg + a.chunk - 1) / a.chunk;
            int k, unused, tot, nfirst;
            block_scan2<kSeedBlock>(nch, first ? 1 : 0, scan_tmp, k, unused, tot, nfirst);
            if (threadIdx.x == 0) {
                if (tot) s_base = atomic_add_dev(&a.chunk_tail[0], tot);
                if (nfirst) (void)atomic_add_dev(a.colored, nfirst);
            }
            __syncthreads();
            if (nch) {
                const long long slot = (long long)s_base + k;
                if (slot + nch <= a.chunk_cap) {
                    for (int c = 0; c < nch; ++c) {
                        const int cb = beg + c * a.chunk;
                        a.chunks[slot + c] = make_int4(v, cb, min(end, cb + a.chunk), (int)a.prio[v]);
                    }
                } else {
                    a.stats->overflowed = 1;
                    for (long long c = slot; c < slot + nch && c < a.chunk_cap; ++c)
                        a.chunks[c] = make_int4(v, 0, 0, 0);
                    a.queue0[atomic_add_dev(&a.qtail[0], 1)] = v;
                }
            }
        }
        __syncthreads();  // s_base is rewritten by the next step
    }
}

struct ColorKernels {
    const void *round, *count, *count_drain, *round_drain;
};

template <int BLOCK>
ColorKernels pick_block(wc_mode mode)
{
    ColorKernels k{nullptr, nullptr, reinterpret_cast<const void *>(&color_count_drain<BLOCK>),
                   reinterpret_cast<const void *>(&color_round_drain<BLOCK>)};
    switch (mode) {
    case WC_FLAT:
        k.round = reinterpret_cast<const void *>(&color_round<WC_FLAT, BLOCK>);
        k.count = reinterpret_cast<const void *>(&color_count<WC_FLAT, BLOCK>);
        break;
    case WC_WAVE:
        k.round = reinterpret_cast<const void *>(&color_round<WC_WAVE, BLOCK>);
        k.count = reinterpret_cast<const void *>(&color_count<WC_WAVE, BLOCK>);
        break;
    case WC_BLOCK:
        k.round = reinterpret_cast<const void *>(&color_round<WC_BLOCK, BLOCK>);
        k.count = reinterpret_cast<const void *>(&color_count<WC_BLOCK, BLOCK>);
        break;
    default:
        k.round = reinterpret_cast<const void *>(&color_round_grid<BLOCK>);
        k.count = reinterpret_cast<const void *>(&color_count<WC_GRID, BLOCK>);
        break;
    }
    return k;
}

ColorKernels pick(wc_mode mode, int block)
{
    switch (block) {
    case 64: return pick_block<64>(mode);
    case 128: return pick_block<128>(mode);
    case 512: return pick_block<512>(mode);
    case 1024: return pick_block<1024>(mode);
    default: return pick_block<256>(mode);
    }
}

}  // namespace
}  // namespace wc

using namespace wc;

extern "C" wc_status wc_color(wc_ctx *ctx, const wc_csr *g, const uint32_t *prio, int32_t *color, wc_mode mode,
                              const wc_tune *tune, hipStream_t stream, wc_stats *stats)
{
    if (!ctx || !g) return fail(WC_EINVAL, "wc_color: NULL context or graph");
    if (mode < WC_FLAT || mode > WC_GRID) return fail(WC_EINVAL, "wc_color: bad mode");
    if (g->n < 0 || g->m < 0) return fail(WC_EINVAL, "wc_color: negative size");
    if (g->n == 0) {
        if (stats) std::memset(stats, 0, sizeof(*stats));
        return WC_OK;
    }
    if (!g->row_ptr || !prio || !color || (g->m > 0 && !g->col)) return fail(WC_EINVAL, "wc_color: NULL array");
    WC_HIP(hipSetDevice(ctx->device));
    int block = (tune && tune->block_threads > 0) ? tune->block_threads : 256;
    ColorKernels ks = pick(mode, block);
    int resident = resident_blocks(ctx, ks.round, block);
    Config cfg;
    wc_status st = resolve_tune(ctx, "color", mode, tune, resident, &cfg);
    if (st != WC_OK) return st;
    if (cfg.driver != 0) return fail(WC_EINVAL, "wc_color: only the relaunch driver (driver = 0) exists");
    if (cfg.block != block) {
        ks = pick(mode, cfg.block);
        resident = resident_blocks(ctx, ks.round, cfg.block);
    }
    const long long n = g->n, m = g->m;
    const int chunk = kWave * cfg.items_per_lane;
    const bool grid_mode = mode == WC_GRID;
    // grid mode: every vertex has ceil(deg / chunk) <= deg / chunk + 1 chunks
    // in the one round that colors it (and in the count pass), so n + m / chunk
    // + 1 entries per buffer never overflow.  Wave and block modes buffer only
    // vertices with more than one chunk of neighbours (ceil(deg / chunk) <
    // 2 deg / chunk each), in the count pass or one round at a time.
    const bool spills = mode == WC_WAVE || mode == WC_BLOCK;
    const long long cap_full = grid_mode ? n + m / chunk + 1 : spills ? 2 * (m / chunk) + 1 : 1;
    const long long cap = cfg.buf_capacity > 0 && mode != WC_FLAT ? std::min(cfg.buf_capacity, cap_full) : cap_full;
    const size_t need = 3 * padded(n * 4) + padded(m * 4) + 3 * padded(3 * kPad * 4) +
                        (grid_mode ? 2 : 1) * padded(cap * 16);
    st = pool_reserve(ctx, need, stream);
    if (st != WC_OK) return st;
    ColorArgs a;
    std::memset(&a, 0, sizeof(a));
    a.row_ptr = g->row_ptr;
    a.col = g->col;
    a.prio = prio;
    a.color = color;
    a.wait = pool_take<int>(ctx, n);
    a.rcol = pool_take<int>(ctx, m);
    a.queue0 = pool_take<int>(ctx, n);
    a.queue1 = pool_take<int>(ctx, n);
    a.qtail = pool_take<int>(ctx, 3 * kPad);
    a.chunk_tail = pool_take<int>(ctx, 3 * kPad);
    a.chunks = pool_take<int4>(ctx, cap);
    a.chunks1 = grid_mode ? pool_take<int4>(ctx, cap) : nullptr;
    a.chunk_cap = cap;
    a.colored = pool_take<int>(ctx, 3 * kPad);
    a.n = (int)n;
    a.threshold = cfg.threshold;
    a.chunk = chunk;
    a.host_ring = ctx->host_ring_dev;
    a.stats = ctx->dstats;
    a.want_stats = stats != nullptr;
    const int grid = std::max(1, std::min<int>(std::min(cfg.grid, resident), (int)((n + cfg.block - 1) / cfg.block)));
    const int dgrid = std::max(1, std::min(cfg.grid, resident));
    st = begin_call(ctx, stream, stats);
    if (st != WC_OK) return st;
    {
        void *args[] = {&a};
        st = launch(ctx, "color_reset", reinterpret_cast<const void *>(&color_reset), dim3(1), dim3(64), args,
                    stream);
        if (st == WC_OK) st = launch(ctx, "color_count", ks.count, dim3(grid), dim3(cfg.block), args, stream);
        if (st == WC_OK && mode != WC_FLAT)
            st = launch(ctx, "color_count_drain", ks.count_drain, dim3(dgrid), dim3(cfg.block), args, stream);
        const int sg = (int)std::min<long long>((n + kSeedBlock - 1) / kSeedBlock, 4096);
        const void *seed = grid_mode ? reinterpret_cast<const void *>(&color_seed<true>)
                                     : reinterpret_cast<const void *>(&color_seed<false>);
        if (st == WC_OK) st = launch(ctx, "color_seed", seed, dim3(sg), dim3(kSeedBlock), args, stream);
        if (st != WC_OK) return st;
    }
    static const char *names[] = {"color_round_flat", "color_round_wave", "color_round_block", "color_round_grid"};
    // relaunch driver: rounds kept in flight (each publishes whether it has
    // work: its queue size, or in grid mode whether chunks or vertices wait);
    // the first empty round ends the loop
    const int window = 4;
    int rounds = 0, launched = 0;
    long long colored = 0;
    for (;;) {
        while (launched < rounds + window) {
            clear_round_slot(ctx, launched);
            void *args[] = {&a, &launched};
            st = launch(ctx, names[mode], ks.round, dim3(grid_mode ? dgrid : grid), dim3(cfg.block), args, stream);
            if (st == WC_OK && spills)
                st = launch(ctx, "color_round_drain", ks.round_drain, dim3(dgrid), dim3(cfg.block), args, stream);
            if (st != WC_OK) return st;
            ++launched;
        }
        int c = 0;
        st = wait_round_count(ctx, rounds, &c);
        if (st != WC_OK) return st;
        if (c == 0) break;
        colored += c;
        ++rounds;
        if (!grid_mode && colored > n) return fail(WC_EINVAL, "wc_color: more queued vertices than vertices");
        if (rounds > n + 1) return fail(WC_ETIMEOUT, "wc_color: more rounds than vertices");
    }
    if (grid_mode) {
        // the last round with work colored the vertices of the largest color;
        // a graph without edges has one color and no round with work
        rounds = std::max(rounds, 1);
        clear_host_slot(ctx, kHostSlotGraph);
        void *args[] = {&a};
        st = launch(ctx, "color_publish", reinterpret_cast<const void *>(&color_publish), dim3(1), dim3(64), args,
                    stream);
        if (st != WC_OK) return st;
        int c = 0;
        st = wait_host_slot(ctx, kHostSlotGraph, &c);
        if (st != WC_OK) return st;
        colored = c;
    }
    st = end_call(ctx, stream, stats, rounds, cfg.fail_on_overflow);
    if (st != WC_OK) return st;
    if (colored != n)
        return fail(WC_EINVAL, "wc_color: some vertices never became ready (the graph is not symmetric)");
    return WC_OK;
}
