// Recursive BFS (the BFS-Rec benchmark of Sec. V) on the recursion path, for
// the wave and block modes.
//
// The recursion: a call visit(v, l) walks v's out-edges; a neighbour u whose
// level it lowers to l + 1 (atomic min) is a recursive call visit(u, l + 1)
// (parallel recursion, Sec. II.B and Fig. 1(c): every recursive call would be
// a child launch under basic dynamic parallelism).  A vertex without out-edges
// makes no call.  Levels only decrease, so whatever the order in which calls
// run, the fixed point is the breadth-first level of every vertex.
//
// Consolidation of the recursive calls (Sec. IV.A-IV.C), as in the packet
// queue of the trees' wave and block modes: the calls a group (one wave, or
// one workgroup) makes are inserted into the group's LDS buffer; a full or
// final buffer becomes one consolidated dispatch, a packet in a device-wide
// queue that any group of the persistent grid picks up, processing the
// concatenated edge ranges of the packet's calls with all its lanes.  A call is
// an entry (u, level, first edge, end edge) of at most `chunk` edges: the call
// of a vertex with more out-edges is handed on as several entries, written by
// the wave straight to the global node list and published as packets of about
// one group's share of work each, so a hub is spread over many groups (the
// child thread-count rule of Sec. IV.E) instead of one.  An entry whose vertex has meanwhile been lowered
// again is stale (a newer call exists) and is skipped.
//
// Termination: a count of outstanding packets (published, not finished).  The
// waits for packets are bounded in time.  When the node list is full, the call
// that does not fit is dropped and the overflow flag is raised; the host then
// recomputes the levels with the frontier rounds of the SSSP path (unit
// weights), so the result is exact either way.
#include <algorithm>
#include <cstring>

#include "wc_block.h"
#include "wc_device.h"
#include "wc_internal.h"
#include "wc_stats.h"

namespace wc {
namespace {

struct BfsArgs {
    const int *row_ptr;
    const int *col;
    uint32_t *level;
    int n;
    int src;
    int chunk;           // edges per call entry
    int work_cap;        // edges per packet: a flush cuts its entries into packets of about this many
    int4 *nl;            // call entries (vertex, level, first edge, end edge)
    long long nl_cap;
    int *nl_tail;
    long long *pq;       // packets: (first entry << 32) | entry count; -1 = not yet written
    long long pq_cap;
    int *pq_head;
    int *pq_tail;
    int *outstanding;
    unsigned long long wait_ticks;
    DevStats *stats;
    int want_stats;
};

// Publishes the entries nl[start, start + count) as packets of at most
// `per` entries.  Called by ONE lane, after the entries were written by the
// wave (the release fence orders them before the packets).
__device__ void publish_entries(const BfsArgs &a, int start, int count, int per, StatAcc &acc)
{
    if (count <= 0) return;
    const int packets = (count + per - 1) / per;
    // one release fence for all the packets: the stores after it are ordered
    // behind the entries
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    atomic_add_dev(a.outstanding, packets);
    const int slot = atomic_add_dev(a.pq_tail, packets);
    for (int p = 0; p < packets; ++p) {
        const int s = start + p * per, k = min(per, count - p * per);
        if ((long long)slot + p < a.pq_cap)
            __hip_atomic_store(&a.pq[slot + p], ((long long)s << 32) | (long long)k, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    if (a.want_stats) acc.items += count;
}

// Appends the calls of the wave's lanes that hold nch > 1 entries (vertices
// with more than `chunk` out-edges) to the node list and publishes them as
// packets of their own, each carrying about a group's share of work
// (work_cap edges), so that a hub's edges spread over many groups.  Every
// lane of the wave calls this.
template <int G>
__device__ void hand_on_big_calls(const BfsArgs &a, int u, uint32_t lvl, int beg, int end, int nch, StatAcc &acc)
{
    const int slot = wave_reserve_n(nch, a.nl_tail);
    const int total = readlane(slot + nch, kWave - 1) - readlane(slot, 0);  // entries reserved by the wave
    const int base = readlane(slot, 0);
    uint64_t m = __ballot(nch > 0);
    while (m) {
        const int b = __builtin_ctzll(m);
        m &= m - 1;
        const int s0 = readlane(slot, b), n0 = readlane(nch, b), rb = readlane(beg, b), re = readlane(end, b);
        const int ub = readlane(u, b);
        const int lb = readlane((int)lvl, b);
        for (int c = lane_id(); c < n0; c += kWave) {
            const int cb = rb + c * a.chunk;
            if ((long long)s0 + c < a.nl_cap) a.nl[s0 + c] = make_int4(ub, lb, cb, min(re, cb + a.chunk));
        }
        if (lane_id() == 0 && (long long)s0 + n0 > a.nl_cap) a.stats->overflowed = 1;
    }
    if (lane_id() == 0) {
        const long long fit = std::min<long long>((long long)base + total, a.nl_cap) - base;
        publish_entries(a, base, (int)std::max<long long>(fit, 0), max(1, a.work_cap / a.chunk), acc);
    }
}

// Group = one wave (G = 64) or one workgroup (G = BLOCK).
template <int G>
struct BfsLds {
    int pk_beg[G];     // first edge of each entry of the packet being processed
    int pk_pre[G + 1]; // exclusive prefix of their edge counts
    uint32_t pk_lvl[G];
    int4 buf[2 * G];   // the group's buffer of small calls
    int hpos[2 * G + 1];  // flush: first buffer entry of each packet, then the count
    int buf_cnt;
    int buf_work;
    int pk_start;
    int pk_count;
    int flag;
    int scan_tmp[2 * (G / kWave) + 2];
};

template <int G>
__device__ __forceinline__ void gsync()
{
    if (G > kWave) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

template <int G>
__device__ __forceinline__ int gtid() { return G > kWave ? (int)threadIdx.x : lane_id(); }

// Exclusive scan of two ints over the group (one wave, or the whole block).
template <int G>
__device__ __forceinline__ void group_scan2(int x, int y, int *tmp, int &ex, int &ey, int &tx, int &ty)
{
    if constexpr (G > kWave) {
        block_scan2<G>(x, y, tmp, ex, ey, tx, ty);
    } else {
        const int ix = wave_incl_scan(x), iy = wave_incl_scan(y);
        ex = ix - x;
        ey = iy - y;
        tx = readlane(ix, kWave - 1);
        ty = readlane(iy, kWave - 1);
    }
}

// Flushes the group's buffer of small calls as packets (consolidated
// dispatches) of at most G entries carrying about work_cap edges each: a
// packet starts at an entry where the edges buffered before it cross a
// multiple of work_cap, or every G entries.  All packets of one flush share
// one reservation of entry slots, one release fence and one reservation of
// queue slots.  Thread t holds buffer entries t and t + G; all threads of the
// group call it.
template <int G>
__device__ void flush_calls(const BfsArgs &a, BfsLds<G> &s, StatAcc &acc)
{
    const int cnt = s.buf_cnt;
    if (cnt == 0) return;
    const int t = gtid<G>();
    const int i0 = t, i1 = t + G;
    const int w0 = i0 < cnt ? s.buf[i0].w - s.buf[i0].z : 0, w1 = i1 < cnt ? s.buf[i1].w - s.buf[i1].z : 0;
    int pre0, pre1, tw0, tw1;
    group_scan2<G>(w0, w1, s.scan_tmp, pre0, pre1, tw0, tw1);
    pre1 += tw0;
    const int cap = a.work_cap;
    // key(i) = before(i) / cap + i / G never decreases; a packet starts where it changes
    bool h0 = false, h1 = false;
    if (i0 < cnt) {
        const int wp = i0 > 0 ? s.buf[i0 - 1].w - s.buf[i0 - 1].z : 0;
        h0 = i0 == 0 || pre0 / cap + i0 / G != (pre0 - wp) / cap + (i0 - 1) / G;
    }
    if (i1 < cnt) {
        const int wp = s.buf[i1 - 1].w - s.buf[i1 - 1].z;
        h1 = pre1 / cap + i1 / G != (pre1 - wp) / cap + (i1 - 1) / G;
    }
    int p0, p1, np0, np1;
    group_scan2<G>(h0 ? 1 : 0, h1 ? 1 : 0, s.scan_tmp, p0, p1, np0, np1);
    p1 += np0;
    const int npk = np0 + np1;
    if (h0) s.hpos[p0] = i0;
    if (h1) s.hpos[p1] = i1;
    if (t == 0) {
        s.hpos[npk] = cnt;
        s.pk_start = atomic_add_dev(a.nl_tail, cnt);
    }
    gsync<G>();
    const int base = s.pk_start;
    if (i0 < cnt && (long long)base + i0 < a.nl_cap) a.nl[base + i0] = s.buf[i0];
    if (i1 < cnt && (long long)base + i1 < a.nl_cap) a.nl[base + i1] = s.buf[i1];
    gsync<G>();
    if (t == 0) {
        // entries beyond the list's end are dropped (the overflow flag makes the
        // host recompute the levels); only packets with entries are published
        const int fit = (int)std::max<long long>(0, std::min<long long>((long long)base + cnt, a.nl_cap) - base);
        if (fit < cnt) a.stats->overflowed = 1;
        int npub = 0;
        while (npub < npk && s.hpos[npub] < fit) ++npub;
        if (npub > 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            atomic_add_dev(a.outstanding, npub);
            const int slot = atomic_add_dev(a.pq_tail, npub);
            for (int p = 0; p < npub; ++p) {
                const int k = min(s.hpos[p + 1], fit) - s.hpos[p];
                if ((long long)slot + p < a.pq_cap)
                    __hip_atomic_store(&a.pq[slot + p], ((long long)(base + s.hpos[p]) << 32) | (long long)k,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (a.want_stats) acc.items += fit;
        }
        s.buf_cnt = 0;
        s.buf_work = 0;
    }
    gsync<G>();
}

// A group flushes its buffer once it holds G calls or this many packets' worth
// of edges (more packets per flush, fewer round trips).
constexpr int kFlushPackets = 8;

__global__ void bfs_rec_init(BfsArgs a, long long pq_cap)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < a.n; i += (long long)gridDim.x * blockDim.x)
        a.level[i] = i == a.src ? 0u : kInf;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < pq_cap;
         i += (long long)gridDim.x * blockDim.x)
        a.pq[i] = -1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *a.pq_head = 0;
        *a.pq_tail = 0;
        *a.nl_tail = 0;
        *a.outstanding = 0;
    }
}

// The source's call: its entries and packets (one wave).
template <int G>
__global__ void bfs_rec_root(BfsArgs a)
{
    StatAcc acc;
    const int beg = a.row_ptr[a.src], end = a.row_ptr[a.src + 1];
    const int nch = lane_id() == 0 ? (end - beg + a.chunk - 1) / a.chunk : 0;
    hand_on_big_calls<G>(a, a.src, 0u, beg, end, nch, acc);
}

template <int G, int BLOCK>
__global__ __launch_bounds__(BLOCK) void bfs_rec_queue(BfsArgs a)
{
    constexpr int GROUPS = BLOCK / G;
    __shared__ BfsLds<G> lds[GROUPS];
    const int gid = G > kWave ? 0 : (int)threadIdx.x / kWave;
    BfsLds<G> &s = lds[gid];
    const int t = gtid<G>();
    StatAcc acc;
    if (t == 0) {
        s.buf_cnt = 0;
        s.buf_work = 0;
    }
    gsync<G>();
    for (;;) {
        // ---- fetch a packet (group leader): the next ticket of the queue; its
        // packet is published later or, once no packet is outstanding, never
        if (t == 0) {
            const int h = atomic_add_dev(a.pq_head, 1);
            const unsigned long long deadline = wait_deadline(a.wait_ticks);
            long long pk = -1;
            int got = -1;
            for (int poll = 0;; ++poll) {
                if (h < a.pq_cap) {
                    pk = __hip_atomic_load(&a.pq[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (pk >= 0) {
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                        got = h;
                        break;
                    }
                }
                if ((poll & 7) == 7 &&
                    __hip_atomic_load(a.outstanding, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
                    break;
                __builtin_amdgcn_s_sleep(2);
                if (past(deadline)) {
                    a.stats->timed_out = 1;
                    break;
                }
            }
            s.flag = got;
            s.pk_start = got >= 0 ? (int)(pk >> 32) : 0;
            s.pk_count = got >= 0 ? (int)(pk & 0xffffffff) : 0;
            if (a.want_stats && got >= 0) acc.dispatches += 1;
        }
        gsync<G>();
        if (s.flag < 0) break;
        // ---- the consolidated child: the packet's calls, their edge ranges
        // concatenated; a call whose vertex was lowered again since is stale
        const int pcount = s.pk_count;
        int len = 0, cb = 0;
        uint32_t lvl = 0;
        if (t < pcount) {
            const int4 e = a.nl[s.pk_start + t];
            lvl = (uint32_t)e.y;
            const uint32_t now = __hip_atomic_load(&a.level[e.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (now == lvl) {
                cb = e.z;
                len = e.w - e.z;
            }
        }
        int pre, dummy, total, dummy_total;
        if constexpr (G > kWave) {
            block_scan2<G>(len, 0, s.scan_tmp, pre, dummy, total, dummy_total);
        } else {
            const int incl = wave_incl_scan(len);
            pre = incl - len;
            total = readlane(incl, kWave - 1);
        }
        if (t < pcount) {
            s.pk_beg[t] = cb;
            s.pk_pre[t] = pre;
            s.pk_lvl[t] = lvl;
        }
        if (t == 0) s.pk_pre[pcount] = total;
        gsync<G>();
        if (a.want_stats && t == 0) acc.edges += total;
        int k = 0;
        for (int jb = 0; jb < total; jb += G) {
            const int j = jb + t;
            int u = -1, ub = 0, ue = 0;
            uint32_t nl = 0;
            if (j < total) {
                while (k + 1 < pcount && s.pk_pre[k + 1] <= j) ++k;
                u = a.col[s.pk_beg[k] + (j - s.pk_pre[k])];
                nl = s.pk_lvl[k] + 1u;
                // the recursive call happens when this edge lowers u's level
                if (nl < a.level[u] && atomic_min_dev(&a.level[u], nl) > nl) {
                    ub = a.row_ptr[u];
                    ue = a.row_ptr[u + 1];
                    if (a.want_stats) acc.updates += 1;
                } else {
                    u = -1;
                }
            }
            const int deg = ue - ub;
            // small calls into the group's buffer; calls of more than one
            // entry are handed on as packets of their own
            const bool small = u >= 0 && deg > 0 && deg <= a.chunk;
            const int nbig = u >= 0 && deg > a.chunk ? (deg + a.chunk - 1) / a.chunk : 0;
            if (__ballot(nbig > 0)) hand_on_big_calls<G>(a, u, nl, ub, ue, nbig, acc);
            if constexpr (G > kWave) {
                int pos, dummy2, add, work;
                block_scan2<G>(small ? 1 : 0, small ? deg : 0, s.scan_tmp, pos, dummy2, add, work);
                if (small) s.buf[s.buf_cnt + pos] = make_int4(u, (int)nl, ub, ue);
                gsync<G>();
                if (t == 0) {
                    s.buf_cnt += add;
                    s.buf_work += work;
                }
            } else {
                const uint64_t m = __ballot(small);
                const int work = wave_sum_i(small ? deg : 0);
                if (small) s.buf[s.buf_cnt + rank_in(m)] = make_int4(u, (int)nl, ub, ue);
                gsync<G>();
                if (t == 0) {
                    s.buf_cnt += __builtin_popcountll(m);
                    s.buf_work += work;
                }
            }
            gsync<G>();
            if (s.buf_cnt >= G || s.buf_work >= kFlushPackets * a.work_cap) flush_calls<G>(a, s, acc);
        }
        flush_calls<G>(a, s, acc);
        // this dispatch is finished (its own follow-up packets are already counted)
        if (t == 0) __hip_atomic_fetch_add(a.outstanding, -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        gsync<G>();
    }
    if (a.want_stats) stat_flush(a.stats, acc);
}

// Publishes the call's flags (timeout, overflow) to the host ring.
__global__ void bfs_rec_flags(DevStats *s, unsigned long long *ring)
{
    if (threadIdx.x == 0) publish_host(ring, kHostSlotFlags, s, (s->timed_out ? 1 : 0) | (s->overflowed ? 2 : 0));
}

template <int BLOCK>
const void *queue_kernel(wc_mode mode)
{
    return mode == WC_WAVE ? reinterpret_cast<const void *>(&bfs_rec_queue<kWave, BLOCK>)
                           : reinterpret_cast<const void *>(&bfs_rec_queue<BLOCK, BLOCK>);
}

template <int BLOCK>
const void *root_kernel(wc_mode mode)
{
    return mode == WC_WAVE ? reinterpret_cast<const void *>(&bfs_rec_root<kWave>)
                           : reinterpret_cast<const void *>(&bfs_rec_root<BLOCK>);
}

}  // namespace

// Wave and block modes of wc_bfs.  Returns WC_OK with *overflowed = 1 when the
// node list was too small (the levels are then incomplete and the caller
// recomputes them).
wc_status run_bfs_rec(wc_ctx *ctx, const wc_csr *g, int32_t src, uint32_t *level, wc_mode mode, const Config &cfg,
                      hipStream_t stream, wc_stats *stats, int *overflowed)
{
    *overflowed = 0;
    const int block = cfg.block;
    const void *qk = nullptr, *rk = nullptr;
    switch (block) {
    case 64: qk = queue_kernel<64>(mode); rk = root_kernel<64>(mode); break;
    case 128: qk = queue_kernel<128>(mode); rk = root_kernel<128>(mode); break;
    case 512: qk = queue_kernel<512>(mode); rk = root_kernel<512>(mode); break;
    case 1024: qk = queue_kernel<1024>(mode); rk = root_kernel<1024>(mode); break;
    default: qk = queue_kernel<256>(mode); rk = root_kernel<256>(mode); break;
    }
    const int resident = resident_blocks(ctx, qk, block);
    const int grid = std::max(1, std::min(cfg.grid, resident));
    const long long n = g->n, m = g->m;
    const int chunk = kWave * cfg.items_per_lane;
    // entries: every improvement of a vertex makes ceil(deg / chunk) of them;
    // room for each reached vertex and edge range twice by default
    long long cap = 2 * (n + m / chunk) + 1024;
    if (cfg.buf_capacity > 0) cap = std::min(cap, cfg.buf_capacity);
    const long long pq_cap = cap;
    const size_t need = padded(cap * 16) + padded(pq_cap * 8) + 4 * padded(4);
    wc_status st = pool_reserve(ctx, need, stream);
    if (st != WC_OK) return st;
    BfsArgs a;
    std::memset(&a, 0, sizeof(a));
    a.row_ptr = g->row_ptr;
    a.col = g->col;
    a.level = level;
    a.n = (int)n;
    a.src = src;
    a.chunk = chunk;
    a.work_cap = (mode == WC_WAVE ? kWave : block) * cfg.items_per_lane;
    a.nl = pool_take<int4>(ctx, cap);
    a.nl_cap = cap;
    a.pq = pool_take<long long>(ctx, pq_cap);
    a.pq_cap = pq_cap;
    a.nl_tail = pool_take<int>(ctx, 1);
    a.pq_head = pool_take<int>(ctx, 1);
    a.pq_tail = pool_take<int>(ctx, 1);
    a.outstanding = pool_take<int>(ctx, 1);
    a.wait_ticks = ctx->wait_ticks;
    a.stats = ctx->dstats;
    a.want_stats = stats != nullptr;
    st = begin_call(ctx, stream, stats);
    if (st != WC_OK) return st;
    long long pqc = pq_cap;
    const int ig = (int)std::min<long long>((std::max(n, pq_cap) + 255) / 256, 4096);
    void *iargs[] = {&a, &pqc};
    st = launch(ctx, "bfs_rec_init", reinterpret_cast<const void *>(&bfs_rec_init), dim3(ig), dim3(256), iargs,
                stream);
    void *args[] = {&a};
    if (st == WC_OK) st = launch(ctx, "bfs_rec_root", rk, dim3(1), dim3(kWave), args, stream);
    if (st == WC_OK)
        st = launch(ctx, mode == WC_WAVE ? "bfs_rec_queue_wave" : "bfs_rec_queue_block", qk, dim3(grid), dim3(block),
                    args, stream);
    if (st != WC_OK) return st;
    // the flags decide whether the levels are complete: wait for them
    void *fargs[] = {&ctx->dstats, &ctx->host_ring_dev};
    clear_host_slot(ctx, kHostSlotFlags);
    st = launch(ctx, "bfs_rec_flags", reinterpret_cast<const void *>(&bfs_rec_flags), dim3(1), dim3(64), fargs,
                stream);
    if (st != WC_OK) return st;
    int flags = 0;
    st = wait_host_slot(ctx, kHostSlotFlags, &flags);
    if (st != WC_OK) return st;
    chain_break(ctx);
    if (flags & 1) return fail(WC_ETIMEOUT, "a device-side wait exceeded its time limit");
    if (flags & 2) {
        *overflowed = 1;
        return WC_OK;
    }
    return end_call(ctx, stream, stats, 0, cfg.fail_on_overflow);
}

}  // namespace wc
