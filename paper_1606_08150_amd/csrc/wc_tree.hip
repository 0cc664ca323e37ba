// Tree descendants / tree heights with workload consolidation (parallel
// recursion, Fig. 1(c)).
//
// The recursive kernel of Fig. 1(c) gives one thread per child c of a node:
// if c has children it launches itself on c (the recursive call), otherwise it
// does the leaf work; afterwards the post-work folds c's result into its
// parent (descendants: + (1 + desc[c]); heights: max with 1 + height[c]).
// Consolidation buffers the recursive calls, i.e. the nodes with children, and
// one consolidated child processes all buffered nodes' children.
//
//   grid  - level-synchronous: the global buffer of level l holds chunks of
//           the children ranges of every node found in level l-1; a grid-wide
//           barrier (the kernel boundary) separates levels.  The post-work is consolidated too (Sec. IV.C,
//           grid-level post-work): after the last level, one pass per level from
//           the deepest up folds every chunk into its node with one atomic.
//   flat  - the same level structure without consolidation: one thread per
//           node of the level handles all of its children serially, and one
//           thread per node folds them back.
//   wave / block - no grid-wide barrier at all.  A wave (block) inserts the
//           nodes with children it finds into its own LDS buffer; a full (or
//           final) buffer becomes one consolidated dispatch: a packet in a
//           device-wide queue that any wave (block) of the persistent grid
//           picks up.  The post-work runs as soon as a node's last child is
//           done: per-node words of pending children and folded value; the thread that
//           completes a node folds it into its parent and climbs on while it
//           keeps completing ancestors.
// Integer folds are associative and commutative, so every mode and schedule
// gives identical results.
#include <algorithm>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "wc_block.h"
#include "wc_device.h"
#include "wc_internal.h"
#include "wc_stats.h"

namespace wc {
namespace {

enum { OP_DESC = 0, OP_HEIGHT = 1 };

// One tree of a batch (wc_tree_batch).
struct TreeInst {
    const int *child_ptr;
    const int *child;
    int *out;
    long long n;
};

struct TreeArgs {
    const int *parent;
    const int *child_ptr;
    const int *child;
    int *out;
    int n;
    int chunk;
    // batch of trees (level-synchronous modes): NULL for a single tree; else
    // items carry their tree's index in .w >> 1 and every array is the tree's
    const TreeInst *inst;
    int count;
    // level-synchronous modes
    int *lvl_start;  // [max_levels + 2]
    int *lvl_count;  // [max_levels + 2]
    int4 *items;     // grid: (node, begin, end, 0) chunks; flat: .x = node
    long long item_cap;
    // packet-queue modes
    int *nl;             // node list the packets point into [n]
    int *nl_tail;
    long long *pq;       // packets: (start << 32) | count; -1 = not yet written
    long long pq_cap;
    int *pq_head;
    int *pq_tail;
    int *outstanding;
    unsigned long long *word;  // per internal node: (children not yet finished << 32) | folded value
    int work_cap;        // children per packet: a flush cuts its nodes into packets of about this many
    unsigned long long wait_ticks;  // bound of the packet queue's waits (100 MHz ticks)
    unsigned long long *host_ring;
    DevStats *stats;
    int want_stats;
};

__device__ __forceinline__ int fanout(const TreeArgs &a, int v) { return a.child_ptr[v + 1] - a.child_ptr[v]; }

// The arrays of the tree an item belongs to (the single tree, or tree i of a batch).
struct TreeView {
    const int *child_ptr;
    const int *child;
    int *out;
};
__device__ __forceinline__ TreeView view(const TreeArgs &a, int i)
{
    if (!a.inst) return TreeView{a.child_ptr, a.child, a.out};
    const TreeInst &t = a.inst[i];
    return TreeView{t.child_ptr, t.child, t.out};
}
__device__ __forceinline__ int fanout(const TreeView &t, int v) { return t.child_ptr[v + 1] - t.child_ptr[v]; }

template <int OP>
__device__ __forceinline__ int fold(int acc, int v)
{
    return OP == OP_DESC ? acc + 1 + v : max(acc, 1 + v);
}

template <int OP>
__device__ __forceinline__ void atomic_fold(int *p, int v)
{
    if (OP == OP_DESC) atomic_add_dev(p, v);
    else atomic_max_dev(p, v);
}

// ---------------------------------------------------------------- level-synchronous (flat, grid)

__global__ void tree_init_levels(TreeArgs a)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.out[0] = 0;
        int f = fanout(a, 0);
        a.lvl_start[0] = 0;
        a.lvl_count[1] = 0;
        if (f == 0) {
            a.lvl_count[0] = 0;
        } else {
            // level 0 buffers the root: the host's launch on the root's children
            int nch = (f + a.chunk - 1) / a.chunk;
            for (int c = 0; c < nch; ++c) {
                int cb = a.child_ptr[0] + c * a.chunk;
                a.items[c] = make_int4(0, cb, min(cb + a.chunk, a.child_ptr[1]), nch == 1);
            }
            a.lvl_count[0] = nch;
        }
    }
}

__global__ void tree_init_levels_flat(TreeArgs a)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.out[0] = 0;
        a.lvl_start[0] = 0;
        a.lvl_count[0] = fanout(a, 0) > 0 ? 1 : 0;
        a.lvl_count[1] = 0;
        a.items[0] = make_int4(0, 0, 0, 0);
    }
}

// Level 0 of a batch: every tree's root is the host's launch on its children.
// One workgroup; grid mode buffers the roots' children as chunks, flat mode the
// roots themselves.
__global__ __launch_bounds__(256) void tree_init_batch(TreeArgs a, int grid_mode)
{
    __shared__ int s_count;
    if (threadIdx.x == 0) {
        s_count = 0;
        a.lvl_start[0] = 0;
        a.lvl_count[1] = 0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < a.count; i += blockDim.x) {
        const TreeView t = view(a, i);
        t.out[0] = 0;
        const int f = fanout(t, 0);
        if (f == 0) continue;
        if (!grid_mode) {
            const int slot = atomicAdd(&s_count, 1);
            a.items[slot] = make_int4(0, 0, 0, i << 1);
            continue;
        }
        const int nch = (f + a.chunk - 1) / a.chunk;
        const int slot = atomicAdd(&s_count, nch);
        for (int c = 0; c < nch; ++c) {
            const int cb = t.child_ptr[0] + c * a.chunk;
            a.items[slot + c] = make_int4(0, cb, min(cb + a.chunk, t.child_ptr[1]), (i << 1) | (nch == 1));
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) a.lvl_count[0] = s_count;
}

// Items per block tile in the grid-mode level passes: up to BLOCK, fewer when
// the level is small, so that every block of the grid gets work.
template <int BLOCK>
__device__ __forceinline__ int tile_items(int count)
{
    const int per_block = (count + (int)gridDim.x - 1) / (int)gridDim.x;
    return max(1, min(BLOCK, per_block));
}

// Top-down step of level l: children of the level's buffered nodes.  Internal
// children are inserted into level l+1's buffer, leaves get the leaf work.
template <int MODE, int BLOCK>
__device__ void level_down(const TreeArgs &a, int l, int start, int count, StatAcc &acc)
{
    const int out_base = start + count;
    int *cnt_next = &a.lvl_count[l + 1];
    if constexpr (MODE == WC_GRID) {
        // The block takes a tile of buffered items at a time and walks their
        // children as one flattened range (most items have a few children), so
        // the next level's buffer is reserved with one atomic per BLOCK
        // children instead of one per item.
        __shared__ int s_pre[BLOCK], s_cb[BLOCK], s_inst[BLOCK], s_tmp[2 * (BLOCK / kWave)];
        __shared__ int s_base;
        const int T = tile_items<BLOCK>(count);
        for (int tile = blockIdx.x * T; tile < count; tile += gridDim.x * T) {
            const int it = tile + threadIdx.x;
            int cb = 0, len = 0, ti = 0;
            if ((int)threadIdx.x < T && it < count) {
                const int4 d = a.items[start + it];
                cb = d.y;
                len = d.z - d.y;
                ti = d.w >> 1;
            }
            if (a.want_stats) acc.edges += len;
            int excl, e0, total, e1;
            block_scan2<BLOCK>(len, 0, s_tmp, excl, e0, total, e1);
            s_pre[threadIdx.x] = excl;
            s_cb[threadIdx.x] = cb;
            s_inst[threadIdx.x] = ti;
            __syncthreads();
            for (int j0 = 0; j0 < total; j0 += BLOCK) {
                const int j = j0 + threadIdx.x;
                int c = -1, f = 0, ci = 0;
                TreeView t{nullptr, nullptr, nullptr};
                if (j < total) {
                    // owner: the last item whose offset is <= j
                    int lo = 0, hi = BLOCK - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_pre[mid] <= j) lo = mid;
                        else hi = mid - 1;
                    }
                    ci = s_inst[lo];
                    t = view(a, ci);
                    c = t.child[s_cb[lo] + (j - s_pre[lo])];
                    f = fanout(t, c);
                    t.out[c] = 0;  // leaf work, or the identity the folds start from
                }
                const int nch = f > 0 ? (f + a.chunk - 1) / a.chunk : 0;
                if (a.want_stats) acc.items += f > 0 ? 1 : 0;
                int x0, x1, tot, x2;
                block_scan2<BLOCK>(nch, 0, s_tmp, x0, x1, tot, x2);
                if (threadIdx.x == 0) s_base = tot ? atomic_add_dev(cnt_next, tot) : 0;
                __syncthreads();
                const int slot = s_base + x0;
                if (nch > 0) {
                    const int c0 = t.child_ptr[c];
                    for (int k = 0; k < nch; ++k) {
                        const int kb = c0 + k * a.chunk;
                        a.items[out_base + slot + k] =
                            make_int4(c, kb, min(kb + a.chunk, c0 + f), (ci << 1) | (nch == 1));
                    }
                }
                __syncthreads();  // s_base is rewritten by the next step
            }
        }
    } else {
        for (int i = blockIdx.x * BLOCK + threadIdx.x; i < count; i += gridDim.x * BLOCK) {
            const int4 d = a.items[start + i];
            const int p = d.x;
            const TreeView t = view(a, d.w >> 1);
            const int cb = t.child_ptr[p], ce = t.child_ptr[p + 1];
            if (a.want_stats) acc.edges += ce - cb;
            for (int e = cb; e < ce; ++e) {
                const int c = t.child[e];
                const bool internal = fanout(t, c) > 0;
                t.out[c] = 0;
                const int slot = wave_reserve(internal, cnt_next);
                if (internal) a.items[out_base + slot] = make_int4(c, 0, 0, d.w & ~1);
            }
        }
    }
}

// Bottom-up post-work of level l (all deeper levels are final).
template <int MODE, int OP, int BLOCK>
__device__ void level_up(const TreeArgs &a, int start, int count)
{
    if constexpr (MODE == WC_GRID) {
        // tiles of items as in the top-down pass: the children's values are
        // folded per item in LDS, then one atomic per item folds into its node
        __shared__ int s_pre[BLOCK], s_cb[BLOCK], s_acc[BLOCK], s_inst[BLOCK], s_tmp[2 * (BLOCK / kWave)];
        const int T = tile_items<BLOCK>(count);
        for (int tile = blockIdx.x * T; tile < count; tile += gridDim.x * T) {
            const int it = tile + threadIdx.x;
            int p = -1, cb = 0, len = 0, whole = 0, ti = 0;
            if ((int)threadIdx.x < T && it < count) {
                const int4 d = a.items[start + it];
                p = d.x;
                cb = d.y;
                len = d.z - d.y;
                whole = d.w & 1;
                ti = d.w >> 1;
            }
            int excl, e0, total, e1;
            block_scan2<BLOCK>(len, 0, s_tmp, excl, e0, total, e1);
            s_pre[threadIdx.x] = excl;
            s_cb[threadIdx.x] = cb;
            s_acc[threadIdx.x] = 0;
            s_inst[threadIdx.x] = ti;
            __syncthreads();
            for (int j = threadIdx.x; j < total; j += BLOCK) {
                int lo = 0, hi = BLOCK - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_pre[mid] <= j) lo = mid;
                    else hi = mid - 1;
                }
                const TreeView t = view(a, s_inst[lo]);
                const int v = 1 + t.out[t.child[s_cb[lo] + (j - s_pre[lo])]];
                if (OP == OP_DESC) atomicAdd(&s_acc[lo], v);
                else atomicMax(&s_acc[lo], v);
            }
            __syncthreads();
            // an item holding all of its node's children is the node's only
            // contribution: a plain store; split nodes fold atomically
            if (p >= 0) {
                int *o = view(a, ti).out;
                if (whole) o[p] = s_acc[threadIdx.x];
                else atomic_fold<OP>(&o[p], s_acc[threadIdx.x]);
            }
            __syncthreads();  // the LDS arrays are rewritten by the next tile
        }
    } else {
        for (int i = blockIdx.x * BLOCK + threadIdx.x; i < count; i += gridDim.x * BLOCK) {
            const int4 d = a.items[start + i];
            const int p = d.x;
            const TreeView t = view(a, d.w >> 1);
            int acc = 0;
            for (int e = t.child_ptr[p]; e < t.child_ptr[p + 1]; ++e) acc = fold<OP>(acc, t.out[t.child[e]]);
            t.out[p] = acc;
        }
    }
}

template <int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void tree_down(TreeArgs a, int l)
{
    const int start = a.lvl_start[l], count = a.lvl_count[l];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.lvl_start[l + 1] = start + count;
        a.lvl_count[l + 2] = 0;
        publish_host(a.host_ring, l % kHostRing, a.stats, count);
        if (a.want_stats && MODE == WC_GRID && count > 0) atomic_add_dev(&a.stats->rep[0].dispatches, 1ull);
    }
    if (count == 0) return;
    StatAcc acc;
    level_down<MODE, BLOCK>(a, l, start, count, acc);
    if (a.want_stats) stat_flush(a.stats, acc);
}

template <int MODE, int OP, int BLOCK>
__global__ __launch_bounds__(BLOCK) void tree_up(TreeArgs a, int l)
{
    level_up<MODE, OP, BLOCK>(a, a.lvl_start[l], a.lvl_count[l]);
}

// Last kernel of a captured graph of levels 0..L: publishes the tree's depth
// (its first empty level), or -2 when level L is not empty (the tree is deeper
// than the recorded one and the levels have to be driven from the host).
__global__ void tree_publish_depth(TreeArgs a, int L)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int d = -2;
        for (int l = 0; l <= L; ++l)
            if (a.lvl_count[l] == 0) {
                d = l;
                break;
            }
        publish_host(a.host_ring, kHostSlotGraph, a.stats, d);
    }
}

// ---------------------------------------------------------------- packet queue (wave, block)

// Post-work state of an internal node is ONE 64-bit word: the number of its
// children not yet finished in the high half and the fold of the finished
// ones in the low half.  A finishing child updates both with a single atomic
// read-modify-write (descendants: one 64-bit add; heights: a compare-and-swap
// loop), so the count can never be seen before the value it guards and no
// memory fence is needed on this path.  The child whose update takes the count
// to zero gets the node's final value back from its own atomic.
template <int OP>
__device__ __forceinline__ unsigned long long fold_finished(unsigned long long *w, int contrib, int count)
{
    if (OP == OP_DESC) {
        // the low half never carries: a node's descendants stay below 2^31
        const unsigned long long add =
            (unsigned long long)(unsigned int)contrib - ((unsigned long long)(unsigned int)count << 32);
        return __hip_atomic_fetch_add(w, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + add;
    }
    unsigned long long old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), nw;
    do {
        const unsigned int lo = (unsigned int)old, hi = (unsigned int)(old >> 32);
        nw = ((unsigned long long)(hi - (unsigned int)count) << 32) | (unsigned int)max((int)lo, contrib);
    } while (!__hip_atomic_compare_exchange_weak(w, &old, nw, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT));
    return nw;
}

// Post-work of a finished node v with value val: fold it into its parent;
// whoever finishes the parent's last child stores the parent's value and
// carries on upward.
template <int OP>
__device__ void complete_upward(const TreeArgs &a, int v, int val)
{
    for (;;) {
        const int p = a.parent[v];
        if (p < 0) return;
        const unsigned long long nw = fold_finished<OP>(&a.word[p], 1 + val, 1);
        if ((nw >> 32) != 0) return;
        val = (int)(unsigned int)nw;
        a.out[p] = val;
        v = p;
    }
}

// nleaf leaf children of p are done (leaf value 0): fold them in at once; if
// they were p's last unfinished children, p is done and its post-work climbs on.
template <int OP>
__device__ void complete_leaves(const TreeArgs &a, int p, int nleaf)
{
    const unsigned long long nw = fold_finished<OP>(&a.word[p], OP == OP_DESC ? nleaf : 1, nleaf);
    if ((nw >> 32) != 0) return;
    const int val = (int)(unsigned int)nw;
    a.out[p] = val;
    complete_upward<OP>(a, p, val);
}

__global__ void tree_init_queue(TreeArgs a, long long pq_cap)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < pq_cap;
         i += (long long)gridDim.x * blockDim.x)
        a.pq[i] = -1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.out[0] = 0;
        const int f = fanout(a, 0);
        *a.pq_head = 0;
        if (f == 0) {
            *a.nl_tail = 0;
            *a.pq_tail = 0;
            *a.outstanding = 0;
        } else {
            a.word[0] = (unsigned long long)(unsigned int)f << 32;
            a.nl[0] = 0;
            *a.nl_tail = 1;
            *a.pq_tail = 1;
            *a.outstanding = 1;
        }
    }
}

__global__ void tree_publish_root(TreeArgs a)
{
    if (threadIdx.x == 0 && fanout(a, 0) > 0)
        __hip_atomic_store(&a.pq[0], (0LL << 32) | 1LL, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Group = one wave (G = 64) or one block (G = BLOCK).  Per group LDS state:
// the packet being processed and the buffer being filled.
template <int G>
struct QueueLds {
    int pk_node[G];
    int pk_beg[G];
    int pk_pre[G + 1];
    int buf[2 * G];
    int buf_w[2 * G];   // children of each buffered node
    int hpos[2 * G + 1];  // flush: first buffer entry of each packet, then the count
    int buf_cnt;
    int buf_work;
    int pk_start;
    int pk_count;
    int flag;
    int slot0;
    int scan_tmp[2 * (G / kWave) + 2];
};

// Group-wide barrier: a wave needs none (lockstep); a block uses __syncthreads.
template <int G>
__device__ __forceinline__ void gsync()
{
    if (G > kWave) {
        __syncthreads();
    } else {
        // one wave runs in lockstep; the fence only keeps the compiler from
        // moving LDS accesses across this point
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

// Flush the group's buffer: its nodes become packets (consolidated
// dispatches) of at most G nodes carrying about work_cap children each: a
// packet starts at a node where the children buffered before it cross a
// multiple of work_cap, or where the node count crosses a multiple of G.  All
// packets of one flush share one reservation of node-list slots, one of queue
// slots and one count update, so that a group that finds many recursive calls
// pays those round trips once, not once per packet.  Thread t holds buffer
// entries t and t + G.
template <int G>
__device__ void flush_buffer(const TreeArgs &a, QueueLds<G> &s, StatAcc &acc)
{
    const int cnt = s.buf_cnt;
    if (cnt == 0) return;
    const int t = gtid<G>();
    const int i0 = t, i1 = t + G;
    const int w0 = i0 < cnt ? s.buf_w[i0] : 0, w1 = i1 < cnt ? s.buf_w[i1] : 0;
    int pre0, pre1, tw0, tw1;
    group_scan2<G>(w0, w1, s.scan_tmp, pre0, pre1, tw0, tw1);
    pre1 += tw0;
    const int cap = a.work_cap;
    // key(i) = before(i) / cap + i / G never decreases; a packet starts where it changes
    bool h0 = false, h1 = false;
    if (i0 < cnt)
        h0 = i0 == 0 || pre0 / cap + i0 / G != (pre0 - s.buf_w[i0 - 1]) / cap + (i0 - 1) / G;
    if (i1 < cnt) h1 = pre1 / cap + i1 / G != (pre1 - s.buf_w[i1 - 1]) / cap + (i1 - 1) / G;
    int p0, p1, np0, np1;
    group_scan2<G>(h0 ? 1 : 0, h1 ? 1 : 0, s.scan_tmp, p0, p1, np0, np1);
    p1 += np0;
    const int npk = np0 + np1;
    if (h0) s.hpos[p0] = i0;
    if (h1) s.hpos[p1] = i1;
    if (t == 0) {
        s.hpos[npk] = cnt;
        s.pk_start = atomic_add_dev(a.nl_tail, cnt);
        s.slot0 = atomic_add_dev(a.pq_tail, npk);
        atomic_add_dev(a.outstanding, npk);
        if (a.want_stats) acc.items += cnt;
    }
    gsync<G>();
    const int base = s.pk_start, slot0 = s.slot0;
    if (i0 < cnt) a.nl[base + i0] = s.buf[i0];
    if (i1 < cnt) a.nl[base + i1] = s.buf[i1];
    gsync<G>();
    // each packet's first node publishes it; the release makes the group's
    // node-list entries (and the nodes' post-work words) visible first
    if (h0)
        __hip_atomic_store(&a.pq[slot0 + p0], ((long long)(base + i0) << 32) | (long long)(s.hpos[p0 + 1] - i0),
                           __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (h1)
        __hip_atomic_store(&a.pq[slot0 + p1], ((long long)(base + i1) << 32) | (long long)(s.hpos[p1 + 1] - i1),
                           __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    gsync<G>();
    if (t == 0) {
        s.buf_cnt = 0;
        s.buf_work = 0;
    }
    gsync<G>();
}

// A group flushes its buffer once it holds G nodes or this many packets' worth
// of children (more packets per flush, fewer round trips).
constexpr int kFlushPackets = 8;

template <int OP, int G, int BLOCK>
__global__ __launch_bounds__(BLOCK) void tree_queue(TreeArgs a)
{
    constexpr int GROUPS = BLOCK / G;
    __shared__ QueueLds<G> lds[GROUPS];
    const int gid = G > kWave ? 0 : (int)threadIdx.x / kWave;
    QueueLds<G> &s = lds[gid];
    const int t = gtid<G>();
    StatAcc acc;
    if (t == 0) {
        s.buf_cnt = 0;
        s.buf_work = 0;
    }
    gsync<G>();
    for (;;) {
        // ---- fetch a packet (group leader): take the next ticket of the queue;
        // its packet is published later or, once no packet is outstanding, never
        if (t == 0) {
            const int h = atomic_add_dev(a.pq_head, 1);
            const unsigned long long deadline = wait_deadline(a.wait_ticks);
            long long pk = -1;
            int got = -1;
            // polls are relaxed loads (an acquire load invalidates the L2 each
            // time); one acquire fence follows the poll that succeeds
            for (int poll = 0;; ++poll) {
                if (h < a.pq_cap) {
                    pk = __hip_atomic_load(&a.pq[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (pk >= 0) {
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                        got = h;
                        break;
                    }
                }
                // the shared counter is read only every 8th poll (thousands of waiting
                // waves would otherwise contend on its line)
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
        // ---- the consolidated child: all buffered nodes' children, flattened
        const int pcount = s.pk_count;
        int node = 0, f = 0, beg = 0;
        if (t < pcount) {
            node = a.nl[s.pk_start + t];
            beg = a.child_ptr[node];
            f = a.child_ptr[node + 1] - beg;
        }
        int pre, dummy, total, dummy_total;
        if constexpr (G > kWave) {
            block_scan2<G>(f, 0, s.scan_tmp, pre, dummy, total, dummy_total);
        } else {
            int incl = wave_incl_scan(f);
            pre = incl - f;
            total = readlane(incl, kWave - 1);
        }
        if (t < pcount) {
            s.pk_node[t] = node;
            s.pk_beg[t] = beg;
            s.pk_pre[t] = pre;
        }
        if (t == 0) s.pk_pre[pcount] = total;
        gsync<G>();
        if (a.want_stats && t == 0) acc.edges += total;
        int k = 0;
        for (int jb = 0; jb < total; jb += G) {
            const int j = jb + t;
            int c = -1, cf = 0, p = -1;
            if (j < total) {
                while (k + 1 < pcount && s.pk_pre[k + 1] <= j) ++k;
                p = s.pk_node[k];
                c = a.child[s.pk_beg[k] + (j - s.pk_pre[k])];
                cf = fanout(a, c);
                if (cf > 0) a.word[c] = (unsigned long long)(unsigned int)cf << 32;  // nothing folded yet
                else a.out[c] = 0;  // leaf work
            }
            // insert the recursive calls into the group's buffer
            if constexpr (G > kWave) {
                int pos, dummy2, add, work;
                block_scan2<G>(cf > 0 ? 1 : 0, cf, s.scan_tmp, pos, dummy2, add, work);
                if (cf > 0) {
                    s.buf[s.buf_cnt + pos] = c;
                    s.buf_w[s.buf_cnt + pos] = cf;
                }
                gsync<G>();
                if (t == 0) {
                    s.buf_cnt += add;
                    s.buf_work += work;
                }
            } else {
                uint64_t m = __ballot(cf > 0);
                int work = wave_sum_i(cf);
                if (cf > 0) {
                    s.buf[s.buf_cnt + rank_in(m)] = c;
                    s.buf_w[s.buf_cnt + rank_in(m)] = cf;
                }
                gsync<G>();
                if (t == 0) {
                    s.buf_cnt += __builtin_popcountll(m);
                    s.buf_work += work;
                }
            }
            // leaves: their post-work right away, aggregated per parent: the
            // lanes of a wave that share a parent are consecutive (a segment),
            // and its first lane folds all of the segment's leaves at once
            {
                const int lane = lane_id();
                const int key = c >= 0 ? k : -1;
                const int prev = __shfl_up(key, 1, kWave);
                const bool head = c >= 0 && (lane == 0 || prev != key);
                const uint64_t heads = __ballot(head);
                const uint64_t leaves = __ballot(c >= 0 && cf == 0);
                if (head) {
                    const uint64_t above = lane == 63 ? 0ull : heads & (~0ull << (lane + 1));
                    const int next = above ? __builtin_ctzll(above) : 64;
                    const uint64_t seg = (next == 64 ? ~0ull : ((1ull << next) - 1)) & (~0ull << lane);
                    const int nleaf = __builtin_popcountll(leaves & seg);
                    if (nleaf) complete_leaves<OP>(a, p, nleaf);
                }
            }
            gsync<G>();
            if (s.buf_cnt >= G || s.buf_work >= kFlushPackets * a.work_cap) flush_buffer<G>(a, s, acc);
        }
        flush_buffer<G>(a, s, acc);
        // this dispatch is finished (its own follow-up packets are already counted)
        if (t == 0) __hip_atomic_fetch_add(a.outstanding, -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        gsync<G>();
    }
    if (a.want_stats) stat_flush(a.stats, acc);
}

// basic dynamic parallelism, emulated for comparison (driver 2): every node
// with children is a recursive call whose child kernel runs over its
// children; the host launches one such kernel per internal node, bottom-up,
// and the post-work folds the children (fixed-order workgroup reduction).
constexpr int kBasicBlock = 256;
template <int OP>
__global__ __launch_bounds__(kBasicBlock) void tree_child_basic(TreeArgs a, int v)
{
    __shared__ int tmp[kBasicBlock / kWave];
    const int beg = a.child_ptr[v], end = a.child_ptr[v + 1];
    int acc = 0;
    for (int i = beg + (int)threadIdx.x; i < end; i += kBasicBlock) acc = fold<OP>(acc, a.out[a.child[i]]);
    acc = OP == OP_DESC ? wave_sum_i(acc) : wave_max_i(acc);
    if (lane_id() == 0) tmp[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int r = 0;
        for (int k = 0; k < kBasicBlock / kWave; ++k) r = OP == OP_DESC ? r + tmp[k] : max(r, tmp[k]);
        a.out[v] = r;
    }
}

__global__ void tree_zero_out(TreeArgs a)
{
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) a.out[v] = 0;
}

// ---------------------------------------------------------------- host side

template <int OP, int BLOCK>
struct TreeKernels {
    const void *down, *up, *queue;
};

template <int OP, int BLOCK>
TreeKernels<OP, BLOCK> kernels_for(wc_mode mode)
{
    TreeKernels<OP, BLOCK> k{nullptr, nullptr, nullptr};
    if (mode == WC_GRID) {
        k.down = reinterpret_cast<const void *>(&tree_down<WC_GRID, BLOCK>);
        k.up = reinterpret_cast<const void *>(&tree_up<WC_GRID, OP, BLOCK>);
    } else if (mode == WC_FLAT) {
        k.down = reinterpret_cast<const void *>(&tree_down<WC_FLAT, BLOCK>);
        k.up = reinterpret_cast<const void *>(&tree_up<WC_FLAT, OP, BLOCK>);
    } else if (mode == WC_WAVE) {
        k.queue = reinterpret_cast<const void *>(&tree_queue<OP, kWave, BLOCK>);
    } else {
        k.queue = reinterpret_cast<const void *>(&tree_queue<OP, BLOCK, BLOCK>);
    }
    return k;
}

// The level-synchronous modes (flat, grid) over one tree or a batch of trees
// (all trees' items of one depth in the same level buffer).  n: total nodes,
// max_n: nodes of the largest tree (bounds the depth).
template <int OP, int BLOCK>
wc_status run_levels(wc_ctx *ctx, TreeArgs a, wc_mode mode, const Config &cfg, int grid, long long n, long long max_n,
                     const std::vector<TreeInst> *batch, hipStream_t stream, wc_stats *stats)
{
    // level-synchronous: levels <= max_n; chunks over all levels <= n + (n-1)/chunk + 1
    // per tree (the relaunch driver may run up to `window` empty levels past the last one)
    TreeKernels<OP, BLOCK> ks = kernels_for<OP, BLOCK>(mode);
    const int count = batch ? (int)batch->size() : 1;
    const long long max_levels = max_n + 1;
    const long long lvl_len = max_levels + 16;
    const int chunk = a.chunk;
    long long cap = mode == WC_GRID ? n + n / chunk + 2LL * count : n + count;
    const size_t inst_bytes = batch ? sizeof(TreeInst) * batch->size() : 0;
    size_t need = 2 * padded(lvl_len * 4) + padded(cap * 16) + padded(inst_bytes);
    wc_status st = pool_reserve(ctx, need, stream);
    if (st != WC_OK) return st;
    a.lvl_start = pool_take<int>(ctx, lvl_len);
    a.lvl_count = pool_take<int>(ctx, lvl_len);
    a.items = pool_take<int4>(ctx, cap);
    a.item_cap = cap;
    if (batch) {
        a.inst = reinterpret_cast<const TreeInst *>(pool_take<char>(ctx, inst_bytes));
        a.count = count;
    }
    st = begin_call(ctx, stream, stats);
    if (st != WC_OK) return st;
    if (batch) {
        st = stage_to_device(ctx, const_cast<TreeInst *>(a.inst), batch->data(), inst_bytes, stream);
        if (st != WC_OK) return st;
    }
    // level 0: the root(s)
    auto init_levels = [&]() -> wc_status {
        void *args[] = {&a};
        if (batch) {
            int grid_mode = mode == WC_GRID;
            void *bargs[] = {&a, &grid_mode};
            return launch(ctx, "tree_init_levels", reinterpret_cast<const void *>(&tree_init_batch), dim3(1),
                          dim3(256), bargs, stream);
        }
        return launch(ctx, "tree_init_levels",
                      mode == WC_GRID ? reinterpret_cast<const void *>(&tree_init_levels)
                                      : reinterpret_cast<const void *>(&tree_init_levels_flat),
                      dim3(1), dim3(64), args, stream);
    };
    st = init_levels();
    if (st != WC_OK) return st;
    // A call repeated on the same tree replays a captured graph of all levels
    // (down to the recorded depth plus one empty level, then up); the empty
    // level publishes its count, and a non-zero count (a deeper tree at the same
    // addresses) sends the call down the ordinary path.
    const char *down_name = mode == WC_GRID ? "tree_down_grid" : "tree_down_flat";
    const char *up_name = mode == WC_GRID ? "tree_up_grid" : "tree_up_flat";
    unsigned long long key = 1469598103934665603ull;
    {
        const unsigned char *b = reinterpret_cast<const unsigned char *>(&a);
        for (size_t k = 0; k < sizeof(a); ++k) key = (key ^ b[k]) * 1099511628211ull;
        const long long extra[4] = {(long long)mode, (long long)OP, (long long)grid, (long long)BLOCK};
        b = reinterpret_cast<const unsigned char *>(extra);
        for (size_t k = 0; k < sizeof(extra); ++k) key = (key ^ b[k]) * 1099511628211ull;
        // a batch is the same call only with the same trees and outputs
        b = reinterpret_cast<const unsigned char *>(batch ? batch->data() : nullptr);
        for (size_t k = 0; k < inst_bytes; ++k) key = (key ^ b[k]) * 1099511628211ull;
    }
    wc_ctx::TreeGraph *tg = nullptr;
    if (!ctx->timing)
        for (auto &e : ctx->tree_graphs)
            if (e.exec && e.key == key) tg = &e;
    if (tg) {
        clear_host_slot(ctx, kHostSlotGraph);
        chain_break(ctx);
        WC_HIP(hipEventRecord(ctx->graph_ready, stream));
        WC_HIP(hipStreamWaitEvent(ctx->capture_stream, ctx->graph_ready, 0));
        WC_HIP(hipGraphLaunch(tg->exec, ctx->capture_stream));
        WC_HIP(hipEventRecord(ctx->graph_done, ctx->capture_stream));
        WC_HIP(hipStreamWaitEvent(stream, ctx->graph_done, 0));
        int depth = 0;
        st = wait_host_slot(ctx, kHostSlotGraph, &depth);
        if (st != WC_OK) return st;
        if (depth >= 0) return end_call(ctx, stream, stats, depth, cfg.fail_on_overflow);
        WC_HIP(hipStreamSynchronize(stream));
        (void)hipGraphExecDestroy(tg->exec);
        *tg = wc_ctx::TreeGraph{};
        st = begin_call(ctx, stream, stats);
        if (st != WC_OK) return st;
        if (batch) {
            st = stage_to_device(ctx, const_cast<TreeInst *>(a.inst), batch->data(), inst_bytes, stream);
            if (st != WC_OK) return st;
        }
        st = init_levels();
        if (st != WC_OK) return st;
    }
    const int window = 4;
    int launched = 0, levels = 0;
    for (;;) {
        while (launched < levels + window) {
            clear_round_slot(ctx, launched);
            void *args[] = {&a, &launched};
            st = launch(ctx, down_name, ks.down, dim3(grid), dim3(BLOCK), args, stream);
            if (st != WC_OK) return st;
            ++launched;
        }
        int c = 0;
        st = wait_round_count(ctx, levels, &c);
        if (st != WC_OK) return st;
        if (c == 0) break;
        ++levels;
        if (levels > n + 1) return fail(WC_ETIMEOUT, "tree: more levels than nodes");
    }
    for (int l = levels - 1; l >= 0; --l) {
        void *args[] = {&a, &l};
        st = launch(ctx, up_name, ks.up, dim3(grid), dim3(BLOCK), args, stream);
        if (st != WC_OK) return st;
    }
    if (levels <= 1024 && !ctx->timing) {
        // record the levels of this tree as a graph for the next call
        hipGraph_t graph = nullptr;
        WC_HIP(hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
        const int saved_timing = ctx->timing;
        ctx->timing = 0;
        for (int l = 0; l <= levels && st == WC_OK; ++l) {
            void *args[] = {&a, &l};
            st = launch(ctx, down_name, ks.down, dim3(grid), dim3(BLOCK), args, ctx->capture_stream);
        }
        for (int l = levels - 1; l >= 0 && st == WC_OK; --l) {
            void *args[] = {&a, &l};
            st = launch(ctx, up_name, ks.up, dim3(grid), dim3(BLOCK), args, ctx->capture_stream);
        }
        if (st == WC_OK) {
            int L = levels;
            void *args[] = {&a, &L};
            st = launch(ctx, "tree_publish_depth", reinterpret_cast<const void *>(&tree_publish_depth), dim3(1),
                        dim3(64), args, ctx->capture_stream);
        }
        ctx->timing = saved_timing;
        hipError_t e = hipStreamEndCapture(ctx->capture_stream, &graph);
        if (st != WC_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        wc_ctx::TreeGraph &slot = ctx->tree_graphs[ctx->tree_graph_next];
        ctx->tree_graph_next = (ctx->tree_graph_next + 1) % 4;
        if (slot.exec) (void)hipGraphExecDestroy(slot.exec);
        slot = wc_ctx::TreeGraph{};
        e = hipGraphInstantiate(&slot.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            slot.exec = nullptr;
            return hip_fail(e, "hipGraphInstantiate");
        }
        slot.key = key;
        slot.levels = levels;
    }
    return end_call(ctx, stream, stats, levels, cfg.fail_on_overflow);
}

template <int OP, int BLOCK>
wc_status run_tree(wc_ctx *ctx, const wc_tree *t, int *out, wc_mode mode, const Config &cfg, hipStream_t stream,
                   wc_stats *stats)
{
    TreeKernels<OP, BLOCK> ks = kernels_for<OP, BLOCK>(mode);
    // the grid is sized to the residency of the kernel that runs: the queue kernel, or the level kernels
    const void *main_kernel = ks.queue ? ks.queue : ks.down;
    const int resident = resident_blocks(ctx, main_kernel, BLOCK);
    const int grid = std::max(1, std::min(cfg.grid, resident));
    const long long n = t->n;
    const int chunk = kWave * cfg.items_per_lane;
    TreeArgs a;
    std::memset(&a, 0, sizeof(a));
    a.parent = t->parent;
    a.child_ptr = t->child_ptr;
    a.child = t->child;
    a.out = out;
    a.n = (int)n;
    a.chunk = chunk;
    a.host_ring = ctx->host_ring_dev;
    a.stats = ctx->dstats;
    a.want_stats = stats != nullptr;
    a.wait_ticks = ctx->wait_ticks;
    a.work_cap = BLOCK * cfg.items_per_lane;
    if (cfg.driver == 2) {
        // no pool workspace (plan-only mode: nothing to record, nothing enqueued)
        if (ctx->plan_only) return pool_reserve(ctx, 0, stream);
        // Basic dynamic parallelism, emulated: the host walks the tree (read back
        // once) and launches one child kernel per internal node, deepest first.
        std::vector<int> cp((size_t)n + 1), ch((size_t)std::max<long long>(n - 1, 1));
        WC_HIP(hipMemcpy(cp.data(), t->child_ptr, sizeof(int) * (size_t)(n + 1), hipMemcpyDeviceToHost));
        if (n > 1) WC_HIP(hipMemcpy(ch.data(), t->child, sizeof(int) * (size_t)(n - 1), hipMemcpyDeviceToHost));
        std::vector<int> order;
        order.reserve((size_t)n);
        order.push_back(0);
        for (size_t i = 0; i < order.size(); ++i) {
            const int v = order[i];
            if (cp[v] < 0 || cp[v + 1] > n - 1 || cp[v] > cp[v + 1])
                return fail(WC_EINVAL, "tree: child_ptr out of range");
            for (int k = cp[v]; k < cp[v + 1]; ++k) {
                if (ch[k] <= 0 || ch[k] >= n || (long long)order.size() >= n)
                    return fail(WC_EINVAL, "tree: child list is not a tree rooted at 0");
                order.push_back(ch[k]);
            }
        }
        wc_status st = begin_call(ctx, stream, stats);
        if (st != WC_OK) return st;
        void *zargs[] = {&a};
        st = launch(ctx, "tree_zero_out", reinterpret_cast<const void *>(&tree_zero_out),
                    dim3((unsigned)std::min<long long>((n + 255) / 256, 4096)), dim3(256), zargs, stream);
        long long launches = 0;
        for (size_t i = order.size(); i-- > 0 && st == WC_OK;) {
            int v = order[i];
            if (cp[v + 1] == cp[v]) continue;
            void *cargs[] = {&a, &v};
            st = launch(ctx, "tree_child_basic", reinterpret_cast<const void *>(&tree_child_basic<OP>), dim3(1),
                        dim3(kBasicBlock), cargs, stream);
            ++launches;
        }
        if (st != WC_OK) return st;
        st = end_call(ctx, stream, stats, 0, cfg.fail_on_overflow);
        if (stats) {
            stats->dispatches = launches;
            stats->items_buffered = launches;
        }
        return st;
    }
    const bool queue_mode = mode == WC_WAVE || mode == WC_BLOCK;
    if (queue_mode) {
        a.work_cap = (mode == WC_WAVE ? kWave : BLOCK) * cfg.items_per_lane;
        long long pq_cap = n;
        size_t need = padded(n * 4) + padded(n * 8) + padded(pq_cap * 8) + 4 * padded(4);
        wc_status st = pool_reserve(ctx, need, stream);
        if (st != WC_OK) return st;
        a.nl = pool_take<int>(ctx, n);
        a.word = pool_take<unsigned long long>(ctx, n);
        a.pq = pool_take<long long>(ctx, pq_cap);
        a.pq_cap = pq_cap;
        a.nl_tail = pool_take<int>(ctx, 1);
        a.pq_head = pool_take<int>(ctx, 1);
        a.pq_tail = pool_take<int>(ctx, 1);
        a.outstanding = pool_take<int>(ctx, 1);
        st = begin_call(ctx, stream, stats);
        if (st != WC_OK) return st;
        int ig = (int)std::min<long long>((pq_cap + 255) / 256, 4096);
        void *iargs[] = {&a, &pq_cap};
        st = launch(ctx, "tree_init_queue", reinterpret_cast<const void *>(&tree_init_queue), dim3(ig), dim3(256),
                    iargs, stream);
        void *args[] = {&a};
        if (st == WC_OK)
            st = launch(ctx, "tree_publish_root", reinterpret_cast<const void *>(&tree_publish_root), dim3(1),
                        dim3(64), args, stream);
        if (st == WC_OK)
            st = launch(ctx, mode == WC_WAVE ? "tree_queue_wave" : "tree_queue_block", ks.queue, dim3(grid),
                        dim3(BLOCK), args, stream);
        if (st != WC_OK) return st;
        // the queue's waits are bounded: a wave that gave up is reported
        return end_call(ctx, stream, stats, 0, cfg.fail_on_overflow, true);
    }
    return run_levels<OP, BLOCK>(ctx, a, mode, cfg, grid, n, n, nullptr, stream, stats);
}

template <int OP>
wc_status run_tree_block(wc_ctx *ctx, const wc_tree *t, int *out, wc_mode mode, const Config &cfg,
                         hipStream_t stream, wc_stats *stats)
{
    switch (cfg.block) {
    case 64: return run_tree<OP, 64>(ctx, t, out, mode, cfg, stream, stats);
    case 128: return run_tree<OP, 128>(ctx, t, out, mode, cfg, stream, stats);
    case 512: return run_tree<OP, 512>(ctx, t, out, mode, cfg, stream, stats);
    case 1024: return run_tree<OP, 1024>(ctx, t, out, mode, cfg, stream, stats);
    default: return run_tree<OP, 256>(ctx, t, out, mode, cfg, stream, stats);
    }
}

wc_status tree_entry(int op, wc_ctx *ctx, const wc_tree *t, int32_t *out, wc_mode mode, const wc_tune *tune,
                     hipStream_t stream, wc_stats *stats)
{
    if (!ctx || !t) return fail(WC_EINVAL, "tree: NULL context or tree");
    if (mode < WC_FLAT || mode > WC_GRID) return fail(WC_EINVAL, "tree: bad mode");
    if (t->n < 1) return fail(WC_EINVAL, "tree: a tree has at least the root");
    if (!t->parent || !t->child_ptr || !out || (t->n > 1 && !t->child)) return fail(WC_EINVAL, "tree: NULL array");
    WC_HIP(hipSetDevice(ctx->device));
    Config cfg;
    wc_status st = resolve_tune(ctx, "tree", mode, tune, ctx->num_cus * 8, &cfg);
    if (st != WC_OK) return st;
    // descendants at block level run 512-thread groups by default: their folds
    // are one 64-bit add, while the heights' compare-and-swap folds contend more
    // in larger groups (2^22-node random tree at 256 / 512 threads: descendants
    // 1.09 / 0.88 ms, heights 2.41 / 2.75 ms; 39.3M-node layered tree,
    // descendants 1.11 / 0.79 ms)
    if (op == OP_DESC && mode == WC_BLOCK && !(tune && tune->block_threads > 0)) cfg.block = 512;
    // refusals come before anything is enqueued
    if (cfg.driver == 2 && mode != WC_GRID) return fail(WC_EINVAL, "tree: driver 2 needs grid mode");
    if (tune && tune->grid_blocks > 0) cfg.grid = tune->grid_blocks;
    else cfg.grid = 1 << 30;  // clamp to the resident count of the chosen kernel
    return op == OP_DESC ? run_tree_block<OP_DESC>(ctx, t, out, mode, cfg, stream, stats)
                         : run_tree_block<OP_HEIGHT>(ctx, t, out, mode, cfg, stream, stats);
}

// Many trees in one sequence of level launches (flat or grid mode): every
// level kernel takes the items of that depth of all trees, so grid mode
// consolidates the recursive calls of every tree into one buffer per level.
template <int OP, int BLOCK>
wc_status run_tree_batch(wc_ctx *ctx, int32_t count, const wc_tree *trees, int32_t *const *out, wc_mode mode,
                         const Config &cfg, hipStream_t stream, wc_stats *stats)
{
    TreeKernels<OP, BLOCK> ks = kernels_for<OP, BLOCK>(mode);
    const int resident = resident_blocks(ctx, ks.down, BLOCK);
    const int grid = std::max(1, std::min(cfg.grid, resident));
    std::vector<TreeInst> inst((size_t)count);
    long long total = 0, max_n = 1;
    for (int i = 0; i < count; ++i) {
        inst[i] = TreeInst{trees[i].child_ptr, trees[i].child, out[i], trees[i].n};
        total += trees[i].n;
        max_n = std::max<long long>(max_n, trees[i].n);
    }
    if (total > 0x7fffffffLL) return fail(WC_EINVAL, "tree batch: more than 2^31 nodes in one batch");
    TreeArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = (int)total;
    a.chunk = kWave * cfg.items_per_lane;
    a.host_ring = ctx->host_ring_dev;
    a.stats = ctx->dstats;
    a.want_stats = stats != nullptr;
    a.wait_ticks = ctx->wait_ticks;
    return run_levels<OP, BLOCK>(ctx, a, mode, cfg, grid, total, max_n, &inst, stream, stats);
}

wc_status tree_batch_entry(int op, wc_ctx *ctx, int32_t count, const wc_tree *trees, int32_t *const *out,
                           wc_mode mode, const wc_tune *tune, hipStream_t stream, wc_stats *stats)
{
    if (!ctx || count < 0 || (count > 0 && (!trees || !out))) return fail(WC_EINVAL, "tree batch: NULL argument");
    if (mode != WC_FLAT && mode != WC_GRID)
        return fail(WC_EINVAL, "tree batch: flat and grid modes only (the queue modes run one tree per call)");
    if (count > (1 << 30)) return fail(WC_EINVAL, "tree batch: too many trees");
    for (int i = 0; i < count; ++i) {
        const wc_tree &t = trees[i];
        if (t.n < 1) return fail(WC_EINVAL, "tree batch: tree " + std::to_string(i) + " has no root");
        if (!t.child_ptr || !out[i] || (t.n > 1 && !t.child))
            return fail(WC_EINVAL, "tree batch: NULL array in tree " + std::to_string(i));
    }
    if (count == 0) {
        if (stats) std::memset(stats, 0, sizeof(*stats));
        return WC_OK;
    }
    WC_HIP(hipSetDevice(ctx->device));
    Config cfg;
    wc_status st = resolve_tune(ctx, "tree", mode, tune, ctx->num_cus * 8, &cfg);
    if (st != WC_OK) return st;
    if (cfg.driver != 0) return fail(WC_EINVAL, "tree batch: only the relaunch driver (driver = 0) applies");
    if (tune && tune->grid_blocks > 0) cfg.grid = tune->grid_blocks;
    else cfg.grid = 1 << 30;
    auto run = [&](auto opc) -> wc_status {
        constexpr int OPV = decltype(opc)::value;
        switch (cfg.block) {
        case 64: return run_tree_batch<OPV, 64>(ctx, count, trees, out, mode, cfg, stream, stats);
        case 128: return run_tree_batch<OPV, 128>(ctx, count, trees, out, mode, cfg, stream, stats);
        case 512: return run_tree_batch<OPV, 512>(ctx, count, trees, out, mode, cfg, stream, stats);
        case 1024: return run_tree_batch<OPV, 1024>(ctx, count, trees, out, mode, cfg, stream, stats);
        default: return run_tree_batch<OPV, 256>(ctx, count, trees, out, mode, cfg, stream, stats);
        }
    };
    return op == OP_DESC ? run(std::integral_constant<int, OP_DESC>{}) : run(std::integral_constant<int, OP_HEIGHT>{});
}

}  // namespace
}  // namespace wc

using namespace wc;

extern "C" wc_status wc_tree_descendants_batch(wc_ctx *ctx, int32_t count, const wc_tree *trees, int32_t *const *desc,
                                               wc_mode mode, const wc_tune *tune, hipStream_t stream, wc_stats *stats)
{
    return tree_batch_entry(OP_DESC, ctx, count, trees, desc, mode, tune, stream, stats);
}

extern "C" wc_status wc_tree_height_batch(wc_ctx *ctx, int32_t count, const wc_tree *trees, int32_t *const *height,
                                          wc_mode mode, const wc_tune *tune, hipStream_t stream, wc_stats *stats)
{
    return tree_batch_entry(OP_HEIGHT, ctx, count, trees, height, mode, tune, stream, stats);
}

extern "C" wc_status wc_tree_descendants(wc_ctx *ctx, const wc_tree *t, int32_t *desc, wc_mode mode,
                                         const wc_tune *tune, hipStream_t stream, wc_stats *stats)
{
    return tree_entry(OP_DESC, ctx, t, desc, mode, tune, stream, stats);
}

extern "C" wc_status wc_tree_height(wc_ctx *ctx, const wc_tree *t, int32_t *height, wc_mode mode,
                                    const wc_tune *tune, hipStream_t stream, wc_stats *stats)
{
    return tree_entry(OP_HEIGHT, ctx, t, height, mode, tune, stream, stats);
}
