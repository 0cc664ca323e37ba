// Batched SSSP: many independent instances in one launch sequence.
//
// The instances' vertices are numbered consecutively (instance i owns global
// ids vbase[i] .. vbase[i+1]-1) and every round runs one parent kernel over
// the whole id range, so one grid serves all instances.  Each instance brings
// its own consolidation granularity and threshold (picked per size bucket by
// the autotuner): a heavy vertex goes to its wave's ballot buffer, its block's
// LDS buffer or the global chunk buffer, according to its instance's mode, and
// the global buffer consolidates heavy items of all grid-mode instances into
// one child (Sec. IV.A: buffering the work of many would-be child launches).
// The round kernels exit at once when no instance has a frontier, so a fixed
// number of rounds can be captured into a HIP graph and replayed as a single
// launch; the host continues with ordinary rounds if they were not enough.
#include <algorithm>
#include <cstring>
#include <vector>

#include "wc_block.h"
#include "wc_device.h"
#include "wc_internal.h"
#include "wc_stats.h"

namespace wc {
namespace {

constexpr int kPad = 32;
constexpr int kUnroll = 4;
constexpr int kWinInst = 256;  // vertices per entry of the instance lookup table

struct Inst {
    const int *row_ptr;
    const int *col;
    const uint32_t *w;
    uint32_t *dist;
    int n;
    int mode;
    int threshold;
    int chunk;
    int src;
    int pad;
};

struct BatchArgs {
    const Inst *inst;
    const int *vbase;  // [count + 1]
    const int *win_inst;  // [total / kWinInst + 1]: instance owning vertex k * kWinInst
    int count;
    int total;         // vbase[count]
    int *stamp;        // [total]
    uint32_t *relaxed_at;  // [total]: the largest distance the vertex's edges were last relaxed with
    int *active;       // ring of 3 (stride kPad)
    int *chunk_tail;   // ring of 3 (stride kPad)
    int4 *chunks;      // (global u, begin, end, instance)
    long long chunk_cap;
    unsigned long long *host_ring;
    DevStats *stats;
    int want_stats;
    int has_wave, has_block, has_grid;  // which consolidation levels occur in this batch
};

// Instance owning global vertex gid: the instance owning vertex
// (gid / kWinInst) * kWinInst, from the window table, then forward.
__device__ __forceinline__ int find_inst(const BatchArgs &a, int gid)
{
    int i = a.win_inst[gid / kWinInst];
    while (gid >= a.vbase[i + 1]) ++i;
    return i;
}

__device__ __forceinline__ uint32_t add_sat(uint32_t du, uint32_t w)
{
    uint32_t s = du + w;
    return s < du ? kInf : s;
}

__device__ __forceinline__ bool relax_loaded(uint32_t *dist, int *stamp_base, int v, uint32_t nd, uint32_t dv,
                                             int next)
{
    // as in single-instance SSSP: stamping on nd < dv gives the same frontier
    // as waiting for the atomic's old value
    if (nd >= dv) return false;
    atomic_min_dev_noret(&dist[v], nd);
    stamp_base[v] = next;
    return true;
}

// kUnroll edges per lane: e_k = first + k * stride (< end) of one instance.
__device__ __forceinline__ bool relax_batch(const Inst &d, int *stamp_base, int first, int stride, int end,
                                            uint32_t du, int next)
{
    int v[kUnroll];
    uint32_t wt[kUnroll], dv[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
        const int e = first + k * stride;
        const bool ok = e < end;
        v[k] = ok ? d.col[e] : -1;
        wt[k] = ok ? d.w[e] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) dv[k] = v[k] >= 0 ? d.dist[v[k]] : 0u;
    bool any = false;
#pragma unroll
    for (int k = 0; k < kUnroll; ++k)
        if (v[k] >= 0) any |= relax_loaded(d.dist, stamp_base, v[k], add_sat(du, wt[k]), dv[k], next);
    return any;
}

__global__ void batch_init(BatchArgs a)
{
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < a.total; g += gridDim.x * blockDim.x) {
        const int i = find_inst(a, g);
        const Inst &d = a.inst[i];
        const int v = g - a.vbase[i];
        const bool s = v == d.src;
        d.dist[v] = s ? 0u : kInf;
        a.stamp[g] = s ? 0 : -1;
        a.relaxed_at[g] = kInf;
    }
    if (blockIdx.x == 0 && threadIdx.x < 3) {
        a.active[threadIdx.x * kPad] = threadIdx.x == 0 ? 1 : 0;
        a.chunk_tail[threadIdx.x * kPad] = 0;
    }
}

template <int BLOCK>
struct BatchLds {
    int inst[BLOCK];
    int beg[BLOCK];
    int end[BLOCK];
    int csz[BLOCK];
    uint32_t du[BLOCK];
    int pre[BLOCK + 1];
    int scan_tmp[2 * (BLOCK / kWave)];
    int base;
};

// Windows of BLOCK vertices whose frontier stamps a block of batch_round
// reads together.
constexpr int kWindowsPerStep = 8;

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void batch_round(BatchArgs a, int r)
{
    __shared__ BatchLds<BLOCK> sb;
    const int act = a.active[(r % 3) * kPad];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.active[((r + 2) % 3) * kPad] = 0;
        a.chunk_tail[((r + 1) % 3) * kPad] = 0;
        publish_host(a.host_ring, r % kHostRing, a.stats, act);
    }
    if (!act) return;
    const int next = r + 1;
    const int lane = lane_id();
    StatAcc acc;
    // the stamps of S windows are read together and a block skips all S at
    // once when none of them holds a frontier vertex
    constexpr int S = kWindowsPerStep;
    const int stride = gridDim.x * BLOCK;
    for (long long wbase = (long long)blockIdx.x * BLOCK; wbase < a.total; wbase += (long long)S * stride) {
        int bits = 0;
#pragma unroll
        for (int w = 0; w < S; ++w) {
            const long long gg = wbase + (long long)w * stride + threadIdx.x;
            if (gg < a.total && a.stamp[gg] == r) bits |= 1 << w;
        }
        if (!__syncthreads_or(bits)) continue;
        for (int w = 0; w < S; ++w) {
            const long long base_l = wbase + (long long)w * stride;
            if (base_l >= a.total) break;  // uniform in the block
            const int base = (int)base_l;
            const int g = base + threadIdx.x;
            const bool member = (bits >> w) & 1;
            int i = 0, beg = 0, end = 0, mode = WC_FLAT;
            uint32_t du = 0;
            if (member) {
                i = find_inst(a, g);
                const Inst &d = a.inst[i];
                const int v = g - a.vbase[i];
                beg = d.row_ptr[v];
                end = d.row_ptr[v + 1];
                du = d.dist[v];
                // already relaxed with its present distance (it improved before its
                // own relaxations read it): nothing to do
                if (a.relaxed_at[g] == du) end = beg;
                mode = end - beg > d.threshold ? d.mode : WC_FLAT;
                // a wave's or block's own child keeps items of up to one chunk;
                // longer ones go to the grid-wide drain (the KC_X rule of
                // Sec. IV.E: a warp's or block's child gets many blocks)
                if ((mode == WC_WAVE || mode == WC_BLOCK) && end - beg > d.chunk) mode = WC_GRID;
                // wave, block and inline work use this reading; grid chunks raise
                // the value from 0 in the drain (or it stays du on overflow)
                if (end > beg && mode != WC_GRID) a.relaxed_at[g] = du;
            }
            const int deg = end - beg;
            const bool heavy = mode != WC_FLAT;
            if (a.want_stats) {
                acc.edges += deg;
                acc.buffered += heavy ? deg : 0;
                acc.items += heavy ? 1 : 0;
            }
            bool any = false;
            if (member && !heavy) any = [&] {
                const Inst &d = a.inst[i];
                int *sbase = a.stamp + a.vbase[i];
                bool f = false;
                for (int e = beg; e < end; e += kUnroll) f |= relax_batch(d, sbase, e, 1, end, du, next);
                return f;
            }();
            // wave-level items: the ballot mask is the buffer, the wave drains it
            uint64_t wmask = a.has_wave ? __ballot(mode == WC_WAVE) : 0ull;
            if (a.want_stats && wmask && lane == 0) acc.dispatches += 1;
            while (wmask) {
                const int b = __builtin_ctzll(wmask);
                wmask &= wmask - 1;
                const int ii = readlane(i, b);
                const Inst &d = a.inst[ii];
                int *sbase = a.stamp + a.vbase[ii];
                const int ub = readlane(beg, b), ue = readlane(end, b);
                const uint32_t ud = readlane_u(du, b);
                for (int e0 = ub; e0 < ue; e0 += kWave * kUnroll)
                    any |= relax_batch(d, sbase, e0 + lane, kWave, ue, ud, next);
            }
            // block-level items: LDS buffer, barrier, flattened drain by the block
            if (a.has_block) {
                const bool bl = mode == WC_BLOCK;
                int k, off, nb, total;
                block_scan2<BLOCK>(bl ? 1 : 0, bl ? deg : 0, sb.scan_tmp, k, off, nb, total);
                if (bl) {
                    sb.inst[k] = i;
                    sb.beg[k] = beg;
                    sb.du[k] = du;
                    sb.pre[k] = off;
                }
                if (threadIdx.x == 0) {
                    sb.pre[nb] = total;
                    if (a.want_stats && nb) acc.dispatches += 1;
                }
                __syncthreads();
                int it = 0;
                for (int j = threadIdx.x; j < total; j += BLOCK) {
                    while (it + 1 < nb && sb.pre[it + 1] <= j) ++it;
                    const Inst &d = a.inst[sb.inst[it]];
                    const int e = sb.beg[it] + (j - sb.pre[it]);
                    const int v = d.col[e];
                    const uint32_t nd = add_sat(sb.du[it], d.w[e]);
                    any |= relax_loaded(d.dist, a.stamp + a.vbase[sb.inst[it]], v, nd, d.dist[v], next);
                }
                __syncthreads();
            }
            // grid-level items: chunks into the global buffer (block-aggregated reservation)
            if (a.has_grid) {
                const bool gr = mode == WC_GRID;
                int chunk = 1, nch = 0;
                if (gr) {
                    chunk = a.inst[i].chunk;
                    nch = (deg + chunk - 1) / chunk;
                }
                int excl, d0, tot, d1;
                block_scan2<BLOCK>(nch, 0, sb.scan_tmp, excl, d0, tot, d1);
                sb.pre[threadIdx.x] = excl;
                sb.inst[threadIdx.x] = i;
                sb.beg[threadIdx.x] = beg;
                sb.end[threadIdx.x] = end;
                sb.csz[threadIdx.x] = chunk;
                sb.du[threadIdx.x] = du;
                if (threadIdx.x == 0) sb.base = tot ? atomic_add_dev(&a.chunk_tail[(r % 3) * kPad], tot) : 0;
                __syncthreads();
                const int slot0 = sb.base;
                if (nch > 0) a.relaxed_at[g] = (long long)slot0 + excl + nch > a.chunk_cap ? du : 0u;
                // the block writes the window's chunks together: chunk j belongs to
                // the last thread whose offset is <= j
                for (int j = threadIdx.x; j < tot; j += BLOCK) {
                    int lo = 0, hi = BLOCK - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (sb.pre[mid] <= j) lo = mid;
                        else hi = mid - 1;
                    }
                    const int ck = sb.csz[lo];
                    const int cb = sb.beg[lo] + (j - sb.pre[lo]) * ck, ce = min(sb.end[lo], cb + ck);
                    const int oi = sb.inst[lo];
                    if ((long long)slot0 + j < a.chunk_cap) {
                        a.chunks[slot0 + j] = make_int4(base + lo, cb, ce, oi);
                    } else {
                        a.stats->overflowed = 1;
                        const Inst &d = a.inst[oi];
                        int *sbase = a.stamp + a.vbase[oi];
                        for (int e = cb; e < ce; e += kUnroll) any |= relax_batch(d, sbase, e, 1, ce, sb.du[lo], next);
                    }
                }
                __syncthreads();
            }
            if (__ballot(any) && lane == 0) a.active[((r + 1) % 3) * kPad] = 1;
        }
    }
    if (a.want_stats) stat_flush(a.stats, acc);
}

// Two chunks at once (uniform arguments; the chunks may belong to different
// instances): each lane keeps 2 * kUnroll edges in flight.  The source
// distances are read after the edges are requested; the distances used are
// returned.  Chunk 1 may be empty (cb1 == ce1).
__device__ __forceinline__ bool relax_pair(const BatchArgs &a, int g0, int i0, int cb0, int ce0, int g1, int i1,
                                           int cb1, int ce1, int next, uint32_t &du0_used, uint32_t &du1_used)
{
    const Inst &d0 = a.inst[i0];
    const Inst &d1 = a.inst[i1];
    const int vb0 = a.vbase[i0], vb1 = a.vbase[i1];
    int *sb0 = a.stamp + vb0;
    int *sb1 = a.stamp + vb1;
    bool any = false;
    du0_used = du1_used = 0u;
    const int len = max(ce0 - cb0, ce1 - cb1);
    for (int o = lane_id(); o - lane_id() < len; o += kWave * kUnroll) {
        int v[2 * kUnroll];
        uint32_t wt[2 * kUnroll], dv[2 * kUnroll];
#pragma unroll
        for (int k = 0; k < 2 * kUnroll; ++k) {
            const bool first = k < kUnroll;
            const int e = (first ? cb0 : cb1) + o + (k % kUnroll) * kWave;
            const bool ok = e < (first ? ce0 : ce1);
            v[k] = ok ? (first ? d0.col[e] : d1.col[e]) : -1;
            wt[k] = ok ? (first ? d0.w[e] : d1.w[e]) : 0u;
        }
        const uint32_t du0 = d0.dist[g0 - vb0];
        const uint32_t du1 = cb1 < ce1 ? d1.dist[g1 - vb1] : 0u;
        du0_used = max(du0_used, du0);
        du1_used = max(du1_used, du1);
#pragma unroll
        for (int k = 0; k < 2 * kUnroll; ++k) dv[k] = v[k] >= 0 ? (k < kUnroll ? d0.dist[v[k]] : d1.dist[v[k]]) : 0u;
#pragma unroll
        for (int k = 0; k < 2 * kUnroll; ++k)
            if (v[k] >= 0) {
                const bool first = k < kUnroll;
                any |= relax_loaded(first ? d0.dist : d1.dist, first ? sb0 : sb1, v[k],
                                    add_sat(first ? du0 : du1, wt[k]), dv[k], next);
            }
    }
    return any;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void batch_drain(BatchArgs a, int r)
{
    if (!a.active[(r % 3) * kPad]) return;
    const int tail = a.chunk_tail[(r % 3) * kPad];
    const int total = (long long)tail < a.chunk_cap ? tail : (int)a.chunk_cap;
    const int next = r + 1;
    const int gw = (blockIdx.x * BLOCK + threadIdx.x) / kWave;
    const int nw = gridDim.x * (BLOCK / kWave);
    if (a.want_stats && blockIdx.x == 0 && threadIdx.x == 0 && total > 0)
        atomic_add_dev(&a.stats->rep[0].dispatches, 1ull);
    bool any = false;
    // two chunks per wave and step; the next pair's entries are fetched before
    // the current pair's edges
    int4 q0 = load_or_zero(a.chunks, gw, gw < total);
    int4 q1 = load_or_zero(a.chunks, gw + nw, gw + nw < total);
    for (int c = gw; c < total; c += 2 * nw) {
        const int g0 = __builtin_amdgcn_readfirstlane(q0.x), i0 = __builtin_amdgcn_readfirstlane(q0.w);
        const int cb0 = __builtin_amdgcn_readfirstlane(q0.y), ce0 = __builtin_amdgcn_readfirstlane(q0.z);
        const int g1 = __builtin_amdgcn_readfirstlane(q1.x), i1 = __builtin_amdgcn_readfirstlane(q1.w);
        const int cb1 = __builtin_amdgcn_readfirstlane(q1.y), ce1 = __builtin_amdgcn_readfirstlane(q1.z);
        const int cn = c + 2 * nw;
        q0 = load_or_zero(a.chunks, cn, cn < total);
        q1 = load_or_zero(a.chunks, cn + nw, cn + nw < total);
        uint32_t du0, du1;
        any |= relax_pair(a, g0, i0, cb0, ce0, g1, i1, cb1, ce1, next, du0, du1);
        if (lane_id() == 0) {
            atomic_max_dev_noret(&a.relaxed_at[g0], du0);
            if (cb1 < ce1) atomic_max_dev_noret(&a.relaxed_at[g1], du1);
        }
    }
    if (__ballot(any) && lane_id() == 0) a.active[((r + 1) % 3) * kPad] = 1;
}

// Publishes whether round r has a frontier (after the graph's last round).
__global__ void batch_publish(BatchArgs a, int r)
{
    if (threadIdx.x == 0) publish_host(a.host_ring, r % kHostRing, a.stats, a.active[(r % 3) * kPad]);
}

struct BatchKernels {
    const void *round, *drain;
};

BatchKernels pick(int block)
{
    switch (block) {
    case 64: return {reinterpret_cast<const void *>(&batch_round<64>), reinterpret_cast<const void *>(&batch_drain<64>)};
    case 128:
        return {reinterpret_cast<const void *>(&batch_round<128>), reinterpret_cast<const void *>(&batch_drain<128>)};
    case 512:
        return {reinterpret_cast<const void *>(&batch_round<512>), reinterpret_cast<const void *>(&batch_drain<512>)};
    case 1024:
        return {reinterpret_cast<const void *>(&batch_round<1024>),
                reinterpret_cast<const void *>(&batch_drain<1024>)};
    default:
        return {reinterpret_cast<const void *>(&batch_round<256>), reinterpret_cast<const void *>(&batch_drain<256>)};
    }
}

}  // namespace
}  // namespace wc

using namespace wc;

static unsigned long long fnv(unsigned long long h, const void *p, size_t n)
{
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t k = 0; k < n; ++k) h = (h ^ b[k]) * 1099511628211ull;
    return h;
}

extern "C" wc_status wc_sssp_batch(wc_ctx *ctx, int32_t count, const wc_csr *graphs, const uint32_t *const *w,
                                   const int32_t *src, uint32_t *const *dist, const wc_mode *modes,
                                   const wc_tune *tunes, int32_t graph_rounds, hipStream_t stream, wc_stats *stats)
{
    if (!ctx || count < 0 || (count > 0 && (!graphs || !w || !src || !dist)))
        return fail(WC_EINVAL, "wc_sssp_batch: NULL argument");
    if (count == 0) {
        if (stats) std::memset(stats, 0, sizeof(*stats));
        return WC_OK;
    }
    if (graph_rounds < 0 || graph_rounds > 4096) return fail(WC_EINVAL, "wc_sssp_batch: graph_rounds out of range");
    WC_HIP(hipSetDevice(ctx->device));
    std::vector<Inst> inst(count);
    std::vector<int> vbase(count + 1);
    long long total = 0, cap = 1;
    int block = 256, has[4] = {0, 0, 0, 0};
    for (int i = 0; i < count; ++i) {
        const wc_csr &g = graphs[i];
        if (g.n < 1 || g.m < 0 || !g.row_ptr || !dist[i] || (g.m > 0 && (!g.col || !w[i])))
            return fail(WC_EINVAL, "wc_sssp_batch: bad instance " + std::to_string(i));
        if (src[i] < 0 || src[i] >= g.n)
            return fail(WC_EINVAL, "wc_sssp_batch: source out of range in instance " + std::to_string(i));
        const wc_mode mode = modes ? modes[i] : WC_GRID;
        if (mode < WC_FLAT || mode > WC_GRID) return fail(WC_EINVAL, "wc_sssp_batch: bad mode");
        Config cfg;
        wc_status st = resolve_tune(ctx, "sssp", mode, tunes ? &tunes[i] : nullptr, 1, &cfg);
        if (st != WC_OK) return st;
        // one workgroup size for the whole batch: the first instance's; later
        // instances that leave block_threads unset adopt it
        if (i == 0) block = cfg.block;
        else if (tunes && tunes[i].block_threads > 0 && tunes[i].block_threads != block)
            return fail(WC_EINVAL, "wc_sssp_batch: all instances must share block_threads");
        if (cfg.driver != 0) return fail(WC_EINVAL, "wc_sssp_batch: the persistent driver is disabled");
        const int chunk = kWave * cfg.items_per_lane;
        inst[i] = Inst{g.row_ptr, g.col, w[i], dist[i], g.n, (int)mode, mode == WC_FLAT ? 0x7fffffff : cfg.threshold,
                       chunk, src[i], 0};
        has[mode] = 1;
        vbase[i] = (int)total;
        total += g.n;
        if (mode == WC_GRID) cap += g.n + g.m / chunk + 1;
        // wave and block levels hand vertices with more than one chunk of edges
        // (at most 2 deg / chunk chunks each) to the grid path
        if (mode == WC_WAVE || mode == WC_BLOCK) {
            has[WC_GRID] = 1;
            cap += 2 * (g.m / chunk) + 1;
        }
        if (total > 0x7fffffffLL) return fail(WC_EINVAL, "wc_sssp_batch: more than 2^31 vertices in one batch");
    }
    vbase[count] = (int)total;
    BatchKernels ks = pick(block);
    const int resident = resident_blocks(ctx, ks.round, block);
    const int windows = (int)((total + block - 1) / block);
    // With wave- or block-level instances the parent takes one step of
    // kWindowsPerStep windows per workgroup, so the hardware hands the steps
    // dense with buffered vertices to CUs as they free up (512 instances, all
    // block / all wave: 15.8 -> 14.1 ms, 20.5 -> 16.9 ms); grid-level
    // instances alone keep the resident grid (15.2 against 15.5 ms).
    const int grid = std::max(1, has[WC_WAVE] || has[WC_BLOCK] ? (windows + kWindowsPerStep - 1) / kWindowsPerStep
                                                              : std::min(resident, windows));
    const int dgrid = std::max(1, resident);
    const long long nwin = total / kWinInst + 1;
    const size_t blob = padded(sizeof(Inst) * count) + padded(4 * (count + 1)) + padded(4 * nwin);
    size_t need = blob + 2 * padded(total * 4) + 2 * padded(3 * kPad * 4) + padded(cap * 16);
    wc_status st = pool_reserve(ctx, need, stream);
    if (st != WC_OK) return st;
    BatchArgs a;
    std::memset(&a, 0, sizeof(a));
    char *d_blob = pool_take<char>(ctx, blob);
    a.inst = reinterpret_cast<const Inst *>(d_blob);
    a.vbase = reinterpret_cast<const int *>(d_blob + padded(sizeof(Inst) * count));
    a.win_inst = reinterpret_cast<const int *>(d_blob + padded(sizeof(Inst) * count) + padded(4 * (count + 1)));
    a.count = count;
    a.total = (int)total;
    a.stamp = pool_take<int>(ctx, total);
    a.relaxed_at = pool_take<uint32_t>(ctx, total);
    a.active = pool_take<int>(ctx, 3 * kPad);
    a.chunk_tail = pool_take<int>(ctx, 3 * kPad);
    a.chunks = pool_take<int4>(ctx, cap);
    a.chunk_cap = cap;
    a.host_ring = ctx->host_ring_dev;
    a.stats = ctx->dstats;
    a.want_stats = stats != nullptr;
    a.has_wave = has[WC_WAVE];
    a.has_block = has[WC_BLOCK];
    a.has_grid = has[WC_GRID];
    // descriptors (instances, then vertex offsets) in one staged upload
    std::vector<char> host_blob(blob, 0);
    std::memcpy(host_blob.data(), inst.data(), sizeof(Inst) * count);
    std::memcpy(host_blob.data() + padded(sizeof(Inst) * count), vbase.data(), 4 * (count + 1));
    {
        int *win = reinterpret_cast<int *>(host_blob.data() + padded(sizeof(Inst) * count) + padded(4 * (count + 1)));
        int i = 0;
        for (long long k = 0; k < nwin; ++k) {
            const long long v = k * kWinInst;
            while (i + 1 < count && v >= vbase[i + 1]) ++i;
            win[k] = i;
        }
    }
    st = stage_to_device(ctx, d_blob, host_blob.data(), blob, stream);
    if (st != WC_OK) return st;
    st = begin_call(ctx, stream, stats);
    if (st != WC_OK) return st;
    {
        void *args[] = {&a};
        const int ig = (int)std::min<long long>((total + 255) / 256, 8192);
        st = launch(ctx, "batch_init", reinterpret_cast<const void *>(&batch_init), dim3(ig), dim3(256), args, stream);
        if (st != WC_OK) return st;
    }
    int rounds_done = 0;
    if (graph_rounds > 0) {
        // graph_rounds rounds captured once into a graph (its kernels exit at
        // once past convergence), replayed as one launch while the arguments stay
        // the same; a final kernel publishes whether more rounds are needed
        unsigned long long key = 1469598103934665603ull;
        key = fnv(key, &a, sizeof(a));
        key = fnv(key, &graph_rounds, sizeof(graph_rounds));
        key = fnv(key, &grid, sizeof(grid));
        key = fnv(key, &dgrid, sizeof(dgrid));
        key = fnv(key, &block, sizeof(block));
        if (!ctx->graph_exec || ctx->graph_key != key) {
            if (ctx->graph_exec) {
                WC_HIP(hipStreamSynchronize(stream));
                WC_HIP(hipStreamSynchronize(ctx->capture_stream));
                (void)hipGraphExecDestroy(ctx->graph_exec);
                ctx->graph_exec = nullptr;
            }
            hipGraph_t graph = nullptr;
            WC_HIP(hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
            const int saved_timing = ctx->timing;
            ctx->timing = 0;  // no event records inside the captured graph
            for (int r = 0; r < graph_rounds && st == WC_OK; ++r) {
                void *args[] = {&a, &r};
                st = launch(ctx, "batch_round", ks.round, dim3(grid), dim3(block), args, ctx->capture_stream);
                if (st == WC_OK)
                    st = launch(ctx, "batch_drain", ks.drain, dim3(dgrid), dim3(block), args, ctx->capture_stream);
            }
            int rr = graph_rounds;
            void *pargs[] = {&a, &rr};
            if (st == WC_OK)
                st = launch(ctx, "batch_publish", reinterpret_cast<const void *>(&batch_publish), dim3(1), dim3(64),
                            pargs, ctx->capture_stream);
            ctx->timing = saved_timing;
            hipError_t e = hipStreamEndCapture(ctx->capture_stream, &graph);
            if (st != WC_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&ctx->graph_exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                ctx->graph_exec = nullptr;
                return hip_fail(e, "hipGraphInstantiate");
            }
            ctx->graph_key = key;
        }
        for (int r = 0; r <= graph_rounds; ++r) clear_round_slot(ctx, r);
        chain_break(ctx);
        WC_HIP(hipEventRecord(ctx->graph_ready, stream));
        WC_HIP(hipStreamWaitEvent(ctx->capture_stream, ctx->graph_ready, 0));
        WC_HIP(hipGraphLaunch(ctx->graph_exec, ctx->capture_stream));
        WC_HIP(hipEventRecord(ctx->graph_done, ctx->capture_stream));
        WC_HIP(hipStreamWaitEvent(stream, ctx->graph_done, 0));
        int c = 0;
        st = wait_round_count(ctx, graph_rounds, &c);
        if (st != WC_OK) return st;
        rounds_done = graph_rounds;
        if (c == 0) return end_call(ctx, stream, stats, graph_rounds, false);
    }
    // ordinary rounds (all of them without a graph, or the ones the graph did not cover)
    const int window = 4;
    int rounds = rounds_done, launched = rounds_done;
    for (;;) {
        while (launched < rounds + window) {
            clear_round_slot(ctx, launched);
            void *args[] = {&a, &launched};
            st = launch(ctx, "batch_round", ks.round, dim3(grid), dim3(block), args, stream);
            if (st == WC_OK) st = launch(ctx, "batch_drain", ks.drain, dim3(dgrid), dim3(block), args, stream);
            if (st != WC_OK) return st;
            ++launched;
        }
        int c = 0;
        st = wait_round_count(ctx, rounds, &c);
        if (st != WC_OK) return st;
        if (c == 0) break;
        ++rounds;
        if (rounds > total + 1) return fail(WC_ETIMEOUT, "wc_sssp_batch: more rounds than vertices");
    }
    return end_call(ctx, stream, stats, rounds, false);
}
