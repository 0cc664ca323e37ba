// Context, pre-allocated pool, error reporting and configuration of libwc.
//
// The pool is the customized allocator of Sec. IV.E: one device allocation
// made up front, from which each call carves its consolidation buffers, so no
// allocation happens while kernels run (the paper measures per-allocation
// overhead as the main cost of the default and halloc allocators, Sec. V.A).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstring>
#include <string>
#include <thread>

#include "wc_internal.h"
#include "wc_stats.h"

namespace wc {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

wc_status fail(wc_status st, const std::string &msg)
{
    set_error(msg);
    return st;
}

wc_status hip_fail(hipError_t e, const char *what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return WC_EHIP;
}

// A growth replaces the pool and drops the captured graphs (they hold pool
// addresses) without waiting: calls in flight on any stream keep the old ones,
// which are retired and released at the next drain of the device by the
// context (no device-wide synchronization that would stall other contexts'
// streams; the cost is the retired memory until then).
static void retire_graphs(wc_ctx *ctx)
{
    if (ctx->graph_exec) ctx->retired_graphs.push_back(ctx->graph_exec);
    ctx->graph_exec = nullptr;
    ctx->graph_key = 0;
    for (auto &tg : ctx->tree_graphs) {
        if (tg.exec) ctx->retired_graphs.push_back(tg.exec);
        tg = wc_ctx::TreeGraph{};
    }
}

// After the device has been drained: frees what growths retired.
static void release_retired(wc_ctx *ctx)
{
    for (char *p : ctx->retired_pools) (void)hipFree(p);
    ctx->retired_pools.clear();
    for (hipGraphExec_t g : ctx->retired_graphs) (void)hipGraphExecDestroy(g);
    ctx->retired_graphs.clear();
}

static wc_status pool_alloc(wc_ctx *ctx, size_t bytes)
{
    char *fresh = nullptr;
    hipError_t e = hipMalloc(&fresh, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(WC_ENOMEM, "cannot allocate a device pool of " + std::to_string(bytes) + " bytes");
    }
    if (ctx->pool) ctx->retired_pools.push_back(ctx->pool);
    ctx->pool = fresh;
    ctx->pool_bytes = bytes;
    return WC_OK;
}

wc_status pool_reserve(wc_ctx *ctx, size_t bytes, hipStream_t stream)
{
    if (ctx->plan_only) {
        ctx->planned = std::max(ctx->planned, bytes);
        return WC_PLANNED;
    }
    (void)stream;
    ctx->pool_off = 0;
    if (bytes <= ctx->pool_bytes) return WC_OK;
    ++ctx->pool_grows;
    // earlier calls may still be using the pool: it is retired, not freed
    const size_t grow = ctx->pool_bytes * 2;
    retire_graphs(ctx);
    return pool_alloc(ctx, bytes > grow ? bytes : grow);
}

void pool_reset(wc_ctx *ctx) { ctx->pool_off = 0; }

int resident_blocks_on(int num_cus, const void *kernel, int block)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    return per_cu * num_cus;
}

int resident_blocks(wc_ctx *ctx, const void *kernel, int block) { return resident_blocks_on(ctx->num_cus, kernel, block); }

static hipEvent_t take_event(wc_ctx *ctx)
{
    if (!ctx->spare_events.empty()) {
        hipEvent_t e = ctx->spare_events.back();
        ctx->spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static void recycle_records(wc_ctx *ctx)
{
    for (auto &r : ctx->records) {
        if (r.own_start) ctx->spare_events.push_back(r.start);
        ctx->spare_events.push_back(r.stop);
    }
    ctx->records.clear();
    chain_break(ctx);
}

wc_status launch(wc_ctx *ctx, const char *name, const void *kernel, dim3 grid, dim3 block, void **args,
                 hipStream_t stream)
{
    if (!ctx || !ctx->timing) {
        WC_HIP(hipLaunchKernel(kernel, grid, block, args, 0, stream));
        return WC_OK;
    }
    // one event per launch: a launch that directly follows a timed launch on
    // the same stream starts at that launch's stop event
    const bool chained = ctx->chain_event && ctx->chain_stream == stream;
    hipEvent_t a = chained ? ctx->chain_event : take_event(ctx);
    hipEvent_t b = take_event(ctx);
    if (!a || !b) return fail(WC_EHIP, "hipEventCreate failed");
    if (!chained) WC_HIP(hipEventRecord(a, stream));
    WC_HIP(hipLaunchKernel(kernel, grid, block, args, 0, stream));
    WC_HIP(hipEventRecord(b, stream));
    ctx->records.push_back({name, a, b, !chained});
    ctx->chain_event = b;
    ctx->chain_stream = stream;
    return WC_OK;
}

static int default_threshold(const char *problem, wc_mode mode)
{
    if (mode == WC_FLAT) return INT_MAX;
    if (!strcmp(problem, "tree")) return 0;  // every node with children is a recursive call (Fig. 1(c))
    // grid level drains with lane groups sized to each item, so only very short
    // items stay inline; so do the wave- and block-level children of SSSP and
    // SpMV (SpMV's rows go to lane groups; SSSP's edges are walked flattened).
    // Scale-22 graph, items_per_lane 2, threshold 8 / 16 / 32: SSSP wave 2.27 /
    // 2.36 / 2.46 ms, block 2.48 / 2.53 / 2.61 ms; SpMV wave 0.93 / 0.92 / 0.95 ms
    if (mode == WC_GRID && strcmp(problem, "color")) return 8;
    if (!strcmp(problem, "sssp") || !strcmp(problem, "spmv")) return 8;
    // coloring at block level: the block's child walks the concatenated
    // ranges, so short ranges gain from it (symmetric R-MAT scale 16 / 22,
    // chunks of 64: 12.4 / 96.6 ms at threshold 8, 16.1 / 106 ms at 32)
    if (!strcmp(problem, "color") && mode == WC_BLOCK) return 8;
    // coloring at grid level buffers every readied vertex's range; the
    // threshold applies to its count pass, where lanes walk up to 64 entries
    if (mode == WC_GRID) return 64;
    return 32;
}

wc_status resolve_tune(wc_ctx *ctx, const char *problem, wc_mode mode, const wc_tune *tune, int resident,
                       Config *out)
{
    (void)ctx;
    wc_tune t;
    wc_status st = wc_default_tune(problem, mode, resident, &t);
    if (st != WC_OK) return st;
    if (tune) {
        if (tune->threshold > 0 && mode != WC_FLAT && strcmp(problem, "tree")) t.threshold = tune->threshold;
        if (tune->block_threads > 0) t.block_threads = tune->block_threads;
        if (tune->grid_blocks > 0) t.grid_blocks = tune->grid_blocks;
        if (tune->items_per_lane > 0) t.items_per_lane = tune->items_per_lane;
        if (tune->driver > 0) t.driver = tune->driver;
        t.allow_fallback = tune->allow_fallback;
        if (tune->buf_capacity > 0) t.buf_capacity = tune->buf_capacity;
        t.buffer_alloc = tune->buffer_alloc;
    }
    int b = t.block_threads;
    if (b != 64 && b != 128 && b != 256 && b != 512 && b != 1024)
        return fail(WC_EINVAL, "block_threads must be one of 64, 128, 256, 512, 1024");
    if (t.items_per_lane > 64) return fail(WC_EINVAL, "items_per_lane must be at most 64");
    if (t.driver < 0 || t.driver > 3)
        return fail(WC_EINVAL,
                    "driver must be 0 (relaunch), 2 (basic; grid mode of SSSP, SpMV and trees) or "
                    "3 (1-1 mapping; SSSP grid only)");
    if (t.driver == 1)
        return fail(WC_EINVAL, "the persistent driver (driver = 1) is not available: use the relaunch driver");
    if (t.driver >= 2 && strcmp(problem, "sssp") &&
        !(t.driver == 2 && (!strcmp(problem, "spmv") || !strcmp(problem, "tree"))))
        return fail(WC_EINVAL, "driver 2 exists for SSSP, SpMV and trees, driver 3 for SSSP only");
    out->threshold = t.threshold;
    out->block = t.block_threads;
    out->grid = t.grid_blocks;
    out->items_per_lane = t.items_per_lane;
    out->driver = t.driver;
    out->fail_on_overflow = t.allow_fallback < 0;
    if (t.buffer_alloc < 0 || t.buffer_alloc > 2)
        return fail(WC_EINVAL, "buffer_alloc must be 0 (registers / LDS), 1 (pool) or 2 (device malloc)");
    if (t.buffer_alloc != 0 && strcmp(problem, "sssp"))
        return fail(WC_EINVAL, "buffer_alloc exists for SSSP only");
    out->buf_capacity = t.buf_capacity;
    out->buffer_alloc = t.buffer_alloc;
    return WC_OK;
}

// Clears the per-call device counters with a kernel rather than a memset node,
// so that a captured graph replays it correctly, and stores the call's epoch,
// which every later kernel of the call tags its host-ring values with.
__global__ void zero_stats(DevStats *s, unsigned int epoch)
{
    unsigned int *w = reinterpret_cast<unsigned int *>(s);
    for (unsigned i = threadIdx.x; i < sizeof(DevStats) / 4; i += blockDim.x) w[i] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) s->epoch = epoch;
}

// Publishes the timeout and overflow flags of the call to the host ring.
__global__ void publish_flags(DevStats *s, unsigned long long *ring)
{
    if (threadIdx.x == 0) publish_host(ring, kHostSlotFlags, s, (s->timed_out ? 1 : 0) | (s->overflowed ? 2 : 0));
}

wc_status begin_call(wc_ctx *ctx, hipStream_t stream, wc_stats *stats)
{
    if (stats) memset(stats, 0, sizeof(*stats));
    chain_break(ctx);  // other work may have been queued since the last call
    if (++ctx->epoch == 0) ctx->epoch = 1;
    void *args[] = {&ctx->dstats, &ctx->epoch};
    wc_status st = launch(ctx, "zero_stats", reinterpret_cast<const void *>(&zero_stats), dim3(1), dim3(64), args,
                          stream);
    if (st != WC_OK) return st;
    if (stats) {
        WC_HIP(hipEventRecord(ctx->ev_start, stream));
        chain_break(ctx);
    }
    return WC_OK;
}

wc_status end_call(wc_ctx *ctx, hipStream_t stream, wc_stats *stats, int rounds, bool fail_on_overflow,
                   bool bounded_waits)
{
    DevStats ds;
    chain_break(ctx);
    if (!stats && bounded_waits) {
        // the flags come back through the host ring once the call's kernels are done
        void *args[] = {&ctx->dstats, &ctx->host_ring_dev};
        clear_host_slot(ctx, kHostSlotFlags);
        wc_status st = launch(ctx, "publish_flags", reinterpret_cast<const void *>(&publish_flags), dim3(1),
                              dim3(64), args, stream);
        if (st != WC_OK) return st;
        int flags = 0;
        st = wait_host_slot(ctx, kHostSlotFlags, &flags);
        if (st != WC_OK) return st;
        chain_break(ctx);
        if (flags & 1) return fail(WC_ETIMEOUT, "a device-side wait exceeded its time limit");
        if (fail_on_overflow && (flags & 2))
            return fail(WC_EOVERFLOW, "a consolidation buffer overflowed (buf_capacity too small)");
        return WC_OK;
    }
    if (stats) {
        WC_HIP(hipEventRecord(ctx->ev_stop, stream));
        WC_HIP(hipMemcpyAsync(&ds, ctx->dstats, sizeof(ds), hipMemcpyDeviceToHost, stream));
        WC_HIP(hipStreamSynchronize(stream));
        float ms = 0.f;
        WC_HIP(hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop));
        stats->rounds = rounds;
        stats->overflowed = ds.overflowed;
        for (int r = 0; r < kStatReps; ++r) {
            stats->items_buffered += (int64_t)ds.rep[r].items_buffered;
            stats->dispatches += (int64_t)ds.rep[r].dispatches;
            stats->edges_processed += (int64_t)ds.rep[r].edges_processed;
            stats->edges_buffered += (int64_t)ds.rep[r].edges_buffered;
            stats->updates += (int64_t)ds.rep[r].updates;
            stats->updates_buffered += (int64_t)ds.rep[r].updates_buffered;
        }
        stats->ms = ms;
    } else if (fail_on_overflow) {
        WC_HIP(hipMemcpyAsync(&ds, ctx->dstats, sizeof(ds), hipMemcpyDeviceToHost, stream));
        WC_HIP(hipStreamSynchronize(stream));
    } else {
        WC_HIP(hipGetLastError());
        return WC_OK;
    }
    WC_HIP(hipGetLastError());
    if (ds.timed_out) return fail(WC_ETIMEOUT, "a device-side wait exceeded its time limit");
    if (fail_on_overflow && ds.overflowed)
        return fail(WC_EOVERFLOW, "a consolidation buffer overflowed (buf_capacity too small)");
    return WC_OK;
}

wc_status stage_to_device(wc_ctx *ctx, void *dst, const void *src, size_t bytes, hipStream_t stream)
{
    if (ctx->staging_pending) {
        WC_HIP(hipEventSynchronize(ctx->staging_done));
        ctx->staging_pending = false;
    }
    if (bytes > ctx->staging_bytes) {
        if (ctx->staging) WC_HIP(hipHostFree(ctx->staging));
        ctx->staging = nullptr;
        ctx->staging_bytes = 0;
        size_t sz = std::max<size_t>(bytes, 1 << 16);
        WC_HIP(hipHostMalloc(&ctx->staging, sz, hipHostMallocDefault));
        ctx->staging_bytes = sz;
    }
    std::memcpy(ctx->staging, src, bytes);
    chain_break(ctx);
    WC_HIP(hipMemcpyAsync(dst, ctx->staging, bytes, hipMemcpyHostToDevice, stream));
    WC_HIP(hipEventRecord(ctx->staging_done, stream));
    ctx->staging_pending = true;
    return WC_OK;
}

void clear_host_slot(wc_ctx *ctx, int index)
{
    reinterpret_cast<volatile unsigned long long *>(ctx->host_ring)[index] = 0ull;  // epoch 0 is never used
}

void clear_round_slot(wc_ctx *ctx, int r)
{
    clear_host_slot(ctx, r % kHostRing);
}

wc_status wait_round_count(wc_ctx *ctx, int r, int *count)
{
    return wait_host_slot(ctx, r % kHostRing, count);
}

wc_status wait_host_slot(wc_ctx *ctx, int index, int *count)
{
    volatile unsigned long long *slot = reinterpret_cast<volatile unsigned long long *>(ctx->host_ring) + index;
    auto t0 = std::chrono::steady_clock::now();
    long spins = 0;
    for (;;) {
        const unsigned long long v = *slot;  // one aligned 8-byte load: tag and value together
        if ((unsigned int)(v >> 32) == ctx->epoch) {
            *count = (int)(unsigned int)(v & 0xffffffffull);
            return WC_OK;
        }
        if (++spins > 2000) {
            std::this_thread::yield();
            if ((spins & 1023) == 0) {
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return hip_fail(e, "kernel launch while waiting for a round count");
                double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                if (s > 120.0) return fail(WC_ETIMEOUT, "round count never published (120 s)");
            }
        }
    }
}

}  // namespace wc

using namespace wc;

extern "C" {

const char *wc_last_error(void) { return g_last_error.c_str(); }

const char *wc_version(void) { return "wc 0.1 (gfx950)"; }

int64_t wc_per_buffer_size(int64_t total_thread, int64_t total_buff_var, int64_t items_per_thread)
{
    return total_thread * total_buff_var * items_per_thread;
}

void wc_kc_config(int64_t blocks, int64_t threads, int64_t x, int64_t *out_blocks, int64_t *out_threads)
{
    if (x < 1) x = 1;
    int64_t b = (blocks + x - 1) / x;
    *out_blocks = b < 1 ? 1 : b;
    *out_threads = threads;
}

wc_status wc_default_tune(const char *problem, wc_mode mode, int32_t resident_blocks, wc_tune *out)
{
    if (!problem || !out) return fail(WC_EINVAL, "NULL argument");
    if (strcmp(problem, "sssp") && strcmp(problem, "spmv") && strcmp(problem, "tree") && strcmp(problem, "color") &&
        strcmp(problem, "bfs"))
        return fail(WC_EINVAL, std::string("unknown problem ") + problem);
    if (mode < WC_FLAT || mode > WC_GRID) return fail(WC_EINVAL, "mode must be flat, wave, block or grid");
    out->threshold = default_threshold(problem, mode);
    // grid level: 512-thread workgroups measured fastest (scale-22 graph,
    // 2^22-node tree) except for coloring; everything else 256
    out->block_threads = mode == WC_GRID && strcmp(problem, "color") ? 512 : 256;
    // the packet queues of recursive BFS and the trees (one persistent grid):
    // larger workgroups measured faster, except for the trees at block level
    // (scale-22 graph, BFS at 256 / 512 / 1024 threads: wave 9.02 / 8.97 /
    // 8.50 ms, block 3.86 / 2.72 / 2.99 ms; 2^22-node random tree, descendants
    // at wave level 3.01 / 2.92 / 2.65 ms, the 39.3M-node layered tree 2.55 /
    // 2.39 / 2.15 ms; at block level 512 threads helped the descendants and
    // slowed the heights)
    if (!strcmp(problem, "bfs") && mode == WC_WAVE) out->block_threads = 1024;
    if (!strcmp(problem, "bfs") && mode == WC_BLOCK) out->block_threads = 512;
    if (!strcmp(problem, "tree") && mode == WC_WAVE) out->block_threads = 1024;
    // The drain grid of every mode is the resident maximum (KC_1 of Sec. IV.E):
    // wave- and block-level drains run inside the parent groups, which are
    // already resident, so no downgrade for concurrency is needed.
    out->grid_blocks = resident_blocks > 0 ? resident_blocks : 1;
    out->items_per_lane = 4;  // "const" of Sec. IV.E
    if (mode == WC_GRID && !strcmp(problem, "spmv")) out->items_per_lane = 8;
    // SSSP and SpMV in wave and block modes: items longer than one chunk of
    // 64 * items_per_lane go to the grid-wide drain, which balances them over
    // the whole device; a group's own child keeps the rest.  Chunks of 128
    // measured fastest (scale-22 graph, threshold 8, items_per_lane 1 / 2 / 4 /
    // 8: SSSP wave 2.26 / 2.27 / 3.13 / 4.51 ms; SpMV wave 1.01 / 0.93 / 1.37 /
    // 2.18 ms; block within 10% of wave)
    if ((mode == WC_WAVE || mode == WC_BLOCK) && (!strcmp(problem, "sssp") || !strcmp(problem, "spmv")))
        out->items_per_lane = 2;
    // SSSP grid chunks of 128 edges: 1.7% faster than 256 on the scale-22 graph
    // (4 x 20 calls each; the drain waves take two chunks per step); BFS's
    // frontier rounds at grid level are the same kernels
    if (mode == WC_GRID && (!strcmp(problem, "sssp") || !strcmp(problem, "bfs"))) out->items_per_lane = 2;
    // coloring rounds are short and bound by their dependent chain of loads and
    // atomics: 128-neighbour chunks in 256-thread groups measured fastest
    // (symmetric R-MAT graphs of scale 16 and 22)
    if (mode == WC_GRID && !strcmp(problem, "color")) out->items_per_lane = 2;
    // coloring in wave and block modes: ranges longer than one chunk go to the
    // grid-wide drain of the pass or round; chunks of 64 measured fastest
    // (symmetric R-MAT scale 16 / 22, wave at threshold 32: 20.5 / 114 ms at
    // 64, 30.3 / 154 ms at 256)
    if ((mode == WC_WAVE || mode == WC_BLOCK) && !strcmp(problem, "color")) out->items_per_lane = 1;
    // tree items are child ranges: most nodes have a few children, and shorter
    // chunks split the few wide nodes over more waves (measured on 2^22 nodes)
    if (mode == WC_GRID && !strcmp(problem, "tree")) out->items_per_lane = 2;
    // recursive BFS in wave and block modes (its packet queue): every packet
    // costs its consumer an acquire, so calls are cut and packets filled eight
    // times coarser (scale-22 graph, wave / block: 13.8 / 5.7 ms at 8, 10.4 /
    // 4.4 ms at 16, 8.9 / 3.8 ms at 32, 9.1 / 4.0 ms at 64)
    if ((mode == WC_WAVE || mode == WC_BLOCK) && !strcmp(problem, "bfs")) out->items_per_lane = 32;
    // with 1024-thread groups at wave level, packets twice as coarse again
    // (8.46 -> 8.13 ms; at block level 64 measured slower, 2.97 against 2.71 ms)
    if (mode == WC_WAVE && !strcmp(problem, "bfs")) out->items_per_lane = 64;
    // the trees' packet queue: packets of 64 x 32 (wave) or block x 32 (block)
    // children; against 4, the 2^22-node random tree's heights took 2.4 instead
    // of 2.9 ms (block) and the wide layered trees 0.24 / 2.5 instead of 0.49 /
    // 3.1 ms (block / wave); from 8 to 64 the times vary within about 30%
    if ((mode == WC_WAVE || mode == WC_BLOCK) && !strcmp(problem, "tree")) out->items_per_lane = 32;
    out->driver = 0;
    out->allow_fallback = 0;
    out->buf_capacity = 0;
    out->buffer_alloc = 0;
    out->reserved = 0;
    return WC_OK;
}

wc_status wc_ctx_create(int device, size_t pool_bytes, wc_ctx **out)
{
    if (!out) return fail(WC_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return fail(WC_EINVAL, "no such HIP device");
    }
    wc_ctx *ctx = new (std::nothrow) wc_ctx();
    if (!ctx) return fail(WC_ENOMEM, "host allocation failed");
    ctx->device = device;
    hipError_t e = hipSetDevice(device);
    hipDeviceProp_t prop;
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        delete ctx;
        return hip_fail(e, "hipGetDeviceProperties");
    }
    ctx->num_cus = prop.multiProcessorCount;
    ctx->max_threads_per_cu = prop.maxThreadsPerMultiProcessor;
    ctx->lds_per_block = prop.sharedMemPerBlock;
    wc_status st = pool_alloc(ctx, pool_bytes ? pool_bytes : (size_t(512) << 20));
    if (st == WC_OK) {
        e = hipHostMalloc(&ctx->host_ring, sizeof(unsigned long long) * kHostSlots,
                          hipHostMallocMapped | hipHostMallocCoherent);
        if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&ctx->host_ring_dev, ctx->host_ring, 0);
        if (e == hipSuccess) e = hipMalloc(&ctx->dstats, sizeof(DevStats));
        if (e == hipSuccess) e = hipEventCreate(&ctx->ev_start);
        if (e == hipSuccess) e = hipEventCreate(&ctx->ev_stop);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->staging_done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->graph_ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->graph_done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess) st = hip_fail(e, "context setup");
    }
    if (st != WC_OK) {
        wc_ctx_destroy(ctx);
        return st;
    }
    for (int i = 0; i < kHostSlots; ++i) ctx->host_ring[i] = 0ull;
    ctx->wait_ticks = kWaitTicks;
    *out = ctx;
    return WC_OK;
}

wc_status wc_ctx_set_timing(wc_ctx *ctx, int enable)
{
    if (!ctx) return fail(WC_EINVAL, "NULL context");
    WC_HIP(hipSetDevice(ctx->device));
    WC_HIP(hipDeviceSynchronize());
    recycle_records(ctx);
    release_retired(ctx);
    ctx->timing = enable ? 1 : 0;
    return WC_OK;
}

wc_status wc_ctx_set_plan_only(wc_ctx *ctx, int enable)
{
    if (!ctx) return fail(WC_EINVAL, "NULL context");
    ctx->plan_only = enable ? 1 : 0;
    ctx->planned = 0;
    return WC_OK;
}

wc_status wc_ctx_planned_bytes(wc_ctx *ctx, size_t *bytes)
{
    if (!ctx || !bytes) return fail(WC_EINVAL, "NULL argument");
    *bytes = ctx->planned;
    return WC_OK;
}

wc_status wc_ctx_pool_info(wc_ctx *ctx, size_t *pool_bytes, int64_t *grows)
{
    if (!ctx || !pool_bytes || !grows) return fail(WC_EINVAL, "NULL argument");
    *pool_bytes = ctx->pool_bytes;
    *grows = ctx->pool_grows;
    return WC_OK;
}

wc_status wc_ctx_reserve(wc_ctx *ctx, size_t bytes)
{
    if (!ctx) return fail(WC_EINVAL, "NULL context");
    if (bytes <= ctx->pool_bytes) return WC_OK;
    WC_HIP(hipSetDevice(ctx->device));
    ++ctx->pool_grows;
    retire_graphs(ctx);
    return pool_alloc(ctx, bytes);
}

wc_status wc_ctx_set_wait_limit(wc_ctx *ctx, int64_t microseconds)
{
    if (!ctx) return fail(WC_EINVAL, "NULL context");
    // the device clock of the bounded waits counts at 100 MHz
    ctx->wait_ticks = microseconds > 0 ? (unsigned long long)microseconds * 100ull : kWaitTicks;
    return WC_OK;
}

wc_status wc_ctx_kernel_stats(wc_ctx *ctx, int32_t index, const char **name, int64_t *launches, double *total_ms,
                              double *max_ms)
{
    if (!ctx || !name || !launches || !total_ms || !max_ms) return fail(WC_EINVAL, "NULL argument");
    // distinct names in first-launch order
    std::vector<const char *> names;
    for (auto &r : ctx->records) {
        bool seen = false;
        for (auto *nm : names) seen = seen || !strcmp(nm, r.name);
        if (!seen) names.push_back(r.name);
    }
    if (index < 0 || index >= (int32_t)names.size()) return fail(WC_EINVAL, "no kernel record with that index");
    WC_HIP(hipSetDevice(ctx->device));
    *name = names[index];
    *launches = 0;
    *total_ms = 0.0;
    *max_ms = 0.0;
    for (auto &r : ctx->records) {
        if (strcmp(r.name, names[index])) continue;
        WC_HIP(hipEventSynchronize(r.stop));
        float ms = 0.f;
        WC_HIP(hipEventElapsedTime(&ms, r.start, r.stop));
        *launches += 1;
        *total_ms += ms;
        if (ms > *max_ms) *max_ms = ms;
    }
    return WC_OK;
}

wc_status wc_ctx_kernel_record(wc_ctx *ctx, int32_t index, const char **name, double *ms)
{
    if (!ctx || !name || !ms) return fail(WC_EINVAL, "NULL argument");
    if (index < 0 || index >= (int32_t)ctx->records.size()) return fail(WC_EINVAL, "no record with that index");
    WC_HIP(hipSetDevice(ctx->device));
    const wc_kernel_record &r = ctx->records[index];
    WC_HIP(hipEventSynchronize(r.stop));
    float t = 0.f;
    WC_HIP(hipEventElapsedTime(&t, r.start, r.stop));
    *name = r.name;
    *ms = t;
    return WC_OK;
}

wc_status wc_ctx_destroy(wc_ctx *ctx)
{
    if (!ctx) return WC_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    recycle_records(ctx);
    for (auto e : ctx->spare_events) (void)hipEventDestroy(e);
    ctx->spare_events.clear();
    if (ctx->pool) (void)hipFree(ctx->pool);
    release_retired(ctx);
    if (ctx->host_ring) (void)hipHostFree(ctx->host_ring);
    if (ctx->dstats) (void)hipFree(ctx->dstats);
    if (ctx->ev_start) (void)hipEventDestroy(ctx->ev_start);
    if (ctx->ev_stop) (void)hipEventDestroy(ctx->ev_stop);
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    for (auto &tg : ctx->tree_graphs)
        if (tg.exec) (void)hipGraphExecDestroy(tg.exec);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    if (ctx->staging) (void)hipHostFree(ctx->staging);
    if (ctx->staging_done) (void)hipEventDestroy(ctx->staging_done);
    if (ctx->graph_ready) (void)hipEventDestroy(ctx->graph_ready);
    if (ctx->graph_done) (void)hipEventDestroy(ctx->graph_done);
    (void)hipGetLastError();
    delete ctx;
    return WC_OK;
}

}  // extern "C"
