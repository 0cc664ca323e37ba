// Host-side internals of libwc: context, pre-allocated pool, error reporting,
// device-published round counts, and the per-call stats block.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/wc.h"

namespace wc {

// Device counters accumulated by kernels when stats are requested.  Each
// workgroup adds its totals to one of kStatReps replicas (on separate cache
// lines) so the counting itself does not serialize on a few addresses; the
// host sums the replicas.
constexpr int kStatReps = 64;
struct StatRep {
    unsigned long long items_buffered;
    unsigned long long dispatches;
    unsigned long long edges_processed;
    unsigned long long edges_buffered;
    unsigned long long updates;
    unsigned long long updates_buffered;
    unsigned long long pad[10];
};
struct DevStats {
    StatRep rep[kStatReps];
    int overflowed;
    int timed_out;
    int rounds;
    unsigned int epoch;  // the call's epoch, written by its first kernel (zero_stats)
};

// Ring of values (round counts, flags) published by kernels to pinned host
// memory, so the host can stop relaunching rounds without a blocking copy per
// round.  Each entry is 64-bit: the call's epoch in the high half, the value in
// the low half.  A call waits only for entries carrying its own epoch, so a
// value left behind by an earlier call's trailing kernels (rounds enqueued past
// the last one with work) is never taken for one of this call.
constexpr int kHostRing = 256;
// host-ring entry after the round slots, written only by a graph's last kernel
constexpr int kHostSlotGraph = kHostRing;
// entry written by the last kernel of a call that has bounded device-side
// waits: bit 0 = a wait timed out, bit 1 = a buffer overflowed
constexpr int kHostSlotFlags = kHostRing + 1;
constexpr int kHostSlots = kHostRing + 2;

}  // namespace wc

struct wc_kernel_record {
    const char *name;
    hipEvent_t start, stop;
    bool own_start;  // false: start is the previous record's stop
};

struct wc_ctx {
    int device = 0;
    int num_cus = 0;
    int max_threads_per_cu = 0;
    size_t lds_per_block = 0;
    char *pool = nullptr;      // device pool (the pre-allocated allocator of Sec. IV.E)
    size_t pool_bytes = 0;
    size_t pool_off = 0;
    unsigned long long *host_ring = nullptr;  // pinned, device-visible; see kHostRing
    unsigned long long *host_ring_dev = nullptr;
    unsigned int epoch = 0;  // of the current call (begin_call advances it; never 0)
    // plan-only mode (wc_ctx_set_plan_only): calls record their workspace and
    // return WC_PLANNED before enqueueing anything
    int plan_only = 0;
    size_t planned = 0;
    long long pool_grows = 0;
    // pools and captured graphs replaced by a growth: calls still in flight on
    // any stream may use them, so they are released only where the context
    // drains the device anyway (wc_ctx_set_timing, wc_ctx_destroy)
    std::vector<char *> retired_pools;
    std::vector<hipGraphExec_t> retired_graphs;
    unsigned long long wait_ticks = 0;  // bound of every device-side wait, in 100 MHz ticks
    wc::DevStats *dstats = nullptr;  // device
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    // optional per-kernel timing: events recorded around every launch
    int timing = 0;
    std::vector<wc_kernel_record> records;
    std::vector<hipEvent_t> spare_events;
    // consecutive timed launches on one stream share an event (the stop of one
    // is the start of the next); any other stream work breaks the chain
    hipEvent_t chain_event = nullptr;
    hipStream_t chain_stream = nullptr;
    // pinned staging buffer for small host-to-device descriptor uploads
    void *staging = nullptr;
    size_t staging_bytes = 0;
    hipEvent_t staging_done = nullptr;
    bool staging_pending = false;
    // batched SSSP: capture stream and the last instantiated round graph
    hipStream_t capture_stream = nullptr;
    hipEvent_t graph_ready = nullptr, graph_done = nullptr;
    unsigned long long graph_key = 0;
    hipGraphExec_t graph_exec = nullptr;
    // level-synchronous trees: captured graphs of all levels, keyed by the call
    struct TreeGraph {
        unsigned long long key = 0;
        hipGraphExec_t exec = nullptr;
        int levels = 0;
    } tree_graphs[4];
    int tree_graph_next = 0;
};

namespace wc {

void set_error(const std::string &msg);
wc_status fail(wc_status st, const std::string &msg);
wc_status hip_fail(hipError_t e, const char *what);

#define WC_HIP(call)                                      \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return wc::hip_fail(e_, #call); \
    } while (0)

// Pool carving: reset at the start of each call, then take aligned slices.
// Grows the pool if a call needs more than it has (the old pool is retired,
// not freed: work in flight may still use it).
// In plan-only mode it records `bytes` and returns WC_PLANNED instead, which
// every caller passes straight up (nothing has been enqueued at that point).
wc_status pool_reserve(wc_ctx *ctx, size_t bytes, hipStream_t stream);
void pool_reset(wc_ctx *ctx);
template <typename T>
T *pool_take(wc_ctx *ctx, size_t count)
{
    size_t off = (ctx->pool_off + 255) & ~size_t(255);
    size_t bytes = count * sizeof(T);
    ctx->pool_off = off + bytes;
    return reinterpret_cast<T *>(ctx->pool + off);
}
inline size_t padded(size_t bytes) { return (bytes + 255) & ~size_t(255); }

// Resolved configuration of one call.
struct Config {
    int threshold;
    int block;
    int grid;
    int items_per_lane;
    int driver;
    bool fail_on_overflow;
    long long buf_capacity;
    int buffer_alloc;
};

int resident_blocks(wc_ctx *ctx, const void *kernel, int block);
// the same for a device with num_cus compute units (no context needed)
int resident_blocks_on(int num_cus, const void *kernel, int block);

// Every kernel launch of the library goes through here so that per-kernel
// timing (wc_ctx_set_timing) can bracket it with events on its stream.  A
// NULL context launches without timing (the entry points that take none).
wc_status launch(wc_ctx *ctx, const char *name, const void *kernel, dim3 grid, dim3 block, void **args,
                 hipStream_t stream);
wc_status resolve_tune(wc_ctx *ctx, const char *problem, wc_mode mode, const wc_tune *tune, int resident, Config *out);

// Call bracket: advances the call epoch, clears the device counters (and sets
// the epoch there for the kernels), records the start event.
wc_status begin_call(wc_ctx *ctx, hipStream_t stream, wc_stats *stats);
// Records the stop event; fills `stats` (synchronizing) when non-NULL; reports
// overflow / timeout flags.  A call whose kernels contain bounded waits passes
// bounded_waits = true: without `stats` the host then waits for a last kernel
// that publishes the flags, so a wait that gave up is reported as WC_ETIMEOUT
// whether or not stats were requested.
wc_status end_call(wc_ctx *ctx, hipStream_t stream, wc_stats *stats, int rounds, bool fail_on_overflow,
                   bool bounded_waits = false);

// Copies `bytes` from host memory to device memory `dst` on `stream` through
// the context's pinned staging buffer (waits for the previous staged copy).
wc_status stage_to_device(wc_ctx *ctx, void *dst, const void *src, size_t bytes, hipStream_t stream);

// Waits (bounded) until a kernel of the current call published the count of
// round `r` to the host ring.
inline void chain_break(wc_ctx *ctx) { ctx->chain_event = nullptr; }
wc_status wait_round_count(wc_ctx *ctx, int r, int *count);
// Clears the entry of round r before that round is launched: within one call
// the ring is reused every kHostRing rounds.
void clear_round_slot(wc_ctx *ctx, int r);
// the same for one host-ring entry by index (0 <= index < kHostSlots)
wc_status wait_host_slot(wc_ctx *ctx, int index, int *value);
void clear_host_slot(wc_ctx *ctx, int index);

// Recursive BFS in the wave and block modes (the recursion path); sets
// *overflowed (levels incomplete) when its call list was too small.
wc_status run_bfs_rec(wc_ctx *ctx, const wc_csr *g, int32_t src, uint32_t *level, wc_mode mode, const Config &cfg,
                      hipStream_t stream, wc_stats *stats, int *overflowed);


}  // namespace wc
