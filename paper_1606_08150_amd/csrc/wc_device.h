// Device primitives shared by the consolidation kernels (gfx950, wave64).
//
//  - wave_append: ballot + mbcnt prefix; one atomic per wavefront reserves the
//    slots of every lane that inserts (the buffer insertion of Fig. 4(b)).
//  - wave reductions in a fixed butterfly order (deterministic results).
//  - device-scope atomics with explicit memory scope.
//  - grid_barrier: the counter barrier of Sec. IV.E, made reusable with a
//    generation word so one persistent grid can cross it once per round.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wc {

constexpr int kWave = 64;
constexpr uint32_t kInf = 0xFFFFFFFFu;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of set bits of `mask` strictly below this lane.
__device__ __forceinline__ int rank_in(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int readlane(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ __forceinline__ uint32_t readlane_u(uint32_t v, int lane)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// ---- guarded loads ---------------------------------------------------------------------------
// arr[i] when ok, else zero, without a select between a global address and a
// local temporary (which the compiler would otherwise materialise on the stack).
__device__ __forceinline__ int4 load_or_zero(const int4 *arr, long long i, bool ok)
{
    int4 v = make_int4(0, 0, 0, 0);
    if (ok) v = arr[i];
    return v;
}

// ---- scoped atomics ---------------------------------------------------------------------------
__device__ __forceinline__ int atomic_add_dev(int *p, int v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long atomic_add_dev(unsigned long long *p, unsigned long long v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t atomic_min_dev(uint32_t *p, uint32_t v)
{
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// result unused: the wave does not wait for the atomic to return
__device__ __forceinline__ void atomic_min_dev_noret(uint32_t *p, uint32_t v)
{
    (void)__hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_max_dev_noret(uint32_t *p, uint32_t v)
{
    (void)__hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int atomic_max_dev(int *p, int v)
{
    return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int atomic_exch_dev(int *p, int v)
{
    return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int atomic_load_dev(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_system(int *p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ---- wave-aggregated append ---------------------------------------------------------------------
// Every active lane must call this (it issues a ballot).  Lanes with pred
// receive distinct consecutive slots starting at the value *tail had; the
// wave performs one atomic.  Returns the lane's slot, or -1 without pred.
__device__ __forceinline__ int wave_reserve(bool pred, int *tail)
{
    uint64_t mask = __ballot(pred);
    if (mask == 0) return -1;
    int leader = __builtin_ctzll(mask);
    int base = 0;
    if (lane_id() == leader) base = atomic_add_dev(tail, __builtin_popcountll(mask));
    base = readlane(base, leader);
    return pred ? base + rank_in(mask) : -1;
}

// Slot reservation of `count` (>= 0, per lane) consecutive entries.  Must be
// called with all 64 lanes active (non-participants pass 0).  Returns the
// lane's first slot (meaningless when count == 0).  One atomic per wave.
__device__ __forceinline__ int wave_reserve_n(int count, int *tail)
{
    int incl = count;
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int other = __shfl_up(incl, d, kWave);
        incl += lane >= d ? other : 0;
    }
    int total = readlane(incl, kWave - 1);
    int base = 0;
    if (total > 0 && lane == 0) base = atomic_add_dev(tail, total);
    base = readlane(base, 0);
    return base + incl - count;
}

// ---- fixed-order wave reductions ----------------------------------------------------------------
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}
__device__ __forceinline__ int wave_sum_i(int v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}
__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d, kWave));
    return v;
}

// ---- bounded waits --------------------------------------------------------------------------------
// Every device-side wait is bounded in wall-clock time (the 100 MHz constant
// clock read by wall_clock64), so a wait that can never end reports a timeout
// instead of holding the GPU.
constexpr unsigned long long kWaitTicks = 200000000ull;  // 2 s at 100 MHz

__device__ __forceinline__ unsigned long long wait_deadline() { return wall_clock64() + kWaitTicks; }
__device__ __forceinline__ bool past(unsigned long long deadline) { return wall_clock64() > deadline; }

// ---- grid barrier ---------------------------------------------------------------------------------
// Counter barrier of Sec. IV.E: the counter starts at the number of blocks and
// each block's first thread decrements it once; the block that takes it to zero
// is the last arrival.  To reuse it across rounds the last arrival resets the
// counter and bumps a generation word that the other blocks wait on.  Requires
// every block of the grid to be co-resident (cooperative launch).
struct GridBarrier {
    int count;
    int generation;
};

// Returns false if the wait passed its deadline (the grid then has to stop; the
// caller reports WC_ETIMEOUT).
__device__ __forceinline__ bool grid_barrier(GridBarrier *b, int nblocks)
{
    __syncthreads();
    bool ok = true;
    if (threadIdx.x == 0) {
        int gen = __hip_atomic_load(&b->generation, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // release this block's writes, then arrive
        int left = __hip_atomic_fetch_add(&b->count, -1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) - 1;
        if (left == 0) {
            __hip_atomic_store(&b->count, nblocks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&b->generation, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const unsigned long long deadline = wait_deadline();
            while (__hip_atomic_load(&b->generation, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(1);
                if (past(deadline)) {
                    ok = false;
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return ok;
}

}  // namespace wc
