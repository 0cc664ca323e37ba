// Device primitives shared by the consolidation kernels (gfx950, wave64).
//
//  - wave_append: ballot + mbcnt prefix; one atomic per wavefront reserves the
//    slots of every lane that inserts (the buffer insertion of Fig. 4(b)).
//  - wave reductions in a fixed butterfly order (deterministic results).
//  - device-scope atomics with explicit memory scope.
//  - wall-clock deadlines for the bounded device-side waits.
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
// One wave runs in lockstep; the fence keeps the compiler from moving the
// wave's LDS accesses across this point.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
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

// ---- summation with a bounded rounding depth -------------------------------------------------------
// A running fp32 sum of N terms rounds the first term N times, so its error
// bound grows with N (N * 2^-24 of the magnitude sum).  Cascade keeps four
// partial sums: terms go into s0; after every 32 terms s0 is added into s1 and
// restarted, after every 32 * 32 terms s1 into s2, after every 32^3 terms s2
// into s3; the total is s3 + (s2 + (s1 + s0)).  A term is then rounded at most
// 32 times in each of the first three levels, ceil(N / 32768) times in s3 and
// 3 times in the final combination: at most 99 + ceil(N / 32768) roundings
// (131 for N <= 2^20) instead of N.  The order is fixed, so sums are bitwise
// reproducible.  Callers either add one term at a time (add) or fuse U terms
// into s0 themselves and then call step<U>() (U divides 32).
struct Cascade {
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    unsigned int steps = 0;

    template <int U>
    __device__ __forceinline__ void step()
    {
        static_assert(U >= 1 && 32 % U == 0, "U must divide 32");
        ++steps;
        if ((steps & (32u / U - 1u)) == 0u) {
            s1 += s0;
            s0 = 0.f;
            if ((steps & (1024u / U - 1u)) == 0u) {
                s2 += s1;
                s1 = 0.f;
                if ((steps & (32768u / U - 1u)) == 0u) {
                    s3 += s2;
                    s2 = 0.f;
                }
            }
        }
    }
    __device__ __forceinline__ void add(float x)
    {
        s0 += x;
        step<1>();
    }
    __device__ __forceinline__ float total() const { return s3 + (s2 + (s1 + s0)); }
};

// ---- bounded waits --------------------------------------------------------------------------------
// Every device-side wait is bounded in wall-clock time (the 100 MHz constant
// clock read by wall_clock64), so a wait that can never end reports a timeout
// instead of holding the GPU.  The bound is the context's (default 2 s).
constexpr unsigned long long kWaitTicks = 200000000ull;  // 2 s at 100 MHz

__device__ __forceinline__ unsigned long long wait_deadline(unsigned long long ticks) { return wall_clock64() + ticks; }
__device__ __forceinline__ bool past(unsigned long long deadline) { return wall_clock64() > deadline; }

}  // namespace wc
