// Device-side building blocks for gfx950 (wave64): lane masks, wave and block
// scans, wave-level digit matching, binary search.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace jp {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of set bits of `m` in lanes below the calling lane.
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Exclusive scan over the threads of a block of BLOCK threads.  `lds` needs
// BLOCK/64 + 1 elements.  *total receives the block sum.  Every thread adds
// up the wave totals itself (BLOCK/64 LDS reads), so the scan takes two
// barriers: one before the reads, one before `lds` may be written again.
template <int BLOCK, class T>
__device__ __forceinline__ T block_excl_scan(T v, T *lds, T *total) {
    constexpr int W = BLOCK / kWave;
    const T inc = wave_incl_scan(v);
    const int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) lds[w] = inc;
    __syncthreads();
    T pre = 0, all = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        const T t = lds[i];
        pre += i < w ? t : T(0);
        all += t;
    }
    *total = all;
    __syncthreads();
    return inc - v + pre;
}

template <int BLOCK, class T>
__device__ __forceinline__ T block_sum(T v, T *lds) {
    T tot;
    (void)block_excl_scan<BLOCK>(v, lds, &tot);
    return tot;
}

// Lanes (among `active`) holding the same BITS-bit digit as the calling lane.
template <int BITS>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t active) {
    uint64_t peers = active;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

// First index i in [lo, hi) with a[i] >= key (hi if none).
template <class T, class I>
__device__ __forceinline__ I lower_bound_dev(const T *a, I lo, I hi, T key) {
    while (lo < hi) {
        I mid = lo + (hi - lo) / 2;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Last index i in [lo, hi) with a[i] <= key, for sorted a with a[lo] <= key.
template <class T, class I>
__device__ __forceinline__ I upper_bound_dev(const T *a, I lo, I hi, T key) {
    while (lo < hi) {
        I mid = lo + (hi - lo) / 2;
        if (a[mid] <= key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

}  // namespace jp
