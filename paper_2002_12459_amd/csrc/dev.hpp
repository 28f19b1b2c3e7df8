// Device-side building blocks for gfx950 (wave64): lane masks, wave and block
// scans, wave-level digit matching, binary search.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace jp {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of set bits of `m` in lanes below the calling lane.
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// x + (x moved by the DPP control CTRL in the rows of ROWS), 64-bit: both
// halves moved, then one 64-bit add.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_add64(uint64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, ROWS, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, ROWS, 0xf, false);
    return x + (((uint64_t)hi << 32) | lo);
}

// Inclusive scan over the 64 lanes of a wave.  32-bit values use DPP:
// shifts by 1, 2, 4 and 8 lanes within each row of 16 (lanes with no
// source add 0), then lane 15's total added to rows 1 and 3 (row_bcast:15)
// and lane 31's to rows 2 and 3 (row_bcast:31); VALU only.  64-bit values
// take the same steps on both halves with a 64-bit add.
template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    static_assert(std::is_integral<T>::value && (sizeof(T) == 4 || sizeof(T) == 8), "32- or 64-bit integers");
    if constexpr (sizeof(T) == 4) {
        int x = (int)v;
        x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
        x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
        x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
        x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
        x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
        x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
        return (T)x;
    } else {
        uint64_t x = (uint64_t)v;
        x = dpp_add64<0x111, 0xf>(x);  // row_shr:1
        x = dpp_add64<0x112, 0xf>(x);  // row_shr:2
        x = dpp_add64<0x114, 0xf>(x);  // row_shr:4
        x = dpp_add64<0x118, 0xf>(x);  // row_shr:8
        x = dpp_add64<0x142, 0xa>(x);  // row_bcast:15 into rows 1, 3
        x = dpp_add64<0x143, 0xc>(x);  // row_bcast:31 into rows 2, 3
        return (T)x;
    }
}

// Value of lane `lane` (the same for the whole wave) to every lane, by
// v_readlane (no LDS crossbar).  The wave must be converged.
template <class T>
__device__ __forceinline__ T wave_lane(T v, int lane) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
    if constexpr (sizeof(T) == 4) {
        return (T)__builtin_amdgcn_readlane((int)v, lane);
    } else {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, lane);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), lane);
        return (T)(((uint64_t)hi << 32) | lo);
    }
}

// Sum over the wave, in every lane (the last lane of the inclusive scan).
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
    return wave_lane(wave_incl_scan(v), kWave - 1);
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
