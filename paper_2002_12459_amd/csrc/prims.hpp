// Device-wide primitives written for this library: grid loops, exclusive
// scan (reduce-then-scan, no inter-block waiting), stable LSD radix sort of
// 32/64-bit keys (per-tile digit counts, scan, wave-ballot ranked scatter
// staged through LDS) and stable stream compaction by wave ballots.
#pragma once

#include <algorithm>

#include "common.hpp"
#include "dev.hpp"

namespace jp {

// ---------------------------------------------------------------------------
// Grid-stride loop
// ---------------------------------------------------------------------------
template <class F>
__global__ __launch_bounds__(256) void k_for_each(int64_t n, F f) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) f(i);
}

template <class F>
void for_each(const Ctx &c, int64_t n, F f) {
    if (n <= 0) return;
    int64_t blocks = std::min<int64_t>(ceil_div(n, 256), (int64_t)c.num_cus * 32);
    hipLaunchKernelGGL(k_for_each<F>, dim3((unsigned)blocks), dim3(256), 0, c.stream, n, f);
    JP_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Exclusive scan of int64 values produced by get(i); put(i, prefix) receives
// the exclusive prefix of element i.  Tiles of 4096 elements: each wave scans
// 1024 consecutive elements in 16 coalesced rounds of 64.
// ---------------------------------------------------------------------------
constexpr int kTileItems = 16;
constexpr int kTileBlock = 256;
constexpr int64_t kTile = kTileItems * kTileBlock;

template <class G>
__global__ __launch_bounds__(kTileBlock) void k_scan_reduce(int64_t n, G get, int64_t *partial) {
    __shared__ int64_t lds[kTileBlock / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    int64_t s = 0;
#pragma unroll 4
    for (int j = 0; j < kTileItems; ++j) {
        int64_t i = base + (int64_t)j * kTileBlock + threadIdx.x;
        if (i < n) s += get(i);
    }
    int64_t tot = block_sum<kTileBlock>(s, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

template <class G, class P>
__global__ __launch_bounds__(kTileBlock) void k_scan_down(int64_t n, G get, const int64_t *partial_scan, P put) {
    __shared__ int64_t lds[kTileBlock / kWave + 1];
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int64_t wbase = (int64_t)blockIdx.x * kTile + (int64_t)w * kWave * kTileItems;
    int64_t v[kTileItems];
    int64_t wtot = 0;
#pragma unroll
    for (int j = 0; j < kTileItems; ++j) {
        int64_t i = wbase + (int64_t)j * kWave + lane;
        v[j] = i < n ? get(i) : 0;
        wtot += v[j];
    }
    wtot = wave_sum(wtot);
    // prefix of the wave totals inside the block
    int64_t dummy;
    int64_t contrib = (lane == 0) ? wtot : 0;
    int64_t wpre = block_excl_scan<kTileBlock>(contrib, lds, &dummy);
    wpre = __shfl(wpre, 0);
    int64_t carry = partial_scan[blockIdx.x] + wpre;
#pragma unroll
    for (int j = 0; j < kTileItems; ++j) {
        int64_t i = wbase + (int64_t)j * kWave + lane;
        int64_t inc = wave_incl_scan(v[j]);
        if (i < n) put(i, carry + inc - v[j]);
        carry += __shfl(inc, kWave - 1);
    }
}

struct ArrayGet {
    const int64_t *a;
    __device__ int64_t operator()(int64_t i) const { return a[i]; }
};
struct ArrayPut {
    int64_t *a;
    __device__ void operator()(int64_t i, int64_t v) const { a[i] = v; }
};

// Exclusive scan; if total_dev is given, the overall sum is stored there.
template <class G, class P>
void scan_exclusive(const Ctx &c, int64_t n, G get, P put, int64_t *total_dev = nullptr) {
    if (n <= 0) {
        if (total_dev) c.zero(total_dev, 1);
        return;
    }
    const int64_t nt = ceil_div(n, kTile);
    DBuf<int64_t> part = c.buf<int64_t>((size_t)nt + 1);
    hipLaunchKernelGGL((k_scan_reduce<G>), dim3((unsigned)nt), dim3(kTileBlock), 0, c.stream, n, get, part.get());
    JP_HIP(hipGetLastError());
    // scan the partials in place (recursively), sum into part[nt]
    DBuf<int64_t> part_scan = c.buf<int64_t>((size_t)nt + 1);
    if (nt == 1) {
        int64_t *ps = part_scan.get(), *p = part.get();
        for_each(c, 1, [=] __device__(int64_t) {
            ps[0] = 0;
            ps[1] = p[0];
        });
    } else {
        scan_exclusive(c, nt, ArrayGet{part.get()}, ArrayPut{part_scan.get()}, part_scan.get() + nt);
    }
    hipLaunchKernelGGL((k_scan_down<G, P>), dim3((unsigned)nt), dim3(kTileBlock), 0, c.stream, n, get,
                       (const int64_t *)part_scan.get(), put);
    JP_HIP(hipGetLastError());
    if (total_dev) JP_HIP(hipMemcpyAsync(total_dev, part_scan.get() + nt, sizeof(int64_t),
                                         hipMemcpyDeviceToDevice, c.stream));
}

// ---------------------------------------------------------------------------
// Sum of get(i) over [0,n) added into *out (device, 64-bit).
// ---------------------------------------------------------------------------
template <class G>
__global__ __launch_bounds__(256) void k_reduce_sum(int64_t n, G get, unsigned long long *out) {
    __shared__ int64_t lds[256 / kWave + 1];
    int64_t s = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) s += get(i);
    int64_t t = block_sum<256>(s, lds);
    if (threadIdx.x == 0 && t) atomicAdd(out, (unsigned long long)t);
}

template <class G>
void reduce_sum(const Ctx &c, int64_t n, G get, unsigned long long *out_dev) {
    c.zero(out_dev, 1);
    if (n <= 0) return;
    int64_t blocks = std::min<int64_t>(ceil_div(n, 256), (int64_t)c.num_cus * 8);
    hipLaunchKernelGGL((k_reduce_sum<G>), dim3((unsigned)blocks), dim3(256), 0, c.stream, n, get, out_dev);
    JP_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Stable compaction: for i in [0,n) with pred(i), emit(i, pos) with pos the
// rank of i among selected elements.  Ballot + mbcnt inside each wave, block
// prefix of wave counts, tile prefix from a scan of per-tile counts.
// ---------------------------------------------------------------------------
template <class Pr>
__global__ __launch_bounds__(kTileBlock) void k_compact_count(int64_t n, Pr pred, int64_t *partial) {
    __shared__ int64_t lds[kTileBlock / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    int64_t s = 0;
    for (int j = 0; j < kTileItems; ++j) {
        int64_t i = base + (int64_t)j * kTileBlock + threadIdx.x;
        if (i < n && pred(i)) ++s;
    }
    int64_t tot = block_sum<kTileBlock>(s, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

template <class Pr, class Em>
__global__ __launch_bounds__(kTileBlock) void k_compact_write(int64_t n, Pr pred, Em emit, const int64_t *partial_scan) {
    __shared__ int64_t lds[kTileBlock / kWave + 1];
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int64_t wbase = (int64_t)blockIdx.x * kTile + (int64_t)w * kWave * kTileItems;
    uint32_t flags = 0;
    int64_t wcnt = 0;
    for (int j = 0; j < kTileItems; ++j) {
        int64_t i = wbase + (int64_t)j * kWave + lane;
        bool f = i < n && pred(i);
        flags |= (uint32_t)f << j;
        wcnt += __popcll(ballot(f));
    }
    int64_t dummy;
    int64_t wpre = block_excl_scan<kTileBlock>(lane == 0 ? wcnt : (int64_t)0, lds, &dummy);
    wpre = __shfl(wpre, 0);
    int64_t pos = partial_scan[blockIdx.x] + wpre;
    for (int j = 0; j < kTileItems; ++j) {
        int64_t i = wbase + (int64_t)j * kWave + lane;
        bool f = (flags >> j) & 1u;
        uint64_t m = ballot(f);
        if (f) emit(i, pos + mbcnt(m));
        pos += __popcll(m);
    }
}

// Returns the number of selected elements in *count_dev (device scalar).
template <class Pr, class Em>
void compact(const Ctx &c, int64_t n, Pr pred, Em emit, int64_t *count_dev) {
    if (n <= 0) {
        c.zero(count_dev, 1);
        return;
    }
    const int64_t nt = ceil_div(n, kTile);
    DBuf<int64_t> part = c.buf<int64_t>((size_t)nt);
    DBuf<int64_t> part_scan = c.buf<int64_t>((size_t)nt);
    hipLaunchKernelGGL((k_compact_count<Pr>), dim3((unsigned)nt), dim3(kTileBlock), 0, c.stream, n, pred, part.get());
    JP_HIP(hipGetLastError());
    scan_exclusive(c, nt, ArrayGet{part.get()}, ArrayPut{part_scan.get()}, count_dev);
    hipLaunchKernelGGL((k_compact_write<Pr, Em>), dim3((unsigned)nt), dim3(kTileBlock), 0, c.stream, n, pred, emit,
                       (const int64_t *)part_scan.get());
    JP_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// LSD radix sort (keys only), 8-bit digits.
// ---------------------------------------------------------------------------
constexpr int kRsBlock = 256;
constexpr int kRsItems = 16;
constexpr int64_t kRsTile = kRsBlock * kRsItems;

// Per-tile digit counts, digit-major: counts[d * ntiles + tile].  Keys are
// read coalesced (each wave takes 64 consecutive keys per step); lanes of a
// wave holding the same digit are matched by ballots and their leader adds
// the group size to the wave's private histogram, so skewed digits cost no
// atomic contention.
template <class K>
__global__ __launch_bounds__(kRsBlock) void k_rs_hist(const K *keys, int64_t n, int shift, uint32_t *counts,
                                                      int64_t ntiles) {
    constexpr int W = kRsBlock / kWave;
    __shared__ uint32_t h[W][256];
    for (int d = threadIdx.x; d < 256; d += kRsBlock)
#pragma unroll
        for (int q = 0; q < W; ++q) h[q][d] = 0;
    __syncthreads();
    const int64_t tile = blockIdx.x;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int64_t wbase = tile * kRsTile + (int64_t)w * kWave * kRsItems;
    K k[kRsItems];
#pragma unroll
    for (int j = 0; j < kRsItems; ++j) {
        const int64_t i = wbase + (int64_t)j * kWave + lane;
        k[j] = i < n ? keys[i] : K(0);
    }
#pragma unroll
    for (int j = 0; j < kRsItems; ++j) {
        const int64_t i = wbase + (int64_t)j * kWave + lane;
        const bool valid = i < n;
        const uint32_t d = (uint32_t)(k[j] >> shift) & 255u;
        const uint64_t peers = match_digit<8>(d, ballot(valid));
        const int leader = peers ? (int)(__ffsll((unsigned long long)peers) - 1) : 0;
        if (valid && lane == leader) h[w][d] += (uint32_t)__popcll(peers);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < 256; d += kRsBlock) {
        uint32_t t = 0;
#pragma unroll
        for (int q = 0; q < W; ++q) t += h[q][d];
        counts[(int64_t)d * ntiles + tile] = t;
    }
}

template <class K>
__global__ __launch_bounds__(kRsBlock) void k_rs_scatter(const K *in, K *out, int64_t n, int shift,
                                                         const int64_t *offs, int64_t ntiles) {
    constexpr int W = kRsBlock / kWave;
    __shared__ K tk[kRsTile];
    __shared__ uint32_t wcnt[W][256];
    __shared__ uint32_t bstart[256];
    __shared__ uint32_t dcount[256];
    __shared__ int64_t goff[256];
    __shared__ uint32_t lds_scan[W + 1];
    const int64_t tile = blockIdx.x;
    const int64_t tbase = tile * kRsTile;
    const int w = threadIdx.x / kWave, lane = lane_id();
    for (int d = threadIdx.x; d < 256; d += kRsBlock) {
        for (int q = 0; q < W; ++q) wcnt[q][d] = 0;
        goff[d] = offs[(int64_t)d * ntiles + tile];
    }
    __syncthreads();
    K k[kRsItems];
    uint32_t rank[kRsItems];
    const int64_t wbase = tbase + (int64_t)w * kWave * kRsItems;
#pragma unroll
    for (int j = 0; j < kRsItems; ++j) {
        int64_t i = wbase + (int64_t)j * kWave + lane;
        bool valid = i < n;
        k[j] = valid ? in[i] : K(0);
        uint32_t d = (uint32_t)(k[j] >> shift) & 255u;
        uint64_t act = ballot(valid);
        uint64_t peers = match_digit<8>(d, act);
        int leader = peers ? (int)(__ffsll((unsigned long long)peers) - 1) : 0;
        uint32_t before = 0;
        if (valid && lane == leader) {
            before = wcnt[w][d];
            wcnt[w][d] = before + (uint32_t)__popcll(peers);
        }
        before = __shfl(before, leader);
        rank[j] = before + mbcnt(peers);
    }
    __syncthreads();
    // digit totals -> per-wave exclusive prefix and block start of each digit
    uint32_t tot = 0;
    if (threadIdx.x < 256) {
        const int d = threadIdx.x;
        for (int q = 0; q < W; ++q) {
            uint32_t t = wcnt[q][d];
            wcnt[q][d] = tot;
            tot += t;
        }
    }
    uint32_t all;
    uint32_t st = block_excl_scan<kRsBlock>(threadIdx.x < 256 ? tot : 0u, lds_scan, &all);
    if (threadIdx.x < 256) {
        bstart[threadIdx.x] = st;
        dcount[threadIdx.x] = tot;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kRsItems; ++j) {
        int64_t i = wbase + (int64_t)j * kWave + lane;
        if (i < n) {
            uint32_t d = (uint32_t)(k[j] >> shift) & 255u;
            tk[bstart[d] + wcnt[w][d] + rank[j]] = k[j];
        }
    }
    __syncthreads();
    const int64_t tile_n = std::min<int64_t>(kRsTile, n - tbase);
    for (int p = threadIdx.x; p < tile_n; p += kRsBlock) {
        K key = tk[p];
        uint32_t d = (uint32_t)(key >> shift) & 255u;
        const uint32_t q = (uint32_t)p - bstart[d];
        if (q < dcount[d]) out[goff[d] + q] = key;  // stays inside digit d's range
    }
}

// Sorts n keys on their low `bits` bits.  Uses `keys` and `tmp` as ping-pong
// buffers and returns the one holding the result.
template <class K>
K *radix_sort(const Ctx &c, K *keys, K *tmp, int64_t n, int bits) {
    if (n <= 1 || bits <= 0) return keys;
    const int passes = (bits + 7) / 8;
    const int64_t nt = ceil_div(n, kRsTile);
    DBuf<uint32_t> counts = c.buf<uint32_t>((size_t)(256 * nt));
    DBuf<int64_t> offs = c.buf<int64_t>((size_t)(256 * nt));
    K *src = keys, *dst = tmp;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL((k_rs_hist<K>), dim3((unsigned)nt), dim3(kRsBlock), 0, c.stream, (const K *)src, n, shift,
                           counts.get(), nt);
        JP_HIP(hipGetLastError());
        const uint32_t *cp = counts.get();
        scan_exclusive(
            c, 256 * nt, [=] __device__(int64_t i) -> int64_t { return (int64_t)cp[i]; }, ArrayPut{offs.get()});
        hipLaunchKernelGGL((k_rs_scatter<K>), dim3((unsigned)nt), dim3(kRsBlock), 0, c.stream, (const K *)src, dst, n,
                           shift, (const int64_t *)offs.get(), nt);
        JP_HIP(hipGetLastError());
        std::swap(src, dst);
    }
    return src;
}

}  // namespace jp
