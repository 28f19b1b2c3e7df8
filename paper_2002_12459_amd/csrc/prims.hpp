// Device-wide primitives written for this library: grid loops, exclusive
// scan and stable stream compaction (one pass each, decoupled look-back
// between tiles), and stable LSD radix sort of 32/64-bit keys (per-tile digit
// counts, scan, wave-ballot ranked scatter staged through LDS).
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
    // one element per thread (loads of different elements overlap), grid-stride beyond 2^26 threads
    int64_t blocks = std::min<int64_t>(ceil_div(n, 256), 1ll << 18);
    hipLaunchKernelGGL(k_for_each<F>, dim3(grid_x(blocks, 256)), dim3(256), 0, c.stream, n, f);
    JP_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Exclusive scan of int64 values produced by get(i); put(i, prefix) receives
// the exclusive prefix of element i.  One pass with decoupled look-back:
// tile t = blockIdx.x holds 256 threads x IT elements (each wave scans 64*IT
// consecutive elements in IT coalesced rounds of 64), publishes its sum, and
// the first wave of each tile sums its predecessors' published values, 64 at
// a time, back to the nearest tile whose inclusive prefix is already known.
//
// Nothing orders the start of workgroups, so a predecessor may not be running
// yet.  A waiting lane gives up after `wait` ticks of the constant-rate device
// clock, and the wave then computes that predecessor's sum itself from the
// input (the summands are pure functions of the index).  Every wait therefore
// ends under any schedule.  With in-order dispatch the fallback is not taken
// in practice; tests force it with wait = 0.  (An ordered ticket per tile
// would also guarantee progress, but its device-scope atomics are serialised,
// about 11 ns each on MI355X: 31 us of a 10M-element pass.)
// ---------------------------------------------------------------------------
constexpr int kTileBlock = 256;
constexpr int kScanItems = 16;
constexpr int64_t kScanTile = (int64_t)kScanItems * kTileBlock;

// status word of a tile: (value << 2) | flag, flag 1 = tile sum, 2 = inclusive prefix
__device__ __forceinline__ void lb_publish(uint64_t *status, int64_t t, int64_t v, uint64_t flag) {
    __hip_atomic_store(status + t, ((uint64_t)v << 2) | flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix of tile t >= 1, computed by one whole wave (all lanes get
// it).  agg(tile) returns a tile's sum to every lane of the wave (whole-wave
// call).
template <class Agg>
__device__ __forceinline__ int64_t lb_lookback(uint64_t *status, int64_t t, int64_t wait, Agg agg) {
    const int lane = lane_id();
    int64_t excl = 0;
    const int64_t start = wall_clock64();
    for (int64_t top = t - 1;; top -= kWave) {
        const int64_t idx = top - lane;
        uint64_t s = 2;  // before tile 0: inclusive prefix 0
        if (idx >= 0) {
            s = __hip_atomic_load(status + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            while ((s & 3u) == 0 && wall_clock64() - start < wait) {
                __builtin_amdgcn_s_sleep(1);
                s = __hip_atomic_load(status + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        for (uint64_t missing = ballot((s & 3u) == 0); missing; missing &= missing - 1) {
            const int l = (int)__ffsll((unsigned long long)missing) - 1;
            const int64_t a = agg(top - l);
            if (lane == l) s = ((uint64_t)a << 2) | 1u;
        }
        const uint64_t inc = ballot((s & 3u) == 2);
        const int stop = inc ? (int)(__ffsll((unsigned long long)inc) - 1) : kWave;
        excl += wave_sum(lane <= stop ? ((int64_t)s >> 2) : (int64_t)0);
        if (inc) break;
    }
    return excl;
}

// Wave 0 resolves the exclusive prefix of tile t from its sum A; returns it
// to all threads.
template <class Agg>
__device__ __forceinline__ int64_t lb_resolve(uint64_t *status, int64_t t, int64_t A, int64_t *sh, int64_t *total,
                                              int64_t ntiles, int64_t wait, Agg agg) {
    if (threadIdx.x < kWave) {
        int64_t excl = 0;
        if (status) {
            if (t == 0) {
                if (threadIdx.x == 0) lb_publish(status, 0, A, 2);
            } else {
                if (threadIdx.x == 0) lb_publish(status, t, A, 1);
                excl = lb_lookback(status, t, wait, agg);
                if (threadIdx.x == 0) lb_publish(status, t, excl + A, 2);
            }
        }
        if (threadIdx.x == 0) {
            *sh = excl;
            if (total && t == ntiles - 1) *total = excl + A;
        }
    }
    __syncthreads();
    return *sh;
}

// A scan element: the summand and a value passed through to put().
template <class V>
struct Sum {
    int64_t add;
    V v;
};
__device__ __forceinline__ int64_t sum_add(int64_t a) { return a; }
template <class V>
__device__ __forceinline__ int64_t sum_add(const Sum<V> &a) { return a.add; }

template <int IT, class G, class P>
__global__ __launch_bounds__(kTileBlock) void k_scan_lb(int64_t n, G get, P put, uint64_t *status, int64_t wait,
                                                        int64_t *total) {
    using R = decltype(get((int64_t)0));
    constexpr int64_t TILE = (int64_t)IT * kTileBlock;
    __shared__ int64_t lds[kTileBlock / kWave + 1];
    __shared__ int64_t sh_excl;
    const int64_t t = blockIdx.x;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int64_t wbase = t * TILE + (int64_t)w * kWave * IT;
    int64_t v[IT];
    R r[IT];
    int64_t wtot = 0;
    // get() on a clamped index for every item, so all loads are in flight at once
#pragma unroll
    for (int j = 0; j < IT; ++j) {
        const int64_t i = wbase + (int64_t)j * kWave + lane;
        r[j] = get(i < n ? i : n - 1);
        v[j] = i < n ? sum_add(r[j]) : 0;
    }
#pragma unroll
    for (int j = 0; j < IT; ++j) wtot += v[j];
    wtot = wave_sum(wtot);
    int64_t A;
    int64_t wpre = block_excl_scan<kTileBlock>(lane == 0 ? wtot : (int64_t)0, lds, &A);
    wpre = wave_lane(wpre, 0);
    auto agg = [&](int64_t tile) {
        const int64_t b = tile * TILE, e = std::min<int64_t>(n, b + TILE);
        int64_t a = 0;
        for (int64_t i = b + lane; i < e; i += kWave) a += sum_add(get(i));
        return wave_sum(a);
    };
    int64_t carry = lb_resolve(status, t, A, &sh_excl, total, gridDim.x, wait, agg) + wpre;
#pragma unroll
    for (int j = 0; j < IT; ++j) {
        int64_t i = wbase + (int64_t)j * kWave + lane;
        int64_t inc = wave_incl_scan(v[j]);
        if (i < n) put(i, carry + inc - v[j], r[j]);
        carry += wave_lane(inc, kWave - 1);
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

// Adapts put(i, prefix) to the kernel's put(i, prefix, value).
template <class P>
struct PutNoValue {
    P put;
    template <class R>
    __device__ void operator()(int64_t i, int64_t pre, const R &) const { put(i, pre); }
};

// Cleared tile status words for a look-back pass over nt tiles (none needed
// for a single tile): a piece of the handle's cleared pool, or a buffer of
// its own when the pass needs more than the pool holds.
struct LookbackState {
    DBuf<uint64_t> buf;
    uint64_t *status = nullptr;
    LookbackState(const Ctx &c, int64_t nt) {
        (void)grid_x(nt, kTileBlock);
        if (nt <= 1) return;
        status = c.take_status((size_t)nt);
        if (!status) {
            buf = c.buf<uint64_t>((size_t)nt);
            c.zero(buf.get(), (size_t)nt);
            status = buf.get();
        }
    }
};

// Exclusive scan where put(i, prefix, value) also receives get(i) (an
// int64 summand, or a Sum<V> whose add is summed), so it needs no loads of
// its own; if total_dev is given, the overall sum is stored there.
template <class G, class P>
void scan_exclusive_v(const Ctx &c, int64_t n, G get, P put, int64_t *total_dev = nullptr) {
    if (n <= 0) {
        if (total_dev) c.zero(total_dev, 1);
        return;
    }
    const int64_t nt = ceil_div(n, kScanTile);
    LookbackState lb(c, nt);
    hipLaunchKernelGGL((k_scan_lb<kScanItems, G, P>), dim3(grid_x(nt, kTileBlock)), dim3(kTileBlock), 0, c.stream, n, get,
                       put, lb.status, c.lookback_wait, total_dev);
    JP_HIP(hipGetLastError());
}

// Exclusive scan, put(i, prefix).
template <class G, class P>
void scan_exclusive(const Ctx &c, int64_t n, G get, P put, int64_t *total_dev = nullptr) {
    scan_exclusive_v(c, n, get, PutNoValue<P>{put}, total_dev);
}

// ---------------------------------------------------------------------------
// Sum of get(i) over [0,n) stored at *out (device, 64-bit).  Each workgroup
// writes its partial sum and one workgroup adds them up: device-scope
// atomics on one address are serialised (about 11 ns each), so thousands of
// workgroups adding into one word would cost tens of microseconds.
// ---------------------------------------------------------------------------
template <class G>
__global__ __launch_bounds__(256) void k_reduce_sum(int64_t n, G get, int64_t *part) {
    __shared__ int64_t lds[256 / kWave + 1];
    int64_t s = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) s += get(i);
    const int64_t t = block_sum<256>(s, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <int BLOCK>  // (a template, so that every translation unit may define it)
__global__ __launch_bounds__(BLOCK) void k_reduce_parts(const int64_t *part, int64_t np, unsigned long long *out) {
    __shared__ int64_t lds[BLOCK / kWave + 1];
    int64_t s = 0;
    for (int64_t i = threadIdx.x; i < np; i += BLOCK) s += part[i];
    const int64_t t = block_sum<BLOCK>(s, lds);
    if (threadIdx.x == 0) *out = (unsigned long long)t;
}

template <class G>
void reduce_sum(const Ctx &c, int64_t n, G get, unsigned long long *out_dev) {
    if (n <= 0) {
        c.zero(out_dev, 1);
        return;
    }
    const int64_t blocks = std::min<int64_t>(ceil_div(n, 256), (int64_t)c.num_cus * 8);
    DBuf<int64_t> part = c.buf<int64_t>((size_t)blocks);
    hipLaunchKernelGGL((k_reduce_sum<G>), dim3(grid_x(blocks, 256)), dim3(256), 0, c.stream, n, get, part.get());
    JP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_parts<256>, dim3(1), dim3(256), 0, c.stream, (const int64_t *)part.get(), blocks, out_dev);
    JP_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Stable compaction: sel(i) returns {keep, value} for i in [0,n); every kept
// i gets emit(i, pos, value) with pos its rank among the kept elements.  One
// pass: ballot + mbcnt inside each wave, block prefix of wave counts, tile
// prefix by decoupled look-back.  sel() runs for all items of a thread before
// any emit, so its loads overlap; emit() should only store.  Tiles and the
// look-back are those of the scan above.
// ---------------------------------------------------------------------------
constexpr int kCompactItems = 16;
constexpr int64_t kCompactTile = (int64_t)kCompactItems * kTileBlock;

template <class V>
struct Pick {
    bool keep;
    V v;
};

template <int IT, class Sel, class Em>
__global__ __launch_bounds__(kTileBlock) void k_compact_lb(int64_t n, Sel sel, Em emit, uint64_t *status, int64_t wait,
                                                           int64_t *count) {
    using V = decltype(sel((int64_t)0).v);
    static_assert(IT <= 64, "at most 64 items per thread");
    constexpr int64_t TILE = (int64_t)IT * kTileBlock;
    __shared__ int64_t lds[kTileBlock / kWave + 1];
    __shared__ int64_t sh_excl;
    const int64_t t = blockIdx.x;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int64_t wbase = t * TILE + (int64_t)w * kWave * IT;
    uint64_t flags = 0;
    int64_t wcnt = 0;
    // sel() on a clamped index for every item, so all loads are in flight at once
    bool fs[IT];
    V vals[IT];
#pragma unroll
    for (int j = 0; j < IT; ++j) {
        const int64_t i = wbase + (int64_t)j * kWave + lane;
        const Pick<V> pk = sel(i < n ? i : n - 1);
        fs[j] = pk.keep;
        vals[j] = pk.v;
    }
#pragma unroll
    for (int j = 0; j < IT; ++j) {
        const int64_t i = wbase + (int64_t)j * kWave + lane;
        const bool f = (i < n) & fs[j];
        flags |= (uint64_t)f << j;
        wcnt += __popcll(ballot(f));
    }
    int64_t A;
    int64_t wpre = block_excl_scan<kTileBlock>(lane == 0 ? wcnt : (int64_t)0, lds, &A);
    wpre = wave_lane(wpre, 0);
    auto agg = [&](int64_t tile) {
        const int64_t b = tile * TILE, e = std::min<int64_t>(n, b + TILE);
        int64_t a = 0;
        for (int64_t i = b + lane; i < e; i += kWave) a += sel(i).keep ? 1 : 0;
        return wave_sum(a);
    };
    int64_t pos = lb_resolve(status, t, A, &sh_excl, count, gridDim.x, wait, agg) + wpre;
#pragma unroll
    for (int j = 0; j < IT; ++j) {
        int64_t i = wbase + (int64_t)j * kWave + lane;
        bool f = (flags >> j) & 1u;
        uint64_t m = ballot(f);
        if (f) emit(i, pos + mbcnt(m), vals[j]);
        pos += __popcll(m);
    }
}

// Compaction with values (see k_compact_lb); the number of kept elements
// goes to *count_dev (device scalar).
template <class Sel, class Em>
void compact_v(const Ctx &c, int64_t n, Sel sel, Em emit, int64_t *count_dev) {
    if (n <= 0) {
        c.zero(count_dev, 1);
        return;
    }
    const int64_t nt = ceil_div(n, kCompactTile);
    LookbackState lb(c, nt);
    hipLaunchKernelGGL((k_compact_lb<kCompactItems, Sel, Em>), dim3(grid_x(nt, kTileBlock)), dim3(kTileBlock), 0, c.stream, n,
                       sel, emit, lb.status, c.lookback_wait, count_dev);
    JP_HIP(hipGetLastError());
}

template <class Pr>
struct PredPick {
    Pr pred;
    __device__ Pick<char> operator()(int64_t i) const { return Pick<char>{(bool)pred(i), 0}; }
};
template <class Em>
struct EmitNoValue {
    Em emit;
    __device__ void operator()(int64_t i, int64_t p, char) const { emit(i, p); }
};

// Compaction with a predicate: emit(i, pos) for every i with pred(i).
template <class Pr, class Em>
void compact(const Ctx &c, int64_t n, Pr pred, Em emit, int64_t *count_dev) {
    compact_v(c, n, PredPick<Pr>{pred}, EmitNoValue<Em>{emit}, count_dev);
}

// ---------------------------------------------------------------------------
// LSD radix sort (keys only), 8-bit digits.
// ---------------------------------------------------------------------------
constexpr int kRsBlock = 256;
constexpr int kRsItems = 16;
constexpr int64_t kRsTile = kRsBlock * kRsItems;

// Where a pass reads its keys: an array, or (first pass only) a function of
// the index that builds each key from the caller's columns.
template <class K>
struct KeyArray {
    const K *p;
    __device__ K operator()(int64_t i) const { return p[i]; }
};

// Workgroups are dealt to the 8 XCDs round-robin by block index.  The radix
// kernels give XCD r (blocks b with b % 8 == r) the r-th eighth of the tiles,
// a contiguous run: the digit-major count and offset tables hold the entries
// of consecutive tiles in one cache line, and with the run on one XCD that
// line is written and read through one L2 instead of up to eight.  Grids are
// padded to a multiple of 8; a padding block returns -1.
__device__ __forceinline__ int64_t rs_tile(int64_t b, int64_t ntiles) {
    const int64_t per = (ntiles + 7) / 8;
    const int64_t t = (b & 7) * per + (b >> 3);
    return t < ntiles ? t : -1;
}
inline int64_t rs_grid(int64_t ntiles) { return 8 * ((ntiles + 7) / 8); }

// Per-tile digit counts, digit-major: counts[d * ntiles + tile].  Keys are
// read coalesced (each wave takes 64 consecutive keys per step) and counted
// with LDS atomic adds into kRsHistCopies copies of the histogram, lane l
// adding to copy l % kRsHistCopies (copies padded by one word so that equal
// digits of different copies fall in different banks).  Lanes of one
// instruction that hit the same counter are serialised by the LDS; the copies
// divide that cost for skewed digits (a Zipf-distributed id's low byte).
constexpr int kRsHistCopies = 8;
template <class K, class Src>
__global__ __launch_bounds__(kRsBlock) void k_rs_hist(Src keys, int64_t n, int shift, uint32_t *counts,
                                                      int64_t ntiles) {
    static_assert(kRsBlock == 256, "one digit per thread in the final sum");
    constexpr int kStride = 257;
    __shared__ uint32_t h[kRsHistCopies * kStride];
    const int64_t tile = rs_tile(blockIdx.x, ntiles);
    if (tile < 0) return;  // grid padding (uniform per workgroup)
    for (int i = threadIdx.x; i < kRsHistCopies * kStride; i += kRsBlock) h[i] = 0;
    __syncthreads();
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int64_t wbase = tile * kRsTile + (int64_t)w * kWave * kRsItems;
    uint32_t *mine = h + (lane % kRsHistCopies) * kStride;
    K k[kRsItems];
#pragma unroll
    for (int j = 0; j < kRsItems; ++j) {
        const int64_t i = wbase + (int64_t)j * kWave + lane;
        k[j] = keys(i < n ? i : n - 1);
    }
#pragma unroll
    for (int j = 0; j < kRsItems; ++j) {
        const int64_t i = wbase + (int64_t)j * kWave + lane;
        if (i < n) atomicAdd(&mine[(uint32_t)(k[j] >> shift) & 255u], 1u);
    }
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int q = 0; q < kRsHistCopies; ++q) t += h[q * kStride + threadIdx.x];
    counts[(int64_t)threadIdx.x * ntiles + tile] = t;
}

// Stable scatter of one tile: ranks within the tile by wave ballots (lanes
// with the same digit matched bit by bit, the group leader bumps the wave's
// digit counter), keys staged in LDS in digit order, then written out in
// digit runs.  Four workgroups fit a CU for keys of up to 8 bytes (under
// 40 KB of LDS and at most 128 VGPRs); 16-byte keys need twice the LDS.
template <class K, class Src>
__global__ __launch_bounds__(kRsBlock, sizeof(K) <= 8 ? 4 : 2) void k_rs_scatter(Src in, K *out, int64_t n, int shift,
                                                            const int64_t *offs, int64_t ntiles) {
    constexpr int W = kRsBlock / kWave;
    __shared__ K tk[kRsTile];
    __shared__ uint32_t wcnt[W][256];
    __shared__ uint32_t bstart[257];  // start of each digit's run in the tile, bstart[256] = tile size
    __shared__ int64_t goff[256];
    __shared__ uint32_t lds_scan[W + 1];
    const int64_t tile = rs_tile(blockIdx.x, ntiles);
    if (tile < 0) return;  // grid padding (uniform per workgroup)
    const int64_t tbase = tile * kRsTile;
    const int w = threadIdx.x / kWave, lane = lane_id();
    K k[kRsItems];
    uint32_t rank[kRsItems];
    const int64_t wbase = tbase + (int64_t)w * kWave * kRsItems;
    // the tile's keys and its 256 digit offsets (one cache line each: the
    // offsets are digit-major) are all in flight before the first wait
#pragma unroll
    for (int j = 0; j < kRsItems; ++j) {
        const int64_t i = wbase + (int64_t)j * kWave + lane;
        k[j] = in(i < n ? i : n - 1);
    }
    for (int d = threadIdx.x; d < 256; d += kRsBlock) {
        for (int q = 0; q < W; ++q) wcnt[q][d] = 0;
        goff[d] = offs[(int64_t)d * ntiles + tile];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kRsItems; ++j) {
        int64_t i = wbase + (int64_t)j * kWave + lane;
        bool valid = i < n;
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
    if (threadIdx.x < 256) bstart[threadIdx.x] = st;
    if (threadIdx.x == 0) bstart[256] = all;
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
        if (q < bstart[d + 1] - bstart[d]) out[goff[d] + q] = key;  // stays inside digit d's range
    }
}

// One stable pass on the digit at `shift`: keys from src into dst.
template <class K, class Src>
void radix_pass(const Ctx &c, Src src, K *dst, int64_t n, int shift, uint32_t *counts, int64_t *offs, int64_t nt) {
    hipLaunchKernelGGL((k_rs_hist<K, Src>), dim3(grid_x(rs_grid(nt), kRsBlock)), dim3(kRsBlock), 0, c.stream, src, n,
                       shift, counts, nt);
    JP_HIP(hipGetLastError());
    const uint32_t *cp = counts;
    scan_exclusive(
        c, 256 * nt, [=] __device__(int64_t i) -> int64_t { return (int64_t)cp[i]; }, ArrayPut{offs});
    hipLaunchKernelGGL((k_rs_scatter<K, Src>), dim3(grid_x(rs_grid(nt), kRsBlock)), dim3(kRsBlock), 0, c.stream, src, dst,
                       n, shift, (const int64_t *)offs, nt);
    JP_HIP(hipGetLastError());
}

// Sorts the n keys key0(i), i in [0, n), on their low `bits` bits, with `a`
// and `b` (n keys each) as ping-pong buffers; returns the one holding the
// result.  The first pass reads the keys through key0, so they are never
// stored unsorted.
template <class K, class F>
K *radix_sort_from(const Ctx &c, F key0, K *a, K *b, int64_t n, int bits) {
    if (n <= 0) return a;
    if (n == 1 || bits <= 0) {
        for_each(c, n, [=] __device__(int64_t i) { a[i] = key0(i); });
        return a;
    }
    const int passes = (bits + 7) / 8;
    const int64_t nt = ceil_div(n, kRsTile);
    DBuf<uint32_t> counts = c.buf<uint32_t>((size_t)(256 * nt));
    DBuf<int64_t> offs = c.buf<int64_t>((size_t)(256 * nt));
    radix_pass<K>(c, key0, a, n, 0, counts.get(), offs.get(), nt);
    K *src = a, *dst = b;
    for (int p = 1; p < passes; ++p) {
        radix_pass<K>(c, KeyArray<K>{src}, dst, n, 8 * p, counts.get(), offs.get(), nt);
        std::swap(src, dst);
    }
    return src;
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
        radix_pass<K>(c, KeyArray<K>{src}, dst, n, 8 * p, counts.get(), offs.get(), nt);
        std::swap(src, dst);
    }
    return src;
}

}  // namespace jp
