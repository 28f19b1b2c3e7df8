// Duplicate removal of the light witnesses, per x (Section 6,
// "Deduplication": for a fixed x, gather every reachable z, then either sort
// the gathered values or mark them in a dense vector, whichever suits the
// count and the domain).
//
// The witnesses of x are its light list entries (one list per R tuple of x,
// see two_path.hip) plus the heavy product's nonzeros in row x.  Outputs with
// different x never collide, so x values are processed independently:
//
//  * small x (<= kUnitCap candidates) are packed, in x order, into units of
//    at most kSegCap candidates.  A unit gathers its candidates as 32-bit keys
//    (x - first_x) << bz | z straight into registers, sorts them with an LDS
//    radix sort over the significant bits only, and keeps the first of every
//    run of equal keys (wave ballot + block scan).
//  * large x get a workgroup with an LDS bitmap over a window of the z
//    domain; candidates set bits, set bits are read back in z order.
//
// Each unit writes its distinct keys to a staging array at its candidate
// offset; a scan of the per-unit counts gives output offsets; a final
// load-balanced pass unranks (x, z) into the sorted output columns.
#include "debug.hpp"
#include "pipeline.hpp"
#include "prims.hpp"
#include "segdedup.hpp"

namespace jp {
namespace {

constexpr int kSegThreads = 512;
constexpr int kSegItems = 16;
constexpr int kSegCap = kSegThreads * kSegItems;  // keys per unit (LDS: 32 KB)
constexpr int64_t kUnitCap = kSegCap / 2;          // larger x go to the bitmap kernel
constexpr int kBmWords = 16384;                    // 64 KB bitmap = 524288 z values per window
constexpr int64_t kBmBits = (int64_t)kBmWords * 32;

struct UnitArgs {
    const int32_t *ustart;   // first x of every unit; ustart[n_units] = dom_x
    const int32_t *ids;      // unit ids this launch handles
    const int64_t *toff;     // candidate offset of every x (dom_x + 1)
    const int64_t *off_x;    // R tuples of x (dom_x + 1)
    const int64_t *eoff;     // light candidate offset of every R tuple (n_e + 1)
    const int64_t *lbase;    // list start of every R tuple in zlist
    const int32_t *r_xr;     // x of every R tuple
    const int32_t *zlist;
    const uint64_t *hkeys;   // heavy nonzeros (x << bz | z), sorted
    const int64_t *hoff;     // heavy nonzeros of every x (dom_x + 1)
    int bz;
    uint32_t zmask;
    int64_t dom_z;
    uint32_t *stage;         // distinct keys, at toff[first x] + i
    int64_t *ucount;         // distinct count of every unit
    int64_t *err;
};

__device__ __forceinline__ int bits_dev(uint32_t v) { return v ? 32 - __clz(v) : 0; }

__global__ __launch_bounds__(kSegThreads) void k_unit_sort(UnitArgs a) {
    constexpr int W = kSegThreads / kWave;
    __shared__ uint32_t sk[kSegCap];
    __shared__ uint32_t wcnt[W][256];
    __shared__ uint32_t bstart[256];
    __shared__ uint32_t lds_scan[W + 1];

    const int u = a.ids[blockIdx.x];
    const int32_t xa = a.ustart[u], xb = a.ustart[u + 1];
    const int64_t e0 = a.off_x[xa], e1 = a.off_x[xb];
    const int64_t c0 = a.eoff[e0];
    const int64_t nL = a.eoff[e1] - c0;
    const int64_t h0 = a.hoff[xa];
    const int64_t nH = a.hoff[xb] - h0;
    const int64_t n = nL + nH;
    if (n > kSegCap) {
        if (threadIdx.x == 0) *a.err = 1;
        return;
    }
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int wbase = w * kWave * kSegItems;

    // gather: light candidates [0, nL), heavy [nL, n)
    uint32_t k[kSegItems];
#pragma unroll
    for (int j = 0; j < kSegItems; ++j) {
        const int p = wbase + j * kWave + lane;
        uint32_t key = 0xffffffffu;
        if (p < nL) {
            const int64_t q = c0 + p;
            const int64_t e = upper_bound_dev(a.eoff, e0, e1, q) - 1;
            const uint32_t z = (uint32_t)a.zlist[a.lbase[e] + (q - a.eoff[e])];
            key = ((uint32_t)(a.r_xr[e] - xa) << a.bz) | z;
        } else if (p < n) {
            const uint64_t hk = a.hkeys[h0 + (p - nL)];
            key = ((uint32_t)((int64_t)(hk >> a.bz) - xa) << a.bz) | ((uint32_t)hk & a.zmask);
        }
        k[j] = key;
    }

    // LSD radix sort over the significant bits
    const int B = max(1, bits_dev((uint32_t)(xb - xa - 1)) + a.bz);
    const int P = (B + 7) / 8;
    const int dbits = P ? (B + P - 1) / P : 0;
    const uint32_t dmask = (1u << dbits) - 1u;
    for (int pass = 0; pass < P; ++pass) {
        const int shift = pass * dbits;
        for (int d = threadIdx.x; d < 256; d += kSegThreads)
#pragma unroll
            for (int q = 0; q < W; ++q) wcnt[q][d] = 0;
        __syncthreads();
        uint32_t rank[kSegItems];
#pragma unroll
        for (int j = 0; j < kSegItems; ++j) {
            const int p = wbase + j * kWave + lane;
            const bool valid = p < n;
            const uint32_t d = (k[j] >> shift) & dmask;
            const uint64_t peers = match_digit<8>(d, ballot(valid));
            const int leader = peers ? (int)(__ffsll((unsigned long long)peers) - 1) : 0;
            uint32_t before = 0;
            if (valid && lane == leader) {
                before = wcnt[w][d];
                wcnt[w][d] = before + (uint32_t)__popcll(peers);
            }
            before = __shfl(before, leader);
            rank[j] = before + mbcnt(peers);
        }
        __syncthreads();
        uint32_t tot = 0;
        if (threadIdx.x < 256) {
            const int d = threadIdx.x;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const uint32_t t = wcnt[q][d];
                wcnt[q][d] = tot;
                tot += t;
            }
        }
        uint32_t all;
        const uint32_t st = block_excl_scan<kSegThreads>(threadIdx.x < 256 ? tot : 0u, lds_scan, &all);
        if (threadIdx.x < 256) bstart[threadIdx.x] = st;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSegItems; ++j) {
            const int p = wbase + j * kWave + lane;
            if (p < n) {
                const uint32_t d = (k[j] >> shift) & dmask;
                const uint32_t dst = bstart[d] + wcnt[w][d] + rank[j];
                sk[dst < (uint32_t)kSegCap ? dst : 0] = k[j];
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSegItems; ++j) {
            const int p = wbase + j * kWave + lane;
            k[j] = p < n ? sk[p] : 0xffffffffu;
        }
        __syncthreads();
    }

    // keep the first of every run; write in order
    uint32_t flags = 0;
    uint32_t mine = 0;
    uint32_t carry = (wbase > 0 && wbase - 1 < n) ? sk[wbase - 1] : 0u;  // key before this wave's first
#pragma unroll
    for (int j = 0; j < kSegItems; ++j) {
        const int p = wbase + j * kWave + lane;
        const uint32_t up = __shfl_up(k[j], 1);
        const uint32_t prev = lane == 0 ? carry : up;
        const bool f = (p < n) & ((p == 0) | (k[j] != prev));
        flags |= (uint32_t)f << j;
        mine += f ? 1u : 0u;
        carry = __shfl(k[j], kWave - 1);
    }
    const uint32_t wtot = wave_sum(mine);
    uint32_t all;
    uint32_t wpre = block_excl_scan<kSegThreads>(lane == 0 ? wtot : 0u, lds_scan, &all);
    wpre = __shfl(wpre, 0);
    uint32_t pos = wpre;
    uint32_t *out = a.stage + a.toff[xa];
#pragma unroll
    for (int j = 0; j < kSegItems; ++j) {
        const bool f = (flags >> j) & 1u;
        const uint64_t m = ballot(f);
        if (f) out[pos + mbcnt(m)] = k[j];
        pos += (uint32_t)__popcll(m);
    }
    if (threadIdx.x == 0) a.ucount[u] = all;
}

// One workgroup per large x: LDS bitmap over z windows of kBmBits values.
__global__ __launch_bounds__(kSegThreads) void k_big_x(UnitArgs a) {
    __shared__ uint32_t bm[kBmWords];
    __shared__ uint32_t lds_scan[kSegThreads / kWave + 1];
    const int u = a.ids[blockIdx.x];
    const int32_t x = a.ustart[u];
    const int64_t e0 = a.off_x[x], e1 = a.off_x[x + 1];
    const int64_t c0 = a.eoff[e0];
    const int64_t nL = a.eoff[e1] - c0;
    const int64_t h0 = a.hoff[x];
    const int64_t nH = a.hoff[x + 1] - h0;
    uint32_t *out = a.stage + a.toff[x];
    constexpr int per = kBmWords / kSegThreads;  // words owned by each thread
    uint32_t written = 0;
    for (int64_t zb0 = 0; zb0 < a.dom_z; zb0 += kBmBits) {
        for (int i = threadIdx.x; i < kBmWords; i += kSegThreads) bm[i] = 0;
        __syncthreads();
        for (int64_t p = threadIdx.x; p < nL; p += kSegThreads) {
            const int64_t q = c0 + p;
            const int64_t e = upper_bound_dev(a.eoff, e0, e1, q) - 1;
            const int64_t zr = (int64_t)a.zlist[a.lbase[e] + (q - a.eoff[e])] - zb0;
            if (zr >= 0 && zr < kBmBits) atomicOr(&bm[zr >> 5], 1u << (zr & 31));
        }
        for (int64_t p = threadIdx.x; p < nH; p += kSegThreads) {
            const int64_t zr = (int64_t)((uint32_t)a.hkeys[h0 + p] & a.zmask) - zb0;
            if (zr >= 0 && zr < kBmBits) atomicOr(&bm[zr >> 5], 1u << (zr & 31));
        }
        __syncthreads();
        uint32_t cnt = 0;
#pragma unroll 8
        for (int i = 0; i < per; ++i) cnt += __popc(bm[threadIdx.x * per + i]);
        uint32_t tot;
        uint32_t pos = written + block_excl_scan<kSegThreads>(cnt, lds_scan, &tot);
        for (int i = 0; i < per; ++i) {
            uint32_t word = bm[threadIdx.x * per + i];
            const uint32_t zbase = (uint32_t)zb0 + (uint32_t)(threadIdx.x * per + i) * 32u;
            while (word) {
                const int b = __ffs(word) - 1;
                out[pos++] = zbase + (uint32_t)b;
                word &= word - 1;
            }
        }
        written += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) a.ucount[u] = written;
}

struct EmitArgs {
    const int64_t *uoff;    // output offset of every unit (n_units + 1)
    int64_t n_units, n_out;
    const int32_t *ustart;
    const int64_t *toff;
    const uint32_t *stage;
    const int32_t *xorig, *zorig;
    int bz;
    uint32_t zmask;
    int64_t dom_x, dom_z;
    int32_t *out_x, *out_z;
    int64_t *err;
};

constexpr int kEmitBlock = 256, kEmitItems = 16;
__global__ __launch_bounds__(kEmitBlock) void k_emit(EmitArgs a) {
    const int64_t o0 = (int64_t)blockIdx.x * kEmitBlock * kEmitItems;
    const int64_t olast = std::min<int64_t>(o0 + kEmitBlock * kEmitItems, a.n_out) - 1;
    const int64_t lo = upper_bound_dev(a.uoff, (int64_t)0, a.n_units, o0) - 1;
    const int64_t hi = upper_bound_dev(a.uoff, lo, a.n_units, olast);
    for (int j = 0; j < kEmitItems; ++j) {
        const int64_t o = o0 + (int64_t)j * kEmitBlock + threadIdx.x;
        if (o <= olast) {
            const int64_t u = upper_bound_dev(a.uoff, lo, hi, o) - 1;
            const int32_t xa = a.ustart[u];
            const uint32_t key = a.stage[a.toff[xa] + (o - a.uoff[u])];
            const int64_t xi = (int64_t)xa + (int64_t)(key >> a.bz);
            const int64_t zi = (int64_t)(key & a.zmask);
            const bool ok = (xi < a.dom_x) & (zi < a.dom_z);
            if (!ok) *a.err = 1;
            a.out_x[o] = a.xorig[ok ? xi : 0];
            a.out_z[o] = a.zorig[ok ? zi : 0];
        }
    }
}

}  // namespace

bool segmented_dedup_fits(int bz) { return bz <= 26; }

void segmented_dedup(const Ctx &c, const SegDedupIn &in, DBuf<int32_t> *out_x, DBuf<int32_t> *out_z,
                     int64_t *n_out, SegDedupStats *stats) {
    JP_CHECK(segmented_dedup_fits(in.bz), JP_EINTERNAL, "segmented dedup needs bz <= 26");
    const int64_t dom_x = in.dom_x;
    DBuf<int64_t> scal = c.buf<int64_t>(8);
    int64_t *S = scal.get();
    c.zero(S, 8);

    // heavy nonzeros per x
    DBuf<int64_t> hoff_own;
    const int64_t *hoff;
    hoff_own = c.buf<int64_t>(dom_x + 1);
    {
        int64_t *ho = hoff_own.get();
        const uint64_t *hk = in.hkeys;
        const int64_t nnz = in.nnz;
        const int bz = in.bz;
        if (nnz > 0) {
            for_each(c, dom_x + 1, [=] __device__(int64_t x) {
                ho[x] = lower_bound_dev(hk, (int64_t)0, nnz, (uint64_t)x << bz);
            });
        } else {
            c.zero(ho, dom_x + 1);
        }
        hoff = ho;
    }
    // candidates per x and their offsets
    DBuf<int64_t> toff = c.buf<int64_t>(dom_x + 1);
    {
        const int64_t *ox = in.off_x, *eo = in.eoff;
        auto tx = [=] __device__(int64_t x) -> int64_t {
            return (eo[ox[x + 1]] - eo[ox[x]]) + (hoff[x + 1] - hoff[x]);
        };
        int64_t *to = toff.get();
        scan_exclusive(c, dom_x, tx, ArrayPut{to}, to + dom_x);
    }
    // units: runs of small x inside one kUnitCap window of candidate offsets
    // (and one 2^(32-bz) block of x, so local keys fit 32 bits); large x alone
    const int kb = 32 - in.bz;
    DBuf<int32_t> ustart = c.buf<int32_t>(dom_x + 1);
    {
        const int64_t *to = toff.get();
        int32_t *us = ustart.get();
        auto big = [=] __device__(int64_t x) -> bool { return to[x + 1] - to[x] > kUnitCap; };
        compact(
            c, dom_x,
            [=] __device__(int64_t x) {
                if (x == 0) return true;
                const bool b0 = big(x), b1 = big(x - 1);
                const bool win = (to[x] / kUnitCap) != (to[x - 1] / kUnitCap);
                const bool blk = kb < 31 ? ((x >> kb) != ((x - 1) >> kb)) : false;
                return (bool)(b0 | b1 | win | blk);
            },
            [=] __device__(int64_t x, int64_t p) { us[p] = (int32_t)x; }, S + 0);
    }
    const int64_t n_units = c.load(S + 0);
    {
        int32_t *us = ustart.get();
        const int64_t nu = n_units, dx = dom_x;
        for_each(c, 1, [=] __device__(int64_t) { us[nu] = (int32_t)dx; });
    }
    DBuf<int32_t> small_ids = c.buf<int32_t>(n_units), big_ids = c.buf<int32_t>(n_units);
    {
        const int64_t *to = toff.get();
        const int32_t *us = ustart.get();
        int32_t *si = small_ids.get(), *bi = big_ids.get();
        auto isbig = [=] __device__(int64_t u) -> bool {
            const int32_t x = us[u];
            return to[x + 1] - to[x] > kUnitCap;
        };
        compact(
            c, n_units, [=] __device__(int64_t u) { return !isbig(u); },
            [=] __device__(int64_t u, int64_t p) { si[p] = (int32_t)u; }, S + 1);
        compact(c, n_units, isbig, [=] __device__(int64_t u, int64_t p) { bi[p] = (int32_t)u; }, S + 2);
    }
    int64_t h3[3];
    c.load_n(h3, S + 1, 2);
    const int64_t n_small = h3[0], n_big = h3[1];
    const int64_t n_cand = c.load(toff.get() + dom_x);

    DBuf<uint32_t> stage = c.buf<uint32_t>(std::max<int64_t>(n_cand, 1));
    DBuf<int64_t> ucount = c.buf<int64_t>(n_units + 1);
    UnitArgs ua;
    ua.ustart = ustart.get();
    ua.toff = toff.get();
    ua.off_x = in.off_x;
    ua.eoff = in.eoff;
    ua.lbase = in.lbase;
    ua.r_xr = in.r_xr;
    ua.zlist = in.zlist;
    ua.hkeys = in.hkeys;
    ua.hoff = hoff;
    ua.bz = in.bz;
    ua.zmask = (uint32_t)((1ull << in.bz) - 1);
    ua.dom_z = in.dom_z;
    ua.stage = stage.get();
    ua.ucount = ucount.get();
    ua.err = S + 3;
    if (n_small > 0) {
        ua.ids = small_ids.get();
        hipLaunchKernelGGL(k_unit_sort, dim3((unsigned)n_small), dim3(kSegThreads), 0, c.stream, ua);
        JP_HIP(hipGetLastError());
    }
    if (n_big > 0) {
        ua.ids = big_ids.get();
        hipLaunchKernelGGL(k_big_x, dim3((unsigned)n_big), dim3(kSegThreads), 0, c.stream, ua);
        JP_HIP(hipGetLastError());
    }
    DBuf<int64_t> uoff = c.buf<int64_t>(n_units + 1);
    scan_exclusive(c, n_units, ArrayGet{ucount.get()}, ArrayPut{uoff.get()}, uoff.get() + n_units);
    int64_t hv[2];
    c.load_n(hv, S + 3, 1);
    JP_CHECK(hv[0] == 0, JP_EINTERNAL, "a dedup unit exceeded its on-chip capacity");
    const int64_t total = c.load(uoff.get() + n_units);
    *out_x = c.buf<int32_t>(std::max<int64_t>(total, 1));
    *out_z = c.buf<int32_t>(std::max<int64_t>(total, 1));
    if (total > 0) {
        EmitArgs ea;
        ea.uoff = uoff.get();
        ea.n_units = n_units;
        ea.n_out = total;
        ea.ustart = ustart.get();
        ea.toff = toff.get();
        ea.stage = stage.get();
        ea.xorig = in.xorig;
        ea.zorig = in.zorig;
        ea.bz = in.bz;
        ea.zmask = ua.zmask;
        ea.out_x = out_x->get();
        ea.out_z = out_z->get();
        ea.dom_x = dom_x;
        ea.dom_z = in.dom_z;
        ea.err = S + 4;
        const int64_t blocks = ceil_div(total, (int64_t)kEmitBlock * kEmitItems);
        hipLaunchKernelGGL(k_emit, dim3((unsigned)blocks), dim3(kEmitBlock), 0, c.stream, ea);
        JP_HIP(hipGetLastError());
    }
    if (total > 0) JP_CHECK(c.load(S + 4) == 0, JP_EINTERNAL, "dedup produced a key outside the rank tables");
    *n_out = total;
    if (stats) {
        stats->n_units = n_units;
        stats->n_small = n_small;
        stats->n_big = n_big;
        stats->n_cand = n_cand;
    }
}

}  // namespace jp
