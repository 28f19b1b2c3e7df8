// Degree indexes of a two-path instance for the threshold choice (Section 5,
// "Indexing relations": for a threshold delta the indexes give sum(y_delta),
// sum(x_delta), cdfx(y_delta) and count(w_delta) by binary search over a
// sorted degree vector).
//
// All six indexes (y key degree with witness sums, deg_R(y), deg_S(y),
// deg_R(x) with witness sums, cdfx, deg_S(z)) are built by one histogram
// launch (grid.y = index, one element per thread; the x workgroups build
// both x indexes from one walk over each x's tuples, reading a per-y table of
// (deg_S(y), key degree) made beforehand): degrees below kLdsBins go to
// per-workgroup LDS bins, which are flushed into one of kCopies copies of the
// low global bins (spreading the atomics of thousands of workgroups over the
// copies) and folded afterwards; degrees below kHist go to global bins,
// larger ones to an append list.  One compaction keeps the nonzero bins; the
// host then waits once for sizes and data together and merges the append
// list.
#include <algorithm>

#include "pipeline.hpp"
#include "prims.hpp"

namespace jp {
namespace {

constexpr int kIdx = 6;              // y, yr, ys, x, xcdf, z
constexpr int64_t kHist = 1 << 16;   // global bins per index
constexpr int kLdsBins = 1024;       // LDS bins per workgroup
constexpr int kHistBlock = 256;
constexpr int kEdgeBatch = 4;        // R tuples of an x read together
constexpr int kCopies = 16;          // copies of the low global bins

struct YDeg {
    int64_t ds, key;  // deg_S(y), key degree of y
};

struct IndexArgs {
    const int32_t *dry, *dsz, *ar;
    const int64_t *oy, *ox;
    const YDeg *yd;  // per y
    int64_t dom_y, dom_x, dom_z;
    bool ronly;
    unsigned long long *cnt;   // [kIdx][kHist]
    unsigned long long *sums;  // [kIdx][kHist]
    unsigned long long *lo;    // [kCopies][kIdx][kLdsBins] counts, then as many sums
    int64_t *big;              // append list: idx << 56 | degree, then sum (pairs)
    unsigned long long *nbig;
    int64_t big_cap;
};

__device__ __forceinline__ int64_t key_deg(const IndexArgs &a, int64_t y) {
    const int64_t dr = a.dry[y], ds = a.oy[y + 1] - a.oy[y];
    return a.ronly ? dr : (dr > ds ? dr : ds);
}

// Degree and summed work of element i of index k (k != 3, 4).
__device__ __forceinline__ void index_value(const IndexArgs &a, int k, int64_t i, int64_t &d, unsigned long long &s) {
    s = 0;
    switch (k) {
        case 0: {  // y: key degree, witnesses deg_R(y) deg_S(y)
            const int64_t ds = a.oy[i + 1] - a.oy[i];
            d = key_deg(a, i);
            s = (unsigned long long)a.dry[i] * (unsigned long long)ds;
            break;
        }
        case 1: d = a.dry[i]; break;
        case 2: d = a.oy[i + 1] - a.oy[i]; break;
        default: d = a.dsz[i]; break;
    }
}

// x index (deg_R(x), witnesses = sum over the y of x of deg_S(y)) and cdfx
// index (smallest key degree among the y of x) of x = i, from one walk.
__device__ __forceinline__ void x_values(const IndexArgs &a, int64_t i, int64_t &d, unsigned long long &w, int64_t &m) {
    const int64_t e0 = a.ox[i], e1 = a.ox[i + 1];
    w = 0;
    m = INT64_MAX;
    for (int64_t e = e0; e < e1; e += kEdgeBatch) {  // kEdgeBatch tuples' loads at once
        int32_t y[kEdgeBatch];
#pragma unroll
        for (int r = 0; r < kEdgeBatch; ++r) y[r] = a.ar[e + r < e1 ? e + r : e0];
        YDeg t[kEdgeBatch];
#pragma unroll
        for (int r = 0; r < kEdgeBatch; ++r) t[r] = a.yd[y[r]];
#pragma unroll
        for (int r = 0; r < kEdgeBatch; ++r)
            if (e + r < e1) {
                w += (unsigned long long)t[r].ds;
                m = t[r].key < m ? t[r].key : m;
            }
    }
    d = e1 - e0;
}

__global__ __launch_bounds__(kHistBlock) void k_index_hist(IndexArgs a) {
    __shared__ unsigned int lc[2][kLdsBins];  // [1]: the cdfx index, in the x workgroups
    __shared__ unsigned long long ls[kLdsBins];
    const int k = blockIdx.y;
    if (k == 4) return;  // cdfx comes from the x workgroups
    const int64_t n = k < 3 ? a.dom_y : (k == 3 ? a.dom_x : a.dom_z);
    if ((int64_t)blockIdx.x * kHistBlock >= n) return;  // whole workgroup idle for this index
    for (int b = threadIdx.x; b < kLdsBins; b += kHistBlock) {
        lc[0][b] = 0;
        lc[1][b] = 0;
        ls[b] = 0;
    }
    __syncthreads();
    auto add = [&](int kk, int slot, int64_t d, unsigned long long s) {
        if (d < kLdsBins) {
            atomicAdd(&lc[slot][d], 1u);
            if (s) atomicAdd(&ls[d], s);
        } else if (d < kHist) {
            atomicAdd(&a.cnt[(int64_t)kk * kHist + d], 1ull);
            if (s) atomicAdd(&a.sums[(int64_t)kk * kHist + d], s);
        } else {
            const unsigned long long p = atomicAdd(a.nbig, 1ull);
            if ((int64_t)p < a.big_cap) {
                a.big[2 * p] = ((int64_t)kk << 56) | (d < (1ll << 56) ? d : (1ll << 56) - 1);
                a.big[2 * p + 1] = (int64_t)s;
            }
        }
    };
    for (int64_t i = (int64_t)blockIdx.x * kHistBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kHistBlock) {
        if (k == 3) {
            int64_t d, m;
            unsigned long long w;
            x_values(a, i, d, w, m);
            add(3, 0, d, w);
            add(4, 1, m, 0);
        } else {
            int64_t d;
            unsigned long long s;
            index_value(a, k, i, d, s);
            add(k, 0, d, s);
        }
    }
    __syncthreads();
    const int64_t copy = (int64_t)(blockIdx.x % kCopies);
    unsigned long long *lo = a.lo + (copy * kIdx + k) * kLdsBins;
    unsigned long long *los = lo + (int64_t)kCopies * kIdx * kLdsBins;
    unsigned long long *lo4 = a.lo + (copy * kIdx + 4) * kLdsBins;
    for (int b = threadIdx.x; b < kLdsBins; b += kHistBlock) {
        if (lc[0][b]) atomicAdd(&lo[b], (unsigned long long)lc[0][b]);
        if (ls[b]) atomicAdd(&los[b], ls[b]);
        if (k == 3 && lc[1][b]) atomicAdd(&lo4[b], (unsigned long long)lc[1][b]);
    }
}

// Low bins: the sum of the copies (these bins receive nothing else).
__global__ __launch_bounds__(kHistBlock) void k_index_fold(IndexArgs a) {
    const int64_t i = (int64_t)blockIdx.x * kHistBlock + threadIdx.x;  // k * kLdsBins + b
    if (i >= (int64_t)kIdx * kLdsBins) return;
    const int64_t k = i / kLdsBins, b = i % kLdsBins;
    const int64_t stride = (int64_t)kIdx * kLdsBins, sum_off = (int64_t)kCopies * kIdx * kLdsBins;
    unsigned long long c = 0, sm = 0;
#pragma unroll
    for (int q = 0; q < kCopies; ++q) {
        c += a.lo[q * stride + i];
        sm += a.lo[sum_off + q * stride + i];
    }
    a.cnt[k * kHist + b] = c;
    a.sums[k * kHist + b] = sm;
}

// Sizes and data of the index read-back in one block of 64-bit words:
// [count, nbig, count records of 3 words, nbig pairs], written to mapped host
// memory when it fits in cap words and nbig is within the list's capacity
// (else only the two sizes).
__global__ __launch_bounds__(256) void k_index_to_host(const int64_t *sizes, const int64_t *rec, const int64_t *big,
                                                       int64_t big_cap, int64_t cap, int64_t *dst) {
    const int64_t n_rec = 3 * sizes[0], n_big = 2 * sizes[1];
    const int64_t total = 2 + n_rec + n_big;
    const int64_t n = ((total <= cap) & (sizes[1] <= big_cap)) ? total : 2;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        dst[i] = i < 2 ? sizes[i] : (i < 2 + n_rec ? rec[i - 2] : big[i - 2 - n_rec]);
}

}  // namespace

void summarize_two_path(const Ctx &c, const Ingest &g, int y_rule, TwoPathSummary &s) {
    HostIndex *out[kIdx] = {&s.y, &s.yr, &s.ys, &s.x, &s.xcdf, &s.z};
    const bool with_sum[kIdx] = {true, false, false, true, false, false};
    for (HostIndex *h : out) *h = HostIndex();
    s.have_indexes = true;
    const int64_t nmax = std::max(g.dom_y, std::max(g.dom_x, g.dom_z));
    if (nmax <= 0) return;

    IndexArgs a;
    a.dry = g.dRy.get();
    a.dsz = g.dSz.get();
    a.ar = g.adj_r.get();
    a.oy = g.off_y.get();
    a.ox = g.off_x.get();
    a.dom_y = g.dom_y;
    a.dom_x = g.dom_x;
    a.dom_z = g.dom_z;
    a.ronly = y_rule == JP_Y_RULE_R_ONLY;
    // one block for counts, sums and the low-bin copies, cleared together
    const int64_t lo_words = 2ll * kCopies * kIdx * kLdsBins;
    DBuf<unsigned long long> bins = c.buf<unsigned long long>(2 * kIdx * kHist + lo_words);
    c.zero(bins.get(), 2 * kIdx * kHist + lo_words);
    a.cnt = bins.get();
    a.sums = bins.get() + kIdx * kHist;
    a.lo = bins.get() + 2 * kIdx * kHist;
    // Values of degree >= kHist: at most 3 dom_y + 2 dom_x + dom_z in all.
    a.big_cap = 3 * g.dom_y + 2 * g.dom_x + g.dom_z;
    DBuf<int64_t> big = c.buf<int64_t>((size_t)(2 * a.big_cap));
    DBuf<int64_t> S = c.buf<int64_t>(2);
    c.zero(S.get(), 2);
    a.big = big.get();
    a.nbig = (unsigned long long *)(S.get() + 1);
    // per y: deg_S(y) and key degree, read by the walk over each x's tuples
    DBuf<YDeg> yd = c.buf<YDeg>((size_t)std::max<int64_t>(g.dom_y, 1));
    {
        YDeg *t = yd.get();
        const IndexArgs ac = a;
        for_each(c, g.dom_y, [=] __device__(int64_t y) { t[y] = YDeg{ac.oy[y + 1] - ac.oy[y], key_deg(ac, y)}; });
    }
    a.yd = yd.get();
    // one element per thread (up to 2^24 threads per index, then strided)
    const int64_t bx = std::min<int64_t>(ceil_div(nmax, kHistBlock), 1ll << 16);
    hipLaunchKernelGGL(k_index_hist, dim3(grid_x(bx, kHistBlock), kIdx), dim3(kHistBlock), 0, c.stream, a);
    JP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_index_fold, dim3(grid_x(ceil_div((int64_t)kIdx * kLdsBins, kHistBlock), kHistBlock)),
                       dim3(kHistBlock), 0, c.stream, a);
    JP_HIP(hipGetLastError());

    // nonzero bins of all indexes, in (index, degree) order
    const int64_t nb = kIdx * kHist;
    DBuf<int64_t> rec = c.buf<int64_t>((size_t)(3 * nb));
    {
        const unsigned long long *cp = a.cnt, *sp = a.sums;
        int64_t *r = rec.get();
        compact(
            c, nb, [=] __device__(int64_t b) { return cp[b] != 0; },
            [=] __device__(int64_t b, int64_t p) {
                r[3 * p] = b;
                r[3 * p + 1] = (int64_t)cp[b];
                r[3 * p + 2] = (int64_t)sp[b];
            },
            S.get());
    }
    // sizes and, when they fit the handle's mapped host buffer, the data too: one wait
    int64_t hn[2];
    std::vector<int64_t> r, e;
    bool fetched = false;
    if (c.replay) {  // a plan is recorded or captured: every read-back goes through load_n
        c.load_n(hn, S.get(), 2);
        JP_CHECK(hn[1] <= a.big_cap, JP_EINTERNAL, "degree index overflow list exceeds its bound");
        r.resize(3 * hn[0]);
        e.resize(2 * hn[1]);
        c.load_n(r.data(), rec.get(), r.size());
        c.load_n(e.data(), big.get(), e.size(), true);  // appended with atomics: any order
        fetched = true;
    } else if (c.pinned && c.pinned->host && c.pinned->bytes >= 64) {
        const int64_t cap = (int64_t)(c.pinned->bytes / sizeof(int64_t));
        hipLaunchKernelGGL(k_index_to_host, dim3(64), dim3(256), 0, c.stream, (const int64_t *)S.get(),
                           (const int64_t *)rec.get(), (const int64_t *)big.get(), a.big_cap, cap,
                           (int64_t *)c.pinned->dev);
        JP_HIP(hipGetLastError());
        c.sync();
        const int64_t *h = (const int64_t *)c.pinned->host;
        hn[0] = h[0];
        hn[1] = h[1];
        JP_CHECK(hn[1] <= a.big_cap, JP_EINTERNAL, "degree index overflow list exceeds its bound");
        if (2 + 3 * hn[0] + 2 * hn[1] <= cap) {
            r.assign(h + 2, h + 2 + 3 * hn[0]);
            e.assign(h + 2 + 3 * hn[0], h + 2 + 3 * hn[0] + 2 * hn[1]);
            fetched = true;
        }
    } else {
        c.load_n(hn, S.get(), 2);
        JP_CHECK(hn[1] <= a.big_cap, JP_EINTERNAL, "degree index overflow list exceeds its bound");
    }
    if (!fetched) {
        r.resize(3 * hn[0]);
        e.resize(2 * hn[1]);
        if (hn[0]) JP_HIP(hipMemcpyAsync(r.data(), rec.get(), r.size() * sizeof(int64_t), hipMemcpyDeviceToHost, c.stream));
        if (hn[1]) JP_HIP(hipMemcpyAsync(e.data(), big.get(), e.size() * sizeof(int64_t), hipMemcpyDeviceToHost, c.stream));
        c.sync();
    }

    for (int64_t i = 0; i < hn[0]; ++i) {
        const int64_t b = r[3 * i];
        HostIndex &h = *out[b / kHist];
        h.deg.push_back(b % kHist);
        h.count.push_back(r[3 * i + 1]);
        if (with_sum[b / kHist]) h.sum.push_back((double)r[3 * i + 2]);
    }
    // append list: sort by (index, degree), merge equal degrees
    std::vector<std::pair<int64_t, int64_t>> bigv(hn[1]);
    for (int64_t i = 0; i < hn[1]; ++i) bigv[i] = {e[2 * i], e[2 * i + 1]};
    std::sort(bigv.begin(), bigv.end());
    for (size_t i = 0; i < bigv.size();) {
        size_t j = i;
        int64_t cn = 0;
        double sm = 0;
        while (j < bigv.size() && bigv[j].first == bigv[i].first) {
            ++cn;
            sm += (double)bigv[j].second;
            ++j;
        }
        const int k = (int)(bigv[i].first >> 56);
        HostIndex &h = *out[k];
        h.deg.push_back(bigv[i].first & ((1ll << 56) - 1));
        h.count.push_back(cn);
        if (with_sum[k]) h.sum.push_back(sm);
        i = j;
    }
}

// ---- sampled output size ---------------------------------------------------
// A selector input (not part of the paper's method): k = min(draws, dom_x)
// draws of an x rank, draw i taking rank splitmix64(seed + i) mod dom_x (x
// ranks follow x values, so rank r is the r-th smallest x kept), and the
// exact number of distinct z each drawn x reaches, summed over the draws.
// The draws' candidate z are gathered as (draw, z) keys, sorted and counted
// distinct.  A prefix of the draws whose candidates exceed `cap` is dropped
// (at least one draw is kept; if that alone exceeds 4 cap, nothing is
// counted and draws = 0).

__device__ __forceinline__ uint64_t splitmix64_next(uint64_t x) {
    uint64_t z = x + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Draws kept under the cap: the longest prefix of draws whose candidates
// total at most cap, at least the first draw, none if that one alone passes
// 4 cap (coff: exclusive prefix of the draws' candidate counts).
__device__ __forceinline__ bool draw_kept(const int64_t *coff, int64_t i, int64_t cap) {
    return coff[i + 1] <= cap || (i == 0 && coff[1] <= 4 * cap);
}

// Distinct z of each kept draw when the z domain fits one LDS bitmap: one
// workgroup per draw marks its candidates (its R tuples' lists, 256 tuples
// at a time, the candidates of those lists spread over the threads) and
// counts the set bits.  Adds the counts to *dsum and the kept draws to *kept.
constexpr int64_t kSampleBitmapBits = int64_t(1) << 20;
constexpr int kSampleBlock = 1024;  // one workgroup per CU fits the bitmap: all its threads for one draw
constexpr int kSampleMarkBatch = 8;  // candidates per thread with loads in flight together
__global__ __launch_bounds__(kSampleBlock) void k_sample_distinct(const int32_t *xr, const int64_t *coff, int64_t cap,
                                                                  const int64_t *ox, const int32_t *ar,
                                                                  const int64_t *oy, const int32_t *as, int64_t dom_z,
                                                                  unsigned long long *dsum, unsigned long long *kept) {
    extern __shared__ uint32_t bm[];
    __shared__ int64_t lpre[kSampleBlock + 1], lbase[kSampleBlock];
    __shared__ int64_t lds64[kSampleBlock / kWave + 1];
    const int64_t i = blockIdx.x;
    if (!draw_kept(coff, i, cap)) return;  // uniform per workgroup
    const int tid = threadIdx.x;
    const int nw = (int)((dom_z + 31) / 32);
    for (int t = tid; t < nw; t += kSampleBlock) bm[t] = 0;
    const int32_t x = xr[i];
    const int64_t e0 = ox[x], e1 = ox[x + 1];
    for (int64_t c0 = e0; c0 < e1; c0 += kSampleBlock) {
        const int64_t e = c0 + tid;
        int64_t len = 0, base = 0;
        if (e < e1) {
            const int32_t y = ar[e];
            base = oy[y];
            len = oy[y + 1] - base;
        }
        int64_t tot;
        const int64_t pre = block_excl_scan<kSampleBlock>(len, lds64, &tot);
        lpre[tid] = pre;
        lbase[tid] = base;
        if (tid == 0) lpre[kSampleBlock] = tot;
        __syncthreads();  // also orders the bitmap clear before the first marks
        const int nl = (int)(e1 - c0 < kSampleBlock ? e1 - c0 : kSampleBlock);
        // kSampleMarkBatch candidates per thread and round, their loads issued
        // together (a draw can reach long lists); slots past the end read the
        // last candidate and mark nothing
        for (int64_t q0 = tid; q0 < tot; q0 += (int64_t)kSampleBlock * kSampleMarkBatch) {
            int32_t z[kSampleMarkBatch];
#pragma unroll
            for (int r = 0; r < kSampleMarkBatch; ++r) {
                const int64_t q1 = q0 + (int64_t)r * kSampleBlock;
                const int64_t q = q1 < tot ? q1 : tot - 1;
                int lo = 0, hi = nl - 1;  // the list holding candidate q: last l with lpre[l] <= q
                while (lo < hi) {
                    const int mid = (lo + hi + 1) / 2;
                    if (lpre[mid] <= q) lo = mid;
                    else hi = mid - 1;
                }
                z[r] = as[lbase[lo] + (q - lpre[lo])];
            }
#pragma unroll
            for (int r = 0; r < kSampleMarkBatch; ++r)
                if (q0 + (int64_t)r * kSampleBlock < tot) atomicOr(&bm[z[r] >> 5], 1u << (z[r] & 31));
        }
        __syncthreads();  // lpre / lbase are refilled by the next chunk
    }
    uint32_t cnt = 0;
    for (int t = tid; t < nw; t += kSampleBlock) cnt += (uint32_t)__popc(bm[t]);
    const int64_t d = block_sum<kSampleBlock>((int64_t)cnt, lds64);
    if (tid == 0) {
        atomicAdd(dsum, (unsigned long long)d);
        atomicAdd(kept, 1ull);
    }
}

SampledOut sampled_out(const Ctx &c, const Ingest &g, uint64_t seed, int64_t max_draws, int64_t cap) {
    SampledOut r;
    const int64_t n = g.dom_x;
    if (n <= 0 || max_draws <= 0) return r;
    int64_t k = std::min(max_draws, n);
    DBuf<int32_t> xr = c.buf<int32_t>((size_t)k);
    DBuf<int64_t> cnt = c.buf<int64_t>((size_t)k), coff = c.buf<int64_t>((size_t)k + 1);
    DBuf<int64_t> tcnt = c.buf<int64_t>((size_t)k), toff = c.buf<int64_t>((size_t)k + 1);
    {
        int32_t *x = xr.get();
        int64_t *ct = cnt.get(), *tc = tcnt.get();
        const int64_t *ox = g.off_x.get(), *oy = g.off_y.get();
        const int32_t *ar = g.adj_r.get();
        const uint64_t sd = seed;
        for_each(c, k, [=] __device__(int64_t i) {
            const int32_t xi = (int32_t)(splitmix64_next(sd + (uint64_t)i) % (uint64_t)n);
            x[i] = xi;
            int64_t t = 0;
            for (int64_t e = ox[xi]; e < ox[xi + 1]; ++e) t += oy[ar[e] + 1] - oy[ar[e]];
            ct[i] = t;
            tc[i] = ox[xi + 1] - ox[xi];
        });
        scan_exclusive(c, k, ArrayGet{ct}, ArrayPut{coff.get()}, coff.get() + k);
    }
    if (g.dom_z <= kSampleBitmapBits) {
        // one LDS bitmap per draw: the cap rule applied on the device, one read-back
        DBuf<int64_t> S2 = c.buf<int64_t>(2);
        c.zero(S2.get(), 2);
        const size_t lds = (size_t)((g.dom_z + 31) / 32) * sizeof(uint32_t);
        hipLaunchKernelGGL(k_sample_distinct, dim3(grid_x(k, kSampleBlock)), dim3(kSampleBlock), lds, c.stream,
                           (const int32_t *)xr.get(), (const int64_t *)coff.get(), cap, (const int64_t *)g.off_x.get(),
                           (const int32_t *)g.adj_r.get(), (const int64_t *)g.off_y.get(),
                           g.adj_s(c), g.dom_z, (unsigned long long *)S2.get(),
                           (unsigned long long *)(S2.get() + 1));
        JP_HIP(hipGetLastError());
        int64_t h[2];
        c.load_n(h, S2.get(), 2);
        r.distinct = h[0];
        r.draws = h[1];
        return r;
    }
    std::vector<int64_t> hoff((size_t)k + 1);
    c.load_n(hoff.data(), coff.get(), hoff.size());
    if (hoff[k] > cap) {  // keep the longest prefix of draws within the cap
        int64_t kk = (int64_t)(std::upper_bound(hoff.begin(), hoff.end(), cap) - hoff.begin()) - 1;
        kk = std::max<int64_t>(kk, 1);
        if (hoff[kk] > 4 * cap) return r;
        k = kk;
    }
    const int64_t T = hoff[k];
    r.draws = k;
    if (T == 0) return r;
    // (draw, tuple) pairs, then candidates by pair
    scan_exclusive(c, k, ArrayGet{tcnt.get()}, ArrayPut{toff.get()}, toff.get() + k);
    const int64_t P = c.load(toff.get() + k);
    DBuf<int32_t> pdraw = c.buf<int32_t>((size_t)P);
    DBuf<int64_t> ptup = c.buf<int64_t>((size_t)P), poff = c.buf<int64_t>((size_t)P + 1);
    {
        const int32_t *x = xr.get();
        const int64_t *to = toff.get(), *ox = g.off_x.get();
        int32_t *pd = pdraw.get();
        int64_t *pt = ptup.get();
        const int64_t kd = k;
        for_each(c, P, [=] __device__(int64_t p) {
            const int64_t i = upper_bound_dev(to, (int64_t)0, kd, p) - 1;
            pd[p] = (int32_t)i;
            pt[p] = ox[x[i]] + (p - to[i]);
        });
        const int64_t *oy = g.off_y.get();
        const int32_t *ar = g.adj_r.get();
        const int64_t *ptc = pt;
        scan_exclusive(
            c, P, [=] __device__(int64_t p) -> int64_t { return oy[ar[ptc[p]] + 1] - oy[ar[ptc[p]]]; },
            ArrayPut{poff.get()}, poff.get() + P);
    }
    const int bz = bits_for((uint64_t)std::max<int64_t>(g.dom_z - 1, 1));
    const int bd = bits_for((uint64_t)std::max<int64_t>(k - 1, 1));
    DBuf<uint64_t> keys = c.buf<uint64_t>((size_t)T), tmp = c.buf<uint64_t>((size_t)T);
    {
        const int64_t *po = poff.get(), *pt = ptup.get(), *oy = g.off_y.get();
        const int32_t *pd = pdraw.get(), *ar = g.adj_r.get(), *as = g.adj_s(c);
        uint64_t *ky = keys.get();
        const int64_t np = P;
        const int bzs = bz;
        for_each(c, T, [=] __device__(int64_t o) {
            const int64_t p = upper_bound_dev(po, (int64_t)0, np, o) - 1;
            const int64_t z = as[oy[ar[pt[p]]] + (o - po[p])];
            ky[o] = ((uint64_t)pd[p] << bzs) | (uint64_t)z;
        });
    }
    const uint64_t *sk = radix_sort(c, keys.get(), tmp.get(), T, bd + bz);
    DBuf<int64_t> nd = c.buf<int64_t>(1);
    compact(
        c, T, [=] __device__(int64_t i) { return i == 0 || sk[i] != sk[i > 0 ? i - 1 : 0]; },
        [=] __device__(int64_t, int64_t) {}, nd.get());
    r.distinct = c.load(nd.get());
    return r;
}

}  // namespace jp
