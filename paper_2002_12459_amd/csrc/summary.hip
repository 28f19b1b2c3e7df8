// Degree indexes of a two-path instance for the threshold choice (Section 5,
// "Indexing relations": for a threshold delta the indexes give sum(y_delta),
// sum(x_delta), cdfx(y_delta) and count(w_delta) by binary search over a
// sorted degree vector).  Built on the device as degree histograms (LDS bins
// for small degrees, global bins up to kHist, a compacted list beyond), then
// compacted to the nonzero degrees and copied to the host.
#include <algorithm>

#include "pipeline.hpp"
#include "prims.hpp"

namespace jp {
namespace {

constexpr int64_t kHist = 1 << 16;
constexpr int kLdsBins = 1024;

template <class DegF, class SumF>
__global__ __launch_bounds__(256) void k_deg_hist(int64_t n, DegF degf, SumF sumf, unsigned long long *cnt,
                                                  unsigned long long *sums) {
    __shared__ unsigned int lc[kLdsBins];
    __shared__ unsigned long long ls[kLdsBins];
    for (int b = threadIdx.x; b < kLdsBins; b += 256) {
        lc[b] = 0;
        ls[b] = 0;
    }
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int64_t d = degf(i);
        const unsigned long long s = sumf(i);
        if (d < kLdsBins) {
            atomicAdd(&lc[d], 1u);
            if (s) atomicAdd(&ls[d], s);
        } else if (d < kHist) {
            atomicAdd(&cnt[d], 1ull);
            if (s) atomicAdd(&sums[d], s);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kLdsBins; b += 256) {
        if (lc[b]) atomicAdd(&cnt[b], (unsigned long long)lc[b]);
        if (ls[b]) atomicAdd(&sums[b], ls[b]);
    }
}

template <class DegF, class SumF>
HostIndex build_index(const Ctx &c, int64_t n, DegF degf, SumF sumf, bool with_sum) {
    HostIndex h;
    if (n <= 0) return h;
    DBuf<unsigned long long> cnt = c.buf<unsigned long long>(kHist), sums = c.buf<unsigned long long>(kHist);
    c.zero(cnt.get(), kHist);
    c.zero(sums.get(), kHist);
    const int64_t blocks = std::min<int64_t>(ceil_div(n, 256), (int64_t)c.num_cus * 4);
    hipLaunchKernelGGL((k_deg_hist<DegF, SumF>), dim3((unsigned)blocks), dim3(256), 0, c.stream, n, degf, sumf,
                       cnt.get(), sums.get());
    JP_HIP(hipGetLastError());
    DBuf<int64_t> S = c.buf<int64_t>(2);
    // nonzero bins
    DBuf<int64_t> bd = c.buf<int64_t>(kHist), bc = c.buf<int64_t>(kHist), bs = c.buf<int64_t>(kHist);
    {
        const unsigned long long *cp = cnt.get(), *sp = sums.get();
        int64_t *d = bd.get(), *cc = bc.get(), *ss = bs.get();
        compact(
            c, kHist, [=] __device__(int64_t b) { return cp[b] != 0; },
            [=] __device__(int64_t b, int64_t p) {
                d[p] = b;
                cc[p] = (int64_t)cp[b];
                ss[p] = (int64_t)sp[b];
            },
            S.get());
    }
    // values with degree >= kHist, listed one by one
    DBuf<int64_t> od = c.buf<int64_t>(n), os = c.buf<int64_t>(n);
    {
        int64_t *d = od.get(), *ss = os.get();
        compact(
            c, n, [=] __device__(int64_t i) { return degf(i) >= kHist; },
            [=] __device__(int64_t i, int64_t p) {
                d[p] = degf(i);
                ss[p] = (int64_t)sumf(i);
            },
            S.get() + 1);
    }
    int64_t hn[2];
    c.load_n(hn, S.get(), 2);
    std::vector<int64_t> d(hn[0]), cc(hn[0]), ss(hn[0]), e(hn[1]), es(hn[1]);
    c.load_n(d.data(), bd.get(), hn[0]);
    c.load_n(cc.data(), bc.get(), hn[0]);
    c.load_n(ss.data(), bs.get(), hn[0]);
    c.load_n(e.data(), od.get(), hn[1]);
    c.load_n(es.data(), os.get(), hn[1]);
    h.deg = d;
    h.count = cc;
    if (with_sum) h.sum.assign(ss.begin(), ss.end());
    if (hn[1]) {
        std::vector<std::pair<int64_t, int64_t>> big(hn[1]);
        for (int64_t i = 0; i < hn[1]; ++i) big[i] = {e[i], es[i]};
        std::sort(big.begin(), big.end());
        for (size_t i = 0; i < big.size();) {
            size_t j = i;
            int64_t cn = 0;
            double sm = 0;
            while (j < big.size() && big[j].first == big[i].first) {
                ++cn;
                sm += (double)big[j].second;
                ++j;
            }
            h.deg.push_back(big[i].first);
            h.count.push_back(cn);
            if (with_sum) h.sum.push_back(sm);
            i = j;
        }
    }
    return h;
}

}  // namespace

void summarize_two_path(const Ctx &c, const Ingest &g, int y_rule, TwoPathSummary &s) {
    const int32_t *dry = g.dRy.get(), *dsz = g.dSz.get(), *ar = g.adj_r.get();
    const int64_t *oy = g.off_y.get(), *ox = g.off_x.get();
    const bool ronly = y_rule == JP_Y_RULE_R_ONLY;
    auto kd = [=] __device__(int64_t y) -> int64_t {
        const int64_t dr = dry[y], ds = oy[y + 1] - oy[y];
        return ronly ? dr : (dr > ds ? dr : ds);
    };
    auto zero = [=] __device__(int64_t) -> unsigned long long { return 0ull; };
    s.y = build_index(
        c, g.dom_y, kd,
        [=] __device__(int64_t y) -> unsigned long long {
            return (unsigned long long)dry[y] * (unsigned long long)(oy[y + 1] - oy[y]);
        },
        true);
    s.yr = build_index(c, g.dom_y, [=] __device__(int64_t y) -> int64_t { return dry[y]; }, zero, false);
    s.ys = build_index(c, g.dom_y, [=] __device__(int64_t y) -> int64_t { return oy[y + 1] - oy[y]; }, zero, false);
    s.x = build_index(
        c, g.dom_x, [=] __device__(int64_t x) -> int64_t { return ox[x + 1] - ox[x]; },
        [=] __device__(int64_t x) -> unsigned long long {
            unsigned long long w = 0;
            for (int64_t e = ox[x]; e < ox[x + 1]; ++e) w += (unsigned long long)(oy[ar[e] + 1] - oy[ar[e]]);
            return w;
        },
        true);
    s.xcdf = build_index(
        c, g.dom_x,
        [=] __device__(int64_t x) -> int64_t {
            int64_t m = INT64_MAX;
            for (int64_t e = ox[x]; e < ox[x + 1]; ++e) {
                const int64_t k = kd(ar[e]);
                m = k < m ? k : m;
            }
            return m;
        },
        zero, false);
    s.z = build_index(c, g.dom_z, [=] __device__(int64_t z) -> int64_t { return dsz[z]; }, zero, false);
    s.have_indexes = true;
}

}  // namespace jp
