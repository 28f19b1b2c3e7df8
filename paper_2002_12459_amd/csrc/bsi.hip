// Batched Boolean set intersection (Section 3.3): a batch T of queries
// (a_i, c_i) asks, for each i, whether the sets {b : (a_i, b) in R} and
// {b : (c_i, b) in S} intersect.  As in the paper's experiments, the batch
// filters the relations (R to the queried a, S to the queried c), the
// filtered two-path query is evaluated by Algorithm 1 (run_two_path, any
// thresholds), and each query is answered by a binary search for its pair in
// the sorted distinct output: the pair is in Q(x,z) = R(x,y), S(z,y) exactly
// when the two sets intersect.
#include "pipeline.hpp"
#include "prims.hpp"

namespace jp {
namespace {

__device__ __forceinline__ uint32_t biased(int32_t v) { return (uint32_t)v ^ 0x80000000u; }

// Sorted distinct biased values of col[0..n): returns their count.
int64_t distinct_sorted(const Ctx &c, const int32_t *col, int64_t n, DBuf<uint32_t> &out, int64_t *S) {
    DBuf<uint32_t> a = c.buf<uint32_t>(std::max<int64_t>(n, 1)), b = c.buf<uint32_t>(std::max<int64_t>(n, 1));
    const uint32_t *s = radix_sort_from<uint32_t>(
        c, [=] __device__(int64_t i) { return biased(col[i]); }, a.get(), b.get(), n, 32);
    out = c.buf<uint32_t>(std::max<int64_t>(n, 1));
    uint32_t *d = out.get();
    compact(
        c, n, [=] __device__(int64_t i) { return i == 0 || s[i] != s[i > 0 ? i - 1 : 0]; },
        [=] __device__(int64_t i, int64_t p) { d[p] = s[i]; }, S);
    return c.load(S);
}

// Rows (a, y) of a relation whose a is among the n_keys sorted keys.
int64_t filter_rows(const Ctx &c, const int32_t *a, const int32_t *y, int64_t n, const uint32_t *keys, int64_t n_keys,
                    DBuf<int32_t> &fa, DBuf<int32_t> &fy, int64_t *S) {
    fa = c.buf<int32_t>(std::max<int64_t>(n, 1));
    fy = c.buf<int32_t>(std::max<int64_t>(n, 1));
    int32_t *oa = fa.get(), *oy = fy.get();
    compact(
        c, n,
        [=] __device__(int64_t i) {
            const uint32_t v = biased(a[i]);
            const int64_t p = lower_bound_dev(keys, (int64_t)0, n_keys, v);
            return (p < n_keys) & (keys[p < n_keys ? p : n_keys - 1] == v);
        },
        [=] __device__(int64_t i, int64_t p) {
            oa[p] = a[i];
            oy[p] = y[i];
        },
        S);
    return c.load(S);
}

}  // namespace

void run_bsi(const Ctx &c, const int32_t *rx, const int32_t *ry, int64_t nr, const int32_t *sz, const int32_t *sy,
             int64_t ns, const int32_t *tx, const int32_t *tz, int64_t nt, const jp_options &o, uint8_t *answers,
             jp_stats *stats) {
    jp_stats st{};
    st.arity = 2;
    st.delta1 = st.delta2 = JP_DELTA_INF;
    st.strategy = o.strategy;
    if (nt == 0) {
        if (stats) *stats = st;
        return;
    }
    c.zero(answers, (size_t)nt);
    DBuf<int64_t> scal = c.buf<int64_t>(4);
    int64_t *S = scal.get();
    // the batch's distinct a and c
    DBuf<uint32_t> qa, qc;
    const int64_t na = distinct_sorted(c, tx, nt, qa, S);
    const int64_t nc = distinct_sorted(c, tz, nt, qc, S + 1);
    // relations filtered by the batch
    DBuf<int32_t> fr_x, fr_y, fs_z, fs_y;
    const int64_t nr2 = filter_rows(c, rx, ry, nr, qa.get(), na, fr_x, fr_y, S + 2);
    const int64_t ns2 = filter_rows(c, sz, sy, ns, qc.get(), nc, fs_z, fs_y, S + 3);
    qa.reset();
    qc.reset();
    std::unique_ptr<jp_result> r(run_two_path(c, fr_x.get(), fr_y.get(), nr2, fs_z.get(), fs_y.get(), ns2, o));
    st = r->stats;
    const int64_t m = r->n;
    if (m > 0) {
        // answer every query by a search for its pair in the sorted output
        const int32_t *ox = r->cols[0].get(), *oz = r->cols[1].get();
        for_each(c, nt, [=] __device__(int64_t i) {
            const uint64_t q = ((uint64_t)biased(tx[i]) << 32) | biased(tz[i]);
            int64_t lo = 0, hi = m;
            while (lo < hi) {
                const int64_t mid = lo + (hi - lo) / 2;
                const uint64_t k = ((uint64_t)biased(ox[mid]) << 32) | biased(oz[mid]);
                if (k < q) lo = mid + 1;
                else hi = mid;
            }
            const int64_t at = lo < m ? lo : m - 1;
            const uint64_t k = ((uint64_t)biased(ox[at]) << 32) | biased(oz[at]);
            answers[i] = (lo < m) & (k == q) ? 1 : 0;
        });
    }
    c.sync();
    if (stats) *stats = st;
}

}  // namespace jp
