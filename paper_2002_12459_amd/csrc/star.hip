// Star join-project Q*_k(x1..xk) = R1(x1,y), ..., Rk(xk,y) (Section 3.2),
// 3 <= k <= 8.  k = 2 is the two-path query and goes to run_two_path.
//
//  ingest     every relation becomes a set indexed by y; y missing from any
//             relation is dropped; y and each x_i get dense ranks; degrees.
//  partition  x_i heavy iff deg_i(x_i) > Delta2.  A tuple (a, b) of R_i is in
//             R_i^- when a is light, in R_i^diamond when b has degree
//             <= Delta1 in every other relation, in R_i^+ otherwise.  A
//             witness (a1..ak, b) is heavy iff all k tuples are in R_i^+,
//             i.e. every a_i is heavy and b is heavy (degree > Delta1) in at
//             least two relations ("star-heavy").
//  light      per y, the witness box N1 x ... x Nk when y is not star-heavy,
//             else the box minus H1 x ... x Hk, written as the k disjoint
//             boxes H1 x .. x H(t-1) x Lt x N(t+1) x .. x Nk (t = 1..k) over
//             lists that hold light x first; every box is enumerated into
//             packed keys x1 << s1 | ... | xk with the output index space cut
//             evenly across workgroups.
//  heavy      C[(a1..ag), (a(g+1)..ak)] = sum_b prod_i M_i[a_i, b] over heavy
//             a_i and star-heavy b, g = ceil(k/2): the product V x W^T of
//             Section 3.2 with the rows of V and W generated from the factor
//             matrices as they are loaded (neither is stored); nonzeros
//             become keys.
//  union      one radix sort of light + heavy keys (64-bit, or 128-bit when
//             the rank widths exceed 64 bits), unique, unrank.
#include <climits>

#include "debug.hpp"
#include "pipeline.hpp"
#include "prims.hpp"

namespace jp {
namespace {

typedef unsigned __int128 u128;

__global__ __launch_bounds__(256) void k_minmax3(const int32_t *a, int64_t n, int *out) {
    __shared__ int smn[4], smx[4];
    int mn = INT_MAX, mx = INT_MIN;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int v = a[i];
        mn = v < mn ? v : mn;
        mx = v > mx ? v : mx;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const int a2 = __shfl_xor(mn, o), b2 = __shfl_xor(mx, o);
        mn = a2 < mn ? a2 : mn;
        mx = b2 > mx ? b2 : mx;
    }
    if (lane_id() == 0) {
        smn[threadIdx.x / kWave] = mn;
        smx[threadIdx.x / kWave] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 4; ++i) {
            mn = smn[i] < mn ? smn[i] : mn;
            mx = smx[i] > mx ? smx[i] : mx;
        }
        atomicMin(&out[0], mn);
        atomicMax(&out[1], mx);
    }
}

void minmax3(const Ctx &c, const int32_t *a, int64_t n, int *out) {
    if (n <= 0) return;
    const int64_t blocks = std::min<int64_t>(ceil_div(n, 256 * 16), (int64_t)c.num_cus);
    hipLaunchKernelGGL(k_minmax3, dim3((unsigned)blocks), dim3(256), 0, c.stream, a, n, out);
    JP_HIP(hipGetLastError());
}

// One relation after ingest: y-major, tuples sorted by (y rank, x), x as a rank.
struct RelIdx {
    int64_t n = 0;           // tuples kept
    int64_t dom_x = 0;
    DBuf<int64_t> off;       // dom_y + 1
    DBuf<int32_t> adj;       // x rank per tuple (light x first per y after partition)
    DBuf<int32_t> dx;        // degree of every x rank
    DBuf<int32_t> xorig;     // x rank -> id
    int bx = 0;              // bits of an x rank
};

// Distinct (y, x) of one relation, sorted by y then x: y and x offsets.
struct RelRaw {
    int64_t n1 = 0, ny = 0;
    DBuf<uint32_t> ty, tx;   // per distinct tuple
    DBuf<uint32_t> ys;       // distinct y offsets
    DBuf<int64_t> ystart;    // run starts of the distinct y (ny + 1)
};

RelRaw ingest_raw(const Ctx &c, const int32_t *x, const int32_t *y, int64_t n, int64_t xmin, int xb, int64_t ymin,
                  int yb, int64_t *S) {
    RelRaw r;
    DBuf<uint64_t> ka = c.buf<uint64_t>(n), kb = c.buf<uint64_t>(n);
    const uint64_t *s = radix_sort_from<uint64_t>(
        c, [=] __device__(int64_t i) { return ((uint64_t)((int64_t)y[i] - ymin) << xb) | (uint64_t)((int64_t)x[i] - xmin); },
        ka.get(), kb.get(), n, xb + yb);
    r.ty = c.buf<uint32_t>(n);
    r.tx = c.buf<uint32_t>(n);
    uint32_t *ty = r.ty.get(), *tx = r.tx.get();
    const uint64_t xm = xb >= 64 ? ~0ull : ((1ull << xb) - 1);
    const int xbs = xb;
    compact(
        c, n, [=] __device__(int64_t i) { return i == 0 || s[i] != s[i - 1]; },
        [=] __device__(int64_t i, int64_t p) {
            ty[p] = (uint32_t)(s[i] >> xbs);
            tx[p] = (uint32_t)(s[i] & xm);
        },
        S);
    r.n1 = c.load(S);
    r.ys = c.buf<uint32_t>(r.n1);
    r.ystart = c.buf<int64_t>(r.n1 + 1);
    uint32_t *ys = r.ys.get();
    int64_t *yst = r.ystart.get();
    compact(
        c, r.n1, [=] __device__(int64_t i) { return i == 0 || ty[i] != ty[i - 1]; },
        [=] __device__(int64_t i, int64_t p) {
            ys[p] = ty[i];
            yst[p] = i;
        },
        S);
    r.ny = c.load(S);
    const int64_t ny = r.ny, n1 = r.n1;
    for_each(c, 1, [=] __device__(int64_t) { yst[ny] = n1; });
    return r;
}

// Keeps the tuples whose y is in Yk (sorted distinct y offsets, rank = index),
// ranks x, returns the y-major index over y ranks [0, dom_y).
RelIdx finish_rel(const Ctx &c, const RelRaw &r, const uint32_t *Yk, int64_t dom_y, int64_t xmin, int xb, int64_t *S) {
    RelIdx o;
    // y rank of every distinct y of this relation (or -1)
    DBuf<int32_t> yr = c.buf<int32_t>(std::max<int64_t>(r.ny, 1));
    {
        int32_t *d = yr.get();
        const uint32_t *ys = r.ys.get();
        const int64_t ndy = dom_y;
        for_each(c, r.ny, [=] __device__(int64_t j) {
            const int64_t p = lower_bound_dev(Yk, (int64_t)0, ndy, ys[j]);
            const int64_t q = p < ndy ? p : ndy - 1;
            d[j] = ((p < ndy) & (Yk[q] == ys[j])) ? (int32_t)q : -1;
        });
    }
    // kept tuples (sorted by y rank then x offset) and the y-major offsets
    DBuf<int32_t> seg = c.buf<int32_t>(std::max<int64_t>(r.n1, 1));
    {
        const uint32_t *ty = r.ty.get();
        int32_t *sg = seg.get();
        auto newy = [=] __device__(int64_t i) -> int64_t { return (i == 0 || ty[i] != ty[i - 1]) ? 1 : 0; };
        scan_exclusive(c, r.n1, newy, [=] __device__(int64_t i, int64_t p) { sg[i] = (int32_t)(p + newy(i) - 1); });
    }
    DBuf<uint32_t> kx = c.buf<uint32_t>(std::max<int64_t>(r.n1, 1));
    DBuf<int32_t> ky = c.buf<int32_t>(std::max<int64_t>(r.n1, 1));
    {
        const int32_t *sg = seg.get(), *d = yr.get();
        const uint32_t *tx = r.tx.get();
        uint32_t *ox = kx.get();
        int32_t *oy = ky.get();
        compact(
            c, r.n1, [=] __device__(int64_t i) { return d[sg[i]] >= 0; },
            [=] __device__(int64_t i, int64_t p) {
                ox[p] = tx[i];
                oy[p] = d[sg[i]];
            },
            S);
    }
    o.n = c.load(S);
    const int64_t n = o.n;
    o.off = c.buf<int64_t>(dom_y + 1);
    {
        const int32_t *oy = ky.get();
        int64_t *of = o.off.get();
        compact(
            c, n, [=] __device__(int64_t e) { return e == 0 || oy[e] != oy[e - 1]; },
            [=] __device__(int64_t e, int64_t p) { of[p] = e; }, S);
        const int64_t ndy = dom_y;
        for_each(c, 1, [=] __device__(int64_t) { of[ndy] = n; });
    }
    // x ranks and degrees (run lengths of the sorted x offsets)
    DBuf<uint32_t> xs = c.buf<uint32_t>(std::max<int64_t>(n, 1));
    DBuf<int64_t> xst = c.buf<int64_t>(n + 1);
    {
        DBuf<uint32_t> a = c.buf<uint32_t>(std::max<int64_t>(n, 1)), b = c.buf<uint32_t>(std::max<int64_t>(n, 1));
        const uint32_t *s = radix_sort_from<uint32_t>(c, KeyArray<uint32_t>{kx.get()}, a.get(), b.get(), n, xb);
        uint32_t *d = xs.get();
        int64_t *st = xst.get();
        compact(
            c, n, [=] __device__(int64_t i) { return i == 0 || s[i] != s[i - 1]; },
            [=] __device__(int64_t i, int64_t p) {
                d[p] = s[i];
                st[p] = i;
            },
            S);
    }
    o.dom_x = c.load(S);
    const int64_t nx = o.dom_x;
    o.bx = bits_for((uint64_t)(nx - 1));
    o.xorig = c.buf<int32_t>(nx);
    o.dx = c.buf<int32_t>(nx);
    o.adj = c.buf<int32_t>(std::max<int64_t>(n, 1));
    {
        const uint32_t *d = xs.get();
        const int64_t *st = xst.get();
        int32_t *xo = o.xorig.get(), *dx = o.dx.get(), *adj = o.adj.get();
        const uint32_t *ox = kx.get();
        for_each(c, nx, [=] __device__(int64_t r2) {
            xo[r2] = (int32_t)((int64_t)d[r2] + xmin);
            dx[r2] = (int32_t)((r2 + 1 < nx ? st[r2 + 1] : n) - st[r2]);
        });
        for_each(c, n, [=] __device__(int64_t e) { adj[e] = (int32_t)lower_bound_dev(d, (int64_t)0, nx, ox[e]); });
    }
    return o;
}

// Stable partition of every y list: light x (deg <= d2) first.  nl[y] gets
// the number of light x of y.
void partition_light_first(const Ctx &c, RelIdx &r, int64_t dom_y, int64_t d2, DBuf<int64_t> *nl, int64_t *S) {
    const int64_t n = r.n;
    DBuf<int64_t> lpos = c.buf<int64_t>(n + 1);
    const int32_t *adj = r.adj.get(), *dx = r.dx.get();
    auto light = [=] __device__(int64_t e) -> int64_t { return (int64_t)dx[adj[e]] <= d2 ? 1 : 0; };
    int64_t *lp = lpos.get();
    scan_exclusive(c, n, light, ArrayPut{lp}, lp + n);
    *nl = c.buf<int64_t>(dom_y);
    int64_t *nlp = nl->get();
    const int64_t *of = r.off.get();
    for_each(c, dom_y, [=] __device__(int64_t y) { nlp[y] = lp[of[y + 1]] - lp[of[y]]; });
    DBuf<int32_t> out = c.buf<int32_t>(std::max<int64_t>(n, 1));
    int32_t *o = out.get();
    // y of every tuple: from the offsets by binary search
    const int64_t ndy = dom_y;
    for_each(c, n, [=] __device__(int64_t e) {
        const int64_t y = upper_bound_dev(of, (int64_t)0, ndy, e) - 1;
        const int64_t s0 = of[y];
        const int64_t lb = lp[s0];
        const bool l = light(e) != 0;
        const int64_t li = lp[e] - lb;          // light tuples of y before e
        const int64_t hi = (e - s0) - li;       // heavy tuples of y before e
        const int64_t dst = s0 + (l ? li : nlp[y] + hi);
        o[dst] = adj[e];
    });
    r.adj = std::move(out);
}

// Light witness boxes, k per y (sizes 0 when unused).
constexpr int kMaxStar = 8;
struct BoxArgs {
    const int64_t *boff;  // exclusive offsets of the k * dom_y box sizes (+1)
    int64_t n_box, J_L;
    int k;
    const int64_t *off[kMaxStar];
    const int64_t *nl[kMaxStar];
    const int32_t *adj[kMaxStar];
    const uint8_t *sh;    // star-heavy flag per y
    int s[kMaxStar];      // key = sum of x_i << s[i]
    void *out;
    int64_t *err;
};

// Range (start, length) of relation i's list in box t of y.  Not star-heavy:
// box 0 = N1 x ... x Nk, the others empty.  Star-heavy: box t takes the heavy
// part of the lists before t, the light part of list t, all of the lists
// after t.
__device__ __forceinline__ void box_list(const BoxArgs &a, int64_t y, int t, int i, int64_t *b0, int64_t *bn) {
    const int64_t o = a.off[i][y], d = a.off[i][y + 1] - o, l = a.nl[i][y];
    const bool h = a.sh[y] != 0;
    const int64_t hs = i < t ? o + l : o;
    const int64_t hn = i < t ? d - l : (i == t ? l : d);
    *b0 = h ? hs : o;
    *bn = h ? hn : (t == 0 ? d : 0);
}

// Product of the box's list lengths, saturated at 2^40 (the caller refuses
// joins that large).
__device__ __forceinline__ int64_t box_size(const BoxArgs &a, int64_t y, int t) {
    int64_t p = 1;
    for (int i = 0; i < a.k; ++i) {
        int64_t b0, bn;
        box_list(a, y, t, i, &b0, &bn);
        const int64_t cap = (int64_t)1 << 40;
        p = (bn != 0 && p > cap / bn) ? cap : p * bn;
    }
    return p;
}

template <class K>
__global__ __launch_bounds__(256) void k_star_expand(BoxArgs a) {
    const int64_t o0 = (int64_t)blockIdx.x * 4096;
    const int64_t olast = std::min<int64_t>(o0 + 4096, a.J_L) - 1;
    const int64_t lo = upper_bound_dev(a.boff, (int64_t)0, a.n_box, o0) - 1;
    const int64_t hi = upper_bound_dev(a.boff, lo, a.n_box, olast);
    K *out = reinterpret_cast<K *>(a.out);
    for (int j = 0; j < 16; ++j) {
        const int64_t o = o0 + (int64_t)j * 256 + threadIdx.x;
        if (o <= olast) {
            const int64_t b = upper_bound_dev(a.boff, lo, hi, o) - 1;
            const int64_t y = b / a.k;
            const int t = (int)(b - (int64_t)a.k * y);
            int64_t q = o - a.boff[b];
            K key = 0;
            bool ok = true;
            for (int i = a.k - 1; i >= 0; --i) {  // last list varies fastest
                int64_t b0, bn;
                box_list(a, y, t, i, &b0, &bn);
                ok &= bn > 0;
                const int64_t n1 = bn > 0 ? bn : 1;
                const int64_t idx = q % n1;
                q /= n1;
                key |= (K)(uint32_t)a.adj[i][bn > 0 ? b0 + idx : 0] << a.s[i];
            }
            ok &= q == 0;
            if (!ok) *a.err = 1;
            out[o] = key;
        }
    }
}

}  // namespace

// Heavy product of the star query (bmm.hip).
void star_bmm_keys(const Ctx &c, int k, const int8_t *const *M, const int64_t *u, int64_t ld,
                   const int32_t *const *xof, const int *s, void *keys, bool wide, int64_t cap,
                   unsigned long long *count_dev, bool f16);

namespace {

// Sorts the candidate keys, removes repeats and writes the k id columns.
template <class K>
int64_t star_union(const Ctx &c, int k, K *cand, int64_t total, int bits, const int *shift, const int *bx,
                   const RelIdx *rel, jp_result *res, int64_t *S) {
    DBuf<K> tmp = c.buf<K>(std::max<int64_t>(total, 1));
    const K *s = radix_sort(c, cand, tmp.get(), total, bits);
    struct Unrank {
        const int32_t *xo[kMaxStar];
        int32_t *col[kMaxStar];
        uint64_t n[kMaxStar];
        int sh[kMaxStar];
        uint64_t mask[kMaxStar];
        int k;
    } u;
    for (int i = 0; i < k; ++i) {
        res->cols[i] = c.buf<int32_t>(std::max<int64_t>(total, 1));
        u.xo[i] = rel[i].xorig.get();
        u.col[i] = res->cols[i].get();
        u.n[i] = (uint64_t)rel[i].dom_x;
        u.sh[i] = shift[i];
        u.mask[i] = bx[i] >= 64 ? ~0ull : ((1ull << bx[i]) - 1);
    }
    u.k = k;
    int64_t *err = S + 11;
    c.zero(err, 1);
    compact(
        c, total, [=] __device__(int64_t i) { return i == 0 || s[i] != s[i > 0 ? i - 1 : 0]; },
        [=] __device__(int64_t i, int64_t p) {
            const K kk = s[i];
            bool ok = true;
            for (int t = 0; t < u.k; ++t) {
                const uint64_t r = (uint64_t)(kk >> u.sh[t]) & u.mask[t];
                ok &= r < u.n[t];
                u.col[t][p] = u.xo[t][r < u.n[t] ? r : 0];
            }
            if (!ok) *err = 1;
        },
        S + 12);
    JP_CHECK(c.load(err) == 0, JP_EINTERNAL, "star output key outside the rank tables");
    return c.load(S + 12);
}

}  // namespace

jp_result *run_star(const Ctx &c, int k, const int32_t *const *X, const int32_t *const *Y, const int64_t *N,
                    const jp_options &o) {
    if (k == 2) return run_two_path(c, X[0], Y[0], N[0], X[1], Y[1], N[1], o);
    JP_CHECK(k >= 3 && k <= kMaxStar, JP_EINVAL, "star queries with 2 <= k <= 8 relations are supported");
    const bool timing = (o.flags & JP_FLAG_TIMING) != 0;
    Timeline tl(c, timing);
    const int ev_start = tl.mark();
    auto res = std::make_unique<jp_result>();
    res->alloc = c.alloc;
    res->arity = k;
    jp_stats &st = res->stats;
    std::memset(&st, 0, sizeof(st));
    st.arity = k;
    st.delta1 = st.delta2 = JP_DELTA_INF;
    st.strategy = o.strategy;
    st.dedup = JP_DEDUP_GLOBAL;
    auto finish_empty = [&]() {
        res->n = 0;
        for (int i = 0; i < k; ++i) res->cols[i] = c.buf<int32_t>(1);
        return res.release();
    };
    for (int i = 0; i < k; ++i)
        if (N[i] == 0) return finish_empty();

    DBuf<int64_t> scal = c.buf<int64_t>(32);
    int64_t *S = scal.get();
    // ranges
    DBuf<int> mmb = c.buf<int>(4 * k);
    int *mm = mmb.get();
    for_each(c, 2 * k, [=] __device__(int64_t i) {
        mm[2 * i] = INT_MAX;
        mm[2 * i + 1] = INT_MIN;
    });
    for (int i = 0; i < k; ++i) {
        minmax3(c, X[i], N[i], mm + 4 * i);
        minmax3(c, Y[i], N[i], mm + 4 * i + 2);
    }
    int hmm[4 * kMaxStar];
    c.load_n(hmm, mm, 4 * k);
    int64_t ymin = INT64_MAX, ymax = INT64_MIN;
    int64_t xmin[kMaxStar], xb[kMaxStar];
    for (int i = 0; i < k; ++i) {
        xmin[i] = hmm[4 * i];
        xb[i] = bits_for((uint64_t)((int64_t)hmm[4 * i + 1] - hmm[4 * i]));
        ymin = std::min<int64_t>(ymin, hmm[4 * i + 2]);
        ymax = std::max<int64_t>(ymax, hmm[4 * i + 3]);
    }
    const int yb = bits_for((uint64_t)(ymax - ymin));

    RelRaw raw[kMaxStar];
    for (int i = 0; i < k; ++i) raw[i] = ingest_raw(c, X[i], Y[i], N[i], xmin[i], (int)xb[i], ymin, yb, S);
    // y present in every relation
    DBuf<uint32_t> Yk = c.buf<uint32_t>(std::max<int64_t>(raw[0].ny, 1));
    {
        struct Lists {
            const uint32_t *p[kMaxStar];
            int64_t n[kMaxStar];
            int k;
        } L;
        for (int i = 0; i < k; ++i) {
            L.p[i] = raw[i].ys.get();
            L.n[i] = raw[i].ny;
        }
        L.k = k;
        uint32_t *d = Yk.get();
        compact(
            c, raw[0].ny,
            [=] __device__(int64_t j) {
                const uint32_t v = L.p[0][j];
                bool all = true;
                for (int i = 1; i < L.k; ++i) {
                    const int64_t n = L.n[i];
                    const int64_t p = lower_bound_dev(L.p[i], (int64_t)0, n, v);
                    all &= (p < n) & (L.p[i][p < n ? p : n - 1] == v);
                }
                return all;
            },
            [=] __device__(int64_t j, int64_t p) { d[p] = L.p[0][j]; }, S + 1);
    }
    const int64_t dom_y = c.load(S + 1);
    if (dom_y == 0) return finish_empty();
    RelIdx rel[kMaxStar];
    for (int i = 0; i < k; ++i) {
        rel[i] = finish_rel(c, raw[i], Yk.get(), dom_y, xmin[i], (int)xb[i], S + 2);
        raw[i] = RelRaw();
    }
    // J = sum over y of the product of the k degrees (each term saturated at 2^40)
    BoxArgs ba;
    ba.k = k;
    for (int i = 0; i < k; ++i) {
        ba.off[i] = rel[i].off.get();
        ba.adj[i] = rel[i].adj.get();
    }
    {
        const BoxArgs bb = ba;
        reduce_sum(
            c, dom_y,
            [=] __device__(int64_t y) -> int64_t {
                int64_t p = 1;
                const int64_t cap = (int64_t)1 << 40;
                for (int i = 0; i < bb.k; ++i) {
                    const int64_t d = bb.off[i][y + 1] - bb.off[i][y];
                    p = (d != 0 && p > cap / d) ? cap : p * d;
                }
                return p;
            },
            (unsigned long long *)(S + 3));
    }
    const int64_t J = c.load(S + 3);
    JP_CHECK(J < ((int64_t)1 << 40), JP_ENOMEM, "the star join has 2^40 or more witnesses");
    const int ev_ingest = tl.mark();
    int64_t n_all = 0, Nmax = 0;
    for (int i = 0; i < k; ++i) {
        n_all += rel[i].n;
        Nmax = std::max(Nmax, rel[i].n);
    }
    st.n_r = n_all;
    st.dom_y = dom_y;
    st.dom_x = rel[0].dom_x;
    st.dom_z = rel[k - 1].dom_x;
    st.J = J;

    // thresholds: FIXED or LIGHT_ONLY; otherwise Section 3.2's balance of the
    // three costs N D1^(k-1) = OUT D2 = (N/D2)^k (the product term with
    // omega = 2; its k = 3 example gives D2 = N^(6/16), D1 = N^(7/16) at
    // OUT = N^(3/2)), with OUT estimated as J: D2 = (N^k / J)^(1/(k+1)),
    // D1 = (J D2 / N)^(1/(k-1)).  J <= 20 N: light only (Section 5's switch).
    int64_t d1 = JP_DELTA_INF, d2 = JP_DELTA_INF;
    if (o.strategy == JP_STRATEGY_FIXED) {
        d1 = o.delta1;
        d2 = o.delta2;
    } else if (o.strategy != JP_STRATEGY_LIGHT_ONLY && (double)J > 20.0 * (double)Nmax) {
        const double n = (double)Nmax, jj = (double)J;
        const double t2 = std::pow(std::pow(n, (double)k) / jj, 1.0 / (double)(k + 1));
        const double t1 = std::pow(jj * t2 / n, 1.0 / (double)(k - 1));
        d2 = std::max<int64_t>(1, std::min<int64_t>(Nmax, (int64_t)t2));
        d1 = std::max<int64_t>(1, std::min<int64_t>(Nmax, (int64_t)t1));
    }
    st.delta1 = d1;
    st.delta2 = d2;

    // partition
    DBuf<int64_t> nl[kMaxStar];
    for (int i = 0; i < k; ++i) partition_light_first(c, rel[i], dom_y, d2, &nl[i], S + 4);
    for (int i = 0; i < k; ++i) {
        ba.adj[i] = rel[i].adj.get();  // reordered: light x first per y
        ba.nl[i] = nl[i].get();
    }
    DBuf<uint8_t> sh = c.buf<uint8_t>(dom_y);
    {
        uint8_t *sp = sh.get();
        const BoxArgs bb = ba;
        const int64_t dd1 = d1;
        for_each(c, dom_y, [=] __device__(int64_t y) {
            int hcnt = 0;
            for (int i = 0; i < bb.k; ++i) hcnt += (int)((bb.off[i][y + 1] - bb.off[i][y]) > dd1);
            sp[y] = hcnt >= 2 ? 1 : 0;
        });
    }
    ba.sh = sh.get();
    // heavy ids of the x_i and of the star-heavy y
    int64_t u[kMaxStar] = {0}, v = 0;
    DBuf<int32_t> hid[kMaxStar], xof[kMaxStar];
    DBuf<int32_t> hy = c.buf<int32_t>(dom_y);
    const bool any_heavy = d2 != JP_DELTA_INF;
    if (any_heavy) {
        for (int i = 0; i < k; ++i) {
            const int64_t nx = rel[i].dom_x;
            hid[i] = c.buf<int32_t>(nx);
            xof[i] = c.buf<int32_t>(nx);
            int32_t *h = hid[i].get(), *xo = xof[i].get();
            const int32_t *dx = rel[i].dx.get();
            for_each(c, nx, [=] __device__(int64_t x) { h[x] = -1; });
            compact(
                c, nx, [=] __device__(int64_t x) { return (int64_t)dx[x] > d2; },
                [=] __device__(int64_t x, int64_t p) {
                    h[x] = (int32_t)p;
                    xo[p] = (int32_t)x;
                },
                S + 13 + i);
        }
        int32_t *hyp = hy.get();
        const uint8_t *sp = sh.get();
        for_each(c, dom_y, [=] __device__(int64_t y) { hyp[y] = -1; });
        compact(
            c, dom_y, [=] __device__(int64_t y) { return sp[y] != 0; },
            [=] __device__(int64_t y, int64_t p) { hyp[y] = (int32_t)p; }, S + 21);
        int64_t hv[kMaxStar + 1];
        c.load_n(hv, S + 13, (size_t)kMaxStar + 1);
        for (int i = 0; i < k; ++i) u[i] = hv[i];
        v = hv[kMaxStar];
    }
    bool has_heavy = v > 0;
    double rows_v = 1, rows_w = 1;
    const int g = (k + 1) / 2;
    for (int i = 0; i < k; ++i) {
        has_heavy &= u[i] > 0;
        (i < g ? rows_v : rows_w) *= (double)u[i];
    }
    st.u = (int64_t)std::min(rows_v, 9.2e18);
    st.v = v;
    st.w = (int64_t)std::min(rows_w, 9.2e18);

    // light boxes
    DBuf<int64_t> boff = c.buf<int64_t>(k * dom_y + 1);
    {
        const BoxArgs bb = ba;
        int64_t *bo = boff.get();
        scan_exclusive(
            c, k * dom_y,
            [=] __device__(int64_t b) -> int64_t {
                const int64_t y = b / bb.k;
                return box_size(bb, y, (int)(b - (int64_t)bb.k * y));
            },
            ArrayPut{bo}, bo + k * dom_y);
    }
    const int64_t J_L = c.load(boff.get() + k * dom_y);
    JP_CHECK(J_L >= 0 && J_L <= J, JP_EINTERNAL, "light witness count exceeds the join size");
    const int64_t J_H = J - J_L;
    JP_CHECK(has_heavy || J_H == 0, JP_EINTERNAL, "heavy witnesses without a heavy part");
    st.J_L = J_L;
    st.J_H = J_H;
    const int ev_plan = tl.mark();

    int bxs[kMaxStar], shift[kMaxStar];
    int bits = 0;
    for (int i = k - 1; i >= 0; --i) {
        bxs[i] = rel[i].bx;
        shift[i] = bits;
        bits += rel[i].bx;
    }
    JP_CHECK(bits <= 128, JP_EINVAL, "the star output's rank widths need more than 128 bits");
    const bool wide = bits > 64;
    for (int i = 0; i < k; ++i) ba.s[i] = shift[i];
    const size_t ksz = wide ? sizeof(u128) : sizeof(uint64_t);
    const int64_t cap_h = has_heavy ? (int64_t)std::min<double>((double)J_H, rows_v * rows_w) : 0;
    const int64_t cap = J_L + cap_h;
    DBuf<uint8_t> cand = c.buf<uint8_t>((size_t)std::max<int64_t>(cap, 1) * ksz);
    if (J_L > 0) {
        ba.boff = boff.get();
        ba.n_box = k * dom_y;
        ba.J_L = J_L;
        ba.out = cand.get();
        ba.err = S + 9;
        c.zero(S + 9, 1);
        const int64_t blocks = ceil_div(J_L, 4096);
        if (wide)
            hipLaunchKernelGGL(k_star_expand<u128>, dim3(grid_x(blocks, 256)), dim3(256), 0, c.stream, ba);
        else
            hipLaunchKernelGGL(k_star_expand<uint64_t>, dim3(grid_x(blocks, 256)), dim3(256), 0, c.stream, ba);
        JP_HIP(hipGetLastError());
        JP_CHECK(c.load(S + 9) == 0, JP_EINTERNAL, "star expansion index outside its box");
    }
    const int ev_light = tl.mark();
    int64_t nnz = 0;
    int ev_b0 = ev_light, ev_b1 = ev_light;
    if (has_heavy) {
        JP_CHECK(o.bmm != JP_BMM_F16 || v < (int64_t(1) << 24), JP_EPRECISION,
                 "fp16 product: counts may reach 2^24 (heavy y), beyond fp32's exact range");
        const int64_t ld = ceil_div(v, kBmmPadK) * kBmmPadK;
        DBuf<int8_t> M[kMaxStar];
        const int8_t *Mp[kMaxStar];
        const int32_t *xp[kMaxStar];
        for (int i = 0; i < k; ++i) {
            M[i] = c.buf<int8_t>((size_t)(u[i] * ld));
            c.zero(M[i].get(), (size_t)(u[i] * ld));
            int8_t *m = M[i].get();
            const int64_t *of = rel[i].off.get();
            const int32_t *adj = rel[i].adj.get(), *h = hid[i].get(), *hyp = hy.get();
            const int64_t ldl = ld, ndy = dom_y;
            for_each(c, rel[i].n, [=] __device__(int64_t e) {
                const int64_t y = upper_bound_dev(of, (int64_t)0, ndy, e) - 1;
                const int32_t a = h[adj[e]], b = hyp[y];
                if ((a >= 0) & (b >= 0)) m[(int64_t)(a >= 0 ? a : 0) * ldl + (b >= 0 ? b : 0)] = 1;
            });
            Mp[i] = M[i].get();
            xp[i] = xof[i].get();
        }
        ev_b0 = tl.mark();
        star_bmm_keys(c, k, Mp, u, ld, xp, shift, cand.get() + (size_t)J_L * ksz, wide, cap_h,
                      (unsigned long long *)(S + 10), o.bmm == JP_BMM_F16);
        ev_b1 = tl.mark();
        nnz = c.load(S + 10);
        JP_CHECK(nnz <= cap_h, JP_EINTERNAL, "star heavy product produced more nonzeros than its bound");
        st.bmm = o.bmm == JP_BMM_F16 ? JP_BMM_F16 : JP_BMM_I8_MFMA;
        st.bmm_ops = 2.0 * rows_v * (double)v * rows_w;
    }
    st.nnz_heavy = nnz;
    const int ev_heavy = tl.mark();

    // union + duplicate removal + unrank
    const int64_t total = J_L + nnz;
    res->n = wide ? star_union<u128>(c, k, (u128 *)cand.get(), total, bits, shift, bxs, rel, res.get(), S)
                  : star_union<uint64_t>(c, k, (uint64_t *)cand.get(), total, bits, shift, bxs, rel, res.get(), S);
    st.n_out = res->n;
    const int ev_end = tl.mark();
    if (timing) {
        st.ms_ingest = tl.ms(ev_start, ev_ingest);
        st.ms_plan = tl.ms(ev_ingest, ev_plan);
        st.ms_light = tl.ms(ev_plan, ev_light);
        st.ms_heavy = tl.ms(ev_light, ev_heavy);
        st.ms_bmm = tl.ms(ev_b0, ev_b1);
        st.ms_dedup = tl.ms(ev_heavy, ev_end);
        st.ms_total = tl.ms(ev_start, ev_end);
    }
    return res.release();
}

}  // namespace jp
