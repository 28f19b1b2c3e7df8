// Star join-project Q*_3(x1,x2,x3) = R1(x1,y), R2(x2,y), R3(x3,y)
// (Section 3.2).  k = 2 is the two-path query and goes to run_two_path.
//
//  ingest     every relation becomes a set indexed by y; y missing from any
//             relation is dropped; y and each x_i get dense ranks; degrees.
//  partition  x_i heavy iff deg_i(x_i) > Delta2.  A tuple (a, b) of R_i is in
//             R_i^- when a is light, in R_i^diamond when b has degree
//             <= Delta1 in every other relation, in R_i^+ otherwise.  A
//             witness (a1, a2, a3, b) is heavy iff all three tuples are in
//             R_i^+, i.e. every a_i is heavy and b is heavy (degree > Delta1)
//             in at least two relations ("star-heavy").
//  light      per y, the witness box N1 x N2 x N3 when y is not star-heavy,
//             else the box minus H1 x H2 x H3, written as the disjoint boxes
//             L1 x N2 x N3, H1 x L2 x N3, H1 x H2 x L3 over lists that hold
//             light x first; every box is enumerated into packed keys
//             x1 << (b2+b3) | x2 << b3 | x3 with the output index space cut
//             evenly across workgroups.
//  heavy      C[(a1,a2), a3] = sum_b M1[a1,b] M2[a2,b] M3[a3,b] over heavy a_i
//             and star-heavy b: the product V x W^T of Section 3.2 with V's
//             rows (a1, a2) generated on the fly as M1[a1,:] AND M2[a2,:]
//             (V is never stored); nonzeros become keys.
//  union      one radix sort of light + heavy keys (64-bit, or 128-bit when
//             the three rank widths exceed 64 bits), unique, unrank.
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

// Light witness boxes, three per y (sizes 0 when unused).
struct BoxArgs {
    const int64_t *boff;  // exclusive offsets of the 3 * dom_y box sizes (+1)
    int64_t n_box, J_L;
    const int64_t *off1, *off2, *off3;
    const int64_t *nl1, *nl2, *nl3;
    const uint8_t *sh;    // star-heavy flag per y
    const int32_t *adj1, *adj2, *adj3;
    int s1, s2;           // shifts: key = x1 << s1 | x2 << s2 | x3
    void *out;
    int wide;             // 1: 128-bit keys
    int64_t *err;
};

// Ranges (start, length) of the three lists of box t of y.
__device__ __forceinline__ void box_ranges(const BoxArgs &a, int64_t y, int t, int64_t *A0, int64_t *An, int64_t *B0,
                                           int64_t *Bn, int64_t *C0, int64_t *Cn) {
    const int64_t o1 = a.off1[y], d1 = a.off1[y + 1] - o1, l1 = a.nl1[y];
    const int64_t o2 = a.off2[y], d2 = a.off2[y + 1] - o2, l2 = a.nl2[y];
    const int64_t o3 = a.off3[y], d3 = a.off3[y + 1] - o3, l3 = a.nl3[y];
    const bool h = a.sh[y] != 0;
    // not star-heavy: box 0 = N1 x N2 x N3.  Star-heavy: box 0 = L1 x N2 x N3,
    // box 1 = H1 x L2 x N3, box 2 = H1 x H2 x L3.
    const bool t0 = t == 0, t1 = t == 1, t2 = t == 2;
    *A0 = t0 ? o1 : o1 + l1;
    *An = t0 ? (h ? l1 : d1) : (h ? d1 - l1 : 0);
    *B0 = t2 ? o2 + l2 : o2;
    *Bn = t0 ? d2 : (t1 ? l2 : d2 - l2);
    *C0 = o3;
    *Cn = t2 ? l3 : d3;
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
            const int64_t y = b / 3;
            const int t = (int)(b - 3 * y);
            int64_t A0, An, B0, Bn, C0, Cn;
            box_ranges(a, y, t, &A0, &An, &B0, &Bn, &C0, &Cn);
            int64_t q = o - a.boff[b];
            const bool ok = (An > 0) & (Bn > 0) & (Cn > 0) & (q < An * Bn * Cn);
            if (!ok) *a.err = 1;
            const int64_t cn = Cn > 0 ? Cn : 1, bn = Bn > 0 ? Bn : 1;
            const int64_t ci = q % cn;
            q /= cn;
            const int64_t bi = q % bn;
            const int64_t ai = q / bn;
            const int32_t x1 = a.adj1[ok ? A0 + ai : 0];
            const int32_t x2 = a.adj2[ok ? B0 + bi : 0];
            const int32_t x3 = a.adj3[ok ? C0 + ci : 0];
            out[o] = ((K)(uint32_t)x1 << a.s1) | ((K)(uint32_t)x2 << a.s2) | (K)(uint32_t)x3;
        }
    }
}

}  // namespace

// Heavy product of the star query (bmm.hip).
void star_bmm_keys(const Ctx &c, const int8_t *M1, const int8_t *M2, const int8_t *M3, int64_t u1, int64_t u2,
                   int64_t u3, int64_t ld, const int32_t *x1_of, const int32_t *x2_of, const int32_t *x3_of, int s1,
                   int s2, void *keys, bool wide, int64_t cap, unsigned long long *count_dev);

jp_result *run_star(const Ctx &c, int k, const int32_t *const *X, const int32_t *const *Y, const int64_t *N,
                    const jp_options &o) {
    if (k == 2) return run_two_path(c, X[0], Y[0], N[0], X[1], Y[1], N[1], o);
    JP_CHECK(k == 3, JP_EINVAL, "star queries with k = 2 or 3 are supported");
    const bool timing = (o.flags & JP_FLAG_TIMING) != 0;
    Timeline tl(c, timing);
    const int ev_start = tl.mark();
    auto res = std::make_unique<jp_result>();
    res->alloc = c.alloc;
    res->arity = 3;
    jp_stats &st = res->stats;
    std::memset(&st, 0, sizeof(st));
    st.arity = 3;
    st.delta1 = st.delta2 = JP_DELTA_INF;
    st.strategy = o.strategy;
    st.dedup = JP_DEDUP_GLOBAL;
    auto finish_empty = [&]() {
        res->n = 0;
        for (int i = 0; i < 3; ++i) res->cols[i] = c.buf<int32_t>(1);
        return res.release();
    };
    for (int i = 0; i < 3; ++i)
        if (N[i] == 0) return finish_empty();

    DBuf<int64_t> scal = c.buf<int64_t>(32);
    int64_t *S = scal.get();
    // ranges
    DBuf<int> mmb = c.buf<int>(12);
    int *mm = mmb.get();
    for_each(c, 6, [=] __device__(int64_t i) {
        mm[2 * i] = INT_MAX;
        mm[2 * i + 1] = INT_MIN;
    });
    for (int i = 0; i < 3; ++i) {
        minmax3(c, X[i], N[i], mm + 4 * i);
        minmax3(c, Y[i], N[i], mm + 4 * i + 2);
    }
    int hmm[12];
    c.load_n(hmm, mm, 12);
    int64_t ymin = INT64_MAX, ymax = INT64_MIN;
    int64_t xmin[3], xb[3];
    for (int i = 0; i < 3; ++i) {
        xmin[i] = hmm[4 * i];
        xb[i] = bits_for((uint64_t)((int64_t)hmm[4 * i + 1] - hmm[4 * i]));
        ymin = std::min<int64_t>(ymin, hmm[4 * i + 2]);
        ymax = std::max<int64_t>(ymax, hmm[4 * i + 3]);
    }
    const int yb = bits_for((uint64_t)(ymax - ymin));

    RelRaw raw[3];
    for (int i = 0; i < 3; ++i) raw[i] = ingest_raw(c, X[i], Y[i], N[i], xmin[i], (int)xb[i], ymin, yb, S);
    // y present in all three
    DBuf<uint32_t> Yk = c.buf<uint32_t>(std::max<int64_t>(raw[0].ny, 1));
    {
        const uint32_t *y0 = raw[0].ys.get(), *y1 = raw[1].ys.get(), *y2 = raw[2].ys.get();
        const int64_t n1 = raw[1].ny, n2 = raw[2].ny;
        uint32_t *d = Yk.get();
        auto in = [=] __device__(const uint32_t *a, int64_t n, uint32_t v) -> bool {
            const int64_t p = lower_bound_dev(a, (int64_t)0, n, v);
            const int64_t q = p < n ? p : n - 1;
            return (p < n) & (a[q] == v);
        };
        compact(
            c, raw[0].ny, [=] __device__(int64_t j) { return (int)in(y1, n1, y0[j]) & (int)in(y2, n2, y0[j]); },
            [=] __device__(int64_t j, int64_t p) { d[p] = y0[j]; }, S + 1);
    }
    const int64_t dom_y = c.load(S + 1);
    if (dom_y == 0) return finish_empty();
    RelIdx rel[3];
    for (int i = 0; i < 3; ++i) {
        rel[i] = finish_rel(c, raw[i], Yk.get(), dom_y, xmin[i], (int)xb[i], S + 2);
        raw[i] = RelRaw();
    }
    // J = sum over y of d1 d2 d3
    {
        const int64_t *o1 = rel[0].off.get(), *o2 = rel[1].off.get(), *o3 = rel[2].off.get();
        reduce_sum(
            c, dom_y,
            [=] __device__(int64_t y) -> int64_t {
                return (o1[y + 1] - o1[y]) * (o2[y + 1] - o2[y]) * (o3[y + 1] - o3[y]);
            },
            (unsigned long long *)(S + 3));
    }
    const int64_t J = c.load(S + 3);
    const int ev_ingest = tl.mark();
    st.n_r = rel[0].n + rel[1].n + rel[2].n;
    st.dom_y = dom_y;
    st.dom_x = rel[0].dom_x;
    st.dom_z = rel[2].dom_x;
    st.J = J;

    // thresholds: FIXED or LIGHT_ONLY; otherwise the k = 3 analysis of
    // Section 3.2 balances N D1^2 = OUT D2 = (N/D2)^3 (its example gives
    // D2 = N^(6/16), D1 = N^(7/16) at OUT = N^(3/2)); with OUT estimated as J
    // this is D2 = (N^3 / J)^(1/4), D1 = sqrt(J D2 / N).
    int64_t d1 = JP_DELTA_INF, d2 = JP_DELTA_INF;
    const int64_t Nmax = std::max(rel[0].n, std::max(rel[1].n, rel[2].n));
    if (o.strategy == JP_STRATEGY_FIXED) {
        d1 = o.delta1;
        d2 = o.delta2;
    } else if (o.strategy != JP_STRATEGY_LIGHT_ONLY && (double)J > 20.0 * (double)Nmax) {
        const double n = (double)Nmax, jj = (double)J;
        const double t2 = std::pow(n * n * n / jj, 0.25);
        const double t1 = std::sqrt(jj * t2 / n);
        d2 = std::max<int64_t>(1, std::min<int64_t>(Nmax, (int64_t)t2));
        d1 = std::max<int64_t>(1, std::min<int64_t>(Nmax, (int64_t)t1));
    }
    st.delta1 = d1;
    st.delta2 = d2;

    // partition
    DBuf<int64_t> nl[3];
    for (int i = 0; i < 3; ++i) partition_light_first(c, rel[i], dom_y, d2, &nl[i], S + 4);
    DBuf<uint8_t> sh = c.buf<uint8_t>(dom_y);
    {
        uint8_t *s = sh.get();
        const int64_t *o1 = rel[0].off.get(), *o2 = rel[1].off.get(), *o3 = rel[2].off.get();
        const int64_t dd1 = d1;
        for_each(c, dom_y, [=] __device__(int64_t y) {
            const int hcnt = (int)((o1[y + 1] - o1[y]) > dd1) + (int)((o2[y + 1] - o2[y]) > dd1) +
                             (int)((o3[y + 1] - o3[y]) > dd1);
            s[y] = hcnt >= 2 ? 1 : 0;
        });
    }
    // heavy ids of x_i and of star-heavy y
    int64_t u[3] = {0, 0, 0}, v = 0;
    DBuf<int32_t> hid[3], xof[3];
    DBuf<int32_t> hy = c.buf<int32_t>(dom_y);
    const bool any_heavy = d2 != JP_DELTA_INF;
    if (any_heavy) {
        for (int i = 0; i < 3; ++i) {
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
                S + 5 + i);
        }
        int32_t *hyp = hy.get();
        const uint8_t *s = sh.get();
        for_each(c, dom_y, [=] __device__(int64_t y) { hyp[y] = -1; });
        compact(
            c, dom_y, [=] __device__(int64_t y) { return s[y] != 0; },
            [=] __device__(int64_t y, int64_t p) { hyp[y] = (int32_t)p; }, S + 8);
        int64_t h4[4];
        c.load_n(h4, S + 5, 4);
        u[0] = h4[0];
        u[1] = h4[1];
        u[2] = h4[2];
        v = h4[3];
    }
    const bool has_heavy = u[0] > 0 && u[1] > 0 && u[2] > 0 && v > 0;
    st.u = u[0] * u[1];
    st.v = v;
    st.w = u[2];

    // light boxes
    DBuf<int64_t> boff = c.buf<int64_t>(3 * dom_y + 1);
    BoxArgs ba;
    ba.off1 = rel[0].off.get();
    ba.off2 = rel[1].off.get();
    ba.off3 = rel[2].off.get();
    ba.nl1 = nl[0].get();
    ba.nl2 = nl[1].get();
    ba.nl3 = nl[2].get();
    ba.sh = sh.get();
    ba.adj1 = rel[0].adj.get();
    ba.adj2 = rel[1].adj.get();
    ba.adj3 = rel[2].adj.get();
    {
        const BoxArgs bb = ba;
        int64_t *bo = boff.get();
        scan_exclusive(
            c, 3 * dom_y,
            [=] __device__(int64_t b) -> int64_t {
                const int64_t y = b / 3;
                int64_t A0, An, B0, Bn, C0, Cn;
                box_ranges(bb, y, (int)(b - 3 * y), &A0, &An, &B0, &Bn, &C0, &Cn);
                return An * Bn * Cn;
            },
            ArrayPut{bo}, bo + 3 * dom_y);
    }
    const int64_t J_L = c.load(boff.get() + 3 * dom_y);
    JP_CHECK(J_L >= 0 && J_L <= J, JP_EINTERNAL, "light witness count exceeds the join size");
    const int64_t J_H = J - J_L;
    JP_CHECK(has_heavy || J_H == 0, JP_EINTERNAL, "heavy witnesses without a heavy part");
    st.J_L = J_L;
    st.J_H = J_H;
    const int ev_plan = tl.mark();

    const int b1 = rel[0].bx, b2 = rel[1].bx, b3 = rel[2].bx;
    const int bits = b1 + b2 + b3;
    const bool wide = bits > 64;
    const int s1 = b2 + b3, s2 = b3;
    const size_t ksz = wide ? sizeof(u128) : sizeof(uint64_t);
    const int64_t cap = J_L + J_H;
    DBuf<uint8_t> cand = c.buf<uint8_t>((size_t)std::max<int64_t>(cap, 1) * ksz);
    if (J_L > 0) {
        ba.boff = boff.get();
        ba.n_box = 3 * dom_y;
        ba.J_L = J_L;
        ba.s1 = s1;
        ba.s2 = s2;
        ba.out = cand.get();
        ba.wide = wide;
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
        const int64_t ld = ceil_div(v, kBmmPadK) * kBmmPadK;
        DBuf<int8_t> M[3];
        for (int i = 0; i < 3; ++i) {
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
        }
        ev_b0 = tl.mark();
        star_bmm_keys(c, M[0].get(), M[1].get(), M[2].get(), u[0], u[1], u[2], ld, xof[0].get(), xof[1].get(),
                      xof[2].get(), s1, s2, cand.get() + (size_t)J_L * ksz, wide, J_H,
                      (unsigned long long *)(S + 10));
        ev_b1 = tl.mark();
        nnz = c.load(S + 10);
        JP_CHECK(nnz <= J_H, JP_EINTERNAL, "star heavy product produced more nonzeros than its bound");
        st.bmm = JP_BMM_I8_MFMA;
        st.bmm_ops = 2.0 * (double)u[0] * (double)u[1] * (double)v * (double)u[2];
    }
    st.nnz_heavy = nnz;
    const int ev_heavy = tl.mark();

    // union + duplicate removal + unrank
    const int64_t total = J_L + nnz;
    DBuf<uint8_t> tmp = c.buf<uint8_t>((size_t)std::max<int64_t>(total, 1) * ksz);
    for (int i = 0; i < 3; ++i) res->cols[i] = c.buf<int32_t>(std::max<int64_t>(total, 1));
    int32_t *c0 = res->cols[0].get(), *c1 = res->cols[1].get(), *c2 = res->cols[2].get();
    const int32_t *xo0 = rel[0].xorig.get(), *xo1 = rel[1].xorig.get(), *xo2 = rel[2].xorig.get();
    const uint64_t m2 = (1ull << b2) - 1, m3 = (1ull << b3) - 1;
    const int64_t n0 = rel[0].dom_x, n1 = rel[1].dom_x, n2 = rel[2].dom_x;
    int64_t *err = S + 11;
    c.zero(err, 1);
    if (wide) {
        const u128 *s = radix_sort(c, (u128 *)cand.get(), (u128 *)tmp.get(), total, bits);
        compact(
            c, total, [=] __device__(int64_t i) { return i == 0 || s[i] != s[i - 1]; },
            [=] __device__(int64_t i, int64_t p) {
                const u128 kk = s[i];
                const uint64_t a = (uint64_t)(kk >> s1), b = (uint64_t)(kk >> s2) & m2, cc = (uint64_t)kk & m3;
                const bool ok = (a < (uint64_t)n0) & (b < (uint64_t)n1) & (cc < (uint64_t)n2);
                if (!ok) *err = 1;
                c0[p] = xo0[ok ? a : 0];
                c1[p] = xo1[ok ? b : 0];
                c2[p] = xo2[ok ? cc : 0];
            },
            S + 12);
    } else {
        const uint64_t *s = radix_sort(c, (uint64_t *)cand.get(), (uint64_t *)tmp.get(), total, bits);
        compact(
            c, total, [=] __device__(int64_t i) { return i == 0 || s[i] != s[i - 1]; },
            [=] __device__(int64_t i, int64_t p) {
                const uint64_t kk = s[i];
                const uint64_t a = kk >> s1, b = (kk >> s2) & m2, cc = kk & m3;
                const bool ok = (a < (uint64_t)n0) & (b < (uint64_t)n1) & (cc < (uint64_t)n2);
                if (!ok) *err = 1;
                c0[p] = xo0[ok ? a : 0];
                c1[p] = xo1[ok ? b : 0];
                c2[p] = xo2[ok ? cc : 0];
            },
            S + 12);
    }
    JP_CHECK(c.load(err) == 0, JP_EINTERNAL, "star output key outside the rank tables");
    res->n = c.load(S + 12);
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
