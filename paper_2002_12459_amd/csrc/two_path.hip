// Two-path join-project Q(x,z) = R(x,y), S(z,y) (Algorithm 1, Section 3.1).
//
//  ingest     relations become sets (duplicate rows dropped), tuples whose y
//             is missing from the other relation are dropped, ids get dense
//             order-preserving ranks, R is indexed x-major and S y-major
//             (Section 5, "Indexing relations"), degrees and J are computed.
//  plan       thresholds (Delta1, Delta2) from the planner.
//  partition  x heavy iff deg_R(x) > Delta2, z heavy iff deg_S(z) > Delta2,
//             y heavy iff its key degree > Delta1 (one y classification shared
//             by R and S).  Light witnesses are exactly the disjoint classes
//             (R^- join S) and (R^+ join S^-): an R tuple with light x or
//             light y meets all of N_S(y); a heavy R tuple meets only the
//             light z of N_S(y).
//  light      per R tuple, its witness list is expanded into packed keys
//             (x_rank << bz | z_rank); the output index space is cut evenly
//             across workgroups.
//  heavy      M1 (heavy x by heavy y) and M2^T (heavy z by heavy y) as int8,
//             their 0/1 product's nonzeros appended as keys.
//  union      one radix sort of light + heavy keys over the significant bits,
//             then unique + unrank into the sorted distinct output.
#include <climits>

#include "debug.hpp"
#include "pipeline.hpp"
#include "prims.hpp"
#include "segdedup.hpp"

namespace jp {
namespace {

// min / max of four int32 columns (R x, R y, S z, S y); grid.y selects the
// column, kMinMaxVec 16-byte loads per thread per step.  Each workgroup
// writes its pair to part[(column * gridDim.x + block) * 2]; k_minmax_fold
// reduces them into out[8] (device-scope atomics on one cache line would be
// serialised, about 11 ns each).
constexpr int kMinMaxVec = 4;
__global__ __launch_bounds__(256) void k_minmax4(const int32_t *c0, const int32_t *c1, int64_t n01, const int32_t *c2,
                                                 const int32_t *c3, int64_t n23, int *part) {
    __shared__ int smn[256 / kWave], smx[256 / kWave];
    const int k = blockIdx.y;
    const int32_t *a = k == 0 ? c0 : (k == 1 ? c1 : (k == 2 ? c2 : c3));
    const int64_t n = k < 2 ? n01 : n23;
    int mn = INT_MAX, mx = INT_MIN;
    // aligned body as int4, the rest one by one
    const int64_t head = std::min<int64_t>(n, (int64_t)((16 - ((uintptr_t)a & 15)) & 15) / 4);
    const int64_t nv = (n - head) / 4;
    const int4 *v = (const int4 *)(a + head);
    const int64_t stride = (int64_t)gridDim.x * 256 * kMinMaxVec;
    for (int64_t i0 = (int64_t)blockIdx.x * 256 * kMinMaxVec + threadIdx.x; i0 < nv; i0 += stride) {
        int4 q[kMinMaxVec];
#pragma unroll
        for (int r = 0; r < kMinMaxVec; ++r) {  // all loads in flight at once
            const int64_t i = i0 + (int64_t)r * 256;
            q[r] = v[i < nv ? i : i0];
        }
#pragma unroll
        for (int r = 0; r < kMinMaxVec; ++r) {
            mn = min(mn, min(min(q[r].x, q[r].y), min(q[r].z, q[r].w)));
            mx = max(mx, max(max(q[r].x, q[r].y), max(q[r].z, q[r].w)));
        }
    }
    const int64_t tail0 = head + 4 * nv, nrest = head + (n - tail0);  // at most 6 values
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < nrest; r += stride) {
        const int t = a[r < head ? r : tail0 + (r - head)];
        mn = t < mn ? t : mn;
        mx = t > mx ? t : mx;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        int a2 = __shfl_xor(mn, o), b2 = __shfl_xor(mx, o);
        mn = a2 < mn ? a2 : mn;
        mx = b2 > mx ? b2 : mx;
    }
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
        smn[w] = mn;
        smx[w] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 256 / kWave; ++i) {
            mn = smn[i] < mn ? smn[i] : mn;
            mx = smx[i] > mx ? smx[i] : mx;
        }
        int *p = part + ((int64_t)k * gridDim.x + blockIdx.x) * 2;
        p[0] = mn;
        p[1] = mx;
    }
}

// One wave per column: min and max over the workgroup pairs.
__global__ __launch_bounds__(256) void k_minmax_fold(const int *part, int64_t nblk, int *out) {
    const int k = threadIdx.x / kWave;
    int mn = INT_MAX, mx = INT_MIN;
    for (int64_t b = lane_id(); b < nblk; b += kWave) {
        const int *p = part + ((int64_t)k * nblk + b) * 2;
        mn = p[0] < mn ? p[0] : mn;
        mx = p[1] > mx ? p[1] : mx;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        int a2 = __shfl_xor(mn, o), b2 = __shfl_xor(mx, o);
        mn = a2 < mn ? a2 : mn;
        mx = b2 > mx ? b2 : mx;
    }
    if (lane_id() == 0) {
        out[2 * k] = mn;
        out[2 * k + 1] = mx;
    }
}

void minmax4(const Ctx &c, const int32_t *rx, const int32_t *ry, int64_t nr, const int32_t *sz, const int32_t *sy,
             int64_t ns, int *out) {
    const int64_t n = std::max<int64_t>(std::max(nr, ns), 1);
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256 * 4 * kMinMaxVec), (int64_t)c.num_cus * 4));
    DBuf<int> part = c.buf<int>((size_t)(8 * blocks));
    hipLaunchKernelGGL(k_minmax4, dim3(grid_x(blocks, 256), 4), dim3(256), 0, c.stream, rx, ry, nr, sz, sy, ns, part.get());
    JP_HIP(hipGetLastError());
    static_assert(256 / kWave == 4, "one wave per column");
    hipLaunchKernelGGL(k_minmax_fold, dim3(1), dim3(256), 0, c.stream, (const int *)part.get(), blocks, out);
    JP_HIP(hipGetLastError());
}

// Light witness expansion.  Block b produces outputs [b*4096, b*4096+4096);
// each output index finds its R tuple by binary search in the tuple offsets
// and reads z from that tuple's list.  All lists live in one array: N_S(y)
// for every y (the y-major S), followed by the light-z part of N_S(y) for
// every heavy y; `lbase` holds each tuple's list start, so the kernel has no
// data-dependent choice of array.  Consecutive lanes read consecutive list
// entries and write consecutive keys.
constexpr int kExpBlock = 256;
constexpr int kExpItems = 16;
constexpr int64_t kExpTile = kExpBlock * kExpItems;

struct ExpandArgs {
    const int64_t *eoff;   // exclusive offsets of the per-tuple witness counts (n_e + 1)
    int64_t n_e, J_L;
    const int32_t *r_xr;   // x rank of each R tuple
    const int64_t *lbase;  // start of each tuple's list in zlist
    const int32_t *zlist;  // concatenated z-rank lists
    int64_t zlist_n;
    int bz;
    int wshift;            // > 0: key = (pair << wshift) | 1 (a counted witness of weight 1)
    void *out;             // K keys
    int64_t *err;          // set when an index falls outside zlist
};

template <class K>
__global__ __launch_bounds__(kExpBlock) void k_light_expand(ExpandArgs a) {
    const int64_t o0 = (int64_t)blockIdx.x * kExpTile;
    const int64_t olast = std::min<int64_t>(o0 + kExpTile, a.J_L) - 1;
    const int64_t lo = upper_bound_dev(a.eoff, (int64_t)0, a.n_e, o0) - 1;
    const int64_t hi = upper_bound_dev(a.eoff, lo, a.n_e, olast);
    for (int j = 0; j < kExpItems; ++j) {
        const int64_t o = o0 + (int64_t)j * kExpBlock + threadIdx.x;
        if (o <= olast) {
            const int64_t e = upper_bound_dev(a.eoff, lo, hi, o) - 1;
            const int64_t idx = a.lbase[e] + (o - a.eoff[e]);
            const bool ok = idx >= 0 && idx < a.zlist_n;
            const int32_t z = a.zlist[ok ? idx : 0];
            if (!ok) *a.err = 1;
            const K pair = ((K)(uint32_t)a.r_xr[e] << a.bz) | (K)(uint32_t)z;
            reinterpret_cast<K *>(a.out)[o] = a.wshift ? ((pair << a.wshift) | (K)1) : pair;
        }
    }
}

}  // namespace

// Dense id-indexed tables are used when an id range is at most a few times
// the input size (and at most 2^26 entries).
static bool dense_range_ok(int64_t span, int64_t n) { return span <= (1ll << 26) && span <= 4 * n + (1ll << 20); }

// Returns false when the instance has no output (no common y).
static bool ingest_two_path(const Ctx &c, const int32_t *rx, const int32_t *ry, int64_t nr, const int32_t *sz,
                            const int32_t *sy, int64_t ns, Ingest &g, int64_t *S) {
    // ---- ranges of the id columns --------------------------------------------
    DBuf<int> mmb = c.buf<int>(8);
    int *mm = mmb.get();
    minmax4(c, rx, ry, nr, sz, sy, ns, mm);
    int hmm[8];
    c.load_n(hmm, mm, 8);
    const int64_t xmin = hmm[0], xmax = hmm[1], zmin = hmm[4], zmax = hmm[5];
    const int64_t ymin = std::min(hmm[2], hmm[6]), ymax = std::max(hmm[3], hmm[7]);
    const int xb = bits_for((uint64_t)(xmax - xmin)), yb = bits_for((uint64_t)(ymax - ymin));
    const int zb = bits_for((uint64_t)(zmax - zmin));
    const uint64_t ymask = yb >= 64 ? ~0ull : ((1ull << yb) - 1), zmask = (1ull << zb) - 1;

    // ---- R: distinct tuples, x-major ----------------------------------------
    DBuf<uint64_t> r1;
    {
        DBuf<uint64_t> ka = c.buf<uint64_t>(nr), kb = c.buf<uint64_t>(nr);
        const uint64_t *s = radix_sort_from<uint64_t>(
            c,
            [=] __device__(int64_t i) {
                return ((uint64_t)((int64_t)rx[i] - xmin) << yb) | (uint64_t)((int64_t)ry[i] - ymin);
            },
            ka.get(), kb.get(), nr, xb + yb);
        r1 = c.buf<uint64_t>(nr);
        uint64_t *d = r1.get();
        compact_v(
            c, nr,
            [=] __device__(int64_t i) {
                const uint64_t k = s[i];
                return Pick<uint64_t>{i == 0 || k != s[i - 1], k};
            },
            [=] __device__(int64_t, int64_t p, uint64_t k) { d[p] = k; }, S + 0);
    }
    // ---- S: distinct tuples, y-major ----------------------------------------
    DBuf<uint64_t> s1;
    {
        DBuf<uint64_t> ka = c.buf<uint64_t>(ns), kb = c.buf<uint64_t>(ns);
        const uint64_t *s = radix_sort_from<uint64_t>(
            c,
            [=] __device__(int64_t i) {
                return ((uint64_t)((int64_t)sy[i] - ymin) << zb) | (uint64_t)((int64_t)sz[i] - zmin);
            },
            ka.get(), kb.get(), ns, yb + zb);
        s1 = c.buf<uint64_t>(ns);
        uint64_t *d = s1.get();
        compact_v(
            c, ns,
            [=] __device__(int64_t i) {
                const uint64_t k = s[i];
                return Pick<uint64_t>{i == 0 || k != s[i - 1], k};
            },
            [=] __device__(int64_t, int64_t p, uint64_t k) { d[p] = k; }, S + 1);
    }
    // ---- distinct y of R with their R degrees (sorted y of the distinct R) -----
    int64_t h2[2];
    c.load_n(h2, S, 2);
    const int64_t n_r1 = h2[0], n_s1 = h2[1];
    DBuf<uint32_t> YR = c.buf<uint32_t>(n_r1);
    DBuf<int64_t> rstart = c.buf<int64_t>(n_r1 + 1);
    {
        DBuf<uint32_t> ya = c.buf<uint32_t>(n_r1), yb2 = c.buf<uint32_t>(n_r1);
        const uint64_t *r = r1.get();
        const uint64_t ym = ymask;
        const uint32_t *s = radix_sort_from<uint32_t>(
            c, [=] __device__(int64_t i) { return (uint32_t)(r[i] & ym); }, ya.get(), yb2.get(), n_r1, yb);
        uint32_t *d = YR.get();
        int64_t *rs = rstart.get();
        compact_v(
            c, n_r1,
            [=] __device__(int64_t i) {
                const uint32_t k = s[i];
                return Pick<uint32_t>{i == 0 || k != s[i - 1], k};
            },
            [=] __device__(int64_t i, int64_t p, uint32_t k) {
                d[p] = k;
                rs[p] = i;
            },
            S + 2);
    }
    {
        // end of the last run, written where the device count says
        int64_t *rs = rstart.get();
        const int64_t *cnt = S + 2;
        const int64_t nr1 = n_r1;
        for_each(c, 1, [=] __device__(int64_t) { rs[*cnt] = nr1; });
    }
    // ---- distinct y of S (from the y-major S) --------------------------------
    DBuf<uint32_t> YS = c.buf<uint32_t>(n_s1);
    {
        const uint64_t *s = s1.get();
        uint32_t *d = YS.get();
        const int zbs = zb;
        compact_v(
            c, n_s1,
            [=] __device__(int64_t i) {
                const uint64_t y = s[i] >> zbs;
                return Pick<uint32_t>{i == 0 || y != (s[i - 1] >> zbs), (uint32_t)y};
            },
            [=] __device__(int64_t, int64_t p, uint32_t y) { d[p] = y; }, S + 3);
    }
    int64_t hy2[2];
    c.load_n(hy2, S + 2, 2);
    const int64_t ny_r = hy2[0], ny_s = hy2[1];

    // ---- semijoin: keep y present in both; dense y ranks; R degree of y -------
    DBuf<int32_t> yrank_js = c.buf<int32_t>(ny_s);
    DBuf<int32_t> dRy = c.buf<int32_t>(ny_s);
    {
        int32_t *yr = yrank_js.get(), *dr = dRy.get();
        const uint32_t *ys = YS.get(), *yrr = YR.get();
        const int64_t *rs = rstart.get();
        const int64_t nyr = ny_r;
        for_each(c, ny_s, [=] __device__(int64_t j) { yr[j] = -1; });
        auto emit = [=] __device__(int64_t j, int64_t p, int32_t deg) {
            yr[j] = (int32_t)p;
            dr[p] = deg;
        };
        const int64_t yspan = ymax - ymin + 1;
        if (dense_range_ok(yspan, nr + ns)) {
            // position of every y in the distinct y of R, from a table over the y range
            DBuf<int32_t> yq = c.buf<int32_t>((size_t)yspan);
            int32_t *yqp = yq.get();
            for_each(c, yspan, [=] __device__(int64_t y) { yqp[y] = -1; });
            for_each(c, nyr, [=] __device__(int64_t q) { yqp[yrr[q]] = (int32_t)q; });
            const int32_t *yqc = yqp;
            compact_v(
                c, ny_s,
                [=] __device__(int64_t j) {
                    const int32_t q = yqc[ys[j]];
                    const int64_t qc = q >= 0 ? q : 0;
                    return Pick<int32_t>{q >= 0, (int32_t)(rs[qc + 1] - rs[qc])};
                },
                emit, S + 4);
        } else {
            compact_v(
                c, ny_s,
                [=] __device__(int64_t j) {
                    const int64_t p = lower_bound_dev(yrr, (int64_t)0, nyr, ys[j]);
                    const int64_t q = p < nyr ? p : nyr - 1;
                    const bool hit = (p < nyr) & (yrr[q] == ys[j]);
                    return Pick<int32_t>{hit, (int32_t)(rs[q + 1] - rs[q])};
                },
                emit, S + 4);
        }
    }
    rstart.reset();
    // Joined y rank of every y value, from a dense table over the y range when
    // that range is small enough (-1: y not in both relations).
    const int64_t yspan = ymax - ymin + 1;
    const bool y_dense = dense_range_ok(yspan, nr + ns);
    DBuf<int32_t> ymap;
    if (y_dense) {
        ymap = c.buf<int32_t>((size_t)yspan);
        int32_t *ymp = ymap.get();
        const uint32_t *ys = YS.get();
        const int32_t *yr = yrank_js.get();
        for_each(c, yspan, [=] __device__(int64_t y) { ymp[y] = -1; });
        for_each(c, ny_s, [=] __device__(int64_t j) { ymp[ys[j]] = yr[j]; });
    }
    // S tuples kept, y-major: y rank + z offset.  Without the dense table the
    // y rank comes from the tuple's run index among the distinct y of S.  A y
    // is kept with all its tuples, so the first kept tuple of a y is the first
    // of its run: it also writes that y's CSR offset (bit 63 of the value).
    DBuf<int32_t> s2_y = c.buf<int32_t>(n_s1);
    DBuf<uint32_t> s2_z = c.buf<uint32_t>(n_s1);
    DBuf<int64_t> off_y = c.buf<int64_t>(ny_s + 1);  // dom_y + 1 used
    {
        const uint64_t *s = s1.get();
        const int zbs = zb;
        const uint64_t zm = zmask;
        int32_t *oy = s2_y.get();
        uint32_t *oz = s2_z.get();
        int64_t *offy = off_y.get();
        auto emit = [=] __device__(int64_t, int64_t p, uint64_t v) {
            const int32_t r = (int32_t)((v >> 32) & 0x7fffffffu);
            oy[p] = r;
            oz[p] = (uint32_t)v;
            if (v >> 63) offy[r] = p;
        };
        auto first_y = [=] __device__(int64_t i, uint64_t k) -> uint64_t {
            return (i == 0 || (k >> zbs) != (s[i - 1] >> zbs)) ? (1ull << 63) : 0ull;
        };
        if (y_dense) {
            const int32_t *ymc = ymap.get();
            compact_v(
                c, n_s1,
                [=] __device__(int64_t i) {
                    const uint64_t k = s[i];
                    const int32_t r = ymc[k >> zbs];
                    return Pick<uint64_t>{r >= 0, first_y(i, k) | ((uint64_t)(uint32_t)r << 32) |
                                                      (uint64_t)(uint32_t)(k & zm)};
                },
                emit, S + 5);
        } else {
            DBuf<int32_t> seg = c.buf<int32_t>(n_s1);
            int32_t *sg = seg.get();
            auto newy = [=] __device__(int64_t i) -> int64_t {
                return (i == 0 || (s[i] >> zbs) != (s[i - 1] >> zbs)) ? 1 : 0;
            };
            scan_exclusive_v(c, n_s1, newy,
                             [=] __device__(int64_t i, int64_t p, int64_t v) { sg[i] = (int32_t)(p + v - 1); });
            const int32_t *yr = yrank_js.get();
            compact_v(
                c, n_s1,
                [=] __device__(int64_t i) {
                    const uint64_t k = s[i];
                    const int32_t r = yr[sg[i]];
                    return Pick<uint64_t>{r >= 0, first_y(i, k) | ((uint64_t)(uint32_t)r << 32) |
                                                      (uint64_t)(uint32_t)(k & zm)};
                },
                emit, S + 5);
        }
    }
    // R tuples kept, x-major: x offset + y rank (from the dense table, else
    // by binary search in the distinct y of S).
    DBuf<uint32_t> r2_x = c.buf<uint32_t>(n_r1);
    DBuf<int32_t> adj_r = c.buf<int32_t>(n_r1);
    {
        const uint64_t *s = r1.get();
        const uint32_t *ys = YS.get();
        const int32_t *yr = yrank_js.get();
        const int64_t nys = ny_s;
        const int ybs = yb;
        const uint64_t ym = ymask;
        uint32_t *ox = r2_x.get();
        int32_t *oy = adj_r.get();
        if (y_dense) {
            const int32_t *ymc = ymap.get();
            compact_v(
                c, n_r1,
                [=] __device__(int64_t i) {
                    const uint64_t k = s[i];
                    const int32_t r = ymc[k & ym];
                    return Pick<uint64_t>{r >= 0, ((uint64_t)(uint32_t)r << 32) | (uint64_t)(uint32_t)(k >> ybs)};
                },
                [=] __device__(int64_t, int64_t p, uint64_t v) {
                    ox[p] = (uint32_t)v;
                    oy[p] = (int32_t)(v >> 32);
                },
                S + 6);
        } else {
            auto find = [=] __device__(int64_t i) -> int32_t {
                uint32_t y = (uint32_t)(s[i] & ym);
                const int64_t p = lower_bound_dev(ys, (int64_t)0, nys, y);
                const int64_t q = p < nys ? p : nys - 1;
                const int32_t r = yr[q];
                return ((p < nys) & (ys[q] == y)) ? r : -1;
            };
            compact_v(
                c, n_r1,
                [=] __device__(int64_t i) {
                    const int32_t r = find(i);
                    return Pick<uint64_t>{r >= 0, ((uint64_t)(uint32_t)r << 32) | (uint64_t)(uint32_t)(s[i] >> ybs)};
                },
                [=] __device__(int64_t, int64_t p, uint64_t v) {
                    ox[p] = (uint32_t)v;
                    oy[p] = (int32_t)(v >> 32);
                },
                S + 6);
        }
    }
    int64_t h7[3];
    c.load_n(h7, S + 4, 3);
    const int64_t dom_y = h7[0], n_s2 = h7[1], n_r2 = h7[2];
    r1.reset();
    s1.reset();
    YR.reset();
    if (n_r2 == 0 || n_s2 == 0) return false;

    // ---- z ranks ---------------------------------------------------------------
    DBuf<uint32_t> ZS = c.buf<uint32_t>(n_s2);
    DBuf<int64_t> zstart = c.buf<int64_t>(n_s2 + 1);
    {
        DBuf<uint32_t> za = c.buf<uint32_t>(n_s2), zb2 = c.buf<uint32_t>(n_s2);
        const uint32_t *s = radix_sort_from<uint32_t>(c, KeyArray<uint32_t>{s2_z.get()}, za.get(), zb2.get(), n_s2, zb);
        uint32_t *d = ZS.get();
        int64_t *zs0 = zstart.get();
        compact_v(
            c, n_s2,
            [=] __device__(int64_t i) {
                const uint32_t k = s[i];
                return Pick<uint32_t>{i == 0 || k != s[i - 1], k};
            },
            [=] __device__(int64_t i, int64_t p, uint32_t k) {
                d[p] = k;
                zs0[p] = i;
            },
            S + 7);
    }
    // ---- x ranks and the x-major CSR of R -----------------------------------------
    // One scan of the first-of-x flags over the x-major tuples gives every
    // tuple its x rank and, at the first tuple of each x, that x's id and
    // CSR offset.
    DBuf<int32_t> xorig = c.buf<int32_t>(n_r2);
    DBuf<int64_t> off_x = c.buf<int64_t>(n_r2 + 1);
    DBuf<int32_t> r_xr = c.buf<int32_t>(n_r2);
    {
        const uint32_t *xs = r2_x.get();
        int32_t *xo = xorig.get(), *xr = r_xr.get();
        int64_t *ox = off_x.get();
        const int64_t xm = xmin;
        scan_exclusive_v(
            c, n_r2,
            [=] __device__(int64_t i) {
                const uint32_t k = xs[i];
                return Sum<uint32_t>{(i == 0 || k != xs[i - 1]) ? 1 : 0, k};
            },
            [=] __device__(int64_t i, int64_t p, const Sum<uint32_t> &it) {
                xr[i] = (int32_t)(p + it.add - 1);
                if (it.add) {
                    xo[p] = (int32_t)((int64_t)it.v + xm);
                    ox[p] = i;
                }
            },
            S + 8);
    }
    // ---- end of the y-major CSR offsets of S and the full join size J ----------
    {
        int64_t *oy = off_y.get();
        const int64_t ny = dom_y, ns2 = n_s2;
        for_each(c, 1, [=] __device__(int64_t) { oy[ny] = ns2; });
        const int32_t *d1 = dRy.get();
        const int64_t *oyc = oy;
        reduce_sum(
            c, dom_y, [=] __device__(int64_t y) -> int64_t { return (int64_t)d1[y] * (oyc[y + 1] - oyc[y]); },
            (unsigned long long *)(S + 10));
    }
    int64_t h9[3];
    c.load_scalars({S + 7, S + 8, S + 10}, h9);
    const int64_t dom_z = h9[0], dom_x = h9[1], J = h9[2];
    {
        int64_t *ox = off_x.get();
        const int64_t nx = dom_x, nr2 = n_r2;
        for_each(c, 1, [=] __device__(int64_t) { ox[nx] = nr2; });
    }
    r2_x.reset();
    // ---- z id of every z rank (the per-tuple z ranks are built on first use) ----
    DBuf<int32_t> zorig = c.buf<int32_t>(dom_z);
    {
        const uint32_t *zs = ZS.get();
        int32_t *zo = zorig.get();
        const int64_t zm = zmin;
        for_each(c, dom_z, [=] __device__(int64_t r) { zo[r] = (int32_t)((int64_t)zs[r] + zm); });
    }
    // ---- degrees (run lengths of the sorts above) and the full join size J ------
    DBuf<int32_t> dSz = c.buf<int32_t>(dom_z);
    {
        int32_t *d2 = dSz.get();
        const int64_t *zs0 = zstart.get();
        const int64_t nz = dom_z, ns2 = n_s2;
        for_each(c, dom_z, [=] __device__(int64_t r) { d2[r] = (int32_t)((r + 1 < nz ? zs0[r + 1] : ns2) - zs0[r]); });
    }
    zstart.reset();
    g.n_r2 = n_r2;
    g.n_s2 = n_s2;
    g.dom_x = dom_x;
    g.dom_y = dom_y;
    g.dom_z = dom_z;
    g.J = J;
    g.r_xr = std::move(r_xr);
    g.adj_r = std::move(adj_r);
    g.zs = std::move(ZS);
    g.n_in = nr + ns;
    g.s2_zoff = std::move(s2_z);
    g.s2_y = std::move(s2_y);
    g.dRy = std::move(dRy);
    g.dSz = std::move(dSz);
    g.xorig = std::move(xorig);
    g.zorig = std::move(zorig);
    if (dom_x == xmax - xmin + 1) g.x_dense_base = xmin;
    if (dom_z == zmax - zmin + 1) g.z_dense_base = zmin;
    g.zmin = zmin;
    g.zspan = zmax - zmin + 1;
    g.off_x = std::move(off_x);
    g.off_y = std::move(off_y);
    return true;
}

const int32_t *Ingest::adj_s(const Ctx &c) const {
    if (adj_s_.get() || n_s2 <= 0) return adj_s_.get();
    DBuf<int32_t> out = c.buf<int32_t>(n_s2);
    int32_t *as = out.get();
    const uint32_t *zsr = zs.get(), *sz2 = s2_zoff.get();
    const int64_t nz = dom_z;
    if (nz == zspan) {
        // every offset of the z range occurs, so a z's rank is its offset
        JP_HIP(hipMemcpyAsync(as, sz2, (size_t)n_s2 * sizeof(int32_t), hipMemcpyDeviceToDevice, c.stream));
    } else if (dense_range_ok(zspan, n_in)) {
        // rank of every z offset from a table over the range (every z of S is
        // among the distinct z, so only their entries are written)
        DBuf<int32_t> zmap = c.buf<int32_t>((size_t)zspan);
        int32_t *zmp = zmap.get();
        for_each(c, nz, [=] __device__(int64_t r) { zmp[zsr[r]] = (int32_t)r; });
        const int32_t *zmc = zmp;
        for_each(c, n_s2, [=] __device__(int64_t e) { as[e] = zmc[sz2[e]]; });
    } else {
        for_each(c, n_s2, [=] __device__(int64_t e) { as[e] = (int32_t)lower_bound_dev(zsr, (int64_t)0, nz, sz2[e]); });
    }
    adj_s_ = std::move(out);
    return adj_s_.get();
}

// Operations the product kernel executed: 2 u v w, or for a symmetric
// product on the tiles on and above the diagonal (256 x 256 tiles) the
// fraction T (T + 1) / 2 of the T^2 tiles.
static double product_ops(int64_t u, int64_t v, int64_t w, bool sym_done) {
    const double full = 2.0 * (double)u * (double)v * (double)w;
    if (!sym_done) return full;
    const double t = (double)ceil_div(u, 256);
    return full * (t * (t + 1) / 2) / (t * t);
}

// ---- overlap output (set similarity join) ---------------------------------
// Every distinct pair with its number of witnesses |N_R(x) & N_S(z)|: the
// light witnesses and the heavy product partition the full join (Algorithm 1),
// so a pair's overlap is its light witness count plus its heavy count C[x][z].
// Candidates carry a weight in their low bits: 1 for a light witness, C[x][z]
// (at most v) for a heavy nonzero; after one sort the run of a pair holds its
// light witnesses and at most one heavy entry, which sorts last, so the
// overlap is (run length - 1) + the last entry's weight.
struct OverlapIn {
    ExpandArgs ex;  // light witnesses; out / wshift / err are set here
    int64_t J_L = 0, cap_h = 0;
    bool has_heavy = false;
    const int8_t *M1 = nullptr, *M2t = nullptr;
    bool sym = false;  // M2t == M1 (self-join)
    int64_t u = 0, v = 0, w = 0, ld = 0;
    const int32_t *x_of_hx = nullptr, *z_of_hz = nullptr;
    int bmm_kind = 0;
    int bx = 0, bz = 0;
    int64_t dom_x = 0, dom_y = 0, dom_z = 0;
    const int32_t *xorig = nullptr, *zorig = nullptr;
    int64_t min_c = 1;
    int order = 0;
    bool force_wide = false;
};

// Ordered variant: selected pairs as (max - overlap) << pbits | pair keys,
// sorted, then unranked.
template <class K, class K2>
static int64_t overlap_ordered(const Ctx &c, const OverlapIn &in, const K *s, const int64_t *en, int64_t n_pairs,
                               int wb, jp_result *res, int64_t *S) {
    const int pbits = in.bx + in.bz;
    const int64_t cmax = std::max<int64_t>(in.dom_y, 1);  // an overlap is at most |dom y|
    const int cb = bits_for((uint64_t)cmax);
    DBuf<K2> k2 = c.buf<K2>(std::max<int64_t>(n_pairs, 1)), t2 = c.buf<K2>(std::max<int64_t>(n_pairs, 1));
    K2 *kk = k2.get();
    const K wmask = ((K)1 << wb) - 1;
    const int64_t minc = in.min_c;
    const int wbs = wb, pb = pbits;
    compact_v(
        c, n_pairs,
        [=] __device__(int64_t p) {
            const int64_t e = en[p], prev = en[p > 0 ? p - 1 : 0], b = p > 0 ? prev + 1 : 0;
            const int64_t cnt = (e - b) + (int64_t)(s[e] & wmask);
            const K2 pair = (K2)(s[e] >> wbs);
            return Pick<K2>{cnt >= minc, ((K2)(uint64_t)(cmax - cnt) << pb) | pair};
        },
        [=] __device__(int64_t, int64_t q, K2 key) { kk[q] = key; }, S + 22);
    const int64_t n = c.load(S + 22);
    const K2 *sorted = radix_sort(c, kk, t2.get(), n, pbits + cb);
    for (int i = 0; i < 3; ++i) res->cols[i] = c.buf<int32_t>(std::max<int64_t>(n, 1));
    int32_t *ox = res->cols[0].get(), *oz = res->cols[1].get(), *oc = res->cols[2].get();
    const int32_t *xo = in.xorig, *zo = in.zorig;
    const uint64_t zm = (1ull << in.bz) - 1;
    const int bzs = in.bz;
    const uint64_t nx = (uint64_t)in.dom_x, nz = (uint64_t)in.dom_z;
    int64_t *err = S + 20;
    c.zero(err, 1);
    for_each(c, n, [=] __device__(int64_t i) {
        const K2 k = sorted[i];
        const uint64_t pair = (uint64_t)(k & (((K2)1 << pb) - 1));
        const uint64_t xi = pair >> bzs, zi = pair & zm;
        const bool ok = (xi < nx) & (zi < nz);
        if (!ok) *err = 1;
        ox[i] = xo[ok ? xi : 0];
        oz[i] = zo[ok ? zi : 0];
        oc[i] = (int32_t)(cmax - (int64_t)(uint64_t)(k >> pb));
    });
    JP_CHECK(c.load(err) == 0, JP_EINTERNAL, "overlap output key outside the rank tables");
    return n;
}

template <class K>
static void overlap_output(const Ctx &c, const OverlapIn &in, jp_result *res, jp_stats &st, int64_t *S) {
    const int wb = bits_for((uint64_t)std::max<int64_t>(in.v, 1));  // heavy counts are at most v
    const int pbits = in.bx + in.bz;
    const int64_t cap = in.J_L + in.cap_h;
    DBuf<K> cand = c.buf<K>(std::max<int64_t>(cap, 1));
    if (in.J_L > 0) {
        ExpandArgs a = in.ex;
        a.wshift = wb;
        a.out = cand.get();
        a.err = S + 19;
        c.zero(S + 19, 1);
        const int64_t blocks = ceil_div(in.J_L, kExpTile);
        hipLaunchKernelGGL(k_light_expand<K>, dim3(grid_x(blocks, kExpBlock)), dim3(kExpBlock), 0, c.stream, a);
        JP_HIP(hipGetLastError());
        JP_CHECK(c.load(S + 19) == 0, JP_EINTERNAL, "light expansion index outside the witness lists");
    }
    int64_t nnz = 0;
    if (in.has_heavy) {
        int used = JP_BMM_I8_MFMA;
        bool sym_done = false;
        Ctx cb = c;
        cb.bmm_used = &used;
        cb.bmm_sym = &sym_done;
        bool_matmul_count_keys(cb, in.M1, in.M2t, in.u, in.w, in.ld, in.bmm_kind, in.x_of_hx, in.z_of_hz, in.bz, wb,
                               cand.get() + in.J_L, sizeof(K) == 16, in.cap_h, (unsigned long long *)(S + 17), in.sym);
        nnz = c.load(S + 17);
        JP_CHECK(nnz <= in.cap_h, JP_EINTERNAL, "heavy product produced more nonzeros than its bound");
        st.bmm = used;
        st.bmm_ops = product_ops(in.u, in.v, in.w, sym_done);
    }
    st.nnz_heavy = nnz;
    const int64_t total = in.J_L + nnz;
    DBuf<K> tmp = c.buf<K>(std::max<int64_t>(total, 1));
    const K *s = radix_sort(c, cand.get(), tmp.get(), total, pbits + wb);
    // last index of every run of equal pairs
    DBuf<int64_t> ends = c.buf<int64_t>(std::max<int64_t>(total, 1));
    int64_t *en = ends.get();
    const int wbs = wb;
    compact(
        c, total,
        [=] __device__(int64_t i) {
            const K next = s[i + 1 < total ? i + 1 : i];  // clamped: loads stay in range
            return (i + 1 == total) | ((s[i] >> wbs) != (next >> wbs));
        },
        [=] __device__(int64_t i, int64_t p) { en[p] = i; }, S + 21);
    const int64_t n_pairs = c.load(S + 21);
    st.J_H = st.J - st.J_L;
    if (in.order == 1) {
        const int cb = bits_for((uint64_t)std::max<int64_t>(in.dom_y, 1));
        res->n = pbits + cb <= 64 && !in.force_wide ? overlap_ordered<K, uint64_t>(c, in, s, en, n_pairs, wb, res, S)
                                  : overlap_ordered<K, unsigned __int128>(c, in, s, en, n_pairs, wb, res, S);
        return;
    }
    for (int i = 0; i < 3; ++i) res->cols[i] = c.buf<int32_t>(std::max<int64_t>(n_pairs, 1));
    int32_t *ox = res->cols[0].get(), *oz = res->cols[1].get(), *oc = res->cols[2].get();
    const int32_t *xo = in.xorig, *zo = in.zorig;
    const K wmask = ((K)1 << wb) - 1;
    const uint64_t zm = (1ull << in.bz) - 1;
    const int bzs = in.bz;
    const uint64_t nx = (uint64_t)in.dom_x, nz = (uint64_t)in.dom_z;
    const int64_t minc = in.min_c;
    int64_t *err = S + 20;
    c.zero(err, 1);
    compact(
        c, n_pairs,
        [=] __device__(int64_t p) {
            const int64_t e = en[p], prev = en[p > 0 ? p - 1 : 0], b = p > 0 ? prev + 1 : 0;
            return (e - b) + (int64_t)(s[e] & wmask) >= minc;
        },
        [=] __device__(int64_t p, int64_t q) {
            const int64_t e = en[p], prev = en[p > 0 ? p - 1 : 0], b = p > 0 ? prev + 1 : 0;
            const uint64_t pair = (uint64_t)(s[e] >> wbs);
            const uint64_t xi = pair >> bzs, zi = pair & zm;
            const bool ok = (xi < nx) & (zi < nz);
            if (!ok) *err = 1;
            ox[q] = xo[ok ? xi : 0];
            oz[q] = zo[ok ? zi : 0];
            oc[q] = (int32_t)((e - b) + (int64_t)(s[e] & wmask));
        },
        S + 18);
    JP_CHECK(c.load(err) == 0, JP_EINTERNAL, "overlap output key outside the rank tables");
    res->n = c.load(S + 18);
}

jp_result *run_two_path(const Ctx &c, const int32_t *rx, const int32_t *ry, int64_t nr, const int32_t *sz,
                        const int32_t *sy, int64_t ns, const jp_options &o, const OverlapSpec *ov) {
    const bool timing = (o.flags & JP_FLAG_TIMING) != 0;
    Timeline tl(c, timing);
    const int ev_start = tl.mark();
    auto res = std::make_unique<jp_result>();
    res->alloc = c.alloc;
    res->arity = ov ? 3 : 2;
    jp_stats &st = res->stats;
    std::memset(&st, 0, sizeof(st));
    st.arity = res->arity;
    st.delta1 = st.delta2 = JP_DELTA_INF;
    st.strategy = o.strategy;
    st.dedup = JP_DEDUP_GLOBAL;

    auto finish_empty = [&]() {
        res->n = 0;
        for (int i = 0; i < res->arity; ++i) res->cols[i] = c.buf<int32_t>(1);
        return res.release();
    };
    if (nr == 0 || ns == 0) return finish_empty();

    DBuf<int64_t> scal = c.buf<int64_t>(32);  // device scalars
    int64_t *S = scal.get();

    Ingest g;
    if (!ingest_two_path(c, rx, ry, nr, sz, sy, ns, g, S)) return finish_empty();
    const int64_t n_r2 = g.n_r2, n_s2 = g.n_s2, dom_x = g.dom_x, dom_y = g.dom_y, dom_z = g.dom_z, J = g.J;
    DBuf<int32_t> &r_xr = g.r_xr, &adj_r = g.adj_r, &s2_y = g.s2_y, &dRy = g.dRy,
                  &dSz = g.dSz, &xorig = g.xorig, &zorig = g.zorig;
    DBuf<int64_t> &off_x = g.off_x, &off_y = g.off_y;
    const int ev_ingest = tl.mark();
    auto check_index = [&](const char *when) {
        std::string w(when);
        check_range(c, (w + ": r_xr").c_str(), r_xr.get(), n_r2, 0, dom_x);
        check_monotone(c, (w + ": r_xr order").c_str(), r_xr.get(), n_r2, 0, -1);
        check_range(c, (w + ": adj_r").c_str(), adj_r.get(), n_r2, 0, dom_y);
        if (checks_on()) check_range(c, (w + ": adj_s").c_str(), g.adj_s(c), n_s2, 0, dom_z);
        check_monotone(c, (w + ": off_x").c_str(), off_x.get(), dom_x + 1, 0, n_r2);
        check_monotone(c, (w + ": off_y").c_str(), off_y.get(), dom_y + 1, 0, n_s2);
        check_range(c, (w + ": s2_y").c_str(), s2_y.get(), n_s2, 0, dom_y);
    };
    check_index("ingest");
    dump(c, "r_xr", r_xr.get(), n_r2);
    dump(c, "adj_r", adj_r.get(), n_r2);
    dump(c, "off_x", off_x.get(), dom_x + 1);
    dump(c, "off_y", off_y.get(), dom_y + 1);
    if (dump_on()) dump(c, "adj_s", g.adj_s(c), n_s2);
    dump(c, "s2_y", s2_y.get(), n_s2);
    dump(c, "dRy", dRy.get(), dom_y);
    dump(c, "dSz", dSz.get(), dom_z);

    st.n_r = n_r2;
    st.n_s = n_s2;
    st.dom_x = dom_x;
    st.dom_y = dom_y;
    st.dom_z = dom_z;
    st.J = J;

    // ---- thresholds ---------------------------------------------------------------
    TwoPathSummary sum;
    sum.n_r = n_r2;
    sum.n_s = n_s2;
    sum.dom_x = dom_x;
    sum.dom_y = dom_y;
    sum.dom_z = dom_z;
    sum.J = J;
    sum.self_join = (rx == sz && ry == sy && nr == ns);
    sum.out_est = estimate_out(dom_x, dom_z, J, std::max(n_r2, n_s2));
    if (o.strategy == JP_STRATEGY_AUTO_COST || o.strategy == JP_STRATEGY_AUTO_MLP)
        summarize_two_path(c, g, o.y_rule, sum);
    if (o.strategy == JP_STRATEGY_AUTO_MLP || (o.flags & JP_FLAG_SAMPLED_OUT)) {
        const SampledOut so = sampled_out(c, g, o.seed);
        sum.sample_draws = so.draws;
        sum.sample_distinct = so.distinct;
        if (so.draws > 0) sum.out_sampled = (double)so.distinct * (double)dom_x / (double)so.draws;
    }
    st.out_est = sum.out_est;
    st.out_sampled = sum.out_sampled;
    st.sample_draws = sum.sample_draws;
    st.sample_distinct = sum.sample_distinct;
    Thresholds th = select_thresholds(c, sum, o);
    st.delta1 = th.d1;
    st.delta2 = th.d2;
    st.strategy = th.strategy;

    // ---- partition ------------------------------------------------------------------
    const int64_t d1 = th.d1, d2 = th.d2;
    const bool rule_r_only = o.y_rule == JP_Y_RULE_R_ONLY;
    int64_t u = 0, v = 0, w = 0;
    DBuf<int32_t> hx_of_x, x_of_hx, hz_of_z, z_of_hz, hy_of_y;
    if (!th.light_only()) {
        hx_of_x = c.buf<int32_t>(dom_x);
        x_of_hx = c.buf<int32_t>(dom_x);
        hz_of_z = c.buf<int32_t>(dom_z);
        z_of_hz = c.buf<int32_t>(dom_z);
        hy_of_y = c.buf<int32_t>(dom_y);
        int32_t *hx = hx_of_x.get(), *xh = x_of_hx.get(), *hz = hz_of_z.get(), *zh = z_of_hz.get();
        int32_t *hy = hy_of_y.get();
        const int64_t *ox = off_x.get(), *oy = off_y.get();
        const int32_t *dry = dRy.get(), *dsz = dSz.get();
        for_each(c, dom_x, [=] __device__(int64_t i) { hx[i] = -1; });
        for_each(c, dom_z, [=] __device__(int64_t i) { hz[i] = -1; });
        for_each(c, dom_y, [=] __device__(int64_t i) { hy[i] = -1; });
        compact(
            c, dom_x, [=] __device__(int64_t x) { return ox[x + 1] - ox[x] > d2; },
            [=] __device__(int64_t x, int64_t p) {
                hx[x] = (int32_t)p;
                xh[p] = (int32_t)x;
            },
            S + 11);
        compact(
            c, dom_z, [=] __device__(int64_t z) { return (int64_t)dsz[z] > d2; },
            [=] __device__(int64_t z, int64_t p) {
                hz[z] = (int32_t)p;
                zh[p] = (int32_t)z;
            },
            S + 12);
        compact(
            c, dom_y,
            [=] __device__(int64_t y) {
                int64_t dr = dry[y], ds = oy[y + 1] - oy[y];
                int64_t key = rule_r_only ? dr : (dr > ds ? dr : ds);
                return key > d1;
            },
            [=] __device__(int64_t y, int64_t p) { hy[y] = (int32_t)p; }, S + 13);
        int64_t h3[3];
        c.load_n(h3, S + 11, 3);
        u = h3[0];
        w = h3[1];
        v = h3[2];
    }
    const bool has_heavy = u > 0 && v > 0 && w > 0;
    if (!th.light_only()) {
        check_range(c, "hx_of_x", hx_of_x.get(), dom_x, -1, u);
        check_range(c, "hz_of_z", hz_of_z.get(), dom_z, -1, w);
        check_range(c, "hy_of_y", hy_of_y.get(), dom_y, -1, v);
        check_range(c, "x_of_hx", x_of_hx.get(), u, 0, dom_x);
        check_range(c, "z_of_hz", z_of_hz.get(), w, 0, dom_z);
        dump(c, "hx_of_x", hx_of_x.get(), dom_x);
        dump(c, "hy_of_y", hy_of_y.get(), dom_y);
        dump(c, "hz_of_z", hz_of_z.get(), dom_z);
    }
    st.u = u;
    st.v = v;
    st.w = w;

    // The per-x dedup may key z by its offset from the smallest z id instead
    // of its rank when the id range is at most a few times the number of
    // distinct z: the output then needs no rank-to-id lookup per pair, and
    // the witness lists are built in offsets from the start.
    const int bzr = bits_for((uint64_t)(dom_z - 1)), bzo = bits_for((uint64_t)(g.zspan - 1));
    const bool z_off = !ov && o.dedup != JP_DEDUP_GLOBAL && segmented_dedup_fits(bzo) && g.zspan <= 4 * dom_z;

    // Heavy matrices: M1 = heavy x by heavy y (R), M2^T = heavy z by heavy y (S).
    // The pass over R also marks the heavy y that some heavy x meets: only
    // those y need the light-z part of their list below.
    DBuf<int8_t> M1, M2t;
    DBuf<int32_t> need_y;  // per heavy y: 1 if a heavy x meets it
    int64_t ld = 0;
    // A self-join (R and S the same columns) has heavy z = heavy x and
    // M2^T = M1: the product is M1 M1^T, computed on half its tiles.
    const bool sym = sum.self_join && u == w;
    if (has_heavy) {
        JP_CHECK(o.bmm != JP_BMM_F16 || v < (int64_t(1) << 24), JP_EPRECISION,
                 "fp16 product: counts may reach 2^24 (heavy y), beyond fp32's exact range");
        ld = ceil_div(v, kBmmPadK) * kBmmPadK;
        M1 = c.buf<int8_t>((size_t)(u * ld));
        if (!sym) M2t = c.buf<int8_t>((size_t)(w * ld));
        need_y = c.buf<int32_t>(v);
        c.zero(M1.get(), (size_t)(u * ld));
        if (!sym) c.zero(M2t.get(), (size_t)(w * ld));
        c.zero(need_y.get(), (size_t)v);
        int8_t *m1 = M1.get(), *m2 = M2t.get();
        int32_t *nd = need_y.get();
        const int32_t *xr = r_xr.get(), *ar = adj_r.get(), *syr = s2_y.get(), *as = g.adj_s(c);
        const int32_t *hx = hx_of_x.get(), *hy = hy_of_y.get(), *hz = hz_of_z.get();
        const int64_t ldl = ld;
        for_each(c, n_r2, [=] __device__(int64_t e) {
            const int32_t a = hx[xr[e]];
            if (a >= 0) {  // the y gather only for heavy x
                const int32_t b = hy[ar[e]];
                if (b >= 0) {
                    m1[(int64_t)a * ldl + b] = 1;
                    nd[b] = 1;
                }
            }
        });
        if (!sym)
            for_each(c, n_s2, [=] __device__(int64_t e) {
                const int32_t cc = hz[as[e]], b = hy[syr[e]];
                if ((cc >= 0) & (b >= 0)) m2[(int64_t)(cc >= 0 ? cc : 0) * ldl + (b >= 0 ? b : 0)] = 1;
            });
    }
    const int8_t *M2use = sym ? M1.get() : M2t.get();
    // Witness lists.  zlist = N_S(y) for all y (adj_s, or the z offsets of
    // the same tuples), then for heavy y the light-z part of N_S(y) (what an
    // R tuple with heavy x and heavy y still meets; empty for heavy y that no
    // heavy x meets, since no tuple reads it).
    DBuf<int64_t> lz_off;
    DBuf<int32_t> zlist_own;
    const int32_t *zfull = z_off ? reinterpret_cast<const int32_t *>(g.s2_zoff.get()) : g.adj_s(c);
    const int32_t *zlist = zfull;
    int64_t zlist_n = n_s2;
    if (has_heavy) {
        // One scan over S (y-major) of the "light z at heavy y" flags gives
        // both the compacted lists and, at the first entry of each heavy y,
        // that y's list start.
        lz_off = c.buf<int64_t>(v + 1);
        int64_t *lo = lz_off.get();
        const int32_t *syr = s2_y.get(), *as = g.adj_s(c), *hy = hy_of_y.get(), *hz = hz_of_z.get();
        const int32_t *ndc = need_y.get();
        zlist_own = c.buf<int32_t>(2 * n_s2);
        int32_t *zl = zlist_own.get();
        JP_HIP(hipMemcpyAsync(zl, zfull, n_s2 * sizeof(int32_t), hipMemcpyDeviceToDevice, c.stream));
        int32_t *la = zl + n_s2;
        struct LzItem {
            int32_t h, z;  // heavy index of the tuple's y (-1: light), z as the lists hold it
            bool first;    // first tuple of its y
        };
        const int32_t *zf = zfull;
        scan_exclusive_v(
            c, n_s2,
            [=] __device__(int64_t e) {
                const int32_t y = syr[e], z = as[e];
                const int32_t h = hy[y];
                const bool first = e == 0 || syr[e - 1] != y;
                // light z at a heavy y that a heavy x meets (z looked up only there)
                const bool keep = h >= 0 && ndc[h] != 0 && hz[z] < 0;
                return Sum<LzItem>{(int64_t)keep, LzItem{h, zf[e], first}};
            },
            [=] __device__(int64_t, int64_t p, const Sum<LzItem> &it) {
                if (it.add) la[p] = it.v.z;
                if ((it.v.h >= 0) & it.v.first) lo[it.v.h] = p;
            },
            lo + v);
        zlist = zl;  // its length n_s2 + lz_off[v] is read back with J_L below
    }

    // Per R tuple: list start and witness count (all loads unconditional,
    // choices by select), then offsets by scan.
    DBuf<int64_t> lbase = c.buf<int64_t>(n_r2);
    DBuf<int64_t> eoff = c.buf<int64_t>(n_r2 + 1);
    {
        DBuf<int64_t> elen = c.buf<int64_t>(n_r2);
        const int32_t *xr = r_xr.get(), *ar = adj_r.get();
        const int64_t *oy = off_y.get();
        int64_t *lb = lbase.get(), *ln = elen.get();
        if (has_heavy) {
            const int32_t *hx = hx_of_x.get(), *hy = hy_of_y.get();
            const int64_t *lo = lz_off.get();
            const int64_t ns2 = n_s2;
            for_each(c, n_r2, [=] __device__(int64_t e) {
                const int32_t y = ar[e];
                const int32_t hyv = hy[y], hxv = hx[xr[e]];
                const bool heavy = (hyv | hxv) >= 0;  // both non-negative
                const int32_t hi2 = heavy ? hyv : 0;
                const int64_t l0 = lo[hi2], l1 = lo[hi2 + 1];
                const int64_t s0 = oy[y], s1v = oy[y + 1];
                lb[e] = heavy ? ns2 + l0 : s0;
                ln[e] = heavy ? l1 - l0 : s1v - s0;
            });
        } else {
            for_each(c, n_r2, [=] __device__(int64_t e) {
                const int32_t y = ar[e];
                lb[e] = oy[y];
                ln[e] = oy[y + 1] - oy[y];
            });
        }
        int64_t *eo = eoff.get();
        scan_exclusive(c, n_r2, ArrayGet{ln}, ArrayPut{eo}, eo + n_r2);
        JP_HIP(hipMemcpyAsync(S + 15, eo + n_r2, sizeof(int64_t), hipMemcpyDeviceToDevice, c.stream));
    }
    // Light and heavy witnesses partition the full join: J_H = J - J_L.
    int64_t J_L = 0;
    if (has_heavy) {
        int64_t hv[2];
        c.load_scalars({S + 15, lz_off.get() + v}, hv);
        J_L = hv[0];
        const int64_t n_lz = hv[1];
        const int32_t *la = zlist_own.get() + n_s2;
        check_monotone(c, "lz_off", lz_off.get(), v + 1, 0, n_lz);
        check_range(c, "lz lists", la, n_lz, 0, z_off ? g.zspan : dom_z);
        dump(c, "lz_off", lz_off.get(), v + 1);
        dump(c, "lz lists", la, n_lz);
        zlist_n = n_s2 + n_lz;
    } else {
        J_L = c.load(S + 15);
    }
    JP_CHECK(J_L >= 0 && J_L <= J, JP_EINTERNAL, "light witness count exceeds the join size");
    const int64_t J_H = J - J_L;
    JP_CHECK(has_heavy || J_H == 0, JP_EINTERNAL, "heavy witnesses without a heavy part");
    st.J_L = J_L;
    st.J_H = J_H;
    const int ev_plan = tl.mark();

    const int bx = bits_for((uint64_t)(dom_x - 1));
    const double uw = (double)u * (double)w;
    const int64_t cap_h = has_heavy ? (int64_t)std::min<double>((double)J_H, uw) : 0;
    const int bz = z_off ? bzo : bzr;
    const bool segmented = !ov && o.dedup != JP_DEDUP_GLOBAL && segmented_dedup_fits(bz);
    int64_t nnz = 0;
    int ev_light = ev_plan, ev_bmm0 = ev_plan, ev_bmm1 = ev_plan, ev_heavy = ev_plan;

    if (ov) {
        // ---- overlap counts: counted light witnesses + heavy counts, one sort ---------
        OverlapIn in;
        ExpandArgs &a = in.ex;
        a.eoff = eoff.get();
        a.n_e = n_r2;
        a.J_L = J_L;
        a.r_xr = r_xr.get();
        a.lbase = lbase.get();
        a.zlist = zlist;
        a.zlist_n = zlist_n;
        a.bz = bz;
        in.J_L = J_L;
        in.cap_h = cap_h;
        in.has_heavy = has_heavy;
        in.M1 = M1.get();
        in.M2t = M2use;
        in.sym = sym;
        in.u = u;
        in.v = v;
        in.w = w;
        in.ld = ld;
        in.x_of_hx = x_of_hx.get();
        in.z_of_hz = z_of_hz.get();
        in.bmm_kind = o.bmm;
        in.bx = bx;
        in.bz = bz;
        in.dom_x = dom_x;
        in.dom_y = dom_y;
        in.dom_z = dom_z;
        in.xorig = xorig.get();
        in.zorig = zorig.get();
        in.min_c = ov->min_c;
        in.order = ov->order;
        const int wb = bits_for((uint64_t)std::max<int64_t>(v, 1));
        in.force_wide = ov->force_wide;
        if (bx + bz + wb <= 64 && !ov->force_wide) overlap_output<uint64_t>(c, in, res.get(), st, S);
        else overlap_output<unsigned __int128>(c, in, res.get(), st, S);
        nnz = st.nnz_heavy;
        st.n_out = res->n;
    } else if (segmented) {
        // ---- heavy nonzeros, sorted; then per-x dedup fused with enumeration ----------
        st.dedup = JP_DEDUP_SEGMENTED;
        // z offsets (see above): the witness lists are already in offsets; the
        // heavy columns are mapped here
        DBuf<int32_t> zo_of_hz;
        const int32_t *zl_used = zlist, *zcol = z_of_hz.get();
        if (z_off) {
            const int32_t *zo = zorig.get();
            const int64_t zm = g.zmin;
            if (has_heavy) {
                zo_of_hz = c.buf<int32_t>((size_t)w);
                int32_t *zh = zo_of_hz.get();
                const int32_t *zoh = z_of_hz.get();
                for_each(c, w, [=] __device__(int64_t j) { zh[j] = (int32_t)((int64_t)zo[zoh[j]] - zm); });
                zcol = zh;
            }
        }
        DBuf<uint64_t> hk, hk_tmp;
        const uint64_t *hks = nullptr;
        if (has_heavy) {
            hk = c.buf<uint64_t>(std::max<int64_t>(cap_h, 1));
            ev_bmm0 = tl.mark();
            int used = JP_BMM_I8_MFMA;
            bool sym_done = false;
            Ctx cb = c;
            cb.bmm_used = &used;
            cb.bmm_sym = &sym_done;
            bool_matmul_keys(cb, M1.get(), M2use, u, w, ld, o.bmm, x_of_hx.get(), zcol, bz, hk.get(), cap_h,
                             (unsigned long long *)(S + 17), sym);
            ev_bmm1 = tl.mark();
            nnz = c.load(S + 17);
            JP_CHECK(nnz <= cap_h, JP_EINTERNAL, "heavy product produced more nonzeros than its bound");
            hk_tmp = c.buf<uint64_t>(std::max<int64_t>(nnz, 1));
            hks = radix_sort(c, hk.get(), hk_tmp.get(), nnz, bx + bz);
            dump(c, "heavy keys", hks, nnz);
            st.bmm = used;
            st.bmm_ops = product_ops(u, v, w, sym_done);
        }
        M1.reset();
        M2t.reset();
        ev_heavy = tl.mark();
        ev_light = ev_heavy;
        SegDedupIn in;
        in.dom_x = dom_x;
        in.dom_z = z_off ? g.zspan : dom_z;
        in.bz = bz;
        in.off_x = off_x.get();
        in.eoff = eoff.get();
        in.lbase = lbase.get();
        in.r_xr = r_xr.get();
        in.zlist = zl_used;
        in.zlist_n = zlist_n;
        in.hkeys = hks;
        in.nnz = nnz;
        in.xorig = xorig.get();
        in.zorig = zorig.get();
        in.x_dense_base = g.x_dense_base;
        in.z_dense_base = z_off ? g.zmin : g.z_dense_base;
        SegDedupStats sst;
        segmented_dedup(c, in, &res->cols[0], &res->cols[1], &res->n, &sst, timing);
        st.n_out = res->n;
        st.ms_kernel_dedup = sst.ms_kernel;
        st.dedup_alg_bytes = 4.0 * (double)(J_L + nnz) + 4.0 * (double)res->n;
        st.dedup_units = sst.n_units;
    } else {
        // ---- candidates: light witnesses + heavy nonzeros, one device-wide sort ------
        st.dedup = JP_DEDUP_GLOBAL;
        const int64_t cap = J_L + cap_h;
        DBuf<uint64_t> cand = c.buf<uint64_t>(std::max<int64_t>(cap, 1));
        if (J_L > 0) {
            ExpandArgs a;
            a.eoff = eoff.get();
            a.n_e = n_r2;
            a.J_L = J_L;
            a.r_xr = r_xr.get();
            a.lbase = lbase.get();
            a.zlist = zlist;
            a.zlist_n = zlist_n;
            a.bz = bz;
            a.wshift = 0;
            a.out = cand.get();
            a.err = S + 19;
            c.zero(S + 19, 1);
            const int64_t blocks = ceil_div(J_L, kExpTile);
            hipLaunchKernelGGL(k_light_expand<uint64_t>, dim3(grid_x(blocks, kExpBlock)), dim3(kExpBlock), 0, c.stream,
                               a);
            JP_HIP(hipGetLastError());
        }
        ev_light = tl.mark();
        if (J_L > 0)
            JP_CHECK(c.load(S + 19) == 0, JP_EINTERNAL, "light expansion index outside the witness lists");
        dump(c, "light keys", cand.get(), J_L);
        if (has_heavy) {
            ev_bmm0 = tl.mark();
            int used = JP_BMM_I8_MFMA;
            bool sym_done = false;
            Ctx cb = c;
            cb.bmm_used = &used;
            cb.bmm_sym = &sym_done;
            bool_matmul_keys(cb, M1.get(), M2use, u, w, ld, o.bmm, x_of_hx.get(), z_of_hz.get(), bz,
                             cand.get() + J_L, cap_h, (unsigned long long *)(S + 17), sym);
            ev_bmm1 = tl.mark();
            nnz = c.load(S + 17);
            JP_CHECK(nnz <= cap_h, JP_EINTERNAL, "heavy product produced more nonzeros than its bound");
            dump(c, "heavy keys", cand.get() + J_L, nnz);
            st.bmm = used;
            st.bmm_ops = product_ops(u, v, w, sym_done);
        }
        M1.reset();
        M2t.reset();
        ev_heavy = tl.mark();

        // ---- union + duplicate removal + unrank -------------------------------------
        const int64_t total = J_L + nnz;
        DBuf<uint64_t> tmp = c.buf<uint64_t>(std::max<int64_t>(total, 1));
        const uint64_t *sorted = radix_sort(c, cand.get(), tmp.get(), total, bx + bz);
        res->cols[0] = c.buf<int32_t>(std::max<int64_t>(total, 1));
        res->cols[1] = c.buf<int32_t>(std::max<int64_t>(total, 1));
        {
            int32_t *ox = res->cols[0].get(), *oz = res->cols[1].get();
            const int32_t *xo = xorig.get(), *zo = zorig.get();
            const uint64_t zm = (1ull << bz) - 1;
            const int bzs = bz;
            const uint64_t nx = (uint64_t)dom_x, nz = (uint64_t)dom_z;
            int64_t *err = S + 20;
            c.zero(err, 1);
            compact(
                c, total, [=] __device__(int64_t i) { return i == 0 || sorted[i] != sorted[i - 1]; },
                [=] __device__(int64_t i, int64_t p) {
                    const uint64_t k = sorted[i];
                    const uint64_t xi = k >> bzs, zi = k & zm;
                    const bool ok = (xi < nx) & (zi < nz);
                    if (!ok) *err = 1;
                    ox[p] = xo[ok ? xi : 0];
                    oz[p] = zo[ok ? zi : 0];
                },
                S + 18);
        }
        JP_CHECK(c.load(S + 20) == 0, JP_EINTERNAL, "output key outside the rank tables");
        res->n = c.load(S + 18);
        st.n_out = res->n;
    }
    st.nnz_heavy = nnz;
    const int ev_end = tl.mark();
    if (timing) {
        st.ms_ingest = tl.ms(ev_start, ev_ingest);
        st.ms_plan = tl.ms(ev_ingest, ev_plan);
        st.ms_light = tl.ms(ev_plan, ev_light);
        st.ms_heavy = tl.ms(ev_light, ev_heavy);
        st.ms_bmm = tl.ms(ev_bmm0, ev_bmm1);
        st.ms_dedup = tl.ms(ev_heavy, ev_end);
        st.ms_total = tl.ms(ev_start, ev_end);
    }
    return res.release();
}

// Index and summarise an instance for the planner entry points; false when
// the join is empty (no summary).
static bool summary_of(const Ctx &c, const int32_t *rx, const int32_t *ry, int64_t nr, const int32_t *sz,
                       const int32_t *sy, int64_t ns, const jp_options &o, TwoPathSummary &sum) {
    if (nr == 0 || ns == 0) return false;
    DBuf<int64_t> scal = c.buf<int64_t>(32);
    Ingest g;
    if (!ingest_two_path(c, rx, ry, nr, sz, sy, ns, g, scal.get())) return false;
    sum.n_r = g.n_r2;
    sum.n_s = g.n_s2;
    sum.dom_x = g.dom_x;
    sum.dom_y = g.dom_y;
    sum.dom_z = g.dom_z;
    sum.J = g.J;
    sum.self_join = (rx == sz && ry == sy && nr == ns);
    sum.out_est = estimate_out(g.dom_x, g.dom_z, g.J, std::max(g.n_r2, g.n_s2));
    summarize_two_path(c, g, o.y_rule, sum);
    const SampledOut so = sampled_out(c, g, o.seed);
    sum.sample_draws = so.draws;
    sum.sample_distinct = so.distinct;
    if (so.draws > 0) sum.out_sampled = (double)so.distinct * (double)g.dom_x / (double)so.draws;
    return true;
}

void plan_two_path(const Ctx &c, const int32_t *rx, const int32_t *ry, int64_t nr, const int32_t *sz,
                   const int32_t *sy, int64_t ns, const jp_options &o, int64_t *d1, int64_t *d2, float *features) {
    *d1 = *d2 = JP_DELTA_INF;
    if (features)
        for (int i = 0; i < kFeatures; ++i) features[i] = 0.f;
    TwoPathSummary sum;
    if (!summary_of(c, rx, ry, nr, sz, sy, ns, o, sum)) return;
    const Thresholds th = select_thresholds(c, sum, o);
    *d1 = th.d1;
    *d2 = th.d2;
    if (features) features16(sum, features);
}

void plan_cells(const Ctx &c, const int32_t *rx, const int32_t *ry, int64_t nr, const int32_t *sz, const int32_t *sy,
                int64_t ns, const jp_options &o, int32_t n_cells, const int64_t *d1, const int64_t *d2,
                double *est_seconds, int64_t *heavy_dims) {
    TwoPathSummary sum;
    const bool any = summary_of(c, rx, ry, nr, sz, sy, ns, o, sum);
    jp_calibration cal_default;
    if (!c.cal) default_calibration(&cal_default);
    const jp_calibration &cal = c.cal ? *c.cal : cal_default;
    if (any) {
        plan_costs(sum.view(), cal, n_cells, d1, d2, est_seconds, heavy_dims);
    } else {
        for (int32_t i = 0; i < n_cells; ++i) {
            if (est_seconds) est_seconds[i] = 0.0;
            if (heavy_dims)
                for (int j = 0; j < 3; ++j) heavy_dims[3 * i + j] = 0;
        }
    }
}

}  // namespace jp
