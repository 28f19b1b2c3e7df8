// Duplicate removal of the light witnesses, per x (Section 6,
// "Deduplication": for a fixed x, gather every reachable z, then either sort
// the gathered values or mark them in a dense vector, whichever suits the
// count and the domain).
//
// The witnesses of x are its light list entries (one list per R tuple of x,
// each sorted by z; see two_path.hip) plus the heavy product's nonzeros in
// row x.  Outputs with different x never collide, so the output is built in
// units that follow x order:
//
//  * small x (at most kUnitCap candidates) are packed into units of at most
//    kDCap candidates.  A unit gathers its candidates as 32-bit keys
//    (x - first_x) << bz | z, sorts them by LSD radix sort in LDS over the
//    significant bits only (5-bit digits, per-thread LDS counters, raking
//    scan), and keeps the first of every run of equal keys.
//  * a large x is cut into z windows; a window unit binary-searches the
//    window's part of every sorted list, marks it in an LDS bitmap and reads
//    the set bits back in z order.
//
// One kernel handles all units.  Workgroups take units in order from a ticket
// counter; a unit publishes its distinct count, finds its output offset by
// looking back over its predecessors' published counts (every predecessor
// already holds a ticket and never waits on a later unit, so the wait ends;
// it is also bounded), and writes its (x, z) pairs, unranked, straight into
// the output columns.
#include "debug.hpp"
#include "pipeline.hpp"
#include "prims.hpp"
#include "segdedup.hpp"

namespace jp {
namespace {

constexpr int kDT = 256;                 // threads per unit
constexpr int kDI = 32;                  // keys per thread
constexpr int kDCap = kDT * kDI;         // keys per unit (LDS 32 KB)
constexpr int64_t kUnitCap = kDCap / 2;  // x with more candidates get window units
constexpr int kRB = 5;                   // radix digit bits
constexpr int kRD = 1 << kRB;            // digits
constexpr int64_t kWinBits = (int64_t)kDCap * 32;  // bitmap window capacity (reuses the key buffer)
constexpr int64_t kWinTarget = 16384;              // candidates per window unit, aimed for
constexpr int kListChunk = kDT;                    // lists handled per round in a window unit

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Windows of a large x: enough to fit the LDS bitmap, about kWinTarget
// candidates each, at least 64 z values wide.
__host__ __device__ inline int64_t windows_of(int64_t tx, int64_t dom_z) {
    const int64_t lo = cdiv(dom_z, kWinBits);
    const int64_t hi = cdiv(dom_z, 64) > lo ? cdiv(dom_z, 64) : lo;
    int64_t want = cdiv(tx, kWinTarget);
    if (want < lo) want = lo;
    if (want > hi) want = hi;
    return want < 1 ? 1 : want;
}

struct DedupArgs {
    const int32_t *ustart;   // x of every unit (first x for packed units); ustart[n_units] = dom_x
    const int32_t *uwin;     // window index of a window unit, -1 for a packed unit
    int64_t n_units;
    const int64_t *toff;     // candidates before x (dom_x + 1)
    const int64_t *off_x;    // R tuples of x (dom_x + 1)
    const int64_t *eoff;     // light candidates before each R tuple (n_e + 1)
    const int64_t *lbase;    // list start of every R tuple in zlist
    const int32_t *r_xr;     // x of every R tuple
    const int32_t *zlist;
    const uint64_t *hkeys;   // heavy nonzeros (x << bz | z), sorted
    const int64_t *hoff;     // heavy nonzeros before x (dom_x + 1)
    int bz;
    uint32_t zmask;
    int64_t dom_x, dom_z;
    const int32_t *xorig, *zorig;
    int32_t *out_x, *out_z;
    int64_t cap;                     // capacity of the output columns
    unsigned long long *status;      // look-back slots, one per unit, zeroed
    unsigned int *ticket;            // unit ticket counter, zeroed
    int64_t *total;                  // distinct pairs overall
    int64_t *err;
};

constexpr unsigned long long kAgg = 1ull << 62, kPre = 2ull << 62, kValMask = (1ull << 62) - 1;

__device__ __forceinline__ unsigned long long ld_status(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Executed by the first wave.  Returns the number of outputs of all earlier
// units and publishes this unit's inclusive count.
__device__ int64_t look_back(const DedupArgs &a, int64_t u, int64_t agg) {
    const int lane = lane_id();
    if (u == 0) {
        if (lane == 0) st_status(&a.status[0], kPre | (unsigned long long)agg);
        return 0;
    }
    if (lane == 0) st_status(&a.status[u], kAgg | (unsigned long long)agg);
    int64_t excl = 0;
    int64_t top = u - 1;
    int spins = 0;
    while (top >= 0) {
        const int64_t idx = top - lane;
        const unsigned long long s = idx >= 0 ? ld_status(&a.status[idx]) : kPre;
        const unsigned long long flag = s & ~kValMask;
        const uint64_t pre = ballot(flag == kPre);
        const uint64_t notready = ballot(flag == 0);
        const int first = pre ? (int)(__ffsll((unsigned long long)pre) - 1) : kWave;
        const uint64_t need = first < kWave ? ((first == 63) ? ~0ull : ((2ull << first) - 1)) : ~0ull;
        if (notready & need) {
            if (++spins > (1 << 22)) {  // bounded: report and continue with what is known
                if (lane == 0) *a.err = 2;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        const int64_t v = (lane <= first) ? (int64_t)(s & kValMask) : 0;
        excl += wave_sum(v);
        if (first < kWave) break;
        top -= kWave;
    }
    if (lane == 0) st_status(&a.status[u], kPre | (unsigned long long)(excl + agg));
    return excl;
}

__global__ __launch_bounds__(kDT) void k_dedup(DedupArgs a) {
    __shared__ uint32_t sk[kDCap];           // keys, then distinct keys; or the window bitmap
    __shared__ uint32_t cnt[kRD * kDT / 2];  // packed 16-bit digit counters [digit][thread]
    __shared__ uint32_t lds_scan[kDT / kWave + 1];
    __shared__ int64_t lds_scan64[kDT / kWave + 1];
    __shared__ int64_t sh[4];
    __shared__ int64_t lpre[kListChunk + 1];  // window units: list prefix counts
    __shared__ int64_t lbeg[kListChunk];      // window units: list sub-range starts

    const int tid = threadIdx.x;
    if (tid == 0) sh[0] = (int64_t)atomicAdd(a.ticket, 1u);
    __syncthreads();
    const int64_t u = sh[0];
    if (u >= a.n_units) return;
    const int32_t xa = a.ustart[u];
    const int32_t win = a.uwin[u];

    if (win < 0) {
        // ------------------------------------------------------------ packed unit
        const int32_t xb = a.ustart[u + 1];
        const int64_t e0 = a.off_x[xa], e1 = a.off_x[xb];
        const int64_t c0 = a.eoff[e0];
        const int64_t nL = a.eoff[e1] - c0;
        const int64_t h0 = a.hoff[xa];
        const int64_t n = nL + (a.hoff[xb] - h0);
        const bool over = n > kDCap;
        if (over && tid == 0) *a.err = 1;
        const int nn = over ? 0 : (int)n;
        const int64_t nLc = over ? 0 : nL;

        // gather candidates [tid*kDI, tid*kDI + kDI): one search, then a walk
        uint32_t k[kDI];
        {
            const int p0 = tid * kDI;
            int64_t e = e0;
            if (p0 < nLc) e = upper_bound_dev(a.eoff, e0, e1, c0 + p0) - 1;
            int64_t eo = a.eoff[e];
            int64_t enext = a.eoff[e + 1];
            int64_t lb = p0 < nLc ? a.lbase[e] : 0;
            uint32_t xl = p0 < nLc ? (uint32_t)(a.r_xr[e] - xa) << a.bz : 0u;
#pragma unroll
            for (int j = 0; j < kDI; ++j) {
                const int p = p0 + j;
                uint32_t key = 0xffffffffu;
                if (p < nLc) {
                    const int64_t q = c0 + p;
                    while (q >= enext) {  // next R tuple with a nonempty list
                        ++e;
                        eo = enext;
                        enext = a.eoff[e + 1];
                        lb = a.lbase[e];
                        xl = (uint32_t)(a.r_xr[e] - xa) << a.bz;
                    }
                    key = xl | (uint32_t)a.zlist[lb + (q - eo)];
                } else if (p < nn) {
                    const uint64_t hk = a.hkeys[h0 + (p - nL)];
                    key = ((uint32_t)((int64_t)(hk >> a.bz) - xa) << a.bz) | ((uint32_t)hk & a.zmask);
                }
                k[j] = key;
            }
        }

        // LSD radix sort: 5-bit digits over the significant bits
        const int xbits = (xb - xa - 1) > 0 ? 32 - __clz((uint32_t)(xb - xa - 1)) : 0;
        const int B = xbits + a.bz > 0 ? xbits + a.bz : 1;
        const int passes = (B + kRB - 1) / kRB;
        uint16_t *c16 = reinterpret_cast<uint16_t *>(cnt);
        for (int pass = 0; pass < passes; ++pass) {
            const int shift = pass * kRB;
            for (int i = tid; i < kRD * kDT / 2; i += kDT) cnt[i] = 0;
            __syncthreads();
            uint16_t loc[kDI];
#pragma unroll
            for (int j = 0; j < kDI; ++j) {
                const int p = tid * kDI + j;
                const uint32_t d = (k[j] >> shift) & (kRD - 1);
                const int ci = (int)d * kDT + tid;
                const uint16_t c = c16[ci];
                loc[j] = c;
                if (p < nn) c16[ci] = (uint16_t)(c + 1);
            }
            __syncthreads();
            // raking exclusive scan over [digit][thread]: thread t owns `per`
            // consecutive words (two 16-bit counters each)
            constexpr int per = kRD * kDT / 2 / kDT;
            uint32_t s = 0;
#pragma unroll
            for (int i = 0; i < per; ++i) {
                const uint32_t wv = cnt[tid * per + i];
                s += (wv & 0xffffu) + (wv >> 16);
            }
            uint32_t all;
            uint32_t run = block_excl_scan<kDT>(s, lds_scan, &all);
#pragma unroll
            for (int i = 0; i < per; ++i) {
                const uint32_t wv = cnt[tid * per + i];
                const uint32_t lo = wv & 0xffffu, hi = wv >> 16;
                const uint32_t p0 = run, p1 = run + lo;
                run += lo + hi;
                cnt[tid * per + i] = (p0 & 0xffffu) | (p1 << 16);
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kDI; ++j) {
                const int p = tid * kDI + j;
                if (p < nn) {
                    const uint32_t d = (k[j] >> shift) & (kRD - 1);
                    const uint32_t dst = (uint32_t)c16[(int)d * kDT + tid] + loc[j];
                    sk[dst < (uint32_t)kDCap ? dst : 0] = k[j];
                }
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kDI; ++j) {
                const int p = tid * kDI + j;
                k[j] = p < nn ? sk[p] : 0xffffffffu;
            }
            __syncthreads();
        }
        // first of every run of equal keys, compacted into sk in order
        uint32_t flags = 0, mine = 0;
        uint32_t prev = (tid > 0 && tid * kDI - 1 < nn) ? sk[tid * kDI - 1] : 0u;
#pragma unroll
        for (int j = 0; j < kDI; ++j) {
            const int p = tid * kDI + j;
            const bool f = (p < nn) & ((p == 0) | (k[j] != prev));
            flags |= (uint32_t)f << j;
            mine += f ? 1u : 0u;
            prev = k[j];
        }
        uint32_t d_all;
        uint32_t pos = block_excl_scan<kDT>(mine, lds_scan, &d_all);
#pragma unroll
        for (int j = 0; j < kDI; ++j)
            if ((flags >> j) & 1u) sk[pos++] = k[j];
        if (tid < kWave) {
            const int64_t ex = look_back(a, u, (int64_t)d_all);
            if (tid == 0) sh[1] = ex;
        }
        __syncthreads();
        const int64_t base = sh[1];
        if (u == a.n_units - 1 && tid == 0) *a.total = base + d_all;
        for (uint32_t i = tid; i < d_all; i += kDT) {
            const uint32_t key = sk[i];
            const int64_t o = base + i;
            const int64_t xi = (int64_t)xa + (key >> a.bz), zi = key & a.zmask;
            const bool ok = (o < a.cap) & (xi < a.dom_x) & (zi < a.dom_z);
            if (!ok) *a.err = 3;
            if (o < a.cap) {
                a.out_x[o] = a.xorig[ok ? xi : 0];
                a.out_z[o] = a.zorig[ok ? zi : 0];
            }
        }
        return;
    }

    // ---------------------------------------------------------------- window unit
    const int64_t x = xa;
    const int64_t tx = a.toff[x + 1] - a.toff[x];
    const int64_t nw = windows_of(tx, a.dom_z);
    const int64_t ws = cdiv(a.dom_z, nw);
    const int64_t zlo = (int64_t)win * ws;
    const int64_t zhi = zlo + ws < a.dom_z ? zlo + ws : a.dom_z;
    const int64_t wbits = zhi > zlo ? zhi - zlo : 0;  // <= kWinBits
    const int nwords = (int)cdiv(wbits, 32);
    for (int i = tid; i < nwords; i += kDT) sk[i] = 0;
    __syncthreads();
    const int64_t e0 = a.off_x[x], e1 = a.off_x[x + 1];
    // lists of x in chunks of kListChunk; the heavy nonzeros of x are one more list
    const int64_t nlists = (e1 - e0) + 1;
    for (int64_t l0 = 0; l0 < nlists; l0 += kListChunk) {
        int64_t b = 0, len = 0;
        const int64_t l = l0 + tid;
        if (l < nlists) {
            if (l < e1 - e0) {
                const int64_t e = e0 + l;
                const int64_t lb = a.lbase[e];
                const int64_t ln = a.eoff[e + 1] - a.eoff[e];
                const int32_t *L = a.zlist + lb;
                const int64_t s0 = lower_bound_dev(L, (int64_t)0, ln, (int32_t)zlo);
                const int64_t s1 = lower_bound_dev(L, s0, ln, (int32_t)zhi);
                b = lb + s0;
                len = s1 - s0;
            } else {
                const int64_t h0 = a.hoff[x], h1 = a.hoff[x + 1];
                const uint64_t kx = (uint64_t)x << a.bz;
                const int64_t s0 = lower_bound_dev(a.hkeys, h0, h1, kx | (uint64_t)zlo);
                const int64_t s1 = lower_bound_dev(a.hkeys, s0, h1, kx | (uint64_t)zhi);
                b = -1 - s0;  // negative: heavy keys starting at s0
                len = s1 - s0;
            }
        }
        int64_t tot;
        const int64_t pre = block_excl_scan<kDT>(len, lds_scan64, &tot);
        lpre[tid] = pre;
        lbeg[tid] = b;
        if (tid == 0) lpre[kListChunk] = tot;
        __syncthreads();
        const int64_t nl = (nlists - l0) < kListChunk ? (nlists - l0) : kListChunk;
        for (int64_t p = tid; p < tot; p += kDT) {
            const int64_t li = upper_bound_dev(lpre, (int64_t)0, nl, p) - 1;
            const int64_t bb = lbeg[li];
            const int64_t off = p - lpre[li];
            const int64_t z = bb >= 0 ? (int64_t)a.zlist[bb + off]
                                      : (int64_t)((uint32_t)a.hkeys[-1 - bb + off] & a.zmask);
            const int64_t zr = z - zlo;
            if ((zr >= 0) & (zr < wbits)) atomicOr(&sk[zr >> 5], 1u << (zr & 31));
        }
        __syncthreads();
    }
    // distinct count, offset, then set bits in z order: rounds of kDT words
    uint32_t c = 0;
    for (int i = tid; i < nwords; i += kDT) c += __popc(sk[i]);
    uint32_t d_all;
    (void)block_excl_scan<kDT>(c, lds_scan, &d_all);
    if (tid < kWave) {
        const int64_t ex = look_back(a, u, (int64_t)d_all);
        if (tid == 0) sh[1] = ex;
    }
    __syncthreads();
    int64_t base = sh[1];
    if (u == a.n_units - 1 && tid == 0) *a.total = base + d_all;
    const int32_t xo = a.xorig[x < a.dom_x ? x : 0];
    for (int r0 = 0; r0 < nwords; r0 += kDT) {
        const int i = r0 + tid;
        uint32_t word = i < nwords ? sk[i] : 0u;
        uint32_t rt;
        int64_t o = base + block_excl_scan<kDT>((uint32_t)__popc(word), lds_scan, &rt);
        while (word) {
            const int bit = __ffs(word) - 1;
            word &= word - 1;
            const int64_t zi = zlo + (int64_t)i * 32 + bit;
            if (o < a.cap) {
                a.out_x[o] = xo;
                a.out_z[o] = a.zorig[zi < a.dom_z ? zi : 0];
            } else {
                *a.err = 3;
            }
            ++o;
        }
        base += rt;
    }
}

}  // namespace

bool segmented_dedup_fits(int bz) { return bz <= 26; }

void segmented_dedup(const Ctx &c, const SegDedupIn &in, DBuf<int32_t> *out_x, DBuf<int32_t> *out_z,
                     int64_t *n_out, SegDedupStats *stats) {
    JP_CHECK(segmented_dedup_fits(in.bz), JP_EINTERNAL, "segmented dedup needs bz <= 26");
    const int64_t dom_x = in.dom_x, dom_z = in.dom_z;
    DBuf<int64_t> scal = c.buf<int64_t>(8);
    int64_t *S = scal.get();
    c.zero(S, 8);

    // heavy nonzeros before every x
    DBuf<int64_t> hoff = c.buf<int64_t>(dom_x + 1);
    {
        int64_t *ho = hoff.get();
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
    }
    // candidates before every x
    DBuf<int64_t> toff = c.buf<int64_t>(dom_x + 1);
    {
        const int64_t *ox = in.off_x, *eo = in.eoff, *ho = hoff.get();
        auto tx = [=] __device__(int64_t x) -> int64_t {
            return (eo[ox[x + 1]] - eo[ox[x]]) + (ho[x + 1] - ho[x]);
        };
        int64_t *to = toff.get();
        scan_exclusive(c, dom_x, tx, ArrayPut{to}, to + dom_x);
    }

    // Units in x order.  A small x starts a packed unit when it is the first
    // x, follows a large x, begins a new kUnitCap window of candidate offsets,
    // or begins a new block of 2^(32-bz) x values (local keys fit 32 bits).
    // A large x contributes windows_of(...) window units.
    const int kb = 32 - in.bz;
    DBuf<int64_t> nunits_x = c.buf<int64_t>(dom_x + 1);
    {
        const int64_t *to = toff.get();
        int64_t *nu = nunits_x.get();
        const int64_t dz = dom_z;
        scan_exclusive(
            c, dom_x,
            [=] __device__(int64_t x) -> int64_t {
                const int64_t t = to[x + 1] - to[x];
                if (t > kUnitCap) return windows_of(t, dz);
                if (x == 0) return 1;
                const bool prev_big = to[x] - to[x - 1] > kUnitCap;
                const bool newwin = (to[x] / kUnitCap) != (to[x - 1] / kUnitCap);
                const bool newblk = kb < 31 ? ((x >> kb) != ((x - 1) >> kb)) : false;
                return (prev_big | newwin | newblk) ? 1 : 0;
            },
            ArrayPut{nu}, nu + dom_x);
    }
    int64_t hn[1];
    c.load_n(hn, nunits_x.get() + dom_x, 1);
    const int64_t n_units = hn[0];
    const int64_t n_cand = c.load(toff.get() + dom_x);
    DBuf<int32_t> ustart = c.buf<int32_t>(n_units + 1), uwin = c.buf<int32_t>(n_units + 1);
    {
        const int64_t *to = toff.get(), *nu = nunits_x.get();
        int32_t *us = ustart.get(), *uw = uwin.get();
        for_each(c, dom_x, [=] __device__(int64_t x) {
            const int64_t b = nu[x], m = nu[x + 1] - b;
            const bool big = to[x + 1] - to[x] > kUnitCap;
            for (int64_t i = 0; i < m; ++i) {
                us[b + i] = (int32_t)x;
                uw[b + i] = big ? (int32_t)i : -1;
            }
        });
        const int64_t nun = n_units, dx = dom_x;
        for_each(c, 1, [=] __device__(int64_t) {
            us[nun] = (int32_t)dx;
            uw[nun] = -1;
        });
    }
    dump(c, "ustart", ustart.get(), n_units + 1);
    dump(c, "uwin", uwin.get(), n_units + 1);

    *out_x = c.buf<int32_t>(std::max<int64_t>(n_cand, 1));
    *out_z = c.buf<int32_t>(std::max<int64_t>(n_cand, 1));
    DBuf<unsigned long long> status = c.buf<unsigned long long>(std::max<int64_t>(n_units, 1));
    DBuf<unsigned int> ticket = c.buf<unsigned int>(1);
    c.zero(status.get(), std::max<int64_t>(n_units, 1));
    c.zero(ticket.get(), 1);
    if (n_units > 0) {
        JP_CHECK(n_units < (1ll << 31), JP_EINVAL, "too many dedup units for one launch");
        DedupArgs a;
        a.ustart = ustart.get();
        a.uwin = uwin.get();
        a.n_units = n_units;
        a.toff = toff.get();
        a.off_x = in.off_x;
        a.eoff = in.eoff;
        a.lbase = in.lbase;
        a.r_xr = in.r_xr;
        a.zlist = in.zlist;
        a.hkeys = in.hkeys;
        a.hoff = hoff.get();
        a.bz = in.bz;
        a.zmask = (uint32_t)((1ull << in.bz) - 1);
        a.dom_x = dom_x;
        a.dom_z = dom_z;
        a.xorig = in.xorig;
        a.zorig = in.zorig;
        a.out_x = out_x->get();
        a.out_z = out_z->get();
        a.cap = n_cand;
        a.status = status.get();
        a.ticket = ticket.get();
        a.total = S + 0;
        a.err = S + 1;
        hipLaunchKernelGGL(k_dedup, dim3((unsigned)n_units), dim3(kDT), 0, c.stream, a);
        JP_HIP(hipGetLastError());
    }
    int64_t h2[2];
    c.load_n(h2, S, 2);
    JP_CHECK(h2[1] != 1, JP_EINTERNAL, "a dedup unit exceeded its on-chip capacity");
    JP_CHECK(h2[1] != 2, JP_EINTERNAL, "dedup look-back did not complete");
    JP_CHECK(h2[1] == 0, JP_EINTERNAL, "dedup produced a key outside the rank tables");
    *n_out = h2[0];
    if (stats) {
        stats->n_units = n_units;
        stats->n_cand = n_cand;
    }
}

}  // namespace jp
