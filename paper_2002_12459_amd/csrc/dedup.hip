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
//    kDCap candidates; a medium x (at most kDCap) is a unit of its own.  A
//    unit gathers its candidates as 32-bit keys (x - first_x) << bz | z,
//    sorts them by LSD radix sort in LDS over the significant bits only
//    (5-bit digits, per-thread 16-bit counters updated by LDS atomics that
//    return the old count, raking scan), and keeps the first of every run of
//    equal keys.  Unit size is set so four workgroups fit a CU (LDS and
//    registers): the kernel is bound by memory and LDS latency.
//  * a large x (more than kDCap) is cut into z windows.  A window unit
//    binary-searches the window's part of every sorted list and counts the
//    candidates; if they fit a unit it gathers and sorts them like a packed
//    unit, else it marks them in an LDS bitmap (kWinBits z values at a time)
//    and reads the set bits back in z order.  Windows of an x with up to
//    4 kDCap candidates are sized to fit a unit; larger x get fewer, wider
//    windows (fewer list searches) that use the bitmap.
//
// One kernel handles all units.  A unit writes its distinct keys to a
// staging array at its candidate offset (an upper bound of its output
// offset, so units never wait on each other); a scan of the per-unit counts
// gives output offsets, and a copy (one workgroup per unit) packs the output
// and turns keys back into ids.
#include "debug.hpp"
#include "pipeline.hpp"
#include "prims.hpp"
#include "segdedup.hpp"

namespace jp {
namespace {

constexpr int kDT = 256;                 // threads per unit
constexpr int kDI = 20;                  // keys per thread (4 workgroups per CU by LDS and registers)
constexpr int kDCap = kDT * kDI;         // keys per unit
constexpr int64_t kUnitCap = kDCap / 2;  // x with more candidates get a unit of their own
constexpr int64_t kSoloCap = kDCap;      // x with more candidates get window units
constexpr int kRB = 5;                   // radix digit bits
constexpr int kRD = 1 << kRB;            // digits
constexpr int64_t kWinBits = (int64_t)kDCap * 32;  // bitmap window capacity (reuses the key buffer)
constexpr int64_t kWinTarget = 16384;              // candidates per bitmap window unit, aimed for
constexpr int64_t kWinSort = (3 * kDCap) / 4;      // candidates per sorted window unit, aimed for
constexpr int kListChunk = kDT;                    // lists handled per round in a window unit
constexpr int kWinBatch = 4;                       // window candidates per thread with loads in flight
constexpr int kWriteBatch = 8;                     // distinct keys per thread read from LDS before storing

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Windows of an x with more than kDCap candidates, at least 64 z values
// wide.  Up to 4 kDCap candidates: about kWinSort each, so a window usually
// fits one unit's sort.  More: about kWinTarget each and at least enough to
// fit the LDS bitmap (fewer, wider windows mean fewer list searches).
__host__ __device__ inline int64_t windows_of(int64_t tx, int64_t dom_z) {
    const int64_t hi = cdiv(dom_z, 64) > 1 ? cdiv(dom_z, 64) : 1;
    int64_t want;
    if (tx <= 4 * kDCap) {
        want = cdiv(tx, kWinSort);
    } else {
        want = cdiv(tx, kWinTarget);
        const int64_t lo = cdiv(dom_z, kWinBits);
        if (want < lo) want = lo;
    }
    if (want > hi) want = hi;
    return want < 1 ? 1 : want;
}

// Where a packed unit's candidates are, computed ahead by a setup kernel so
// the unit starts with one load instead of a chain of dependent ones.
struct UnitDesc {
    int64_t e0, e1;  // R tuples of the unit's x range
    int64_t c0;      // light candidates before tuple e0
    int64_t h0;      // heavy nonzeros before the unit's first x
    int64_t nL, n;   // light candidates, all candidates
};

struct DedupArgs {
    const UnitDesc *udesc;   // per unit (packed units only)
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
    uint32_t *stage;         // distinct keys (x - unit's first x) << bz | z of every unit, at ubase[u]
    int64_t *ucount;         // distinct pairs of every unit
    int64_t *ubase;          // where the unit's pairs start in stage
    int64_t *err;
    unsigned long long *clk; // optional per-phase cycle totals (JP_PHASE_CLOCKS)
    // Window boundaries in the lists of every large x: for list l of x and
    // boundary b (0..nw), wpos[wposx[x] + l*(nw + 1) + b] is the first entry
    // of the list at or above min(b*ws, dom_z) (ws = window width).
    const uint32_t *wpos;    // (list positions are below 2^32); nullptr: search instead
    const int64_t *wposx;    // dom_x + 1
};

// Phase clock: thread 0 adds the cycles since the last mark to clk[phase].
// The last mark lives in LDS, so that a launch without clocks keeps no
// timestamp in registers.
struct PhaseClock {
    unsigned long long *clk;
    long long *t;  // LDS
    __device__ PhaseClock(unsigned long long *c, long long *slot) : clk(c), t(slot) {
        if (clk && threadIdx.x == 0) *t = clock64();
    }
    __device__ void mark(int phase) {
        if (clk && threadIdx.x == 0) {
            const long long now = clock64();
            atomicAdd(&clk[phase], (unsigned long long)(now - *t));
            *t = now;
        }
    }
};
enum { kPhGather, kPhSort, kPhUnique, kPhWritePacked, kPhLists, kPhWriteWin, kPhUnitsPacked, kPhUnitsWin,
       kPhCount };

// LDS layouts padded against bank conflicts: key slot i and counter word w.
// (one pad word after every kDI keys: thread t's own keys t*kDI + j sit at
// t*(kDI + 1) + j, one base register and immediate offsets, and an odd row
// stride puts the 64 lanes of a wave in 64 different banks)
__device__ __forceinline__ int kpad(int i) { return i + i / kDI; }
__device__ __forceinline__ int cpad(int w) { return w + (w >> 4); }
constexpr int kSkWords = kDCap + kDCap / kDI;
constexpr int kCntWords = kRD * kDT / 2;
constexpr int kCntPadded = kCntWords + kCntWords / 16;
constexpr int kMaxStagedEdges = 1024;  // R tuples of a packed unit staged in LDS for the gather
static_assert(4 * (kMaxStagedEdges + 2) + 12 * kMaxStagedEdges <= 4 * kCntPadded, "staging fits the counters");


// max(x, x moved by the DPP control CTRL in the rows of ROWS); a lane with
// no source (or in a row outside ROWS) takes 0, which leaves x unchanged.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_max(uint32_t x) {
    const uint32_t t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xf, false);
    return t > x ? t : x;
}

// Exclusive max-scan over the threads of the workgroup (0 for thread 0); the
// wave part by DPP in the steps of wave_incl_scan.
__device__ __forceinline__ uint32_t block_excl_max(uint32_t v, uint32_t *lds) {
    const int lane = lane_id(), w = threadIdx.x / kWave;
    uint32_t inc = v;
    inc = dpp_max<0x111, 0xf>(inc);  // row_shr:1
    inc = dpp_max<0x112, 0xf>(inc);  // row_shr:2
    inc = dpp_max<0x114, 0xf>(inc);  // row_shr:4
    inc = dpp_max<0x118, 0xf>(inc);  // row_shr:8
    inc = dpp_max<0x142, 0xa>(inc);  // row_bcast:15 into rows 1, 3
    inc = dpp_max<0x143, 0xc>(inc);  // row_bcast:31 into rows 2, 3
    if (lane == kWave - 1) lds[w] = inc;
    __syncthreads();
    uint32_t r = __shfl_up(inc, 1);
    if (lane == 0) r = 0;
    for (int q = 0; q < w; ++q) r = lds[q] > r ? lds[q] : r;
    __syncthreads();
    return r;
}

// Thread t's counter of digit d is counter d * kDT + t: the 16-bit half
// (t & 1) of word cpad((d * kDT + t) / 2) = d * kDigitWords + t / 2 + t / 32
// (kDT / 2 is a multiple of 16, so the digit's part of the pad splits off).
static_assert(kDT % 32 == 0, "counter word split");
constexpr int kDigitWords = kDT / 2 + kDT / 32;

// One LSD pass over digit (k >> shift) & (kRD - 1) of the unit's keys.
// STR: the keys are in the striped layout (slot j of thread t holds position
// j * kDT + t) and positions from nn on are not counted; otherwise the
// layout is t * kDI + j and every slot is counted: slots from nn on hold
// 0xffffffff, which sorts after every key of the sorted bits (its bits above
// them are ones) or, where those bits tie, keeps its place after the keys
// (ties keep their order, and those slots are last).  Leaves the layout
// t * kDI + j, with 0xffffffff from nn on.
template <bool STR>
__device__ __forceinline__ void unit_pass(uint32_t (&k)[kDI], int nn, int shift, bool clear_after, uint32_t *sk,
                                          uint32_t *cnt, uint32_t *lds_scan) {
    const int tid = threadIdx.x;
    const int tword = (tid >> 1) + (tid >> 5);
    const int tsh = 16 * (tid & 1);
    // count with LDS atomics that return the old value: the updates of one
    // thread issue back to back instead of as dependent read-modify-writes (a
    // thread's counter stays below 2^16)
    uint16_t loc[kDI];
#pragma unroll
    for (int j = 0; j < kDI; ++j) {
        const int d = (int)((k[j] >> shift) & (kRD - 1));
        const bool valid = !STR || j * kDT + tid < nn;
        const uint32_t old = atomicAdd(&cnt[d * kDigitWords + tword], (valid ? 1u : 0u) << tsh);
        loc[j] = (uint16_t)(old >> tsh);
    }
    __syncthreads();
    // raking exclusive scan over [digit][thread]: thread t owns `per`
    // consecutive counter words (two 16-bit counters each)
    constexpr int per = kCntWords / kDT;
    constexpr int kGrp = 8;
    static_assert(per % kGrp == 0, "whole groups");
    uint32_t s = 0;
#pragma unroll
    for (int g = 0; g < per; g += kGrp) {
        uint32_t wv[kGrp];
#pragma unroll
        for (int i = 0; i < kGrp; ++i) wv[i] = cnt[cpad(tid * per + g + i)];
#pragma unroll
        for (int i = 0; i < kGrp; ++i) s += (wv[i] & 0xffffu) + (wv[i] >> 16);
    }
    uint32_t all;
    uint32_t run = block_excl_scan<kDT>(s, lds_scan, &all);
    // write-back in groups of eight words as well: the group's reads are
    // issued together, then its writes (one LDS round trip per group)
#pragma unroll
    for (int g = 0; g < per; g += kGrp) {
        uint32_t wv[kGrp];
#pragma unroll
        for (int i = 0; i < kGrp; ++i) wv[i] = cnt[cpad(tid * per + g + i)];
#pragma unroll
        for (int i = 0; i < kGrp; ++i) {
            const uint32_t lo = wv[i] & 0xffffu, hi = wv[i] >> 16;
            const uint32_t q0 = run, q1 = run + lo;
            run += lo + hi;
            cnt[cpad(tid * per + g + i)] = (q0 & 0xffffu) | (q1 << 16);
        }
    }
    __syncthreads();
    // scatter without branches, in groups whose counter reads issue together
    // (a striped slot past nn writes the last row's pad word, which no key
    // slot uses)
    constexpr int kScatGrp = 5;
    static_assert(kDI % kScatGrp == 0, "whole groups");
#pragma unroll
    for (int g = 0; g < kDI; g += kScatGrp) {
        uint32_t cb[kScatGrp];
#pragma unroll
        for (int i = 0; i < kScatGrp; ++i)
            cb[i] = (cnt[(int)((k[g + i] >> shift) & (kRD - 1)) * kDigitWords + tword] >> tsh) & 0xffffu;
#pragma unroll
        for (int i = 0; i < kScatGrp; ++i) {
            const int j = g + i;
            const uint32_t dst = cb[i] + loc[j];
            const int slot = kpad(dst < (uint32_t)kDCap ? (int)dst : 0);
            sk[(STR && j * kDT + tid >= nn) ? kSkWords - 1 : slot] = k[j];
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kDI; ++j) {
        const uint32_t v = sk[kpad(tid * kDI + j)];
        k[j] = (STR && tid * kDI + j >= nn) ? 0xffffffffu : v;
    }
    if (clear_after)
        for (int i = tid; i < kCntPadded; i += kDT) cnt[i] = 0;
    __syncthreads();
}

// Sorts the nn keys in k[] on their low B bits by LSD radix sort in LDS:
// 5-bit digits, per-thread 16-bit counters updated by LDS atomics, raking
// scan.  Thread t's slot j holds key t*kDI + j of the current order (valid
// below nn; 0xffffffff from nn on), or, when `striped`, key j*kDT + t (valid
// below nn) on entry; every pass leaves the first layout.  Leaves the
// distinct keys in sk[kpad(0 .. result)), in order.
__device__ __forceinline__ uint32_t sort_unique(uint32_t (&k)[kDI], int nn, int B, uint32_t *sk, uint32_t *cnt,
                                                uint32_t *lds_scan, PhaseClock &pc, bool striped = false) {
    const int tid = threadIdx.x;
    const int passes = (B > 0 ? B + kRB - 1 : kRB) / kRB;
    // counters cleared here for the first pass, then by each pass's read-back
    // for the next (no barrier of their own)
    for (int i = tid; i < kCntPadded; i += kDT) cnt[i] = 0;
    __syncthreads();
    int pass = 0;
    if (striped) {
        unit_pass<true>(k, nn, 0, passes > 1, sk, cnt, lds_scan);
        pass = 1;
    }
    for (; pass < passes; ++pass) unit_pass<false>(k, nn, pass * kRB, pass + 1 < passes, sk, cnt, lds_scan);
    pc.mark(kPhSort);
    // first of every run of equal keys, compacted into sk in order
    uint32_t flags = 0, mine = 0;
    uint32_t prev = (tid > 0 && tid * kDI - 1 < nn) ? sk[kpad(tid * kDI - 1)] : 0u;
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
        if ((flags >> j) & 1u) sk[kpad((int)pos++)] = k[j];
    __syncthreads();
    return d_all;
}

__global__ __launch_bounds__(kDT, 4) void k_dedup(DedupArgs a) {  // 4 workgroups per CU: at most 128 VGPRs
    __shared__ uint32_t sk[kSkWords];     // keys, then distinct keys; or the window bitmap
    __shared__ __attribute__((aligned(8))) uint32_t cnt[kCntPadded];  // digit counters; before that, staged tuples
    __shared__ uint32_t lds_scan[kDT / kWave + 1];
    __shared__ int64_t lds_scan64[kDT / kWave + 1];

    __shared__ long long clock_slot;
    const int tid = threadIdx.x;
    PhaseClock pc(a.clk, &clock_slot);
    const int64_t u = blockIdx.x;
    const int32_t xa = a.ustart[u];
    const int32_t win = a.uwin[u];

    if (win < 0) {
        // ------------------------------------------------------------ packed unit
        const int32_t xb = a.ustart[u + 1];
        const UnitDesc ud = a.udesc[u];
        const int64_t e0 = ud.e0, e1 = ud.e1, c0 = ud.c0, nL = ud.nL, h0 = ud.h0, n = ud.n;
        const bool over = n > kDCap;
        if (over && tid == 0) *a.err = 1;
        const int nn = over ? 0 : (int)n;
        const int nLc = over ? 0 : (int)nL;

        // stage the unit's R tuples (offsets relative to the unit, list
        // starts, local x) in LDS when they fit
        const int64_t ne = e1 - e0;
        const bool staged = ne <= kMaxStagedEdges;
        int64_t *slb = reinterpret_cast<int64_t *>(cnt);               // ne
        int32_t *seo = reinterpret_cast<int32_t *>(slb + kMaxStagedEdges);  // ne + 1
        int32_t *sxl = seo + kMaxStagedEdges + 2;                          // ne
        if (staged) {
            for (int i = tid; i <= ne; i += kDT) seo[i] = (int32_t)(a.eoff[e0 + i] - c0);
            for (int i = tid; i < ne; i += kDT) {
                slb[i] = a.lbase[e0 + i];
                sxl[i] = a.r_xr[e0 + i] - xa;
            }
        }
        __syncthreads();

        uint32_t k[kDI];
        if (staged) {
            // Candidate p of the unit belongs to the tuple whose list covers
            // it: each nonempty tuple i writes i + 1 at its first candidate,
            // and an inclusive max-scan over the candidates fills the rest
            // (sk is free until the sort).  Thread t then takes candidates
            // j*kDT + t, so each load instruction reads 64 consecutive
            // candidates, mostly consecutive list entries.
            uint16_t *ct = reinterpret_cast<uint16_t *>(sk);  // kDCap entries
            for (int i = tid; i < kDCap / 2; i += kDT) sk[i] = 0u;
            __syncthreads();
            for (int i = tid; i < ne; i += kDT) {
                const int32_t s0 = seo[i];
                if (seo[i + 1] > s0 && s0 < nLc) ct[s0] = (uint16_t)(i + 1);
            }
            __syncthreads();
            uint32_t m = 0;
#pragma unroll
            for (int j = 0; j < kDI; ++j) {
                const uint32_t h = ct[tid * kDI + j];
                m = h > m ? h : m;
            }
            uint32_t run = block_excl_max(m, lds_scan);
#pragma unroll
            for (int j = 0; j < kDI; ++j) {
                const uint32_t h = ct[tid * kDI + j];
                run = h > run ? h : run;
                ct[tid * kDI + j] = (uint16_t)run;
            }
            __syncthreads();
            // each list load is issued as soon as its position is known (no
            // array of positions stays live); the ORs come after all loads
            uint32_t z[kDI];
#pragma unroll
            for (int j = 0; j < kDI; ++j) {
                const int p = j * kDT + tid;
                uint32_t key = 0xffffffffu, sj = 0;
                if (p < nLc) {
                    const int e = (int)ct[p] - 1;
                    key = (uint32_t)sxl[e] << a.bz;
                    sj = (uint32_t)(slb[e] + (p - seo[e]));
                } else if (p < nn) {
                    const uint64_t hk = a.hkeys[h0 + (p - nL)];
                    key = ((uint32_t)((int64_t)(hk >> a.bz) - xa) << a.bz) | ((uint32_t)hk & a.zmask);
                }
                k[j] = key;
                z[j] = (uint32_t)a.zlist[sj];
            }
#pragma unroll
            for (int j = 0; j < kDI; ++j) k[j] = j * kDT + tid < nLc ? (k[j] | z[j]) : k[j];
        } else {
            // tuples not staged: thread t takes candidates [t*kDI, t*kDI + kDI),
            // found by one search in the offsets and then a walk
            const int p0 = tid * kDI;
            int64_t e = 0;  // relative to e0
            if (p0 < nLc) e = upper_bound_dev(a.eoff, e0, e1, c0 + p0) - 1 - e0;
            int32_t eo = 0, enext = 0;
            int64_t lb = 0;
            uint32_t xl = 0;
            if (p0 < nLc) {
                eo = (int32_t)(a.eoff[e0 + e] - c0);
                enext = (int32_t)(a.eoff[e0 + e + 1] - c0);
                lb = a.lbase[e0 + e];
                xl = (uint32_t)(a.r_xr[e0 + e] - xa) << a.bz;
            }
            // list positions first, then every list load in one straight run
            // so all of them are in flight
            uint32_t src[kDI];
#pragma unroll
            for (int j = 0; j < kDI; ++j) {
                const int p = p0 + j;
                uint32_t key = 0xffffffffu, sj = 0;
                if (p < nLc) {
                    while (p >= enext) {  // next R tuple with a nonempty list
                        ++e;
                        eo = enext;
                        enext = (int32_t)(a.eoff[e0 + e + 1] - c0);
                        lb = a.lbase[e0 + e];
                        xl = (uint32_t)(a.r_xr[e0 + e] - xa) << a.bz;
                    }
                    key = xl;
                    sj = (uint32_t)(lb + (p - eo));
                } else if (p < nn) {
                    const uint64_t hk = a.hkeys[h0 + (p - nL)];
                    key = ((uint32_t)((int64_t)(hk >> a.bz) - xa) << a.bz) | ((uint32_t)hk & a.zmask);
                }
                k[j] = key;
                src[j] = sj;
            }
#pragma unroll
            for (int j = 0; j < kDI; ++j) {
                const uint32_t z = (uint32_t)a.zlist[src[j]];
                k[j] = p0 + j < nLc ? (k[j] | z) : k[j];
            }
        }
        __syncthreads();  // staged tuple data is overwritten by the counters below
        pc.mark(kPhGather);

        const int xbits = (xb - xa - 1) > 0 ? 32 - __clz((uint32_t)(xb - xa - 1)) : 0;
        const uint32_t d_all = sort_unique(k, nn, xbits + a.bz, sk, cnt, lds_scan, pc, staged);
        pc.mark(kPhUnique);
        const int64_t base = a.toff[xa];
        for (uint32_t i0 = tid; i0 < d_all; i0 += kDT * kWriteBatch) {  // LDS reads, then stores
            uint32_t v[kWriteBatch];
#pragma unroll
            for (int r = 0; r < kWriteBatch; ++r) {
                const uint32_t i = i0 + r * kDT;
                v[r] = sk[kpad((int)(i < d_all ? i : i0))];
            }
#pragma unroll
            for (int r = 0; r < kWriteBatch; ++r)
                if (i0 + r * kDT < d_all) a.stage[base + i0 + r * kDT] = v[r];
        }
        if (tid == 0) {
            a.ucount[u] = d_all;
            a.ubase[u] = base;
        }
        pc.mark(kPhWritePacked);
        if (a.clk && tid == 0) atomicAdd(&a.clk[kPhUnitsPacked], 1ull);
        return;
    }

    // ---------------------------------------------------------------- window unit
    const int64_t x = xa;
    const int64_t tx = a.toff[x + 1] - a.toff[x];
    const int64_t nw = windows_of(tx, a.dom_z);
    const int64_t ws = cdiv(a.dom_z, nw);
    const int64_t zlo = (int64_t)win * ws;
    const int64_t zhi = zlo + ws < a.dom_z ? zlo + ws : a.dom_z;
    int64_t *lpre = reinterpret_cast<int64_t *>(cnt);  // kListChunk + 1
    int64_t *lbeg = lpre + kListChunk + 1;             // kListChunk
    const int64_t e0 = a.off_x[x], e1 = a.off_x[x + 1];
    // The lists of x, in chunks of kListChunk, plus the heavy nonzeros of x as
    // one more list.  list_range(l, lo, hi): start (negative: heavy keys at
    // -1 - start) and length of list l's part in [lo, hi), and how many of
    // its entries lie below lo.
    const int64_t nlists = (e1 - e0) + 1;
    auto list_range = [&](int64_t l, int64_t lo, int64_t hi, int64_t &b, int64_t &len, int64_t &below) {
        b = 0;
        len = 0;
        below = 0;
        if (l >= nlists) return;
        if (a.wpos && l < e1 - e0 && lo == zlo && hi == zhi) {  // the window itself: from the boundary table
            const int64_t e = e0 + l;
            const uint32_t *P = a.wpos + a.wposx[x] + l * (nw + 1) + win;
            const int64_t s0 = P[0], s1 = P[1];
            b = a.lbase[e] + s0;
            len = s1 - s0;
            below = s0;
        } else if (l < e1 - e0) {
            const int64_t e = e0 + l;
            const int64_t lb = a.lbase[e];
            const int64_t ln = a.eoff[e + 1] - a.eoff[e];
            const int32_t *L = a.zlist + lb;
            // first entries >= lo and >= hi, searched in lockstep (two
            // independent loads per step instead of two chains of steps):
            // p0 / p1 end at the last entry below lo / hi
            int64_t p0 = -1, p1 = -1;
            for (int64_t step = ln > 0 ? (int64_t)1 << (63 - __clzll((unsigned long long)ln)) : 0; step > 0;
                 step >>= 1) {
                const int64_t q0 = p0 + step, q1 = p1 + step;
                const int64_t v0 = q0 < ln ? (int64_t)L[q0] : INT64_MAX;
                const int64_t v1 = q1 < ln ? (int64_t)L[q1] : INT64_MAX;
                p0 = v0 < lo ? q0 : p0;
                p1 = v1 < hi ? q1 : p1;
            }
            const int64_t s0 = p0 + 1, s1 = p1 + 1;
            b = lb + s0;
            len = s1 - s0;
            below = s0;
        } else {
            const int64_t h0 = a.hoff[x], h1 = a.hoff[x + 1];
            const uint64_t kx = (uint64_t)x << a.bz;
            const int64_t s0 = lower_bound_dev(a.hkeys, h0, h1, kx | (uint64_t)lo);
            const int64_t s1 = lower_bound_dev(a.hkeys, s0, h1, kx | (uint64_t)hi);
            b = -1 - s0;
            len = s1 - s0;
            below = s0 - h0;
        }
    };
    // fills lpre / lbeg for lists [l0, l0 + kListChunk) over [lo, hi); returns the chunk's candidates
    auto load_chunk = [&](int64_t l0, int64_t lo, int64_t hi) -> int64_t {
        int64_t b, len, below, tot;
        list_range(l0 + tid, lo, hi, b, len, below);
        const int64_t pre = block_excl_scan<kDT>(len, lds_scan64, &tot);
        lpre[tid] = pre;
        lbeg[tid] = b;
        if (tid == 0) lpre[kListChunk] = tot;
        __syncthreads();
        return tot;
    };
    // z of candidate q of the loaded chunk (nl lists).  li is the caller's
    // list of its previous candidate (-1: none); a thread's candidates come
    // in increasing order, so a short forward walk usually finds the list,
    // else a search in the rest of the table.
    auto chunk_z = [&](int64_t q, int64_t nl, int64_t &li) -> int64_t {
        if (li < 0) {
            li = upper_bound_dev(lpre, (int64_t)0, nl, q) - 1;
        } else {
            int steps = 0;
            while (li + 1 < nl && lpre[li + 1] <= q) {
                ++li;
                if (++steps == 4) {
                    li = upper_bound_dev(lpre, li, nl, q) - 1;
                    break;
                }
            }
        }
        const int64_t bb = lbeg[li];
        const int64_t off = q - lpre[li];
        return bb >= 0 ? (int64_t)a.zlist[bb + off] : (int64_t)((uint32_t)a.hkeys[-1 - bb + off] & a.zmask);
    };

    // count the window's candidates and those of x below it (stage offset);
    // with one chunk of lists, its table for the gather is kept
    int64_t before = 0, total = 0;
    const bool one_chunk = nlists <= kListChunk;
    for (int64_t l0 = 0; l0 < nlists; l0 += kListChunk) {
        int64_t b, len, below, t1, t2;
        list_range(l0 + tid, zlo, zhi, b, len, below);
        (void)block_excl_scan<kDT>(below, lds_scan64, &t1);
        const int64_t pre = block_excl_scan<kDT>(len, lds_scan64, &t2);
        if (one_chunk) {
            lpre[tid] = pre;
            lbeg[tid] = b;
            if (tid == 0) lpre[kListChunk] = t2;
        }
        before += t1;
        total += t2;
    }
    __syncthreads();
    const int64_t base = a.toff[x] + before;
    uint32_t d_all = 0;
    if (total <= kDCap) {
        // few enough to sort: gather z - zlo into the key buffer, then registers
        int64_t off = 0;
        for (int64_t l0 = 0; l0 < nlists; l0 += kListChunk) {
            const int64_t tot = one_chunk ? total : load_chunk(l0, zlo, zhi);
            const int64_t nl = (nlists - l0) < kListChunk ? (nlists - l0) : kListChunk;
            int64_t li = -1;
            for (int64_t q0 = tid; q0 < tot; q0 += (int64_t)kDT * kWinBatch) {
                int64_t z[kWinBatch];
#pragma unroll
                for (int r = 0; r < kWinBatch; ++r) {
                    const int64_t q = q0 + (int64_t)r * kDT;
                    z[r] = chunk_z(q < tot ? q : tot - 1, nl, li);
                }
#pragma unroll
                for (int r = 0; r < kWinBatch; ++r) {
                    const int64_t q = q0 + (int64_t)r * kDT;
                    const int64_t dst = off + q;
                    if ((q < tot) & (dst < kDCap)) sk[kpad((int)dst)] = (uint32_t)(z[r] - zlo);
                }
            }
            off += tot;
            __syncthreads();  // lpre / lbeg are refilled by the next chunk
        }
        pc.mark(kPhLists);
        const int nn = (int)total;
        uint32_t k[kDI];
#pragma unroll
        for (int j = 0; j < kDI; ++j) {
            const int p = tid * kDI + j;
            k[j] = p < nn ? sk[kpad(p)] : 0xffffffffu;
        }
        __syncthreads();  // the list tables in the counter space are dead from here
        const int64_t span = zhi - zlo;
        const int B = span > 1 ? 64 - __clzll((unsigned long long)(span - 1)) : 1;
        d_all = sort_unique(k, nn, B, sk, cnt, lds_scan, pc);
        for (uint32_t i0 = tid; i0 < d_all; i0 += kDT * kWriteBatch) {  // local x 0
            uint32_t v[kWriteBatch];
#pragma unroll
            for (int r = 0; r < kWriteBatch; ++r) {
                const uint32_t i = i0 + r * kDT;
                v[r] = sk[kpad((int)(i < d_all ? i : i0))];
            }
#pragma unroll
            for (int r = 0; r < kWriteBatch; ++r)
                if (i0 + r * kDT < d_all) a.stage[base + i0 + r * kDT] = (uint32_t)(zlo + v[r]);
        }
    } else {
        // bitmap of kWinBits z values at a time, set bits read back in z order
        for (int64_t s0 = zlo; s0 < zhi; s0 += kWinBits) {
            const int64_t s1 = s0 + kWinBits < zhi ? s0 + kWinBits : zhi;
            const int64_t wbits = s1 - s0;
            const int nwords = (int)cdiv(wbits, 32);
            for (int i = tid; i < nwords; i += kDT) sk[i] = 0;
            __syncthreads();
            // the counting pass's table is this range's when the window is one range of one chunk
            const bool reuse = one_chunk && s0 == zlo && s1 == zhi;
            for (int64_t l0 = 0; l0 < nlists; l0 += kListChunk) {
                const int64_t tot = reuse ? total : load_chunk(l0, s0, s1);
                const int64_t nl = (nlists - l0) < kListChunk ? (nlists - l0) : kListChunk;
                int64_t li = -1;
                // kWinBatch candidates per thread per round: searches, then loads, then bits
                for (int64_t q0 = tid; q0 < tot; q0 += (int64_t)kDT * kWinBatch) {
                    int64_t z[kWinBatch];
#pragma unroll
                    for (int r = 0; r < kWinBatch; ++r) {
                        const int64_t q = q0 + (int64_t)r * kDT;
                        z[r] = chunk_z(q < tot ? q : tot - 1, nl, li);
                    }
#pragma unroll
                    for (int r = 0; r < kWinBatch; ++r) {
                        const int64_t zr = z[r] - s0;
                        if ((q0 + (int64_t)r * kDT < tot) & (zr >= 0) & (zr < wbits))
                            atomicOr(&sk[zr >> 5], 1u << (zr & 31));
                    }
                }
                __syncthreads();
            }
            pc.mark(kPhLists);
            // set bits in z order: thread t owns a contiguous run of words
            const int per = (nwords + kDT - 1) / kDT;
            const int w0 = tid * per;
            const int w1 = w0 + per < nwords ? w0 + per : nwords;
            uint32_t c = 0;
            for (int i = w0; i < w1; ++i) c += __popc(sk[i]);
            uint32_t sub;
            uint32_t pos = d_all + block_excl_scan<kDT>(c, lds_scan, &sub);
            for (int i = w0; i < w1; ++i) {
                uint32_t word = sk[i];
                while (word) {
                    const int bit = __ffs(word) - 1;
                    word &= word - 1;
                    a.stage[base + pos] = (uint32_t)(s0 + (int64_t)i * 32 + bit);  // local x 0
                    ++pos;
                }
            }
            d_all += sub;
            __syncthreads();  // the bitmap is cleared again for the next range
        }
    }
    if (tid == 0) {
        a.ucount[u] = d_all;
        a.ubase[u] = base;
    }
    pc.mark(kPhWriteWin);
    if (a.clk && tid == 0) atomicAdd(&a.clk[kPhUnitsWin], 1ull);
}

// Window boundary table (see DedupArgs::wpos): entry i belongs to the large
// x whose range of wposx holds it; one binary search in one list per entry.
struct WposArgs {
    const int64_t *wposx, *toff, *off_x, *eoff, *lbase;
    const int32_t *zlist;
    int64_t dom_x, dom_z, n;
    uint32_t *wpos;
};
__global__ __launch_bounds__(256) void k_window_bounds(WposArgs a) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    const int64_t x = upper_bound_dev(a.wposx, (int64_t)0, a.dom_x, i) - 1;
    const int64_t nw = windows_of(a.toff[x + 1] - a.toff[x], a.dom_z);
    const int64_t ws = cdiv(a.dom_z, nw);
    const int64_t r = i - a.wposx[x], l = r / (nw + 1), bnd = r % (nw + 1);
    const int64_t e = a.off_x[x] + l;
    const int64_t ln = a.eoff[e + 1] - a.eoff[e];
    const int64_t z = bnd * ws < a.dom_z ? bnd * ws : a.dom_z;
    a.wpos[i] = (uint32_t)lower_bound_dev(a.zlist + a.lbase[e], (int64_t)0, ln, (int32_t)z);
}

// Copies every unit's pairs from the stage to its output offset, turning
// the unit-local keys back into ids: one workgroup per unit, coalesced reads
// and writes, id lookups in the rank tables.
struct CopyArgs {
    const int64_t *uoff;   // output offset of every unit
    const int64_t *ubase;  // stage offset of every unit
    const int64_t *ucount;
    const int32_t *ustart; // first x of every unit
    const uint32_t *stage;
    int bz;
    uint32_t zmask;
    int64_t dom_x, dom_z;
    const int32_t *xorig, *zorig;
    int64_t xbase, zbase;  // dense id ranges (INT64_MIN: use the tables)
    int32_t *out_x, *out_z;
    int64_t *err;
};
constexpr int kCopyBlock = 256;
constexpr int kCopyBatch = 16;  // keys per thread whose loads are in flight together
__global__ __launch_bounds__(kCopyBlock) void k_stage_copy(CopyArgs a) {
    const int64_t u = blockIdx.x;
    const int64_t n = a.ucount[u], src = a.ubase[u], dst = a.uoff[u];
    const int64_t xa = a.ustart[u];
    const bool xdense = a.xbase != INT64_MIN, zdense = a.zbase != INT64_MIN;
    bool bad = false;
    for (int64_t i0 = threadIdx.x; i0 < n; i0 += (int64_t)kCopyBlock * kCopyBatch) {
        uint32_t key[kCopyBatch];
#pragma unroll
        for (int r = 0; r < kCopyBatch; ++r) {
            const int64_t i = i0 + (int64_t)r * kCopyBlock;
            key[r] = a.stage[src + (i < n ? i : i0)];
        }
        int32_t ox[kCopyBatch], oz[kCopyBatch];
#pragma unroll
        for (int r = 0; r < kCopyBatch; ++r) {
            const int64_t xi = xa + (key[r] >> a.bz), zi = key[r] & a.zmask;
            const bool ok = (xi < a.dom_x) & (zi < a.dom_z);
            bad |= !ok;
            ox[r] = xdense ? (int32_t)(a.xbase + xi) : a.xorig[ok ? xi : 0];
            oz[r] = zdense ? (int32_t)(a.zbase + zi) : a.zorig[ok ? zi : 0];
        }
#pragma unroll
        for (int r = 0; r < kCopyBatch; ++r) {
            const int64_t i = i0 + (int64_t)r * kCopyBlock;
            if (i < n) {
                a.out_x[dst + i] = ox[r];
                a.out_z[dst + i] = oz[r];
            }
        }
    }
    if (bad) *a.err = 3;
}

}  // namespace

bool segmented_dedup_fits(int bz) { return bz <= 26; }

void segmented_dedup(const Ctx &c, const SegDedupIn &in, DBuf<int32_t> *out_x, DBuf<int32_t> *out_z,
                     int64_t *n_out, SegDedupStats *stats, bool timing) {
    JP_CHECK(segmented_dedup_fits(in.bz), JP_EINTERNAL, "segmented dedup needs bz <= 26");
    JP_CHECK(in.zlist_n >= 1 && in.zlist_n < (1ll << 32), JP_EINTERNAL, "witness lists must hold 1 to 2^32-1 entries");
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
    // candidates before every x: the light candidates before x's first R
    // tuple (the tuples are x-major) plus the heavy nonzeros before x
    DBuf<int64_t> toff = c.buf<int64_t>(dom_x + 1);
    {
        const int64_t *ox = in.off_x, *eo = in.eoff, *ho = hoff.get();
        int64_t *to = toff.get();
        for_each(c, dom_x + 1, [=] __device__(int64_t x) { to[x] = eo[ox[x]] + ho[x]; });
    }

    // Units in x order.  A small x starts a packed unit when it is the first
    // x, follows a medium or large x, begins a new kUnitCap window of candidate offsets,
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
                if (t > kSoloCap) return windows_of(t, dz);
                if (t > kUnitCap) return 1;
                if (x == 0) return 1;
                const bool prev_big = to[x] - to[x - 1] > kUnitCap;
                const bool newwin = (to[x] / kUnitCap) != (to[x - 1] / kUnitCap);
                const bool newblk = kb < 31 ? ((x >> kb) != ((x - 1) >> kb)) : false;
                return (prev_big | newwin | newblk) ? 1 : 0;
            },
            ArrayPut{nu}, nu + dom_x);
    }
    // window boundary table: (lists + 1 boundaries) entries per large x
    DBuf<int64_t> wposx = c.buf<int64_t>(dom_x + 1);
    {
        const int64_t *to = toff.get(), *ox = in.off_x;
        const int64_t dz = dom_z;
        int64_t *wx = wposx.get();
        scan_exclusive(
            c, dom_x,
            [=] __device__(int64_t x) -> int64_t {
                const int64_t t = to[x + 1] - to[x];
                return t > kSoloCap ? (ox[x + 1] - ox[x]) * (windows_of(t, dz) + 1) : 0;
            },
            ArrayPut{wx}, wx + dom_x);
    }
    int64_t hn[3];
    c.load_scalars({nunits_x.get() + dom_x, toff.get() + dom_x, wposx.get() + dom_x}, hn);
    const int64_t n_units = hn[0], n_cand = hn[1], n_wpos = hn[2];
    // (beyond 2^31 entries the window units search their lists instead)
    const bool use_wpos = n_wpos > 0 && n_wpos < (1ll << 31);
    DBuf<uint32_t> wpos = c.buf<uint32_t>((size_t)(use_wpos ? n_wpos : 1));
    if (use_wpos) {
        WposArgs w;
        w.wposx = wposx.get();
        w.toff = toff.get();
        w.off_x = in.off_x;
        w.eoff = in.eoff;
        w.lbase = in.lbase;
        w.zlist = in.zlist;
        w.dom_x = dom_x;
        w.dom_z = dom_z;
        w.n = n_wpos;
        w.wpos = wpos.get();
        hipLaunchKernelGGL(k_window_bounds, dim3(grid_x(ceil_div(n_wpos, 256), 256)), dim3(256), 0, c.stream, w);
        JP_HIP(hipGetLastError());
    }
    DBuf<int32_t> ustart = c.buf<int32_t>(n_units + 1), uwin = c.buf<int32_t>(n_units + 1);
    {
        const int64_t *to = toff.get(), *nu = nunits_x.get();
        int32_t *us = ustart.get(), *uw = uwin.get();
        for_each(c, dom_x, [=] __device__(int64_t x) {
            const int64_t b = nu[x], m = nu[x + 1] - b;
            const bool big = to[x + 1] - to[x] > kSoloCap;
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
    DBuf<UnitDesc> udesc = c.buf<UnitDesc>(n_units + 1);
    {
        const int32_t *us = ustart.get(), *uw = uwin.get();
        const int64_t *ox = in.off_x, *eo = in.eoff, *ho = hoff.get();
        UnitDesc *ud = udesc.get();
        for_each(c, n_units, [=] __device__(int64_t u) {
            UnitDesc d{0, 0, 0, 0, 0, 0};
            if (uw[u] < 0) {
                const int32_t xa = us[u], xb = us[u + 1];
                d.e0 = ox[xa];
                d.e1 = ox[xb];
                d.c0 = eo[d.e0];
                d.nL = eo[d.e1] - d.c0;
                d.h0 = ho[xa];
                d.n = d.nL + (ho[xb] - d.h0);
            }
            ud[u] = d;
        });
    }
    dump(c, "ustart", ustart.get(), n_units + 1);
    dump(c, "uwin", uwin.get(), n_units + 1);

    DBuf<uint32_t> stage = c.buf<uint32_t>(std::max<int64_t>(n_cand, 1));
    DBuf<int64_t> ucount = c.buf<int64_t>(n_units + 1), ubase = c.buf<int64_t>(n_units + 1);
    if (n_units > 0) {
        JP_CHECK(n_units < (1ll << 31), JP_EINVAL, "too many dedup units for one launch");
        DedupArgs a;
        a.udesc = udesc.get();
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
        a.stage = stage.get();
        a.ucount = ucount.get();
        a.ubase = ubase.get();
        a.err = S + 1;
        a.wpos = use_wpos ? wpos.get() : nullptr;
        a.wposx = wposx.get();
        DBuf<unsigned long long> clk;
        a.clk = nullptr;
        if (std::getenv("JP_PHASE_CLOCKS")) {
            clk = c.buf<unsigned long long>(kPhCount);
            c.zero(clk.get(), kPhCount);
            a.clk = clk.get();
        }
        Timeline tk(c, timing);
        const int k0 = tk.mark();
        hipLaunchKernelGGL(k_dedup, dim3(grid_x(n_units, kDT)), dim3(kDT), 0, c.stream, a);
        JP_HIP(hipGetLastError());
        const int k1 = tk.mark();
        if (stats && timing) stats->ms_kernel = tk.ms(k0, k1);
        if (a.clk) {
            unsigned long long hc[kPhCount];
            c.load_n(hc, clk.get(), kPhCount);
            static const char *nm[kPhCount] = {"gather", "sort", "unique", "write", "win.lists", "win.write",
                                               "units.packed", "units.window"};
            std::fprintf(stderr, "[jp] dedup phase cycles (thread 0, summed over units):");
            for (int i = 0; i < kPhCount; ++i) std::fprintf(stderr, " %s=%llu", nm[i], hc[i]);
            std::fprintf(stderr, "\n");
        }
    }
    DBuf<int64_t> uoff = c.buf<int64_t>(n_units + 1);
    scan_exclusive(c, n_units, ArrayGet{ucount.get()}, ArrayPut{uoff.get()}, uoff.get() + n_units);
    int64_t h2[2];
    c.load_scalars({S + 1, uoff.get() + n_units}, h2);
    JP_CHECK(h2[0] != 1, JP_EINTERNAL, "a dedup unit exceeded its on-chip capacity");
    JP_CHECK(h2[0] == 0, JP_EINTERNAL, "dedup produced a key outside the rank tables");
    const int64_t total = n_units > 0 ? h2[1] : 0;
    *out_x = c.buf<int32_t>(std::max<int64_t>(total, 1));
    *out_z = c.buf<int32_t>(std::max<int64_t>(total, 1));
    if (total > 0) {
        CopyArgs ca;
        ca.uoff = uoff.get();
        ca.ubase = ubase.get();
        ca.ucount = ucount.get();
        ca.ustart = ustart.get();
        ca.stage = stage.get();
        ca.bz = in.bz;
        ca.zmask = (uint32_t)((1ull << in.bz) - 1);
        ca.dom_x = dom_x;
        ca.dom_z = dom_z;
        ca.xorig = in.xorig;
        ca.zorig = in.zorig;
        ca.xbase = in.x_dense_base;
        ca.zbase = in.z_dense_base;
        ca.out_x = out_x->get();
        ca.out_z = out_z->get();
        ca.err = S + 4;
        hipLaunchKernelGGL(k_stage_copy, dim3(grid_x(n_units, kCopyBlock)), dim3(kCopyBlock), 0, c.stream, ca);
        JP_HIP(hipGetLastError());
        // reads are clamped, so a bad key cannot fault; checked mode reports it
        if (checks_on()) JP_CHECK(c.load(S + 4) == 0, JP_EINTERNAL, "dedup produced a key outside the rank tables");
    }
    *n_out = total;
    if (stats) {
        stats->n_units = n_units;
        stats->n_cand = n_cand;
    }
}

}  // namespace jp
