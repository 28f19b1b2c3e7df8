// Heavy part of the method: the 0/1 matrix product M = M1 x M2 over the
// heavy x / y / z values (the heavy step of Algorithm 1; the Boolean-product
// view of Section 2.2).  Every entry is 0 or 1 and every count is at most the number
// of heavy y values, so int8 inputs with int32 accumulation are exact.  The
// product is never stored: the epilogue tests each accumulator for > 0 in
// registers and appends the nonzero coordinates (one atomic per tile).
//
// Operands: A = M1 (u rows) and Bt = M2 transposed (w rows), both int8
// row-major with the heavy-y index contiguous, row stride `ld` bytes (a
// multiple of 128, zero padded).
#include "pipeline.hpp"
#include "prims.hpp"

namespace jp {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

// ---- int8 MFMA kernel ------------------------------------------------------
// Block tile 128 x 128, K stage 128 bytes, 256 threads = 2 x 2 waves, each
// wave a 64 x 64 sub-tile of 4 x 4 MFMA 16x16x64 blocks.  Operand rows are
// staged in LDS with a 16-byte row pad; the next stage is prefetched into
// registers while the current one is multiplied.
constexpr int BM = 128, BN = 128, BK = 128;
constexpr int LDS_STRIDE = BK + 16;

// Epilogue functors: emit(pos, i, j, cnt) stores the nonzero C[i][j] = cnt
// at output slot pos.  kCounts: the functor uses cnt (the split-K path, which
// keeps only cnt > 0, is then not taken).
struct KeyEmit {  // nonzero (i, j) -> (rowmap[i] << shift) | colmap[j]
    static constexpr bool kCounts = false;
    const int32_t *rowmap, *colmap;
    int shift;
    uint64_t *keys;
    __device__ void operator()(int64_t pos, int64_t i, int64_t j, uint32_t) const {
        keys[pos] = ((uint64_t)(uint32_t)rowmap[i] << shift) | (uint64_t)(uint32_t)colmap[j];
    }
};
struct PairEmit {  // nonzero (i, j) -> rows[pos] = i, cols[pos] = j
    static constexpr bool kCounts = false;
    int32_t *rows, *cols;
    __device__ void operator()(int64_t pos, int64_t i, int64_t j, uint32_t) const {
        rows[pos] = (int32_t)i;
        cols[pos] = (int32_t)j;
    }
};

template <class K>
struct CountKeyEmit {  // nonzero (i, j) -> ((rowmap[i] << shift | colmap[j]) << wshift) | C[i][j]
    static constexpr bool kCounts = true;
    const int32_t *rowmap, *colmap;
    int shift, wshift;
    K *keys;
    __device__ void operator()(int64_t pos, int64_t i, int64_t j, uint32_t cnt) const {
        const K pair = ((K)(uint32_t)rowmap[i] << shift) | (K)(uint32_t)colmap[j];
        keys[pos] = (pair << wshift) | (K)cnt;
    }
};

// Row sources of an operand.  row(r) resolves row r once (per tile); load(h,
// k) then returns its 16 bytes starting at byte k.
struct PlainRows {  // A stored row-major
    const int8_t *A;
    int64_t ld;
    struct Row {
        const int8_t *p;
    };
    __device__ Row row(int64_t r) const { return Row{A + r * ld}; }
    __device__ v4i load(const Row &h, int64_t k) const { return *(const v4i *)(h.p + k); }
};
// Row (a_0, ..., a_{N-1}) of a product of N factor matrices (the V and W of
// the star query, Section 3.2): the AND of the factors' rows M_i[a_i, :] (0/1
// bytes), with r = mixed-radix number of the a_i over the factor heights
// u_i, the last factor varying fastest.  V and W are never stored.
// The mixed-radix decode (integer divisions) happens once per row in row();
// each 16-byte load is then N loads and ANDs.
template <int N>
struct TupleRows {
    const int8_t *M[N];
    int64_t u[N];
    int64_t ld;
    struct Row {
        const int8_t *p[N];
    };
    __device__ Row row(int64_t r) const {
        Row h;
#pragma unroll
        for (int i = N - 1; i >= 0; --i) {
            const int64_t a = i > 0 ? r % u[i] : r;
            if (i > 0) r /= u[i];
            h.p[i] = M[i] + a * ld;
        }
        return h;
    }
    __device__ v4i load(const Row &h, int64_t k) const {
        v4i acc = {-1, -1, -1, -1};
#pragma unroll
        for (int i = 0; i < N; ++i) acc &= *(const v4i *)(h.p[i] + k);
        return acc;
    }
};

// Nonzero (i, j) of V x W^T: i numbers (a_0..a_{G-1}) over u[0..G), j numbers
// (a_G..a_{G+H-1}) over u[G..G+H) (last fastest); the key is the k-tuple of
// their x ranks, x_t << s[t] for every position t.
template <class K, int G, int H>
struct TupleEmit {
    static constexpr bool kCounts = false;
    const int32_t *xof[G + H];
    int64_t u[G + H];
    int s[G + H];
    K *keys;
    __device__ void operator()(int64_t pos, int64_t i, int64_t j, uint32_t) const {
        K key = 0;
#pragma unroll
        for (int t = G - 1; t >= 0; --t) {
            const int64_t a = t > 0 ? i % u[t] : i;
            if (t > 0) i /= u[t];
            key |= (K)(uint32_t)xof[t][a] << s[t];
        }
#pragma unroll
        for (int t = G + H - 1; t >= G; --t) {
            const int64_t a = t > G ? j % u[t] : j;
            if (t > G) j /= u[t];
            key |= (K)(uint32_t)xof[t][a] << s[t];
        }
        keys[pos] = key;
    }
};

// Work items are dealt to the 8 XCDs round-robin by block index.  Item
// sequence index -> work item: XCD r (blocks b with b % 8 == r, grids are
// multiples of 8) takes the r-th eighth of the items, a contiguous run, so
// tiles next to each other in tile_of_block's order share that XCD's L2.
// The item space is padded to a multiple of 8; padding returns -1.
__device__ __forceinline__ int64_t xcd_item(int64_t bid, int64_t total) {
    const int64_t per = (total + 7) / 8;
    const int64_t t = (bid & 7) * per + (bid >> 3);
    return t < total ? t : -1;
}
__host__ __device__ inline int64_t xcd_padded(int64_t total) { return 8 * ((total + 7) / 8); }

// Tile index -> tile: groups of 8 tile-rows swept column-major, so a run of
// consecutive tiles forms a compact 2-D patch (tiles sharing A rows / B rows).
__device__ __forceinline__ void tile_of_block(int64_t t, int64_t tiles_m, int64_t tiles_n, int64_t *tm,
                                              int64_t *tn) {
    // group of 8 tile-rows swept column-major inside the group
    const int64_t G = 8;
    const int64_t group = t / (G * tiles_n);
    const int64_t first_m = group * G;
    const int64_t gm = (tiles_m - first_m) < G ? (tiles_m - first_m) : G;
    const int64_t in = t - group * G * tiles_n;
    *tm = first_m + in % gm;
    *tn = in / gm;
}

// Output slots of one workgroup's tile: the waves' counts are summed in LDS
// and one device-scope atomic reserves them all.  Atomics on one address are
// serialised (about 11 ns each on MI355X), so one per wave (3.8M for a
// 177K x 174K product of 256 x 256 tiles) would cost more than the MFMA
// work.  Returns this wave's first slot, or -1 when the tile has no nonzero
// (the same for the whole workgroup).  Must be reached by every thread; the
// caller's next write to sh/shbase must be separated from this call by a
// workgroup barrier (each kernel's main loop has one).
template <int WAVES>
__device__ __forceinline__ int64_t tile_reserve(uint32_t wtot, unsigned long long *count, uint32_t *sh,
                                                unsigned long long *shbase) {
    const int wv = threadIdx.x / kWave;
    if (lane_id() == 0) sh[wv] = wtot;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int q = 0; q < WAVES; ++q) {
        const uint32_t t = sh[q];
        before += q < wv ? t : 0u;
        all += t;
    }
    if (all == 0) return -1;
    if (threadIdx.x == 0) *shbase = atomicAdd(count, (unsigned long long)all);
    __syncthreads();
    return (int64_t)*shbase + before;
}

// With kchunk < ld the K range is split into chunks (split-K, for products
// with few output tiles and long rows): workgroup item = (tile, chunk), and
// the epilogue ORs "count > 0" into a u x w bitmap instead of emitting
// (entries are sums of non-negative chunk counts, so the OR of the chunk
// tests is the test of the sum).
template <class ARows, class BRows, class Emit>
__global__ __launch_bounds__(256) void k_bmm_i8(ARows arows, BRows brows, int64_t u, int64_t w,
                                                int64_t ld, int64_t tiles_m, int64_t tiles_n, Emit emit, int64_t cap,
                                                unsigned long long *count, int64_t kchunk, uint32_t *bitmap) {
    __shared__ __attribute__((aligned(16))) int8_t sA[BM * LDS_STRIDE];
    __shared__ __attribute__((aligned(16))) int8_t sB[BN * LDS_STRIDE];
    __shared__ uint32_t sh_cnt[4];
    __shared__ unsigned long long sh_base;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
    const int wm = wv >> 1, wn = wv & 1;
    // global -> register staging: each thread moves 4 x 16 B of A and of B
    // per stage: row = (tid / 8) + 32 * q, byte offset = (tid % 8) * 16
    const int lr = tid / 8, lc = (tid % 8) * 16;
    const int fr = lane % 16, fk = (lane / 16) * 16;
    // Workgroups loop over tiles when the tile count exceeds the grid (the
    // grid is a multiple of 8, so a workgroup stays on its XCD's tile patch).
    const int64_t nchunks = (ld + kchunk - 1) / kchunk;
    const int64_t total = tiles_m * tiles_n * nchunks;
    for (int64_t bid = blockIdx.x; bid < xcd_padded(total); bid += gridDim.x) {
        const int64_t item = xcd_item(bid, total);
        if (item < 0) continue;  // padding (uniform per workgroup)
        int64_t tm, tn;
        tile_of_block(item / nchunks, tiles_m, tiles_n, &tm, &tn);
        const int64_t kbeg = (item % nchunks) * kchunk;
        const int64_t kend = kbeg + kchunk < ld ? kbeg + kchunk : ld;
        const int64_t row0 = tm * BM, col0 = tn * BN;
        // this thread's 4 A rows and 4 B rows, resolved once for the tile
        // (rows past the edge resolve row 0 and load zeros)
        typename ARows::Row ha[4];
        typename BRows::Row hb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t r = row0 + lr + 32 * q, c = col0 + lr + 32 * q;
            ha[q] = arows.row(r < u ? r : 0);
            hb[q] = brows.row(c < w ? c : 0);
        }
        v4i ra[4], rb[4];
        auto load_stage = [&](int64_t k0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                ra[q] = row0 + lr + 32 * q < u ? arows.load(ha[q], k0 + lc) : v4i{0, 0, 0, 0};
                rb[q] = col0 + lr + 32 * q < w ? brows.load(hb[q], k0 + lc) : v4i{0, 0, 0, 0};
            }
        };
        auto store_stage = [&]() {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                *(v4i *)(sA + (lr + 32 * q) * LDS_STRIDE + lc) = ra[q];
                *(v4i *)(sB + (lr + 32 * q) * LDS_STRIDE + lc) = rb[q];
            }
        };

        v4i acc[4][4];
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int g = 0; g < 4; ++g) acc[f][g] = v4i{0, 0, 0, 0};

        load_stage(kbeg);
        for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
            __syncthreads();
            store_stage();
            __syncthreads();
            if (k0 + BK < kend) load_stage(k0 + BK);
#pragma unroll
            for (int kk = 0; kk < BK; kk += 64) {
                v4i a[4], b[4];
#pragma unroll
                for (int f = 0; f < 4; ++f)
                    a[f] = *(const v4i *)(sA + (wm * 64 + f * 16 + fr) * LDS_STRIDE + kk + fk);
#pragma unroll
                for (int g = 0; g < 4; ++g)
                    b[g] = *(const v4i *)(sB + (wn * 64 + g * 16 + fr) * LDS_STRIDE + kk + fk);
#pragma unroll
                for (int f = 0; f < 4; ++f)
#pragma unroll
                    for (int g = 0; g < 4; ++g)
                        acc[f][g] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[f], b[g], acc[f][g], 0, 0, 0);
            }
        }

        // Epilogue: C[row][col] with row = 4*(lane/16) + r inside the 16x16
        // block, col = lane % 16.  Entries past the matrix edge are dropped
        // first (edge tiles only); the counts are >= 0, so min(count, 1) is
        // the nonzero test.  One atomic per tile; a wave without a nonzero
        // skips the emission.
        {
            const int rlim = (int)(u - row0 < BM ? u - row0 : BM), clim = (int)(w - col0 < BN ? w - col0 : BN);
            if (rlim < BM || clim < BN) {
#pragma unroll
                for (int f = 0; f < 4; ++f)
#pragma unroll
                    for (int g = 0; g < 4; ++g)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (!(wm * 64 + f * 16 + (lane / 16) * 4 + r < rlim && wn * 64 + g * 16 + (lane % 16) < clim))
                                acc[f][g][r] = 0;
            }
        }
        if (bitmap) {
#pragma unroll
            for (int f = 0; f < 4; ++f)
#pragma unroll
                for (int g = 0; g < 4; ++g)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t i = row0 + wm * 64 + f * 16 + (lane / 16) * 4 + r;
                        const int64_t j = col0 + wn * 64 + g * 16 + (lane % 16);
                        if (acc[f][g][r] > 0) {
                            const int64_t b = i * w + j;
                            atomicOr(&bitmap[b >> 5], 1u << (b & 31));
                        }
                    }
            continue;
        }
        uint32_t mine = 0;
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) mine += (uint32_t)min(acc[f][g][r], 1);
        uint32_t incl = wave_incl_scan(mine);
        uint32_t wtot = wave_lane(incl, kWave - 1);
        const int64_t base = tile_reserve<4>(wtot, count, sh_cnt, &sh_base);
        if (base < 0 || wtot == 0) continue;
        int64_t pos = base + (incl - mine);
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (acc[f][g][r] > 0) {
                        const int64_t i = row0 + wm * 64 + f * 16 + (lane / 16) * 4 + r;
                        const int64_t j = col0 + wn * 64 + g * 16 + (lane % 16);
                        if (pos < cap) emit(pos, i, j, (uint32_t)acc[f][g][r]);
                        ++pos;
                    }
                }
    }
}

// ---- int8 MFMA kernel, large tiles ---------------------------------------------
// Block tile 256 x 256, K stage 128 bytes, 512 threads = 2 x 4 waves, each
// wave a 128 x 64 sub-tile of 8 x 4 MFMA 16x16x64 blocks (128 accumulator
// registers).  Operands go from global memory straight into LDS
// (global_load_lds_dwordx4, 16 bytes per lane), double buffered: the next
// stage streams in while the current one is multiplied.  LDS rows are 128
// bytes with the 16-byte chunk c of row r stored at position c ^ (r & 7), so
// the MFMA operand reads of 8 consecutive rows hit 8 different bank groups.
// Twice the block tile of the 128 x 128 kernel halves the operand traffic
// per operation.
constexpr int BM2 = 256, BN2 = 256, BK2 = 128;
constexpr int kBig = 512;                       // threads
constexpr int kStageBytes = (BM2 + BN2) * BK2;  // 64 KB: A rows then B rows

__device__ __forceinline__ int swz(int r, int c) { return r * BK2 + ((c ^ (r & 7)) << 4); }

// Upper-triangle tile t (column by column: (0,0), (0,1), (1,1), (0,2), ...)
// of a symmetric product.
__device__ __forceinline__ void tri_tile(int64_t t, int64_t *tm, int64_t *tn) {
    int64_t c = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((c + 1) * (c + 2) / 2 <= t) ++c;
    while (c * (c + 1) / 2 > t) --c;
    *tn = c;
    *tm = t - c * (c + 1) / 2;
}

// sym: A == Bt (a self-join's C = M1 M1^T, symmetric): only tiles with
// tm <= tn are computed, and a nonzero of a tile off the diagonal is
// emitted as (i, j) and (j, i).
template <class Emit>
__global__ __launch_bounds__(kBig) void k_bmm_i8_big(const int8_t *__restrict__ A, const int8_t *__restrict__ Bt,
                                                     int64_t u, int64_t w, int64_t ld, int64_t tiles_m,
                                                     int64_t tiles_n, Emit emit, int64_t cap,
                                                     unsigned long long *count, bool sym) {
    extern __shared__ __attribute__((aligned(16))) int8_t lds[];  // 2 stages
    __shared__ uint32_t sh_cnt[kBig / kWave];
    __shared__ unsigned long long sh_base;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
    const int wm = wv >> 2, wn = wv & 3;
    const int fr = lane % 16, fq = lane / 16;
    const int64_t total = sym ? tiles_m * (tiles_m + 1) / 2 : tiles_m * tiles_n;
    const int64_t nk = ld / BK2;
    for (int64_t bid = blockIdx.x; bid < xcd_padded(total); bid += gridDim.x) {
        const int64_t item = xcd_item(bid, total);
        if (item < 0) continue;  // padding (uniform per workgroup)
        int64_t tm, tn;
        if (sym) tri_tile(item, &tm, &tn);
        else tile_of_block(item, tiles_m, tiles_n, &tm, &tn);
        const uint32_t mult = (sym && tm != tn) ? 2u : 1u;  // uniform per workgroup
        const int64_t row0 = tm * BM2, col0 = tn * BN2;
        // Stage s: 4096 chunks of 16 bytes, 8 rounds of 512; chunk P holds
        // (row P / 8, K chunk (P % 8) ^ (row & 7)); rows 0..255 are A, 256..511 B.
        // Rows past the matrix edge read row 0 (their results are never emitted).
        auto issue = [&](int64_t k0, int buf) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int P = q * kBig + tid;
                const int r = P >> 3, c = (P & 7) ^ (r & 7);
                const int8_t *src;
                if (r < BM2) {
                    const int64_t gr = row0 + r;
                    src = A + (gr < u ? gr : 0) * ld + k0 + c * 16;
                } else {
                    const int64_t gc = col0 + (r - BM2);
                    src = Bt + (gc < w ? gc : 0) * ld + k0 + c * 16;
                }
                // LDS destination of the wave: its 64 consecutive chunks
                int8_t *dst = lds + buf * kStageBytes + (q * kBig + wv * kWave) * 16;
                __builtin_amdgcn_global_load_lds((const void *)src, (__attribute__((address_space(3))) void *)dst,
                                                 16, 0, 0);
            }
        };
        v4i acc[8][4];
#pragma unroll
        for (int f = 0; f < 8; ++f)
#pragma unroll
            for (int g = 0; g < 4; ++g) acc[f][g] = v4i{0, 0, 0, 0};

        __syncthreads();  // the previous tile's last reads of both buffers are done
        issue(0, 0);
        for (int64_t s = 0; s < nk; ++s) {
            const int buf = (int)(s & 1);
            __builtin_amdgcn_s_waitcnt(0);  // this thread's loads of stage s have landed
            __syncthreads();                // everyone's have; buffer buf ^ 1 is free
            if (s + 1 < nk) issue((s + 1) * BK2, buf ^ 1);
            const int8_t *sa = lds + buf * kStageBytes;
            const int8_t *sb = sa + BM2 * BK2;
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {  // two K steps of 64 bytes
                const int c = kk * 4 + fq;
                v4i a[8], b[4];
#pragma unroll
                for (int f = 0; f < 8; ++f) {
                    const int r = wm * 128 + f * 16 + fr;
                    a[f] = *(const v4i *)(sa + swz(r, c));
                }
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int r = wn * 64 + g * 16 + fr;
                    b[g] = *(const v4i *)(sb + swz(r, c));
                }
#pragma unroll
                for (int f = 0; f < 8; ++f)
#pragma unroll
                    for (int g = 0; g < 4; ++g)
                        acc[f][g] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[f], b[g], acc[f][g], 0, 0, 0);
            }
        }

        // Epilogue as in the 128 x 128 kernel, in tile-local 32-bit
        // coordinates: rows and columns past the matrix edge are cut by two
        // limits (the tile size for interior tiles).  A wave without a
        // nonzero skips the emission.
        const int rlim = (int)(u - row0 < BM2 ? u - row0 : BM2), clim = (int)(w - col0 < BN2 ? w - col0 : BN2);
        const bool interior = rlim == BM2 && clim == BN2;  // uniform per workgroup
        const int ib = wm * 128 + fq * 4, jb = wn * 64 + fr;
        if (!interior) {  // edge tile: entries past the matrix edge are dropped
#pragma unroll
            for (int f = 0; f < 8; ++f)
#pragma unroll
                for (int g = 0; g < 4; ++g)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (!(ib + f * 16 + r < rlim && jb + g * 16 < clim)) acc[f][g][r] = 0;
        }
        uint32_t mine = 0;  // counts are >= 0: min(count, 1) is the nonzero test
#pragma unroll
        for (int f = 0; f < 8; ++f)
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) mine += (uint32_t)min(acc[f][g][r], 1);
        mine *= mult;
        const uint32_t incl = wave_incl_scan(mine);
        const uint32_t wtot = wave_lane(incl, kWave - 1);
        const int64_t base = tile_reserve<kBig / kWave>(wtot, count, sh_cnt, &sh_base);
        if (base < 0 || wtot == 0) continue;
        int64_t pos = base + (incl - mine);
#pragma unroll
        for (int f = 0; f < 8; ++f)
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (acc[f][g][r] > 0) {
                        const int64_t i = row0 + ib + f * 16 + r, j = col0 + jb + g * 16;
                        if (pos < cap) emit(pos, i, j, (uint32_t)acc[f][g][r]);
                        if (mult == 2u && pos + 1 < cap) emit(pos + 1, j, i, (uint32_t)acc[f][g][r]);
                        pos += mult;
                    }
                }
    }
}

template <class Emit>
void launch_bmm_big(const Ctx &c, const int8_t *A, const int8_t *Bt, int64_t u, int64_t w, int64_t ld, Emit emit,
                    int64_t cap, unsigned long long *count_dev, bool sym = false) {
    JP_CHECK(ld % BK2 == 0, JP_EINTERNAL, "heavy matrix stride must be a multiple of 128");
    JP_CHECK(!sym || (A == Bt && u == w), JP_EINTERNAL, "a symmetric product needs A == Bt");
    c.zero(count_dev, 1);
    if (u <= 0 || w <= 0 || ld <= 0) return;
    const int64_t tm = ceil_div(u, BM2), tn = ceil_div(w, BN2);
    const int64_t total = xcd_padded(sym ? tm * (tm + 1) / 2 : tm * tn);
    constexpr int64_t kMaxGrid = 1ll << 21;  // multiple of 8
    const int64_t blocks = total < kMaxGrid ? total : kMaxGrid;
    hipLaunchKernelGGL((k_bmm_i8_big<Emit>), dim3(grid_x(blocks, kBig)), dim3(kBig), 2 * kStageBytes, c.stream, A,
                       Bt, u, w, ld, tm, tn, emit, cap, count_dev, sym);
    JP_HIP(hipGetLastError());
}

// Nonzeros of a u x w bitmap, emitted with one atomic per wave.
template <class Emit>
__global__ __launch_bounds__(256) void k_emit_bitmap(const uint32_t *bitmap, int64_t u, int64_t w, Emit emit,
                                                     int64_t cap, unsigned long long *count) {
    const int lane = lane_id();
    const int64_t nwords = (u * w + 31) / 32;
    const int64_t stride = (int64_t)gridDim.x * 256;
    const int64_t iters = (nwords + stride - 1) / stride;  // the same for every lane: ballots stay uniform
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t q = it * stride + (int64_t)blockIdx.x * 256 + threadIdx.x;
        const uint32_t word = q < nwords ? bitmap[q] : 0u;
        const uint32_t mine = (uint32_t)__popc(word);
        const uint32_t incl = wave_incl_scan(mine);
        const uint32_t wtot = wave_lane(incl, kWave - 1);
        if (wtot == 0) continue;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(count, (unsigned long long)wtot);
        base = __shfl(base, 0);
        int64_t pos = (int64_t)base + (incl - mine);
        uint32_t bits = word;
        while (bits) {
            const int b = __ffs(bits) - 1;
            bits &= bits - 1;
            const int64_t e = q * 32 + b;
            if (pos < cap) emit(pos, e / w, e % w, 0u);  // split-K: only cnt > 0 is known
            ++pos;
        }
    }
}

// ---- fp16 MFMA kernel ----------------------------------------------------------
// The 128 x 128 block tile of k_bmm_i8 with fp16 operands: the 0/1 bytes
// staged from global memory become fp16 ones and zeros in LDS, and
// v_mfma_f32_16x16x32_f16 accumulates in fp32.  Every partial sum is an
// integer of at most the row length, so the fp32 counts are exact while that
// is below 2^24 (the caller checks).  The int8 storage of the matrices is
// kept; only the LDS tile is twice as wide.
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kF16Stride = 2 * BK + 32;                  // bytes per LDS row: 128 fp16 values + pad
constexpr int kF16Lds = (BM + BN) * kF16Stride;          // dynamic LDS of one workgroup

// Four 0/1 bytes -> four fp16 (1.0 = 0x3C00), as two words.
__device__ __forceinline__ void bytes_to_f16(uint32_t w, uint32_t &lo, uint32_t &hi) {
    lo = ((w & 1u) | ((w & 0x100u) << 8)) * 0x3C00u;
    hi = (((w >> 16) & 1u) | ((w >> 8) & 0x10000u)) * 0x3C00u;
}

template <class ARows, class BRows, class Emit>
__global__ __launch_bounds__(256) void k_bmm_f16(ARows arows, BRows brows, int64_t u, int64_t w, int64_t ld,
                                                 int64_t tiles_m, int64_t tiles_n, Emit emit, int64_t cap,
                                                 unsigned long long *count) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds16[];
    uint8_t *sA = lds16, *sB = lds16 + BM * kF16Stride;
    __shared__ uint32_t sh_cnt[4];
    __shared__ unsigned long long sh_base;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
    const int wm = wv >> 1, wn = wv & 1;
    const int lr = tid / 8, lc = (tid % 8) * 16;
    const int fr = lane % 16, fq = lane / 16;
    const int64_t total = tiles_m * tiles_n;
    for (int64_t bid = blockIdx.x; bid < xcd_padded(total); bid += gridDim.x) {
        const int64_t item = xcd_item(bid, total);
        if (item < 0) continue;  // padding (uniform per workgroup)
        int64_t tm, tn;
        tile_of_block(item, tiles_m, tiles_n, &tm, &tn);
        const int64_t row0 = tm * BM, col0 = tn * BN;
        typename ARows::Row ha[4];
        typename BRows::Row hb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t r = row0 + lr + 32 * q, c = col0 + lr + 32 * q;
            ha[q] = arows.row(r < u ? r : 0);
            hb[q] = brows.row(c < w ? c : 0);
        }
        v4i ra[4], rb[4];
        auto load_stage = [&](int64_t k0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                ra[q] = row0 + lr + 32 * q < u ? arows.load(ha[q], k0 + lc) : v4i{0, 0, 0, 0};
                rb[q] = col0 + lr + 32 * q < w ? brows.load(hb[q], k0 + lc) : v4i{0, 0, 0, 0};
            }
        };
        auto store_row = [&](uint8_t *base, v4i v) {
            uint32_t h[8];
#pragma unroll
            for (int i = 0; i < 4; ++i) bytes_to_f16((uint32_t)v[i], h[2 * i], h[2 * i + 1]);
            *(v4i *)base = v4i{(int)h[0], (int)h[1], (int)h[2], (int)h[3]};
            *(v4i *)(base + 16) = v4i{(int)h[4], (int)h[5], (int)h[6], (int)h[7]};
        };
        f4 acc[4][4];
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int g = 0; g < 4; ++g) acc[f][g] = f4{0.f, 0.f, 0.f, 0.f};
        load_stage(0);
        for (int64_t k0 = 0; k0 < ld; k0 += BK) {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                store_row(sA + (lr + 32 * q) * kF16Stride + 2 * lc, ra[q]);
                store_row(sB + (lr + 32 * q) * kF16Stride + 2 * lc, rb[q]);
            }
            __syncthreads();
            if (k0 + BK < ld) load_stage(k0 + BK);
#pragma unroll
            for (int kk = 0; kk < BK; kk += 32) {
                half8 a[4], b[4];
#pragma unroll
                for (int f = 0; f < 4; ++f)
                    a[f] = *(const half8 *)(sA + (wm * 64 + f * 16 + fr) * kF16Stride + 2 * kk + 16 * fq);
#pragma unroll
                for (int g = 0; g < 4; ++g)
                    b[g] = *(const half8 *)(sB + (wn * 64 + g * 16 + fr) * kF16Stride + 2 * kk + 16 * fq);
#pragma unroll
                for (int f = 0; f < 4; ++f)
#pragma unroll
                    for (int g = 0; g < 4; ++g)
                        acc[f][g] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[f], b[g], acc[f][g], 0, 0, 0);
            }
        }
        // Epilogue as in k_bmm_i8: C[row][col], row = 4 (lane / 16) + r, col = lane % 16.
        {
            const int rlim = (int)(u - row0 < BM ? u - row0 : BM), clim = (int)(w - col0 < BN ? w - col0 : BN);
            if (rlim < BM || clim < BN) {
#pragma unroll
                for (int f = 0; f < 4; ++f)
#pragma unroll
                    for (int g = 0; g < 4; ++g)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (!(wm * 64 + f * 16 + fq * 4 + r < rlim && wn * 64 + g * 16 + fr < clim))
                                acc[f][g][r] = 0.0f;
            }
        }
        uint32_t mine = 0;
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) mine += acc[f][g][r] > 0.5f ? 1u : 0u;
        const uint32_t incl = wave_incl_scan(mine);
        const uint32_t wtot = wave_lane(incl, kWave - 1);
        const int64_t base = tile_reserve<4>(wtot, count, sh_cnt, &sh_base);
        if (base < 0 || wtot == 0) continue;
        int64_t pos = base + (incl - mine);
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t i = row0 + wm * 64 + f * 16 + fq * 4 + r;
                    const int64_t j = col0 + wn * 64 + g * 16 + fr;
                    if (acc[f][g][r] > 0.5f) {
                        if (pos < cap) emit(pos, i, j, (uint32_t)(acc[f][g][r] + 0.5f));
                        ++pos;
                    }
                }
    }
}

template <class ARows, class BRows, class Emit>
void launch_bmm_f16(const Ctx &c, ARows arows, BRows brows, int64_t u, int64_t w, int64_t ld, Emit emit, int64_t cap,
                    unsigned long long *count_dev) {
    JP_CHECK(ld % kBmmPadK == 0, JP_EINTERNAL, "heavy matrix stride must be a multiple of 128");
    JP_CHECK(ld < (int64_t(1) << 24), JP_EPRECISION, "fp16 product: counts may reach 2^24, beyond fp32's exact range");
    c.zero(count_dev, 1);
    if (u <= 0 || w <= 0 || ld <= 0) return;
    const int64_t tm = ceil_div(u, BM), tn = ceil_div(w, BN);
    const int64_t total = xcd_padded(tm * tn);
    constexpr int64_t kMaxGrid = 1ll << 22;  // multiple of 8
    const int64_t blocks = total < kMaxGrid ? total : kMaxGrid;
    hipLaunchKernelGGL((k_bmm_f16<ARows, BRows, Emit>), dim3(grid_x(blocks, 256)), dim3(256), kF16Lds, c.stream, arows,
                       brows, u, w, ld, tm, tn, emit, cap, count_dev);
    JP_HIP(hipGetLastError());
}

template <class ARows, class BRows, class Emit>
void launch_bmm_rows(const Ctx &c, ARows arows, BRows brows, int64_t u, int64_t w, int64_t ld, Emit emit, int64_t cap,
                     unsigned long long *count_dev) {
    JP_CHECK(ld % kBmmPadK == 0, JP_EINTERNAL, "heavy matrix stride must be a multiple of 128");
    c.zero(count_dev, 1);
    if (u <= 0 || w <= 0 || ld <= 0) return;
    const int64_t tm = ceil_div(u, BM), tn = ceil_div(w, BN);
    const int64_t tiles = tm * tn;
    // Split K when the tiles alone would leave most of the chip idle and the
    // rows are long: about two workgroups per compute unit, chunks of at least
    // 1024 bytes.
    int64_t kchunk = ld;
    if (!Emit::kCounts && tiles < c.num_cus && ld >= 4 * 1024) {
        const int64_t want = std::max<int64_t>(1, (2 * c.num_cus) / tiles);
        kchunk = std::max<int64_t>(1024, ceil_div(ceil_div(ld, want), BK) * BK);
    }
    const int64_t nchunks = ceil_div(ld, kchunk);
    const int64_t total = xcd_padded(tiles * nchunks);
    constexpr int64_t kMaxGrid = 1ll << 22;  // items beyond this are looped over (multiple of 8)
    const int64_t blocks = total < kMaxGrid ? total : kMaxGrid;
    if (nchunks == 1) {
        hipLaunchKernelGGL((k_bmm_i8<ARows, BRows, Emit>), dim3(grid_x(blocks, 256)), dim3(256), 0, c.stream, arows,
                           brows, u, w, ld, tm, tn, emit, cap, count_dev, kchunk, (uint32_t *)nullptr);
        JP_HIP(hipGetLastError());
        return;
    }
    const int64_t nwords = ceil_div(u * w, 32);
    DBuf<uint32_t> bitmap = c.buf<uint32_t>((size_t)nwords);
    c.zero(bitmap.get(), (size_t)nwords);
    hipLaunchKernelGGL((k_bmm_i8<ARows, BRows, Emit>), dim3(grid_x(blocks, 256)), dim3(256), 0, c.stream, arows, brows,
                       u, w, ld, tm, tn, emit, cap, count_dev, kchunk, bitmap.get());
    JP_HIP(hipGetLastError());
    const int64_t eb = std::max<int64_t>(1, std::min<int64_t>(ceil_div(nwords, 256), (int64_t)c.num_cus * 4));
    hipLaunchKernelGGL((k_emit_bitmap<Emit>), dim3(grid_x(eb, 256)), dim3(256), 0, c.stream,
                       (const uint32_t *)bitmap.get(), u, w, emit, cap, count_dev);
    JP_HIP(hipGetLastError());
}

template <class ARows, class Emit>
void launch_bmm(const Ctx &c, ARows arows, const int8_t *Bt, int64_t u, int64_t w, int64_t ld, Emit emit, int64_t cap,
                unsigned long long *count_dev) {
    launch_bmm_rows(c, arows, PlainRows{Bt, ld}, u, w, ld, emit, cap, count_dev);
}

}  // namespace

// ---- bit-packed AND + popcount kernel ----------------------------------------
// The 0/1 rows packed 64 per word; C[i][j] = sum over words of
// popcount(A[i][w] & B[j][w]) on the vector units (no matrix cores).  Block
// tile 128 x 128, 256 threads as 16 x 16; thread (ty, tx) owns rows
// ty + 16 i and columns tx + 16 j (i, j < 8), so the 16 threads of a row
// group read 16 consecutive B words from LDS.  K is staged through LDS 8
// words (512 columns) at a time, stored word-major.
constexpr int PB = 128, PKW = 8;

__global__ __launch_bounds__(256) void k_pack_bits(const int8_t *__restrict__ M, int64_t rows, int64_t ld,
                                                   uint64_t *__restrict__ P) {
    const int64_t nw = ld / 64, n = rows * nw;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += stride) {
        const int64_t r = t / nw, wd = t - r * nw;
        const v4i *src = (const v4i *)(M + r * ld + wd * 64);
        uint64_t bits = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const v4i v = src[q];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t x = (uint32_t)v[e];
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    bits |= (uint64_t)(((x >> (8 * b)) & 0xffu) != 0) << (q * 16 + e * 4 + b);
            }
        }
        P[t] = bits;
    }
}

template <class Emit>
__global__ __launch_bounds__(256) void k_bmm_bitpop(const uint64_t *__restrict__ A, const uint64_t *__restrict__ B,
                                                    int64_t u, int64_t w, int64_t nw, int64_t tiles_m,
                                                    int64_t tiles_n, Emit emit, int64_t cap,
                                                    unsigned long long *count) {
    __shared__ uint64_t sA[PKW][PB], sB[PKW][PB];
    __shared__ uint32_t sh_cnt[4];
    __shared__ unsigned long long sh_base;
    const int tid = threadIdx.x, lane = lane_id();
    const int ty = tid / 16, tx = tid % 16;
    const int64_t total = tiles_m * tiles_n;
    for (int64_t bid = blockIdx.x; bid < xcd_padded(total); bid += gridDim.x) {
        const int64_t item = xcd_item(bid, total);
        if (item < 0) continue;  // padding (uniform per workgroup)
        int64_t tm, tn;
        tile_of_block(item, tiles_m, tiles_n, &tm, &tn);
        const int64_t row0 = tm * PB, col0 = tn * PB;
        uint32_t acc[8][8];
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[i][j] = 0;
        for (int64_t k0 = 0; k0 < nw; k0 += PKW) {
            __syncthreads();
            // 128 rows x 8 words of A and of B: 1024 words each, 4 per thread
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = q * 256 + tid, r = e / PKW, kw = e % PKW;
                const int64_t gr = row0 + r, gc = col0 + r, gk = k0 + kw;
                sA[kw][r] = (gr < u && gk < nw) ? A[gr * nw + gk] : 0ull;
                sB[kw][r] = (gc < w && gk < nw) ? B[gc * nw + gk] : 0ull;
            }
            __syncthreads();
#pragma unroll 2
            for (int kw = 0; kw < PKW; ++kw) {
                uint64_t a[8], b[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) a[i] = sA[kw][ty + 16 * i];
#pragma unroll
                for (int j = 0; j < 8; ++j) b[j] = sB[kw][tx + 16 * j];
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int j = 0; j < 8; ++j) acc[i][j] += (uint32_t)__popcll(a[i] & b[j]);
            }
        }
        uint32_t mine = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j)
                mine += (acc[i][j] > 0 && row0 + ty + 16 * i < u && col0 + tx + 16 * j < w) ? 1u : 0u;
        const uint32_t incl = wave_incl_scan(mine);
        const uint32_t wtot = wave_lane(incl, kWave - 1);
        const int64_t base = tile_reserve<4>(wtot, count, sh_cnt, &sh_base);
        if (base < 0) continue;
        int64_t pos = base + (incl - mine);
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int64_t gi = row0 + ty + 16 * i, gj = col0 + tx + 16 * j;
                if (acc[i][j] > 0 && gi < u && gj < w) {
                    if (pos < cap) emit(pos, gi, gj, acc[i][j]);
                    ++pos;
                }
            }
    }
}

template <class Emit>
void launch_bitpop(const Ctx &c, const int8_t *A, const int8_t *Bt, int64_t u, int64_t w, int64_t ld, Emit emit,
                   int64_t cap, unsigned long long *count_dev) {
    JP_CHECK(ld % 64 == 0, JP_EINTERNAL, "heavy matrix stride must be a multiple of 64");
    c.zero(count_dev, 1);
    if (u <= 0 || w <= 0 || ld <= 0) return;
    const int64_t nw = ld / 64;
    DBuf<uint64_t> pa = c.buf<uint64_t>((size_t)(u * nw)), pb = c.buf<uint64_t>((size_t)(w * nw));
    const int64_t gp = std::min<int64_t>(ceil_div(std::max(u, w) * nw, 256), (int64_t)c.num_cus * 16);
    hipLaunchKernelGGL(k_pack_bits, dim3(grid_x(gp, 256)), dim3(256), 0, c.stream, A, u, ld, pa.get());
    hipLaunchKernelGGL(k_pack_bits, dim3(grid_x(gp, 256)), dim3(256), 0, c.stream, Bt, w, ld, pb.get());
    JP_HIP(hipGetLastError());
    const int64_t tm = ceil_div(u, PB), tn = ceil_div(w, PB);
    const int64_t total = xcd_padded(tm * tn);
    constexpr int64_t kMaxGrid = 1ll << 22;  // multiple of 8
    const int64_t blocks = total < kMaxGrid ? total : kMaxGrid;
    hipLaunchKernelGGL((k_bmm_bitpop<Emit>), dim3(grid_x(blocks, 256)), dim3(256), 0, c.stream,
                       (const uint64_t *)pa.get(), (const uint64_t *)pb.get(), u, w, nw, tm, tn, emit, cap,
                       count_dev);
    JP_HIP(hipGetLastError());
}

// Kernel choice: explicit, or for JP_BMM_AUTO / JP_BMM_I8_MFMA by shape
// (large tiles need both sides to fill several 256-row tiles); AUTO also
// races the popcount kernel against the int8 kernel once per shape class on
// the handle (autotune), keeping the faster.
enum class BmmVariant { T128, T256, BITPOP, F16 };

static BmmVariant by_shape(int64_t u, int64_t w) {
    return (u >= 1024 && w >= 1024) ? BmmVariant::T256 : BmmVariant::T128;
}

template <class Emit>
static void run_variant(const Ctx &c, BmmVariant v, const int8_t *A, const int8_t *Bt, int64_t u, int64_t w,
                        int64_t ld, Emit emit, int64_t cap, unsigned long long *count_dev, bool sym = false) {
    switch (v) {
        case BmmVariant::T256:
            launch_bmm_big(c, A, Bt, u, w, ld, emit, cap, count_dev, sym);
            if (sym && c.bmm_sym) *c.bmm_sym = true;
            break;
        case BmmVariant::BITPOP: launch_bitpop(c, A, Bt, u, w, ld, emit, cap, count_dev); break;
        case BmmVariant::F16: launch_bmm_f16(c, PlainRows{A, ld}, PlainRows{Bt, ld}, u, w, ld, emit, cap, count_dev); break;
        default: launch_bmm(c, PlainRows{A, ld}, Bt, u, w, ld, emit, cap, count_dev); break;
    }
}

// Shape class: log2 buckets of u, w and the stride.
uint64_t product_shape_class(int64_t u, int64_t w, int64_t ld) {
    return ((uint64_t)bits_for((uint64_t)u) << 16) | ((uint64_t)bits_for((uint64_t)w) << 8) |
           (uint64_t)bits_for((uint64_t)ld);
}

static uint64_t shape_class(int64_t u, int64_t w, int64_t ld) {
    return ((uint64_t)bits_for((uint64_t)u) << 16) | ((uint64_t)bits_for((uint64_t)w) << 8) |
           (uint64_t)bits_for((uint64_t)ld);
}

template <class Emit>
static void bool_matmul_any(const Ctx &c, const int8_t *A, const int8_t *Bt, int64_t u, int64_t w, int64_t ld,
                            int kind, Emit emit, int64_t cap, unsigned long long *count_dev, bool sym = false) {
    BmmVariant v;
    switch (kind) {
        case JP_BMM_I8_T128: v = BmmVariant::T128; break;
        case JP_BMM_I8_T256: v = BmmVariant::T256; break;
        case JP_BMM_BITPOP: v = BmmVariant::BITPOP; break;
        case JP_BMM_I8_MFMA: v = by_shape(u, w); break;
        case JP_BMM_F16: v = BmmVariant::F16; break;
        default: {
            v = by_shape(u, w);
            // race once per shape class (products too small to matter are not raced)
            if (c.tune && (double)u * (double)w * (double)ld >= 1e9) {
                const uint64_t key = shape_class(u, w, ld);
                auto it = c.tune->find(key);
                if (it != c.tune->end()) {
                    v = (BmmVariant)it->second;
                } else {
                    const BmmVariant cand[2] = {v, BmmVariant::BITPOP};
                    float best = -1;
                    for (BmmVariant q : cand) {
                        EventPair ev;
                        JP_HIP(hipEventRecord(ev.a, c.stream));
                        run_variant(c, q, A, Bt, u, w, ld, emit, 0, count_dev, sym);  // count only
                        JP_HIP(hipEventRecord(ev.b, c.stream));
                        JP_HIP(hipEventSynchronize(ev.b));
                        float ms = 0;
                        JP_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
                        if (best < 0 || ms < best) {
                            best = ms;
                            v = q;
                        }
                    }
                    (*c.tune)[key] = (int)v;
                }
            }
        }
    }
    if (c.bmm_used)
        *c.bmm_used = v == BmmVariant::BITPOP ? JP_BMM_BITPOP : (v == BmmVariant::F16 ? JP_BMM_F16 : JP_BMM_I8_MFMA);
    run_variant(c, v, A, Bt, u, w, ld, emit, cap, count_dev, sym);
}

void bool_matmul_pairs(const Ctx &c, const int8_t *A, const int8_t *Bt, int64_t u, int64_t w, int64_t ld, int kind,
                       int32_t *out_i, int32_t *out_j, int64_t cap, unsigned long long *count_dev) {
    bool_matmul_any(c, A, Bt, u, w, ld, kind, PairEmit{out_i, out_j}, cap, count_dev);
}

void bool_matmul_keys(const Ctx &c, const int8_t *A, const int8_t *Bt, int64_t u, int64_t w, int64_t ld, int kind,
                      const int32_t *rowmap, const int32_t *colmap, int shift, uint64_t *keys, int64_t cap,
                      unsigned long long *count_dev, bool sym) {
    bool_matmul_any(c, A, Bt, u, w, ld, kind, KeyEmit{rowmap, colmap, shift, keys}, cap, count_dev, sym);
}

void bool_matmul_count_keys(const Ctx &c, const int8_t *A, const int8_t *Bt, int64_t u, int64_t w, int64_t ld,
                            int kind, const int32_t *rowmap, const int32_t *colmap, int shift, int wshift, void *keys,
                            bool wide, int64_t cap, unsigned long long *count_dev, bool sym) {
    if (wide)
        bool_matmul_any(c, A, Bt, u, w, ld, kind,
                        CountKeyEmit<unsigned __int128>{rowmap, colmap, shift, wshift, (unsigned __int128 *)keys}, cap,
                        count_dev, sym);
    else
        bool_matmul_any(c, A, Bt, u, w, ld, kind, CountKeyEmit<uint64_t>{rowmap, colmap, shift, wshift,
                                                                          (uint64_t *)keys},
                        cap, count_dev, sym);
}

// Star query heavy product C = V x W^T (Section 3.2) over k factor matrices
// M_t (u[t] x ld, 0/1): V rows are the ceil(k/2)-tuples of the first factors,
// W rows the floor(k/2)-tuples of the rest, both generated from the factors'
// rows as they are loaded.  Nonzeros become k-tuple keys (xof[t][a_t] << s[t]).
template <class K, int G, int H>
static void star_product(const Ctx &c, const int8_t *const *M, const int64_t *u, int64_t ld, const int32_t *const *xof,
                         const int *s, void *keys, int64_t cap, unsigned long long *count_dev, bool f16) {
    TupleRows<G> a;
    TupleRows<H> b;
    TupleEmit<K, G, H> e;
    int64_t rows_a = 1, rows_b = 1;
    for (int t = 0; t < G; ++t) {
        a.M[t] = M[t];
        a.u[t] = u[t];
        rows_a *= u[t];
    }
    for (int t = 0; t < H; ++t) {
        b.M[t] = M[G + t];
        b.u[t] = u[G + t];
        rows_b *= u[G + t];
    }
    a.ld = b.ld = ld;
    for (int t = 0; t < G + H; ++t) {
        e.xof[t] = xof[t];
        e.u[t] = u[t];
        e.s[t] = s[t];
    }
    e.keys = (K *)keys;
    if (f16) launch_bmm_f16(c, a, b, rows_a, rows_b, ld, e, cap, count_dev);
    else launch_bmm_rows(c, a, b, rows_a, rows_b, ld, e, cap, count_dev);
}

template <class K>
static void star_product_k(const Ctx &c, int k, const int8_t *const *M, const int64_t *u, int64_t ld,
                           const int32_t *const *xof, const int *s, void *keys, int64_t cap,
                           unsigned long long *count_dev, bool f16) {
    switch (k) {
        case 3: star_product<K, 2, 1>(c, M, u, ld, xof, s, keys, cap, count_dev, f16); break;
        case 4: star_product<K, 2, 2>(c, M, u, ld, xof, s, keys, cap, count_dev, f16); break;
        case 5: star_product<K, 3, 2>(c, M, u, ld, xof, s, keys, cap, count_dev, f16); break;
        case 6: star_product<K, 3, 3>(c, M, u, ld, xof, s, keys, cap, count_dev, f16); break;
        case 7: star_product<K, 4, 3>(c, M, u, ld, xof, s, keys, cap, count_dev, f16); break;
        case 8: star_product<K, 4, 4>(c, M, u, ld, xof, s, keys, cap, count_dev, f16); break;
        default: fail(JP_EINTERNAL, "star product needs 3 <= k <= 8");
    }
}

void star_bmm_keys(const Ctx &c, int k, const int8_t *const *M, const int64_t *u, int64_t ld,
                   const int32_t *const *xof, const int *s, void *keys, bool wide, int64_t cap,
                   unsigned long long *count_dev, bool f16) {
    if (wide) star_product_k<unsigned __int128>(c, k, M, u, ld, xof, s, keys, cap, count_dev, f16);
    else star_product_k<uint64_t>(c, k, M, u, ld, xof, s, keys, cap, count_dev, f16);
}

}  // namespace jp
