// Heavy part of the method: the 0/1 matrix product M = M1 x M2 over the
// heavy x / y / z values (Algorithm 1, lines 4-6; the Boolean-product view of
// Section 2.2).  Every entry is 0 or 1 and every count is at most the number
// of heavy y values, so int8 inputs with int32 accumulation are exact.  The
// product is never stored: the epilogue tests each accumulator for > 0 in
// registers and appends the nonzero coordinates (one atomic per wave).
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

struct KeyEmit {  // nonzero (i, j) -> (rowmap[i] << shift) | colmap[j]
    const int32_t *rowmap, *colmap;
    int shift;
    uint64_t *keys;
    __device__ void operator()(int64_t pos, int64_t i, int64_t j) const {
        keys[pos] = ((uint64_t)(uint32_t)rowmap[i] << shift) | (uint64_t)(uint32_t)colmap[j];
    }
};
struct PairEmit {  // nonzero (i, j) -> rows[pos] = i, cols[pos] = j
    int32_t *rows, *cols;
    __device__ void operator()(int64_t pos, int64_t i, int64_t j) const {
        rows[pos] = (int32_t)i;
        cols[pos] = (int32_t)j;
    }
};

// Row sources of the A operand: 16 bytes of row r starting at byte k.
struct PlainRows {  // A stored row-major
    const int8_t *A;
    int64_t ld;
    __device__ v4i load(int64_t r, int64_t k) const { return *(const v4i *)(A + r * ld + k); }
};
struct PairRows {  // row (a1, a2) = M1[a1,:] AND M2[a2,:] (0/1 bytes), a1 = r / u2, a2 = r % u2
    const int8_t *M1, *M2;
    int64_t ld, u2;
    __device__ v4i load(int64_t r, int64_t k) const {
        const int64_t a1 = r / u2, a2 = r - a1 * u2;
        const v4i p = *(const v4i *)(M1 + a1 * ld + k), q = *(const v4i *)(M2 + a2 * ld + k);
        return p & q;
    }
};
template <class K>
struct TripleEmit {  // nonzero ((a1,a2), a3) -> x1 << s1 | x2 << s2 | x3
    const int32_t *x1_of, *x2_of, *x3_of;
    int64_t u2;
    int s1, s2;
    K *keys;
    __device__ void operator()(int64_t pos, int64_t i, int64_t j) const {
        const int64_t a1 = i / u2, a2 = i - a1 * u2;
        keys[pos] = ((K)(uint32_t)x1_of[a1] << s1) | ((K)(uint32_t)x2_of[a2] << s2) | (K)(uint32_t)x3_of[j];
    }
};

// Block index -> tile, grouping consecutive blocks of one XCD (blocks are
// dealt round-robin to the 8 XCDs) onto a compact 2-D patch of tiles so that
// tiles sharing A rows / B rows share that XCD's L2.
__device__ __forceinline__ void tile_of_block(int64_t bid, int64_t tiles_m, int64_t tiles_n, int64_t *tm,
                                              int64_t *tn) {
    const int64_t total = tiles_m * tiles_n;
    int64_t t = bid;
    if (total % 8 == 0) {
        const int64_t per = total / 8;
        t = (bid % 8) * per + bid / 8;
    }
    // group of 8 tile-rows swept column-major inside the group
    const int64_t G = 8;
    const int64_t group = t / (G * tiles_n);
    const int64_t first_m = group * G;
    const int64_t gm = (tiles_m - first_m) < G ? (tiles_m - first_m) : G;
    const int64_t in = t - group * G * tiles_n;
    *tm = first_m + in % gm;
    *tn = in / gm;
}

template <class ARows, class Emit>
__global__ __launch_bounds__(256) void k_bmm_i8(ARows arows, const int8_t *__restrict__ Bt, int64_t u, int64_t w,
                                                int64_t ld, int64_t tiles_m, int64_t tiles_n, Emit emit, int64_t cap,
                                                unsigned long long *count) {
    __shared__ __attribute__((aligned(16))) int8_t sA[BM * LDS_STRIDE];
    __shared__ __attribute__((aligned(16))) int8_t sB[BN * LDS_STRIDE];
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
    const int wm = wv >> 1, wn = wv & 1;
    // global -> register staging: each thread moves 4 x 16 B of A and of B
    // per stage: row = (tid / 8) + 32 * q, byte offset = (tid % 8) * 16
    const int lr = tid / 8, lc = (tid % 8) * 16;
    const int fr = lane % 16, fk = (lane / 16) * 16;
    // Workgroups loop over tiles when the tile count exceeds the grid (the
    // grid is a multiple of 8, so a workgroup stays on its XCD's tile patch).
    const int64_t total = tiles_m * tiles_n;
    for (int64_t bid = blockIdx.x; bid < total; bid += gridDim.x) {
        int64_t tm, tn;
        tile_of_block(bid, tiles_m, tiles_n, &tm, &tn);
        const int64_t row0 = tm * BM, col0 = tn * BN;
        v4i ra[4], rb[4];
        auto load_stage = [&](int64_t k0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                int64_t r = row0 + lr + 32 * q;
                ra[q] = r < u ? arows.load(r, k0 + lc) : v4i{0, 0, 0, 0};
                int64_t c = col0 + lr + 32 * q;
                rb[q] = c < w ? *(const v4i *)(Bt + c * ld + k0 + lc) : v4i{0, 0, 0, 0};
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

        load_stage(0);
        for (int64_t k0 = 0; k0 < ld; k0 += BK) {
            __syncthreads();
            store_stage();
            __syncthreads();
            if (k0 + BK < ld) load_stage(k0 + BK);
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
        // block, col = lane % 16.  Count this lane's nonzeros, one atomic per wave.
        uint32_t mine = 0;
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    int64_t i = row0 + wm * 64 + f * 16 + (lane / 16) * 4 + r;
                    int64_t j = col0 + wn * 64 + g * 16 + (lane % 16);
                    mine += (acc[f][g][r] > 0 && i < u && j < w) ? 1u : 0u;
                }
        uint32_t incl = wave_incl_scan(mine);
        uint32_t wtot = __shfl(incl, kWave - 1);
        if (wtot == 0) continue;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(count, (unsigned long long)wtot);
        base = __shfl(base, 0);
        int64_t pos = (int64_t)base + (incl - mine);
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    int64_t i = row0 + wm * 64 + f * 16 + (lane / 16) * 4 + r;
                    int64_t j = col0 + wn * 64 + g * 16 + (lane % 16);
                    if (acc[f][g][r] > 0 && i < u && j < w) {
                        if (pos < cap) emit(pos, i, j);
                        ++pos;
                    }
                }
    }
}

template <class ARows, class Emit>
void launch_bmm(const Ctx &c, ARows arows, const int8_t *Bt, int64_t u, int64_t w, int64_t ld, int kind, Emit emit,
                int64_t cap, unsigned long long *count_dev) {
    JP_CHECK(ld % kBmmPadK == 0, JP_EINTERNAL, "heavy matrix stride must be a multiple of 128");
    c.zero(count_dev, 1);
    if (u <= 0 || w <= 0 || ld <= 0) return;
    (void)kind;
    const int64_t tm = ceil_div(u, BM), tn = ceil_div(w, BN);
    const int64_t total = tm * tn;
    constexpr int64_t kMaxGrid = 1ll << 22;  // tiles beyond this are looped over (multiple of 8)
    const int64_t blocks = total < kMaxGrid ? total : kMaxGrid;
    hipLaunchKernelGGL((k_bmm_i8<ARows, Emit>), dim3(grid_x(blocks, 256)), dim3(256), 0, c.stream, arows, Bt, u, w, ld,
                       tm, tn, emit, cap, count_dev);
    JP_HIP(hipGetLastError());
}

}  // namespace

void bool_matmul_pairs(const Ctx &c, const int8_t *A, const int8_t *Bt, int64_t u, int64_t w, int64_t ld, int kind,
                       int32_t *out_i, int32_t *out_j, int64_t cap, unsigned long long *count_dev) {
    launch_bmm(c, PlainRows{A, ld}, Bt, u, w, ld, kind, PairEmit{out_i, out_j}, cap, count_dev);
}

void bool_matmul_keys(const Ctx &c, const int8_t *A, const int8_t *Bt, int64_t u, int64_t w, int64_t ld, int kind,
                      const int32_t *rowmap, const int32_t *colmap, int shift, uint64_t *keys, int64_t cap,
                      unsigned long long *count_dev) {
    launch_bmm(c, PlainRows{A, ld}, Bt, u, w, ld, kind, KeyEmit{rowmap, colmap, shift, keys}, cap, count_dev);
}

void star_bmm_keys(const Ctx &c, const int8_t *M1, const int8_t *M2, const int8_t *M3, int64_t u1, int64_t u2,
                   int64_t u3, int64_t ld, const int32_t *x1_of, const int32_t *x2_of, const int32_t *x3_of, int s1,
                   int s2, void *keys, bool wide, int64_t cap, unsigned long long *count_dev) {
    const PairRows rows{M1, M2, ld, u2};
    if (wide)
        launch_bmm(c, rows, M3, u1 * u2, u3, ld, JP_BMM_I8_MFMA,
                   TripleEmit<unsigned __int128>{x1_of, x2_of, x3_of, u2, s1, s2, (unsigned __int128 *)keys}, cap,
                   count_dev);
    else
        launch_bmm(c, rows, M3, u1 * u2, u3, ld, JP_BMM_I8_MFMA,
                   TripleEmit<uint64_t>{x1_of, x2_of, x3_of, u2, s1, s2, (uint64_t *)keys}, cap, count_dev);
}

}  // namespace jp
