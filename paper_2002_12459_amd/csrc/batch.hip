// Many independent two-path instances in one evaluation.
//
// The instances are placed side by side in disjoint id ranges: instance i's
// x ids become off_x[i] + (x - min x_i), and likewise for y and z (when the
// ranges of all instances add up to more than 2^31 values, the ids are
// replaced by dense ranks of the pairs (instance, id) instead).  Because
// no y is shared between instances, the join of the combined relations is
// the disjoint union of the instances' joins, and so is the projection
// (Section 2.1): one run of Algorithm 1 over the combined input gives every
// instance's exact output.  The combined output is sorted by (x, z) and the
// x ranges are increasing in i, so instance i's output is one contiguous
// slice; a last pass finds the slice bounds and maps ids back.  All
// instances share one threshold pair (the output does not depend on it).
//
// The point is launch amortisation: the pipeline runs a fixed number of
// kernels whatever the number of instances, so hundreds of small instances
// cost about as much as one instance of their combined size.
#include <climits>

#include "pipeline.hpp"
#include "prims.hpp"

namespace jp {
namespace {

struct BatchDesc {
    const int32_t *rx, *ry, *sz, *sy;
    int64_t nr, ns;          // 0 for instances skipped (an empty relation)
    int64_t r_base, s_base;  // position in the combined columns
};

constexpr int kBatchBlock = 256;

__device__ __forceinline__ void wave_minmax(int &mn, int &mx) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const int a = __shfl_xor(mn, o), b = __shfl_xor(mx, o);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
}

// mm[6 i ..] = min x, max x, min y, max y, min z, max z of instance i (y over R and S)
__global__ __launch_bounds__(kBatchBlock) void k_batch_minmax(const BatchDesc *d, int *mm) {
    __shared__ int sm[kBatchBlock / kWave][6];
    const BatchDesc b = d[blockIdx.y];
    int v[6] = {INT_MAX, INT_MIN, INT_MAX, INT_MIN, INT_MAX, INT_MIN};
    const int64_t stride = (int64_t)gridDim.x * kBatchBlock;
    for (int64_t e = (int64_t)blockIdx.x * kBatchBlock + threadIdx.x; e < b.nr; e += stride) {
        const int x = b.rx[e], y = b.ry[e];
        v[0] = x < v[0] ? x : v[0];
        v[1] = x > v[1] ? x : v[1];
        v[2] = y < v[2] ? y : v[2];
        v[3] = y > v[3] ? y : v[3];
    }
    for (int64_t e = (int64_t)blockIdx.x * kBatchBlock + threadIdx.x; e < b.ns; e += stride) {
        const int z = b.sz[e], y = b.sy[e];
        v[4] = z < v[4] ? z : v[4];
        v[5] = z > v[5] ? z : v[5];
        v[2] = y < v[2] ? y : v[2];
        v[3] = y > v[3] ? y : v[3];
    }
    wave_minmax(v[0], v[1]);
    wave_minmax(v[2], v[3]);
    wave_minmax(v[4], v[5]);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0)
        for (int q = 0; q < 6; ++q) sm[w][q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kBatchBlock / kWave; ++i)
            for (int q = 0; q < 6; q += 2) {
                v[q] = sm[i][q] < v[q] ? sm[i][q] : v[q];
                v[q + 1] = sm[i][q + 1] > v[q + 1] ? sm[i][q + 1] : v[q + 1];
            }
        int *o = mm + 6 * (int64_t)blockIdx.y;
        for (int q = 0; q < 6; q += 2) {
            atomicMin(&o[q], v[q]);
            atomicMax(&o[q + 1], v[q + 1]);
        }
    }
}

// Combined columns: id + add[3 i + {0, 1, 2}] for x, y, z of instance i.
__global__ __launch_bounds__(kBatchBlock) void k_batch_pack(const BatchDesc *d, const int64_t *add, int32_t *Rx,
                                                            int32_t *Ry, int32_t *Sz, int32_t *Sy) {
    const int64_t i = blockIdx.y;
    const BatchDesc b = d[i];
    const int64_t ax = add[3 * i], ay = add[3 * i + 1], az = add[3 * i + 2];
    const int64_t stride = (int64_t)gridDim.x * kBatchBlock;
    for (int64_t e = (int64_t)blockIdx.x * kBatchBlock + threadIdx.x; e < b.nr; e += stride) {
        Rx[b.r_base + e] = (int32_t)((int64_t)b.rx[e] + ax);
        Ry[b.r_base + e] = (int32_t)((int64_t)b.ry[e] + ay);
    }
    for (int64_t e = (int64_t)blockIdx.x * kBatchBlock + threadIdx.x; e < b.ns; e += stride) {
        Sz[b.s_base + e] = (int32_t)((int64_t)b.sz[e] + az);
        Sy[b.s_base + e] = (int32_t)((int64_t)b.sy[e] + ay);
    }
}

// 64-bit key of (instance, id): unsigned order equals (instance, signed id) order.
__device__ __forceinline__ uint64_t inst_key(int64_t i, int32_t v) {
    return ((uint64_t)i << 32) | (uint64_t)((uint32_t)v ^ 0x80000000u);
}

// Keys of one column of every instance: which = 0 (R x), 1 (R y), 2 (S y), 3 (S z).
__global__ __launch_bounds__(kBatchBlock) void k_batch_keys(const BatchDesc *d, int which, uint64_t *out) {
    const int64_t i = blockIdx.y;
    const BatchDesc b = d[i];
    const bool r = which < 2;
    const int32_t *col = which == 0 ? b.rx : (which == 1 ? b.ry : (which == 2 ? b.sy : b.sz));
    const int64_t n = r ? b.nr : b.ns, base = r ? b.r_base : b.s_base;
    const int64_t stride = (int64_t)gridDim.x * kBatchBlock;
    for (int64_t e = (int64_t)blockIdx.x * kBatchBlock + threadIdx.x; e < n; e += stride)
        out[base + e] = inst_key(i, col[e]);
}

// Combined ids of the output back to each instance's own ids.  Block b
// takes outputs [b * kSliceChunk, (b + 1) * kSliceChunk): one search finds
// the instances whose slices meet the chunk, their slice starts are staged
// in LDS, and each output finds its instance there (the last whose slice
// starts at or before it; instances with empty slices precede the one that
// holds the output).  bd: slice starts, n_inst + 1 entries, bd[n_inst] = n.
constexpr int64_t kSliceChunk = 4096;
constexpr int kSliceStage = 256;
__global__ __launch_bounds__(kBatchBlock) void k_batch_unshift(int32_t *X, int32_t *Z, int64_t n, const int64_t *bd,
                                                               int n_inst, const int64_t *add) {
    __shared__ int64_t sb[kSliceStage];
    __shared__ int sh_i0, sh_cnt;
    const int64_t k0 = (int64_t)blockIdx.x * kSliceChunk;
    const int64_t k1 = k0 + kSliceChunk < n ? k0 + kSliceChunk : n;
    auto last_at_or_before = [&](int lo, int hi, int64_t k) {  // last i in [lo, hi] with bd[i] <= k (bd[lo] <= k)
        while (lo < hi) {
            const int mid = lo + (hi - lo + 1) / 2;
            if (bd[mid] <= k) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    };
    if (threadIdx.x == 0) {
        const int i0 = last_at_or_before(0, n_inst, k0);
        sh_i0 = i0;
        sh_cnt = last_at_or_before(i0, n_inst, k1 - 1) - i0 + 1;
    }
    __syncthreads();
    const int i0 = sh_i0, cnt = sh_cnt;
    if (cnt <= kSliceStage) {
        for (int t = threadIdx.x; t < cnt; t += kBatchBlock) sb[t] = bd[i0 + t];
        __syncthreads();
        for (int64_t k = k0 + threadIdx.x; k < k1; k += kBatchBlock) {
            int lo = 0, hi = cnt - 1;
            while (lo < hi) {
                const int mid = lo + (hi - lo + 1) / 2;
                if (sb[mid] <= k) lo = mid;
                else hi = mid - 1;
            }
            const int64_t i = i0 + lo;
            X[k] = (int32_t)((int64_t)X[k] - add[3 * i]);
            Z[k] = (int32_t)((int64_t)Z[k] - add[3 * i + 2]);
        }
    } else {  // more instances meet the chunk than LDS stages: search bd itself
        for (int64_t k = k0 + threadIdx.x; k < k1; k += kBatchBlock) {
            const int64_t i = last_at_or_before(i0, i0 + cnt - 1, k);
            X[k] = (int32_t)((int64_t)X[k] - add[3 * i]);
            Z[k] = (int32_t)((int64_t)Z[k] - add[3 * i + 2]);
        }
    }
}

// Dense ranks of (instance, id) keys: sorted distinct keys in *uniq, their count returned.
struct RankTable {
    DBuf<uint64_t> uniq;
    int64_t n = 0;
};

RankTable rank_table(const Ctx &c, DBuf<uint64_t> &keys, int64_t n, int bits, int64_t *S) {
    RankTable t;
    DBuf<uint64_t> tmp = c.buf<uint64_t>((size_t)n);
    const uint64_t *k = radix_sort(c, keys.get(), tmp.get(), n, bits);
    t.uniq = c.buf<uint64_t>((size_t)n);
    uint64_t *u = t.uniq.get();
    compact(
        c, n, [=] __device__(int64_t i) { return i == 0 || k[i] != k[i - 1]; },
        [=] __device__(int64_t i, int64_t p) { u[p] = k[i]; }, S);
    t.n = c.load(S);
    return t;
}

}  // namespace

jp_result *run_two_path_batch(const Ctx &c, int n_inst, const jp_instance *inst, const jp_options &o) {
    JP_CHECK(n_inst <= 65535, JP_EINVAL, "a batch holds at most 65535 instances");
    std::vector<BatchDesc> hd(n_inst);
    int64_t NR = 0, NS = 0, nmax = 0;
    for (int i = 0; i < n_inst; ++i) {
        const jp_instance &q = inst[i];
        const bool use = q.n_r > 0 && q.n_s > 0;
        hd[i] = BatchDesc{q.r_x, q.r_y, q.s_z, q.s_y, use ? q.n_r : 0, use ? q.n_s : 0, NR, NS};
        NR += hd[i].nr;
        NS += hd[i].ns;
        nmax = std::max(nmax, std::max(hd[i].nr, hd[i].ns));
    }
    auto empty = [&]() {
        auto r = std::make_unique<jp_result>();
        r->alloc = c.alloc;
        r->arity = 2;
        r->stats.arity = 2;
        r->batch_off.assign((size_t)n_inst + 1, 0);
        return r.release();
    };
    if (NR == 0 || NS == 0) return empty();

    DBuf<BatchDesc> dd = c.buf<BatchDesc>((size_t)n_inst);
    c.upload(dd.get(), hd.data(), hd.size() * sizeof(BatchDesc));
    DBuf<int> mmb = c.buf<int>((size_t)6 * n_inst);
    int *mm = mmb.get();
    for_each(c, 6 * (int64_t)n_inst, [=] __device__(int64_t i) { mm[i] = (i & 1) ? INT_MIN : INT_MAX; });
    const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(nmax, kBatchBlock * 16), 64));
    hipLaunchKernelGGL(k_batch_minmax, dim3(gx, (unsigned)n_inst), dim3(kBatchBlock), 0, c.stream,
                       (const BatchDesc *)dd.get(), mm);
    JP_HIP(hipGetLastError());
    std::vector<int> hm((size_t)6 * n_inst);
    c.load_n(hm.data(), mm, hm.size());

    // disjoint ranges: off[i] = sum of the spans of instances before i
    std::vector<int64_t> add((size_t)3 * n_inst), offx((size_t)n_inst + 1);
    int64_t ox = 0, oy = 0, oz = 0;
    for (int i = 0; i < n_inst; ++i) {
        const int *m = &hm[6 * (size_t)i];
        offx[i] = ox;
        if (hd[i].nr == 0) {
            add[3 * i] = add[3 * i + 1] = add[3 * i + 2] = 0;
            continue;
        }
        add[3 * i] = ox - m[0];
        add[3 * i + 1] = oy - m[2];
        add[3 * i + 2] = oz - m[4];
        ox += (int64_t)m[1] - m[0] + 1;
        oy += (int64_t)m[3] - m[2] + 1;
        oz += (int64_t)m[5] - m[4] + 1;
    }
    offx[n_inst] = ox;
    const bool ranked = ox > INT_MAX || oy > INT_MAX || oz > INT_MAX;
    JP_CHECK(NR <= INT_MAX && NS <= INT_MAX, JP_EINVAL, "a batch holds at most 2^31 - 1 tuples per relation");
    DBuf<int64_t> addd = c.buf<int64_t>(add.size());
    DBuf<int64_t> offd = c.buf<int64_t>((size_t)n_inst + 1);
    DBuf<int32_t> Rx = c.buf<int32_t>(NR), Ry = c.buf<int32_t>(NR), Sz = c.buf<int32_t>(NS), Sy = c.buf<int32_t>(NS);
    RankTable tx, tz;
    if (!ranked) {
        c.upload(addd.get(), add.data(), add.size() * sizeof(int64_t));
        c.upload(offd.get(), offx.data(), offx.size() * sizeof(int64_t));
        hipLaunchKernelGGL(k_batch_pack, dim3(gx, (unsigned)n_inst), dim3(kBatchBlock), 0, c.stream,
                           (const BatchDesc *)dd.get(), (const int64_t *)addd.get(), Rx.get(), Ry.get(), Sz.get(),
                           Sy.get());
        JP_HIP(hipGetLastError());
    } else {
        // dense ranks of (instance, id): x over R, z over S, y over both
        DBuf<int64_t> S = c.buf<int64_t>(1);
        const int bits = 32 + bits_for((uint64_t)(n_inst - 1));
        auto keys_of = [&](int which, uint64_t *out) {
            hipLaunchKernelGGL(k_batch_keys, dim3(gx, (unsigned)n_inst), dim3(kBatchBlock), 0, c.stream,
                               (const BatchDesc *)dd.get(), which, out);
            JP_HIP(hipGetLastError());
        };
        auto rank_into = [&](const RankTable &t, const uint64_t *k, int64_t n, int32_t *dst) {
            const uint64_t *u = t.uniq.get();
            const int64_t nu = t.n;
            for_each(c, n, [=] __device__(int64_t e) {
                dst[e] = (int32_t)lower_bound_dev(u, (int64_t)0, nu, k[e]);
            });
        };
        {
            DBuf<uint64_t> kx = c.buf<uint64_t>(NR), kx2 = c.buf<uint64_t>(NR);
            keys_of(0, kx.get());
            JP_HIP(hipMemcpyAsync(kx2.get(), kx.get(), NR * sizeof(uint64_t), hipMemcpyDeviceToDevice, c.stream));
            tx = rank_table(c, kx2, NR, bits, S.get());
            rank_into(tx, kx.get(), NR, Rx.get());
        }
        {
            DBuf<uint64_t> kz = c.buf<uint64_t>(NS), kz2 = c.buf<uint64_t>(NS);
            keys_of(3, kz.get());
            JP_HIP(hipMemcpyAsync(kz2.get(), kz.get(), NS * sizeof(uint64_t), hipMemcpyDeviceToDevice, c.stream));
            tz = rank_table(c, kz2, NS, bits, S.get());
            rank_into(tz, kz.get(), NS, Sz.get());
        }
        {
            DBuf<uint64_t> ky = c.buf<uint64_t>(NR + NS), ky2 = c.buf<uint64_t>(NR + NS);
            keys_of(1, ky.get());
            // S keys after R keys: shift the S bases by NR
            std::vector<BatchDesc> hs = hd;
            for (auto &q : hs) q.s_base += NR;
            DBuf<BatchDesc> ds = c.buf<BatchDesc>((size_t)n_inst);
            c.upload(ds.get(), hs.data(), hs.size() * sizeof(BatchDesc));
            hipLaunchKernelGGL(k_batch_keys, dim3(gx, (unsigned)n_inst), dim3(kBatchBlock), 0, c.stream,
                               (const BatchDesc *)ds.get(), 2, ky.get());
            JP_HIP(hipGetLastError());
            JP_HIP(hipMemcpyAsync(ky2.get(), ky.get(), (NR + NS) * sizeof(uint64_t), hipMemcpyDeviceToDevice,
                                  c.stream));
            RankTable ty = rank_table(c, ky2, NR + NS, bits, S.get());
            rank_into(ty, ky.get(), NR, Ry.get());
            rank_into(ty, ky.get() + NR, NS, Sy.get());
            c.sync();  // hs is read by the copy above
        }
        // first rank of each instance's x: lower bound of (i << 32) in the x table
        const uint64_t *ux = tx.uniq.get();
        const int64_t nux = tx.n;
        int64_t *od = offd.get();
        for_each(c, (int64_t)n_inst + 1, [=] __device__(int64_t i) {
            od[i] = lower_bound_dev(ux, (int64_t)0, nux, (uint64_t)i << 32);
        });
    }
    // the host arrays above are read by the copies before they go out of scope
    c.sync();

    std::unique_ptr<jp_result> res(run_two_path(c, Rx.get(), Ry.get(), NR, Sz.get(), Sy.get(), NS, o));
    Rx.reset();
    Ry.reset();
    Sz.reset();
    Sy.reset();
    const int64_t n = res->n;
    res->batch_off.assign((size_t)n_inst + 1, 0);
    if (n == 0) return res.release();

    // slice bounds: first output whose combined x reaches the instance's first x
    DBuf<int64_t> bnd = c.buf<int64_t>((size_t)n_inst + 1);
    int32_t *X = res->cols[0].get(), *Z = res->cols[1].get();
    const int64_t *od = offd.get();
    int64_t *bd = bnd.get();
    for_each(c, (int64_t)n_inst + 1, [=] __device__(int64_t i) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if ((int64_t)X[mid] < od[i]) lo = mid + 1;
            else hi = mid;
        }
        bd[i] = lo;
    });
    if (ranked) {
        const uint64_t *ux = tx.uniq.get(), *uz = tz.uniq.get();
        for_each(c, n, [=] __device__(int64_t k) {
            X[k] = (int32_t)((uint32_t)ux[X[k]] ^ 0x80000000u);
            Z[k] = (int32_t)((uint32_t)uz[Z[k]] ^ 0x80000000u);
        });
    } else {
        hipLaunchKernelGGL(k_batch_unshift, dim3(grid_x(ceil_div(n, kSliceChunk), kBatchBlock)), dim3(kBatchBlock), 0,
                           c.stream, X, Z, n, (const int64_t *)bd, n_inst, (const int64_t *)addd.get());
        JP_HIP(hipGetLastError());
    }
    c.load_n(res->batch_off.data(), bd, (size_t)n_inst + 1);
    JP_CHECK(res->batch_off[n_inst] == n, JP_EINTERNAL, "batched output slices do not cover the output");
    return res.release();
}

}  // namespace jp
