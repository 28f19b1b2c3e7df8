// Internal interfaces between the host planner, the pipelines and the C ABI.
#pragma once

#include "common.hpp"

struct jp_result {
    std::shared_ptr<jp::Allocator> alloc;
    int32_t arity = 0;
    int64_t n = 0;
    jp::DBuf<int32_t> cols[8];
    jp_stats stats{};
};

namespace jp {

// Degree summary of an indexed two-path instance, on the host: the inputs of
// the threshold choice (Section 5 indexes and Algorithm 2).
struct TwoPathSummary {
    int64_t n_r = 0, n_s = 0, dom_x = 0, dom_y = 0, dom_z = 0;
    int64_t J = 0;
    bool self_join = false;
    // Histograms by degree (index = degree, capped at the max degree):
    std::vector<int64_t> cnt_x;   // number of x with deg_R(x) = d
    std::vector<int64_t> cnt_z;   // number of z with deg_S(z) = d
    std::vector<int64_t> cnt_y;   // number of y with key degree = d (key degree per the y rule)
    std::vector<int64_t> jy;      // sum over y with key degree d of deg_R(y) * deg_S(y)
    std::vector<int64_t> sx;      // sum over x with deg_R(x) = d of the full per-x join work
    std::vector<int64_t> ry;      // sum over y with key degree d of deg_R(y)
    double out_est = 0;           // output-size estimate
};

struct Thresholds {
    int64_t d1 = JP_DELTA_INF, d2 = JP_DELTA_INF;
    int32_t strategy = JP_STRATEGY_LIGHT_ONLY;
    bool light_only() const { return d1 == JP_DELTA_INF && d2 == JP_DELTA_INF; }
};

// Planner (host).
Thresholds choose_thresholds(const TwoPathSummary &s, const jp_options &o);
double estimate_out(int64_t dom_x, int64_t dom_z, int64_t J, int64_t N);
Thresholds theory_thresholds(int64_t N, double out);

// Pipelines.
jp_result *run_two_path(const Ctx &c, const int32_t *rx, const int32_t *ry, int64_t nr, const int32_t *sz,
                        const int32_t *sy, int64_t ns, const jp_options &o);
jp_result *run_star(const Ctx &c, int k, const int32_t *const *x, const int32_t *const *y, const int64_t *n,
                    const jp_options &o);

// Heavy product: A (u x ld) and Bt (w x ld) int8 0/1, K = ld (multiple of 64).
// For every nonzero C[i][j] calls the emitter through a pair buffer: writes
// rows/cols into out_i / out_j (capacity cap) and counts into *count_dev.
void bool_matmul_pairs(const Ctx &c, const int8_t *A, const int8_t *Bt, int64_t u, int64_t w, int64_t ld,
                       int kind, int32_t *out_i, int32_t *out_j, int64_t cap, unsigned long long *count_dev);
// Same, emitting packed keys (rowmap[i] << shift) | colmap[j] (u64).
void bool_matmul_keys(const Ctx &c, const int8_t *A, const int8_t *Bt, int64_t u, int64_t w, int64_t ld, int kind,
                      const int32_t *rowmap, const int32_t *colmap, int shift, uint64_t *keys, int64_t cap,
                      unsigned long long *count_dev);

constexpr int64_t kBmmPadK = 128;  // K padding of the heavy matrices (bytes)

}  // namespace jp
