// Internal interfaces between the host planner, the pipelines and the C ABI.
#pragma once

#include <climits>

#include "common.hpp"

struct jp_result {
    std::shared_ptr<jp::Allocator> alloc;
    int32_t arity = 0;
    int64_t n = 0;
    jp::DBuf<int32_t> cols[8];
    jp_stats stats{};
    std::vector<int64_t> batch_off;  // batched results: instance i owns tuples [off[i], off[i+1])
};

namespace jp {

// One Section 5 index on the host: ascending distinct degrees with the
// number of values of each degree and their summed work.
struct HostIndex {
    std::vector<int64_t> deg, count;
    std::vector<double> sum;
    jp_degree_index view() const {
        jp_degree_index d;
        d.n = (int64_t)deg.size();
        d.deg = deg.data();
        d.count = count.data();
        d.sum = sum.empty() ? nullptr : sum.data();
        return d;
    }
};

// Degree summary of an indexed two-path instance, on the host: the inputs of
// the threshold choice (Section 5 indexes and Algorithm 2).
struct TwoPathSummary {
    int64_t n_r = 0, n_s = 0, dom_x = 0, dom_y = 0, dom_z = 0;
    int64_t J = 0;
    bool self_join = false;
    double out_est = 0;   // output-size estimate (Section 5)
    double out_sampled = 0;  // sampled estimate (selector input); 0 when not computed
    int64_t sample_distinct = 0, sample_draws = 0;
    bool have_indexes = false;
    HostIndex y;          // key degree of y; sum = deg_R(y) deg_S(y)
    HostIndex x;          // deg_R(x); sum = witnesses of x
    HostIndex xcdf;       // smallest key degree among the y of x
    HostIndex z;          // deg_S(z)
    HostIndex yr, ys;     // deg_R(y), deg_S(y) (features)
    jp_two_path_summary view() const {
        jp_two_path_summary v;
        v.n_r = n_r;
        v.n_s = n_s;
        v.dom_x = dom_x;
        v.dom_y = dom_y;
        v.dom_z = dom_z;
        v.J = J;
        v.out_est = out_est;
        v.y = y.view();
        v.x = x.view();
        v.xcdf = xcdf.view();
        v.z = z.view();
        return v;
    }
};

struct PlanResult {
    int64_t d1 = JP_DELTA_INF, d2 = JP_DELTA_INF;
    double cost = 0, cost_light_only = 0;
};

struct Thresholds {
    int64_t d1 = JP_DELTA_INF, d2 = JP_DELTA_INF;
    int32_t strategy = JP_STRATEGY_LIGHT_ONLY;
    bool light_only() const { return d1 == JP_DELTA_INF && d2 == JP_DELTA_INF; }
};

// Learned threshold selector: weights on the device, input normalisation on
// the host (mlp.hip).
constexpr int kFeatures = 16;
constexpr int kSelectorCells = 65;  // 8 x 8 geometric (Delta1, Delta2) grid + light only
struct Selector {
    int32_t n_out = 0;
    DBuf<float> params;
    float mean[kFeatures] = {}, scale[kFeatures] = {};
    bool ready() const { return n_out > 0 && params.get() != nullptr; }
};
int64_t mlp_param_count(int n_out);
void mlp_forward(const Ctx &c, const float *params, int K, const float *x, int64_t batch, float *y);
void mlp_grad(const Ctx &c, const float *params, int K, const float *x, const float *target, const float *mask,
              int64_t batch, float *grad, float *loss);
void mlp_adam(const Ctx &c, float *params, float *m, float *v, const float *grad, int64_t n, int step, float lr,
              float b1, float b2, float eps);
void selector_cells(const float *features, int64_t *d1, int64_t *d2);

// Planner (host).
Thresholds choose_thresholds(const TwoPathSummary &s, const jp_options &o, const jp_calibration &cal);
double estimate_out(int64_t dom_x, int64_t dom_z, int64_t J, int64_t N);
Thresholds theory_thresholds(int64_t N, double out);
PlanResult algorithm2(const jp_two_path_summary &s, const jp_calibration &c);
void default_calibration(jp_calibration *c);
void features16(const TwoPathSummary &s, float *f);
// Algorithm 2's cost of one threshold pair and the heavy dimensions u, v, w.
double plan_cost(const jp_two_path_summary &s, const jp_calibration &c, int64_t d1, int64_t d2, int64_t *uvw);
// The same for n pairs at once (cost and / or uvw may be null).
void plan_costs(const jp_two_path_summary &s, const jp_calibration &c, int n, const int64_t *d1, const int64_t *d2,
                double *cost, int64_t *uvw);
// Its heavy part alone: M-hat(u, v, w) plus the heavy matrices' bytes (0 without a product).
double heavy_cost(const jp_calibration &c, int64_t u, int64_t v, int64_t w);
// Threshold choice for any strategy, running the selector for AUTO_MLP when
// the context holds one (otherwise Algorithm 2).
Thresholds select_thresholds(const Ctx &c, const TwoPathSummary &s, const jp_options &o);

// Two-path index + summary (+ thresholds) without the join (jp_plan_two_path).
void plan_two_path(const Ctx &c, const int32_t *rx, const int32_t *ry, int64_t nr, const int32_t *sz,
                   const int32_t *sy, int64_t ns, const jp_options &o, int64_t *d1, int64_t *d2, float *features);
// Cost-model estimates of given threshold pairs on one instance (jp_plan_cells).
void plan_cells(const Ctx &c, const int32_t *rx, const int32_t *ry, int64_t nr, const int32_t *sz, const int32_t *sy,
                int64_t ns, const jp_options &o, int32_t n_cells, const int64_t *d1, const int64_t *d2,
                double *est_seconds, int64_t *heavy_dims);

// Index build of a two-path instance (Section 5, "Indexing relations"):
// R x-major (off_x, adj_r = y rank, r_xr = x rank per tuple), S y-major
// (off_y, adj_s = z rank, s2_y = y rank per tuple), degrees, rank tables, J.
struct Ingest {
    int64_t n_r2 = 0, n_s2 = 0, dom_x = 0, dom_y = 0, dom_z = 0, J = 0;
    int64_t x_dense_base = INT64_MIN, z_dense_base = INT64_MIN;  // see SegDedupIn
    int64_t zmin = 0, zspan = 0;                                  // range of the z ids kept
    int64_t n_in = 0;                                             // input tuples, |R| + |S|
    DBuf<int32_t> r_xr, adj_r, s2_y, dRy, dSz, xorig, zorig;
    DBuf<uint32_t> s2_zoff;  // z - zmin of every kept S tuple, y-major
    DBuf<uint32_t> zs;       // the distinct z - zmin, ascending (dom_z)
    DBuf<int64_t> off_x, off_y;
    // z rank of every kept S tuple (y-major), built on first use: an
    // evaluation that works in z offsets without a heavy part never reads it.
    const int32_t *adj_s(const Ctx &c) const;
    mutable DBuf<int32_t> adj_s_;
};

// Builds the Section 5 degree indexes of an indexed instance (summary.hip).
void summarize_two_path(const Ctx &c, const Ingest &g, int y_rule, TwoPathSummary &s);

// Sampled output size of an indexed instance (summary.hip): the distinct z
// reached by `draws` x ranks drawn with splitmix64 from `seed` (see there).
struct SampledOut {
    int64_t distinct = 0, draws = 0;
};
SampledOut sampled_out(const Ctx &c, const Ingest &g, uint64_t seed, int64_t max_draws = 1024,
                       int64_t cap = int64_t(1) << 26);

// Set similarity output of a two-path instance (Section 2.1): pairs whose
// sets share at least min_c elements, with the overlap as a third column;
// order 1 sorts by overlap descending, then (x, z).
struct OverlapSpec {
    int64_t min_c = 1;
    int order = 0;
    bool force_wide = false;  // 128-bit candidate and order keys even when 64 bits hold them (tests)
};
// Process-wide switch behind force_wide (jp_test_set_wide_overlap_keys).
inline int &wide_overlap_keys_flag() {
    static int on = 0;
    return on;
}

// Pipelines.
jp_result *run_two_path(const Ctx &c, const int32_t *rx, const int32_t *ry, int64_t nr, const int32_t *sz,
                        const int32_t *sy, int64_t ns, const jp_options &o, const OverlapSpec *ov = nullptr);
jp_result *run_two_path_batch(const Ctx &c, int n_inst, const jp_instance *inst, const jp_options &o);
// Batched Boolean set intersection (bsi.hip): answers[i] (device, nt bytes)
// = 1 iff the sets of tx[i] in R and of tz[i] in S intersect.
void run_bsi(const Ctx &c, const int32_t *rx, const int32_t *ry, int64_t nr, const int32_t *sz, const int32_t *sy,
             int64_t ns, const int32_t *tx, const int32_t *tz, int64_t nt, const jp_options &o, uint8_t *answers,
             jp_stats *stats);
jp_result *run_star(const Ctx &c, int k, const int32_t *const *x, const int32_t *const *y, const int64_t *n,
                    const jp_options &o);

// Heavy product: A (u x ld) and Bt (w x ld) int8 0/1, K = ld (multiple of 128).
// For every nonzero C[i][j] calls the emitter through a pair buffer: writes
// rows/cols into out_i / out_j (capacity cap) and counts into *count_dev.
void bool_matmul_pairs(const Ctx &c, const int8_t *A, const int8_t *Bt, int64_t u, int64_t w, int64_t ld,
                       int kind, int32_t *out_i, int32_t *out_j, int64_t cap, unsigned long long *count_dev);
// Same, emitting ((rowmap[i] << shift | colmap[j]) << wshift) | C[i][j]: the
// key of the pair with its count (u64 keys, or 128-bit keys when wide).
void bool_matmul_count_keys(const Ctx &c, const int8_t *A, const int8_t *Bt, int64_t u, int64_t w, int64_t ld,
                            int kind, const int32_t *rowmap, const int32_t *colmap, int shift, int wshift, void *keys,
                            bool wide, int64_t cap, unsigned long long *count_dev, bool sym = false);
// Same, emitting packed keys (rowmap[i] << shift) | colmap[j] (u64).
// sym: A == Bt and u == w (a self-join): the product is symmetric, and the
// 256 x 256 kernel computes only the tiles on and above the diagonal,
// emitting each nonzero of an off-diagonal tile twice (mirrored).
void bool_matmul_keys(const Ctx &c, const int8_t *A, const int8_t *Bt, int64_t u, int64_t w, int64_t ld, int kind,
                      const int32_t *rowmap, const int32_t *colmap, int shift, uint64_t *keys, int64_t cap,
                      unsigned long long *count_dev, bool sym = false);

constexpr int64_t kBmmPadK = 128;  // K padding of the heavy matrices (bytes)

// Shape class of a product (log2 buckets of u, w and the row stride): the key
// under which JP_BMM_AUTO keeps its kernel choice.
uint64_t product_shape_class(int64_t u, int64_t w, int64_t ld);

}  // namespace jp
