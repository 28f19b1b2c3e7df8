/*
 * jp.h: C ABI of libjoinproject, an MI355X (gfx950) implementation of the
 * join-project method of "Fast Join Project Query Evaluation using Matrix
 * Multiplication" (Deep, Hu, Koutris).
 *
 * Queries (paper Section 2.1):
 *   two-path  Q(x,z)      = R(x,y), S(z,y)           projected on (x,z)
 *   star      Q(x1..xk)   = R1(x1,y), ..., Rk(xk,y)   projected on (x1..xk)
 * The result is the set of distinct output tuples.  The method (Algorithm 1,
 * Section 3.1; star: Section 3.2) splits each relation at integer degree
 * thresholds Delta1 (on the join variable y) and Delta2 (on the free
 * variables); light tuples are joined by per-y expansion followed by
 * duplicate removal, heavy tuples through a 0/1 matrix product whose nonzero
 * entries are the heavy output, and the two outputs are unioned.  Thresholds
 * are given by the caller or chosen automatically (Section 5, Algorithm 2, or
 * Lemma 3's closed forms).  The result does not depend on the thresholds.
 *
 * Conventions for every call:
 *  - Relation columns are DEVICE pointers to int32 values on the handle's
 *    device, borrowed for the duration of the call, never written.  Any int32
 *    value is a valid id.  Rows may repeat (relations are sets: repeats do
 *    not change the result).  A column may be NULL only when its length is 0.
 *  - All device work is ordered on the handle's stream (jp_set_stream); a
 *    call returns after the output size is known (the host waits on the
 *    stream), with the output data possibly still being written in stream
 *    order.
 *  - Output tuples are distinct and sorted ascending, lexicographically by
 *    signed int32, stored as structure-of-arrays int32 device columns owned
 *    by the library until jp_result_free.
 *  - No C++ exception crosses this boundary.  On any status other than JP_OK
 *    no result is returned (*out is set to NULL), nothing leaks, and
 *    jp_last_error(h) describes the failure.
 *  - A handle must not be used by two threads at the same time.
 */
#ifndef JP_H
#define JP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JP_ABI_VERSION 1

typedef enum jp_status {
    JP_OK = 0,
    JP_EINVAL = 1,      /* bad argument: NULL with n > 0, n < 0, k out of range, Delta < 1 */
    JP_ENOMEM = 2,      /* device allocation failed */
    JP_EHIP = 3,        /* a HIP runtime call failed; message has hipGetErrorString */
    JP_ECAPACITY = 4,   /* a caller-supplied capacity was too small; the needed size is reported */
    JP_EPRECISION = 5,  /* JP_BMM_F16 was requested where counts could reach 2^24 (v, or ld, >= 2^24) */
    JP_EINTERNAL = 6    /* internal consistency check failed */
} jp_status;

/* How the thresholds (Delta1, Delta2) are chosen. */
typedef enum jp_strategy {
    JP_STRATEGY_AUTO_COST = 0,  /* Algorithm 2 (Section 5) with device-calibrated constants */
    JP_STRATEGY_THEORY = 1,     /* Lemma 3 closed forms from N and the estimated |OUT| */
    JP_STRATEGY_FIXED = 2,      /* use options.delta1 / options.delta2 as given */
    JP_STRATEGY_LIGHT_ONLY = 3, /* no heavy part: every tuple is light (Delta = infinity) */
    JP_STRATEGY_AUTO_MLP = 4    /* learned selector; falls back to AUTO_COST without weights */
} jp_strategy;

/* Kernel used for the heavy 0/1 matrix product. */
typedef enum jp_bmm_kind {
    JP_BMM_AUTO = 0,     /* int8 MFMA unless the planner prefers the popcount kernel */
    JP_BMM_I8_MFMA = 1,  /* int8 inputs, int32 accumulation on the matrix cores; tile by shape */
    JP_BMM_BITPOP = 2,   /* bit-packed rows, AND + popcount on the vector units */
    JP_BMM_I8_T128 = 3,  /* int8 MFMA, 128 x 128 block tiles */
    JP_BMM_I8_T256 = 4,  /* int8 MFMA, 256 x 256 block tiles */
    JP_BMM_F16 = 5       /* 0/1 operands as fp16, fp32 accumulation (exact below 2^24; JP_EPRECISION otherwise) */
} jp_bmm_kind;

/* Which y-degree decides whether y is heavy (two-path).  MAX: y is heavy when
 * its degree in R or in S exceeds Delta1; R_ONLY: its degree in R. */
typedef enum jp_y_rule { JP_Y_RULE_MAX = 0, JP_Y_RULE_R_ONLY = 1 } jp_y_rule;

/* Duplicate-removal strategy for the light witnesses (Section 6,
 * "Deduplication": append-then-sort or a dense per-x marker vector). */
typedef enum jp_dedup {
    JP_DEDUP_AUTO = 0,     /* per-x segments: sort small ones on chip, dense bitmap for large ones */
    JP_DEDUP_GLOBAL = 1,   /* one device-wide radix sort of all witnesses, then unique */
    JP_DEDUP_SEGMENTED = 2 /* same as AUTO */
} jp_dedup;

#define JP_DELTA_INF INT64_MAX

typedef struct jp_options {
    int64_t delta1;     /* FIXED only: threshold on y degrees, >= 1 (JP_DELTA_INF allowed) */
    int64_t delta2;     /* FIXED only: threshold on x / z degrees, >= 1 (JP_DELTA_INF allowed) */
    int32_t strategy;   /* jp_strategy */
    int32_t bmm;        /* jp_bmm_kind */
    int32_t y_rule;     /* jp_y_rule */
    int32_t dedup;      /* jp_dedup */
    uint64_t seed;      /* seed of the sampled output-size estimate */
    uint64_t flags;     /* JP_FLAG_* */
} jp_options;

#define JP_FLAG_TIMING 1ull      /* record per-phase device times (HIP events) */
#define JP_FLAG_SAMPLED_OUT 2ull /* compute the sampled output-size estimate (always done for AUTO_MLP) */

/* Statistics of one evaluation.  Sizes refer to the relations after duplicate
 * removal and after dropping tuples whose y appears in only one relation. */
typedef struct jp_stats {
    int64_t n_r, n_s;            /* edges kept (two-path); star: n_r = sum over relations */
    int64_t dom_x, dom_y, dom_z; /* distinct values kept; star: dom_x, dom_z = product terms unused */
    int64_t delta1, delta2;      /* thresholds used (JP_DELTA_INF for light only) */
    int32_t strategy;            /* strategy that produced them */
    int32_t bmm;                 /* kernel used for the heavy product (jp_bmm_kind) */
    int32_t dedup;               /* jp_dedup actually used */
    int32_t arity;               /* output arity */
    int64_t u, v, w;             /* heavy x / y / z counts (star: u = rows of V, w = rows of W) */
    int64_t J;                   /* full join size (witness count) */
    int64_t J_L;                 /* light witnesses enumerated */
    int64_t J_H;                 /* heavy witnesses (covered by the product) */
    int64_t nnz_heavy;           /* nonzero entries of the heavy product */
    int64_t n_out;               /* distinct output tuples */
    double bmm_ops;              /* operations the product ran: 2*u*v*w (star: 2*u1*u2*v*u3); a self-join
                                    product on the tiles on and above the diagonal counts only those */
    double ms_ingest;            /* index build: dedup, semijoin, ranks, CSR, degrees */
    double ms_plan;              /* threshold choice + partition */
    double ms_light;             /* light witness enumeration */
    double ms_heavy;             /* heavy matrix build + product */
    double ms_bmm;               /* the product kernel alone */
    double ms_dedup;             /* duplicate removal, union, output */
    double ms_total;             /* whole call, device time */
    double ms_kernel_dedup;      /* per-x duplicate-removal kernel alone (segmented strategy) */
    double dedup_alg_bytes;      /* its algorithmic HBM bytes: 4 per witness read + 4 per distinct pair key written */
    int64_t dedup_units;         /* on-chip units it processed */
    double out_est;              /* Section 5 output-size estimate */
    double out_sampled;          /* sampled estimate (0 when not computed): with k = sample_draws x ranks drawn
                                    as splitmix64(seed + i) mod dom_x, i < k, and D = sample_distinct the sum of
                                    the distinct z each reaches, D * dom_x / k */
    int64_t sample_draws, sample_distinct;
} jp_stats;

typedef struct jp_handle jp_handle;
typedef struct jp_result jp_result;

/*
 * Device constants of the cost-based optimizer (Section 5, Table "Symbol
 * definitions" and Algorithm 2), measured for this library on one GPU.
 */
typedef struct jp_calibration {
    double t_witness;  /* T_I: seconds per light witness (gather + duplicate removal) */
    double t_seq;      /* T_s: seconds per sequential element of a per-x dense marker pass */
    double t_byte;     /* T_m / 32: seconds per byte of heavy matrix allocated and filled */
    double t_x;        /* T_m per x value: fixed per-x cost of the light path */
    double eps;        /* search step: Delta1 <- (1 - eps) Delta1 */
    int32_t literal;   /* 1: start at Delta1 = N and stop when the cost does not decrease */
    int32_t n_mm;      /* entries of the product time table */
    double mm_p[24];   /* table of M-hat(p, p, p): cube sizes p ... */
    double mm_s[24];   /* ... and measured seconds */
    int32_t light_once; /* 1: each light witness is priced once: T_I (sum(y_D1) + sum(x_D2) (1 - sum(y_D1) / J)),
                           the witnesses of light x at light y taken out of sum(x_D2) under independent
                           x and y degree classes, and a plan without a product priced at J witnesses;
                           0: T_I (sum(y_D1) + sum(x_D2)) as printed */
    int32_t k_pad;      /* > 1: the product's inner dimension v is priced padded to a multiple of k_pad (the
                           matrices are u x v_pad and w x v_pad and the product runs over v_pad); 0 or 1: v */
} jp_calibration;

/* Sorted degree vector with per-degree count and summed work: the indexes of
 * Section 5 ("sum", "cdfx", "count"), queried by binary search.  Host arrays. */
typedef struct jp_degree_index {
    int64_t n;            /* distinct degrees */
    const int64_t *deg;   /* ascending */
    const int64_t *count; /* values with that degree */
    const double *sum;    /* summed work of those values (may be NULL for count-only indexes) */
} jp_degree_index;

/* Inputs of the two-path threshold choice. */
typedef struct jp_two_path_summary {
    int64_t n_r, n_s, dom_x, dom_y, dom_z, J;
    double out_est;
    jp_degree_index y;    /* key degree of y (y rule); sum = deg_R(y) * deg_S(y) */
    jp_degree_index x;    /* deg_R(x); sum = witnesses of x = sum over y in N(x) of deg_S(y) */
    jp_degree_index xcdf; /* per x, the smallest key degree among its y (count only): cdfx */
    jp_degree_index z;    /* deg_S(z) (count only) */
} jp_two_path_summary;

/* Create a handle bound to HIP device `device`.  *h receives the handle. */
jp_status jp_create(jp_handle **h, int device);

/* Destroy a handle and release its cached device memory.  NULL is a no-op.
 * Results created by the handle stay valid until freed. */
void jp_destroy(jp_handle *h);

/* Order all later device work of this handle on `stream` (a hipStream_t; NULL
 * means the default stream). */
jp_status jp_set_stream(jp_handle *h, void *stream);

/*
 * Source of the handle's device memory.  Every device buffer a later call of
 * this handle needs (working buffers and result columns) is requested with
 * alloc_fn(bytes, user) and returned with free_fn(ptr, user); the library
 * keeps nothing cached from them.  alloc_fn must return memory of the
 * handle's device, aligned to 256 bytes, usable on the handle's stream, or
 * NULL when it has none: the call then fails with JP_ENOMEM after returning
 * every block it got.  A buffer is released once the work that used it has
 * been queued on the stream, so the allocator must order reuse after that
 * work (a stream-ordered caching allocator such as PyTorch's does).  Both
 * functions NULL restore the built-in caching pool (the default).  Mixing
 * NULL and non-NULL is JP_EINVAL.  The call waits for the handle's stream,
 * releases the built-in pool's cached blocks and moves the handle's own
 * buffers (selector weights) to the new source; results that are still
 * alive return their columns to the source they came from, which must stay
 * valid until they are freed.  This lets the library and the caller's
 * framework (PyTorch's caching allocator) draw on one pool of device memory.
 */
jp_status jp_set_allocator(jp_handle *h, void *(*alloc_fn)(size_t bytes, void *user),
                           void (*free_fn)(void *ptr, void *user), void *user);

/* Message describing the last non-OK status returned for this handle. */
const char *jp_last_error(const jp_handle *h);

/* Fill *opt with the defaults: AUTO_COST, AUTO kernels, MAX y rule. */
void jp_default_options(jp_options *opt);

/* Built-in calibration of the optimizer's constants. */
void jp_default_calibration(jp_calibration *cal);

/* Replace / read the calibration a handle's optimizer uses. */
jp_status jp_set_calibration(jp_handle *h, const jp_calibration *cal);
jp_status jp_get_calibration(const jp_handle *h, jp_calibration *cal);

/*
 * Algorithm 2 (Section 5) on a host summary; no GPU needed.  Writes the
 * thresholds to *delta1 / *delta2 (JP_DELTA_INF for both when the join is
 * small enough for the plain worst-case optimal join, J <= 20 N) and the
 * estimated costs of the chosen plan and of the all-light plan (seconds).
 * cal may be NULL (built-in constants).
 */
jp_status jp_plan_summary(const jp_two_path_summary *s, const jp_calibration *cal, int64_t *delta1,
                          int64_t *delta2, double *cost, double *cost_light_only);

/*
 * Lemma 3 (Section 3.1 analysis, omega = 2): the minimisers of
 * f(D1, D2) = N + N D1 + OUT D2 + N^2 / (D2 min(D1, D2)), namely
 *   OUT <= N:  D1 = OUT^(1/3),  D2 = N / OUT^(2/3);
 *   OUT >  N:  D1 = D2 = (2 N^2 / (N + OUT))^(1/3),
 * rounded down to integers and clamped to [1, N] (integer degrees make the
 * floor exact).  n = max(|R|, |S|), out = the output-size estimate.  Writes
 * JP_DELTA_INF to both when n <= 0 or out <= 0.  Host only; JP_EINVAL when a
 * pointer is NULL or out is not finite.
 */
jp_status jp_plan_theory(int64_t n, double out, int64_t *delta1, int64_t *delta2);

/*
 * Section 5 output-size estimate: the geometric mean of the lower bound
 * max(|dom x|, (J / N)^2) and the upper bound min(|dom x| |dom z|, J), the
 * lower bound first capped at the upper one.  0 when J <= 0.  Host only.
 */
double jp_estimate_out(int64_t dom_x, int64_t dom_z, int64_t J, int64_t n);

/*
 * Index and summarise a two-path instance on the GPU (the first phase of
 * jp_two_path) and return the optimizer's thresholds plus 16 features for a
 * learned selector: log N_R, log N_S, log estimated |OUT|, y-degree quantiles
 * in R and in S (p50, p90, p99, p99.9, max), x-degree p99 and max, z-degree
 * max (logs of degree + 1).  features may be NULL.
 */
jp_status jp_plan_two_path(jp_handle *h, const int32_t *r_x, const int32_t *r_y, int64_t n_r, const int32_t *s_z,
                           const int32_t *s_y, int64_t n_s, const jp_options *opt, int64_t *delta1,
                           int64_t *delta2, float *features);

/*
 * Cost-model view of given thresholds on one instance (for threshold sweeps):
 * indexes and summarises the instance like jp_plan_two_path, then writes for
 * each i < n_cells Algorithm 2's estimated seconds of (delta1[i], delta2[i])
 * (Section 5 cost terms with the handle's calibration) to est_seconds[i], and
 * the heavy dimensions u, v, w the pair would give to heavy_dims[3i .. 3i+2].
 * delta1 / delta2 are host arrays of values >= 1 (JP_DELTA_INF allowed);
 * est_seconds and heavy_dims are host arrays and may be NULL.  An instance
 * whose join is empty gives 0 everywhere.
 */
jp_status jp_plan_cells(jp_handle *h, const int32_t *r_x, const int32_t *r_y, int64_t n_r, const int32_t *s_z,
                        const int32_t *s_y, int64_t n_s, const jp_options *opt, int32_t n_cells,
                        const int64_t *delta1, const int64_t *delta2, double *est_seconds, int64_t *heavy_dims);

/*
 * The heavy part of Algorithm 2's cost (Section 5) for heavy dimensions
 * u, v, w: M-hat(u, v, w) plus the heavy matrices' bytes, in seconds, with
 * the calibration cal (NULL: the library's default).  0 when u, v or w is 0.
 * The learned selector takes a grid cell only when this is below the
 * light-only plan's estimate.  Host only; no GPU needed.
 */
double jp_heavy_cost(const jp_calibration *cal, int64_t u, int64_t v, int64_t w);

/*
 * Learned threshold selector (strategy AUTO_MLP).  It replaces Algorithm 2's
 * search (Section 5) by a fixed-size multilayer perceptron; any thresholds
 * keep the result exact (Section 3.1), so only the run time depends on it.
 *
 * Network: the 16 features of jp_plan_two_path, normalised as
 * (f - mean) / scale, then 16 -> 64 (ReLU) -> 64 (ReLU) -> n_out, fp32.
 * Output k is the predicted log run-time ratio of threshold cell k.  The
 * candidates are the light-only cell and every cell whose heavy part alone
 * (jp_heavy_cost of its u, v, w) is estimated below the light-only plan's
 * Algorithm 2 cost; the candidate with the smallest output is used.
 * Parameters are one flat fp32 array:
 * W1[64][16], b1[64], W2[64][64], b2[64], W3[n_out][64], b3[n_out]
 * (jp_mlp_param_count(n_out) floats).
 */

/* Threshold cells scored by the selector, fixed by the features: cell
 * 8 i + j (i, j < 8) has Delta1 = round(2 (Ymax / 2)^(i/7)) and
 * Delta2 = round(Xmax^(j/7)), with Ymax = max(2, largest y degree in R or S)
 * and Xmax = max(1, largest x degree) read back from features 7, 12 and 14;
 * cell 64 is light only (both JP_DELTA_INF).  Writes 65 entries to each
 * host array and returns 65 (0 if an argument is NULL). */
int32_t jp_selector_cells(const float *features, int64_t *delta1, int64_t *delta2);

/* Number of parameters of the selector network with n_out outputs. */
int64_t jp_mlp_param_count(int32_t n_out);

/* Install selector weights in the handle (host arrays, copied; n_out must be
 * 65; feat_mean / feat_scale hold 16 values, scale > 0).  params == NULL
 * removes the selector, after which AUTO_MLP behaves as AUTO_COST. */
jp_status jp_set_selector(jp_handle *h, const float *params, int32_t n_out, const float *feat_mean,
                          const float *feat_scale);

/* Forward pass for a batch: x is batch x 16 and y is batch x n_out, row-major
 * device fp32 arrays; params is the device parameter array.  1 <= n_out <= 256. */
jp_status jp_mlp_forward(jp_handle *h, const float *params, int32_t n_out, const float *x, int64_t batch, float *y);

/* Gradient of the weighted squared error
 *   L = (1/batch) sum_s [sum_k m[s,k] (y[s,k] - t[s,k])^2] / max(1, sum_k m[s,k])
 * with respect to params, for targets t (batch x n_out) and weights
 * m >= 0 (batch x n_out; 0 marks a missing label).  Device arrays; grad
 * (jp_mlp_param_count floats) and *loss (1 float) are overwritten.  The
 * per-sample terms are summed with atomics, so the last bits vary between
 * runs. */
jp_status jp_mlp_grad(jp_handle *h, const float *params, int32_t n_out, const float *x, const float *target,
                      const float *weight, int64_t batch, float *grad, float *loss);

/* One Adam step (bias-corrected, step counted from 1) on n device fp32
 * values: m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
 * p <- p - lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps). */
jp_status jp_mlp_adam(jp_handle *h, float *params, float *m, float *v, const float *grad, int64_t n, int32_t step,
                      float lr, float beta1, float beta2, float eps);

/*
 * Two-path join-project (Algorithm 1, Section 3.1).
 * R = (r_x[i], r_y[i]) for i < n_r and S = (s_z[i], s_y[i]) for i < n_s.
 * opt may be NULL (defaults).  With strategy FIXED, delta1 and delta2 must be
 * >= 1.  On JP_OK, *out holds a result of arity 2: column 0 = x, column 1 = z.
 */
jp_status jp_two_path(jp_handle *h,
                      const int32_t *r_x, const int32_t *r_y, int64_t n_r,
                      const int32_t *s_z, const int32_t *s_y, int64_t n_s,
                      const jp_options *opt, jp_result **out);

/*
 * jp_two_path without device allocation, for callers that cannot allocate
 * device memory (code that forbids hipMalloc/hipFree, tight serving loops).
 * Same inputs and options as jp_two_path; the distinct sorted pairs are
 * written to the caller's device columns out_x / out_z (capacity cap each)
 * and their count to *n_out; *stats (may be NULL) receives the statistics.
 * Working memory is a fixed 256 MiB device array inside the library, one per
 * GPU, held from the first jp_create on that GPU until the process ends; no
 * call here allocates or frees device memory.
 *  - Inputs of more than 2^19 edges per relation: JP_EINVAL.
 *  - Working memory exhausted (an input whose joins need more than the
 *    array): JP_ENOMEM; use jp_two_path.
 *  - More pairs than cap: JP_ECAPACITY with *n_out = the number needed and
 *    nothing written to out_x / out_z.
 * The array keeps the contents of the previous call; whatever must start at
 * zero is cleared by the call.  Calls on one GPU share the array: calls from
 * threads of one process are serialised by the library (each returns after
 * its device work is complete), and calls that overlap on one GPU through
 * any other route race.  The timing flag is ignored, and JP_BMM_AUTO picks
 * the product kernel by shape without the timed race.
 */
jp_status jp_two_path_static(jp_handle *h,
                             const int32_t *r_x, const int32_t *r_y, int64_t n_r,
                             const int32_t *s_z, const int32_t *s_y, int64_t n_s,
                             const jp_options *opt, int32_t *out_x, int32_t *out_z, int64_t cap,
                             int64_t *n_out, jp_stats *stats);

/*
 * Set similarity join (Section 2.1, "Set Similarity"; Section 4, the heavy
 * and light parts of SizeAware++ and the ordered variant): R(x, y) says set
 * x holds element y, S(z, y) that set z holds y; the result is every pair
 * (a, c) with |{b : (a,b) in R} & {b : (c,b) in S}| >= min_overlap, with
 * that overlap.  Evaluated by Algorithm 1 with counts kept: the light
 * witnesses are counted per pair after one sort, the heavy part adds the
 * product's exact int32 counts C[a][c] (light and heavy witnesses partition
 * the join, so the sum is the overlap).  min_overlap = 1 gives the two-path
 * result.  Options as for jp_two_path (the dedup field is ignored).
 * On JP_OK *out holds a result of arity 3: column 0 = x, column 1 = z,
 * column 2 = overlap (int32).  order 0: pairs ascending by (x, z); order 1
 * (ordered SSJ): by overlap descending, ties by (x, z) ascending.
 * JP_EINVAL for min_overlap < 1 or an order other than 0 and 1.
 */
jp_status jp_ssj(jp_handle *h,
                 const int32_t *r_x, const int32_t *r_y, int64_t n_r,
                 const int32_t *s_z, const int32_t *s_y, int64_t n_s,
                 int64_t min_overlap, int32_t order, const jp_options *opt, jp_result **out);

/*
 * Batched Boolean set intersection (Section 2.1, "Boolean Set Intersection";
 * Section 3.3): R(x, y) says set x holds element y, S(z, y) likewise; the
 * batch holds n_t queries (t_x[i], t_z[i]), device int32 columns.  For every
 * i, answers[i] (device, n_t bytes, caller-owned) becomes 1 when the sets
 * {b : (t_x[i], b) in R} and {b : (t_z[i], b) in S} intersect, else 0.  As
 * in the paper's experiments, the batch filters R to the queried x and S to
 * the queried z, the filtered two-path query runs through Algorithm 1 with
 * the given options, and each query is answered from its sorted output.
 * Queries may repeat and may name ids absent from the relations (answer 0).
 * *stats (may be NULL) receives the statistics of the filtered two-path
 * evaluation.  The call returns after the answers are written.
 */
jp_status jp_bsi(jp_handle *h,
                 const int32_t *r_x, const int32_t *r_y, int64_t n_r,
                 const int32_t *s_z, const int32_t *s_y, int64_t n_s,
                 const int32_t *t_x, const int32_t *t_z, int64_t n_t,
                 const jp_options *opt, uint8_t *answers, jp_stats *stats);

/* One two-path instance of a batch: device columns as for jp_two_path. */
typedef struct jp_instance {
    const int32_t *r_x, *r_y;
    int64_t n_r;
    const int32_t *s_z, *s_y;
    int64_t n_s;
} jp_instance;

/*
 * Many independent two-path instances in one evaluation (Algorithm 1 run
 * once over all of them).  inst is a host array of n_inst descriptors
 * (0 <= n_inst <= 65535).  The instances are laid side by side in disjoint id ranges,
 * which keeps each instance's output exact (no y is shared between
 * instances), and share one threshold pair chosen by opt for the combined
 * input.  The sum over instances of (max id - min id + 1) must stay below
 * 2^31 for each of x, y and z (JP_EINVAL otherwise).  On JP_OK, *out holds
 * one arity-2 result with all instances' tuples, instance by instance, each
 * instance's tuples distinct and sorted as in jp_two_path; the slice of
 * instance i is given by jp_result_batch_offsets.
 */
jp_status jp_two_path_batch(jp_handle *h, int32_t n_inst, const jp_instance *inst, const jp_options *opt,
                            jp_result **out);

/*
 * A reusable, graph-captured evaluation of a batch of two-path instances
 * (the serving form of jp_two_path_batch).  Making the plan runs the batch
 * once, recording every value the pipeline reads back from the device and
 * its peak working memory, then runs it again under HIP stream capture with
 * every working buffer carved from one device arena, which gives one HIP
 * graph of the whole evaluation (no host waits, no allocation, no host
 * decisions inside it).  jp_plan_launch replays the graph on the handle's
 * stream.
 *  - arena: device memory of arena_bytes (256-byte aligned) owned by the
 *    caller and used by the plan until jp_plan_free, or NULL: the plan takes
 *    arena_bytes from the handle's allocator.
 *  - JP_ECAPACITY: arena_bytes is too small for this batch; *arena_needed
 *    receives a size that suffices (make the plan again with it).  On JP_OK
 *    *arena_needed receives the size the plan needed.
 *  - The plan keeps the instance descriptors: the graph reads the same
 *    device columns at every launch.  Its host decisions (thresholds, grid
 *    and buffer sizes) are those of the recorded run, so a launch is valid
 *    only for the contents the plan was made on: jp_plan_launch first
 *    fingerprints the columns on the device and returns JP_ECAPACITY without
 *    replaying when they changed (make a new plan); inside the graph every
 *    recorded read-back is compared with the live value and a difference
 *    raises a device flag (JP_EINTERNAL after the replay).
 * Options as for jp_two_path_batch; the timing flag is ignored.
 */
typedef struct jp_plan jp_plan;
jp_status jp_two_path_batch_plan(jp_handle *h, int32_t n_inst, const jp_instance *inst, const jp_options *opt,
                                 void *arena, int64_t arena_bytes, jp_plan **plan, int64_t *arena_needed);

/* Replay the plan's graph on the handle's stream and wait for it.  The
 * handle must be on the plan's device.  JP_ECAPACITY: the inputs changed
 * since the plan was made (nothing replayed). */
jp_status jp_plan_launch(jp_handle *h, jp_plan *plan);

/* The plan's output after a launch: cols receives 2 device column pointers
 * (x, z; valid until the next launch or jp_plan_free), *n_tuples their
 * length, offsets (n_inst + 1 host values, may be NULL) the instance slices
 * as in jp_result_batch_offsets.  Any argument but plan may be NULL. */
jp_status jp_plan_result(const jp_plan *plan, const int32_t **cols, int64_t *n_tuples, int64_t *offsets);

/* Copy the plan's output into caller-allocated device columns (2 pointers,
 * each with room for n_tuples int32), ordered on the handle's stream. */
jp_status jp_plan_copy(jp_handle *h, const jp_plan *plan, int32_t *const *cols);

/* Release a plan (its graph, stream and device buffers).  NULL is a no-op. */
void jp_plan_free(jp_plan *plan);

/* Slices of a batched result: *n_inst receives the instance count; when
 * offsets is not NULL it receives n_inst + 1 host values, instance i owning
 * tuples [offsets[i], offsets[i+1]).  A result that is not batched reports
 * n_inst = 0. */
jp_status jp_result_batch_offsets(const jp_result *r, int32_t *n_inst, int64_t *offsets);

/*
 * Star join-project Q*_k (Section 3.2), 2 <= k <= 8.  Relation i has columns
 * x[i], y[i] of n[i] rows (host arrays of device pointers).  On JP_OK, *out
 * holds a result of arity k; column i holds x_i.  k = 2 is jp_two_path.  The
 * heavy part is the product V x W^T of Section 3.2, V over the first
 * ceil(k/2) relations and W over the rest.  Thresholds: FIXED, LIGHT_ONLY,
 * or (any other strategy) Section 3.2's balance of the light, output and
 * product costs with |OUT| estimated by J, light only when J <= 20 N.
 * JP_EINVAL when k is out of range or the k dense rank widths of the output
 * exceed 128 bits; JP_ENOMEM when the join has 2^40 or more witnesses.
 */
jp_status jp_star(jp_handle *h, int k,
                  const int32_t *const *x, const int32_t *const *y, const int64_t *n,
                  const jp_options *opt, jp_result **out);

/* Number of tuples and arity of a result. */
jp_status jp_result_size(const jp_result *r, int64_t *n_tuples, int32_t *arity);

/* Borrow the result's device columns: cols[i] receives column i (arity
 * entries).  Valid until jp_result_free. */
jp_status jp_result_columns(const jp_result *r, const int32_t **cols);

/* Copy the result into caller-allocated device columns (arity pointers, each
 * with room for n_tuples int32), ordered on the handle's stream. */
jp_status jp_result_copy(jp_handle *h, const jp_result *r, int32_t *const *cols);

/* Statistics of the evaluation that produced r. */
jp_status jp_result_stats(const jp_result *r, jp_stats *s);

/* Release a result.  NULL is a no-op. */
void jp_result_free(jp_result *r);

/*
 * Product kernel choice by shape (the project's autotuner, autotune.py,
 * writes the table).  JP_BMM_AUTO keeps one kernel per shape class, the
 * log2 buckets of (u, w, ld) given by jp_product_shape_class; a class
 * without an entry is raced once on the handle (its int8 kernel against the
 * popcount kernel, timed) and the faster kept.  jp_set_product_table enters
 * n classes with their kernel (JP_BMM_I8_T128, JP_BMM_I8_T256 or
 * JP_BMM_BITPOP; host arrays, copied), so that no race is needed for them.
 */
uint64_t jp_product_shape_class(int64_t u, int64_t w, int64_t ld);
jp_status jp_set_product_table(jp_handle *h, int32_t n, const uint64_t *classes, const int32_t *kinds);

/*
 * Heavy-product kernel on its own (the heavy step of Algorithm 1; Section 2.2's
 * Boolean matrix product): A is u x k and Bt is w x k, both 0/1 int8
 * row-major device matrices with row stride `ld` bytes (ld >= k, ld a
 * multiple of 128, padding bytes zero).  For every (i, j) with
 * sum_t A[i][t] * Bt[j][t] > 0 the pair (i, j) is written to rows[] / cols[]
 * (device int32 arrays of capacity `cap`), in no particular order, and the
 * count to *nnz.  If the count exceeds cap, JP_ECAPACITY is returned with
 * *nnz = the needed count (only cap pairs written).  `kind` selects the
 * kernel (jp_bmm_kind).  *ms receives the product kernel's device time.
 */
jp_status jp_bool_matmul(jp_handle *h, const int8_t *A, const int8_t *Bt,
                         int64_t u, int64_t w, int64_t k, int64_t ld, int32_t kind,
                         int32_t *rows, int32_t *cols, int64_t cap, int64_t *nnz, double *ms);

#ifdef __cplusplus
}
#endif
#endif /* JP_H */
