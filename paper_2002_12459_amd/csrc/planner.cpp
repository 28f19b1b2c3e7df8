// Threshold choice for the two-path method (host).
//
//  FIXED       the caller's (Delta1, Delta2).
//  LIGHT_ONLY  no heavy part.
//  THEORY      Lemma 3's minimisers of the omega = 2 cost
//                f(D1,D2) = N + N D1 + OUT D2 + N^2 / (D2 min(D1,D2)):
//                OUT <= N:  D1 = OUT^(1/3),  D2 = N / OUT^(2/3)
//                OUT >  N:  D1 = D2 = (2 N^2 / (N + OUT))^(1/3)
//              with OUT the Section 5 estimate; rounded down to integers and
//              clamped to [1, N].
//  AUTO_COST   Algorithm 2 (Section 5) on the degree indexes of the instance
//              with this device's measured constants.
//  AUTO_MLP    learned selector (mlp.hip); Algorithm 2 when the handle has none.
#include <algorithm>
#include <cmath>

#include "pipeline.hpp"

namespace jp {

// Section 5: the output lies between max(|dom x|, (J/N)^2) and
// min(|dom x| |dom z|, J); the estimate is the geometric mean of the two.
double estimate_out(int64_t dom_x, int64_t dom_z, int64_t J, int64_t N) {
    if (J <= 0) return 0.0;
    double r = (double)J / (double)std::max<int64_t>(N, 1);
    double lo = std::max((double)dom_x, r * r);
    double hi = std::min((double)dom_x * (double)dom_z, (double)J);
    lo = std::min(lo, hi);
    return std::sqrt(lo * hi);
}

static int64_t clamp_delta(double t, int64_t N) {
    if (!(t >= 1.0)) return 1;
    if (t >= (double)N) return std::max<int64_t>(N, 1);
    return (int64_t)std::floor(t);
}

Thresholds theory_thresholds(int64_t N, double out) {
    Thresholds th;
    th.strategy = JP_STRATEGY_THEORY;
    if (N <= 0 || out <= 0) return th;  // light only
    double d1, d2;
    if (out <= (double)N) {
        d1 = std::cbrt(out);
        d2 = (double)N / (d1 * d1);
    } else {
        d1 = d2 = std::cbrt(2.0 * (double)N * (double)N / ((double)N + out));
    }
    th.d1 = clamp_delta(d1, N);
    th.d2 = clamp_delta(d2, N);
    return th;
}

void default_calibration(jp_calibration *c) {
    std::memset(c, 0, sizeof(*c));
    // measured on MI355X with this library (paper_2002_12459_amd.calibrate):
    // light witness cost, per-x index cost, heavy-matrix bytes, and the int8
    // product on p x p x p operands; replaced at run time by jp_set_calibration
    c->t_witness = 1.3522e-11;
    c->t_seq = 0.0;
    c->t_byte = 3.0775e-13;
    c->t_x = 1.7849e-09;
    c->eps = 0.05;
    c->literal = 0;
    c->light_once = 1;
    c->k_pad = 128;  // the heavy matrices' stride and the product's K stage
    const double p[] = {1024, 2048, 4096, 8192, 12288, 16384, 20480};
    const double s[] = {3.4316e-05, 4.8074e-05, 7.7510e-05, 4.8934e-04, 1.5718e-03, 3.8439e-03, 7.8472e-03};
    c->n_mm = (int32_t)(sizeof(p) / sizeof(p[0]));
    for (int i = 0; i < c->n_mm; ++i) {
        c->mm_p[i] = p[i];
        c->mm_s[i] = s[i];
    }
}

namespace {

// Section 5 index: sorted degree vector, prefix counts and sums.
struct Index {
    const int64_t *deg = nullptr;
    int64_t n = 0;
    std::vector<int64_t> ccnt;  // ccnt[i] = values with degree <= deg[i-1]
    std::vector<double> csum;
    explicit Index(const jp_degree_index &d) : deg(d.deg), n(d.n), ccnt(d.n + 1, 0), csum(d.n + 1, 0.0) {
        for (int64_t i = 0; i < n; ++i) {
            ccnt[i + 1] = ccnt[i] + d.count[i];
            csum[i + 1] = csum[i] + (d.sum ? d.sum[i] : 0.0);
        }
    }
    int64_t pos(int64_t delta) const {  // number of entries with degree <= delta
        return std::upper_bound(deg, deg + n, delta) - deg;
    }
    int64_t count_le(int64_t delta) const { return ccnt[pos(delta)]; }
    double sum_le(int64_t delta) const { return csum[pos(delta)]; }
    int64_t total() const { return ccnt[n]; }
    int64_t max_deg() const { return n ? deg[n - 1] : 0; }
};

// M-hat(u, v, w): time of the nearest measured cube, scaled by u v w / p^3;
// below the smallest cube, that cube's time (a product launch costs at least
// what the smallest measured one does: its tiles do not fill the GPU).
double mm_hat(const jp_calibration &c, double u, double v, double w) {
    if (u <= 0 || v <= 0 || w <= 0 || c.n_mm <= 0) return 0.0;
    const double p = std::cbrt(u * v * w);
    int best = 0, small = 0;
    for (int i = 1; i < c.n_mm; ++i) {
        if (std::fabs(c.mm_p[i] - p) < std::fabs(c.mm_p[best] - p)) best = i;
        if (c.mm_p[i] < c.mm_p[small]) small = i;
    }
    if (p <= c.mm_p[small]) return c.mm_s[small];
    const double pb = c.mm_p[best];
    return c.mm_s[best] * (u * v * w) / (pb * pb * pb);
}

}  // namespace

double heavy_cost(const jp_calibration &c, int64_t u, int64_t v, int64_t w) {
    if (u <= 0 || v <= 0 || w <= 0) return 0.0;
    const double vp = c.k_pad > 1 ? (double)((v + c.k_pad - 1) / c.k_pad * c.k_pad) : (double)v;
    return mm_hat(c, (double)u, vp, (double)w) + c.t_byte * ((double)u * vp + (double)w * vp);
}

namespace {

// Algorithm 2's cost of a threshold pair on one instance's indexes.
struct CostModel {
    const jp_two_path_summary &s;
    const jp_calibration &c;
    Index Y, X, XC, Z;
    CostModel(const jp_two_path_summary &s_, const jp_calibration &c_)
        : s(s_), c(c_), Y(s_.y), X(s_.x), XC(s_.xcdf), Z(s_.z) {}
    double operator()(int64_t d1, int64_t d2, int64_t *uvw = nullptr) const {
        const int64_t u = s.dom_x - X.count_le(d2), v = s.dom_y - Y.count_le(d1), w = s.dom_z - Z.count_le(d2);
        // light: T_I sum(y_D1) + T_I sum(x_D2) + T_m |dom x| + T_s cdfx(y_D1) |dom x|; with
        // light_once the witnesses of light x at light y (already in sum(y_D1)) are taken
        // out of sum(x_D2), estimated as sum(x_D2) sum(y_D1) / J, and a plan without a
        // product leaves all J witnesses to the light side
        const double sy = Y.sum_le(d1), sx = X.sum_le(d2);
        double wit = sy + sx;
        if (c.light_once && s.J > 0)
            wit = (u > 0 && v > 0 && w > 0) ? sy + sx * std::max(0.0, 1.0 - sy / (double)s.J) : (double)s.J;
        const double light = c.t_witness * wit + c.t_x * (double)s.dom_x +
                             c.t_seq * (double)XC.count_le(d1) * (double)s.dom_x;
        // heavy: M-hat(u, v, w) + allocation of the heavy matrices
        if (uvw) {
            uvw[0] = u;
            uvw[1] = v;
            uvw[2] = w;
        }
        return light + heavy_cost(c, u, v, w);
    }
};

}  // namespace

double plan_cost(const jp_two_path_summary &s, const jp_calibration &c, int64_t d1, int64_t d2, int64_t *uvw) {
    return CostModel(s, c)(d1, d2, uvw);
}

void plan_costs(const jp_two_path_summary &s, const jp_calibration &c, int n, const int64_t *d1, const int64_t *d2,
                double *cost, int64_t *uvw) {
    const CostModel cm(s, c);  // the indexes' prefix tables, built once for all pairs
    for (int i = 0; i < n; ++i) {
        int64_t t[3] = {0, 0, 0};
        const double v = cm(d1[i], d2[i], t);
        if (cost) cost[i] = v;
        if (uvw)
            for (int j = 0; j < 3; ++j) uvw[3 * i + j] = t[j];
    }
}

PlanResult algorithm2(const jp_two_path_summary &s, const jp_calibration &c) {
    PlanResult r;
    const int64_t N = std::max(s.n_r, s.n_s);
    const double out = std::max(s.out_est, 1.0);
    const CostModel cm(s, c);
    const Index &Y = cm.Y;
    auto cost = [&](int64_t d1, int64_t d2) { return cm(d1, d2); };
    r.cost_light_only = cost(JP_DELTA_INF, JP_DELTA_INF);
    if ((double)s.J <= 20.0 * (double)N || N <= 0) {  // small join: plain worst-case optimal join
        r.d1 = r.d2 = JP_DELTA_INF;
        r.cost = r.cost_light_only;
        return r;
    }
    const double eps = c.literal ? 0.95 : (c.eps > 0 && c.eps < 1 ? c.eps : 0.05);
    auto delta2_of = [&](int64_t d1) { return clamp_delta((double)N * (double)d1 / out, N); };
    // Start: literal reading Delta1 = N; otherwise the largest key degree (any
    // larger Delta1 gives the same, all-light partition).
    int64_t d1 = c.literal ? std::max<int64_t>(N, 1) : std::max<int64_t>(Y.max_deg(), 1);
    int64_t d2 = delta2_of(d1);
    double prev = cost(d1, d2);
    for (int it = 0; it < 10000; ++it) {
        int64_t nd1 = (int64_t)std::floor((1.0 - eps) * (double)d1);
        if (nd1 >= d1) nd1 = d1 - 1;
        if (nd1 < 1) break;
        const int64_t nd2 = delta2_of(nd1);
        const double cnow = cost(nd1, nd2);
        const bool stop = c.literal ? (prev <= cnow) : (prev < cnow);
        if (stop) break;
        prev = cnow;
        d1 = nd1;
        d2 = nd2;
    }
    r.d1 = d1;
    r.d2 = d2;
    r.cost = prev;
    if (!(r.cost < r.cost_light_only)) {  // nothing beats the plain join
        r.d1 = r.d2 = JP_DELTA_INF;
        r.cost = r.cost_light_only;
    }
    return r;
}

Thresholds choose_thresholds(const TwoPathSummary &s, const jp_options &o, const jp_calibration &cal) {
    const int64_t N = std::max(s.n_r, s.n_s);
    Thresholds th;
    switch (o.strategy) {
        case JP_STRATEGY_FIXED:
            th.d1 = o.delta1;
            th.d2 = o.delta2;
            th.strategy = JP_STRATEGY_FIXED;
            return th;
        case JP_STRATEGY_LIGHT_ONLY:
            th.strategy = JP_STRATEGY_LIGHT_ONLY;
            return th;
        case JP_STRATEGY_THEORY:
            return theory_thresholds(N, s.out_est);
        default:
            break;
    }
    const jp_two_path_summary cs = s.view();
    const PlanResult r = algorithm2(cs, cal);
    th.d1 = r.d1;
    th.d2 = r.d2;
    th.strategy = JP_STRATEGY_AUTO_COST;
    return th;
}

// Learned-selector features (see jp_plan_two_path).
static double quantile(const jp_degree_index &d, double q) {
    int64_t tot = 0;
    for (int64_t i = 0; i < d.n; ++i) tot += d.count[i];
    if (tot == 0) return 0.0;
    const double want = q * (double)tot;
    int64_t run = 0;
    for (int64_t i = 0; i < d.n; ++i) {
        run += d.count[i];
        if ((double)run >= want) return (double)d.deg[i];
    }
    return (double)d.deg[d.n - 1];
}

void features16(const TwoPathSummary &s, float *f) {
    const jp_two_path_summary v = s.view();
    const jp_degree_index yr = s.yr.view(), ys = s.ys.view();
    f[0] = (float)std::log((double)std::max<int64_t>(s.n_r, 1));
    f[1] = (float)std::log((double)std::max<int64_t>(s.n_s, 1));
    f[2] = (float)std::log(1.0 + (s.out_sampled > 0 ? s.out_sampled : s.out_est));
    const double qs[5] = {0.5, 0.9, 0.99, 0.999, 1.0};
    for (int i = 0; i < 5; ++i) {
        f[3 + i] = (float)std::log(1.0 + quantile(yr, qs[i]));
        f[8 + i] = (float)std::log(1.0 + quantile(ys, qs[i]));
    }
    f[13] = (float)std::log(1.0 + quantile(v.x, 0.99));
    f[14] = (float)std::log(1.0 + quantile(v.x, 1.0));
    f[15] = (float)std::log(1.0 + quantile(v.z, 1.0));
}

}  // namespace jp
