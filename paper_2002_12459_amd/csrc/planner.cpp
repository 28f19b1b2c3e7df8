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
//  AUTO_COST   Algorithm 2 (Section 5) with device-calibrated constants.
//  AUTO_MLP    learned selector; without loaded weights, AUTO_COST.
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
        d2 = (double)N / std::pow(out, 2.0 / 3.0);
    } else {
        d1 = d2 = std::cbrt(2.0 * (double)N * (double)N / ((double)N + out));
    }
    th.d1 = clamp_delta(d1, N);
    th.d2 = clamp_delta(d2, N);
    return th;
}

Thresholds choose_thresholds(const TwoPathSummary &s, const jp_options &o) {
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
    // AUTO_COST / AUTO_MLP
    th = theory_thresholds(N, s.out_est);
    th.strategy = JP_STRATEGY_AUTO_COST;
    if ((double)s.J <= 20.0 * (double)N) {  // Algorithm 2: small join, plain join only
        th.d1 = th.d2 = JP_DELTA_INF;
    }
    return th;
}

}  // namespace jp
