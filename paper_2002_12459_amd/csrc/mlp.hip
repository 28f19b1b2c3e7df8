// Learned threshold selector: a 16 -> 64 -> 64 -> K multilayer perceptron in
// fp32 with ReLU hidden layers.  It maps 16 features of an instance (sizes,
// output estimate, degree quantiles) to a predicted log run time for each of
// K threshold cells; the cell with the smallest prediction is used.  The
// output stays exact whatever cell is picked (the correctness argument of
// Section 3.1 holds for any thresholds).
//
// Parameters are one flat fp32 array: W1 [64][16], b1 [64], W2 [64][64],
// b2 [64], W3 [K][64], b3 [K].
//
// Kernels: forward (one workgroup of 64 threads per sample), loss gradient of
// the masked mean squared error (per-sample gradients reduced with atomics),
// and Adam.
#include <algorithm>
#include <cmath>

#include "pipeline.hpp"
#include "prims.hpp"

namespace jp {

constexpr int kIn = 16, kH = 64;

int64_t mlp_param_count(int n_out) { return (int64_t)kH * kIn + kH + kH * kH + kH + (int64_t)n_out * kH + n_out; }

namespace {

struct MlpView {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
    __host__ __device__ MlpView(const float *p, int K)
        : W1(p), b1(p + kH * kIn), W2(b1 + kH), b2(W2 + kH * kH), W3(b2 + kH), b3(W3 + (int64_t)K * kH) {}
};

// One sample per workgroup: thread j computes hidden unit j of both layers,
// then threads compute the K outputs.
__global__ __launch_bounds__(kH) void k_mlp_fwd(const float *params, int K, const float *x, int64_t batch,
                                               float *y) {
    __shared__ float in[kIn], h1[kH], h2[kH];
    const int64_t s = blockIdx.x;
    const int j = threadIdx.x;
    const MlpView p(params, K);
    if (j < kIn) in[j] = x[s * kIn + j];
    __syncthreads();
    float a = p.b1[j];
    for (int i = 0; i < kIn; ++i) a += p.W1[j * kIn + i] * in[i];
    h1[j] = a > 0.f ? a : 0.f;
    __syncthreads();
    a = p.b2[j];
    for (int i = 0; i < kH; ++i) a += p.W2[j * kH + i] * h1[i];
    h2[j] = a > 0.f ? a : 0.f;
    __syncthreads();
    for (int k = j; k < K; k += kH) {
        float o = p.b3[k];
        for (int i = 0; i < kH; ++i) o += p.W3[k * kH + i] * h2[i];
        y[s * K + k] = o;
    }
}

// Gradient of the weighted mean squared error
//   L = (1/B) sum_s [ sum_k m[s,k] (y[s,k] - t[s,k])^2 ] / max(1, sum_k m[s,k])
// with m >= 0 the per-target weights (0 = no label).  Each workgroup
// back-propagates one sample and adds its share into grad with atomics.
__global__ __launch_bounds__(kH) void k_mlp_grad(const float *params, int K, const float *x, const float *target,
                                                const float *mask, int64_t batch, float *grad, float *loss) {
    __shared__ float in[kIn], z1[kH], h1[kH], z2[kH], h2[kH], g2[kH], g1[kH];
    __shared__ float dy[256];
    __shared__ float red[kH];
    const int64_t s = blockIdx.x;
    const int j = threadIdx.x;
    const MlpView p(params, K);
    const int64_t P1 = 0, Pb1 = kH * kIn, P2 = Pb1 + kH, Pb2 = P2 + kH * kH, P3 = Pb2 + kH,
                  Pb3 = P3 + (int64_t)K * kH;
    if (j < kIn) in[j] = x[s * kIn + j];
    __syncthreads();
    float a = p.b1[j];
    for (int i = 0; i < kIn; ++i) a += p.W1[j * kIn + i] * in[i];
    z1[j] = a;
    h1[j] = a > 0.f ? a : 0.f;
    __syncthreads();
    a = p.b2[j];
    for (int i = 0; i < kH; ++i) a += p.W2[j * kH + i] * h1[i];
    z2[j] = a;
    h2[j] = a > 0.f ? a : 0.f;
    __syncthreads();
    // per-sample normalisation by the number of valid targets
    float mcount = 0.f;
    for (int k = j; k < K; k += kH) mcount += mask[s * K + k];
    red[j] = mcount;
    __syncthreads();
    if (j == 0) {
        float t = 0.f;
        for (int i = 0; i < kH; ++i) t += red[i];
        red[0] = t > 1.f ? t : 1.f;
    }
    __syncthreads();
    const float norm = 1.f / (red[0] * (float)batch);
    __syncthreads();
    float lsum = 0.f;
    for (int k = j; k < K; k += kH) {
        float o = p.b3[k];
        for (int i = 0; i < kH; ++i) o += p.W3[k * kH + i] * h2[i];
        const float m = mask[s * K + k];
        const float e = o - target[s * K + k];
        lsum += m * e * e * norm;
        dy[k] = 2.f * m * e * norm;
        atomicAdd(&grad[Pb3 + k], dy[k]);
    }
    red[j] = lsum;
    __syncthreads();
    if (j == 0) {
        float t = 0.f;
        for (int i = 0; i < kH; ++i) t += red[i];
        atomicAdd(loss, t);
    }
    // layer 3: dW3[k][i] = dy[k] h2[i]; dh2[i] = sum_k dy[k] W3[k][i]
    float dh2 = 0.f;
    for (int k = 0; k < K; ++k) {
        atomicAdd(&grad[P3 + (int64_t)k * kH + j], dy[k] * h2[j]);
        dh2 += dy[k] * p.W3[k * kH + j];
    }
    g2[j] = z2[j] > 0.f ? dh2 : 0.f;
    __syncthreads();
    atomicAdd(&grad[Pb2 + j], g2[j]);
    float dh1 = 0.f;
    for (int k = 0; k < kH; ++k) {
        atomicAdd(&grad[P2 + k * kH + j], g2[k] * h1[j]);
        dh1 += g2[k] * p.W2[k * kH + j];
    }
    g1[j] = z1[j] > 0.f ? dh1 : 0.f;
    __syncthreads();
    atomicAdd(&grad[Pb1 + j], g1[j]);
    for (int i = 0; i < kIn; ++i) atomicAdd(&grad[P1 + j * kIn + i], g1[j] * in[i]);
}

__global__ __launch_bounds__(256) void k_adam(float *params, float *m, float *v, const float *grad, int64_t n,
                                              float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    params[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

void mlp_forward(const Ctx &c, const float *params, int K, const float *x, int64_t batch, float *y) {
    JP_CHECK(K >= 1 && K <= 256, JP_EINVAL, "selector outputs must be in [1, 256]");
    if (batch <= 0) return;
    hipLaunchKernelGGL(k_mlp_fwd, dim3(grid_x(batch, kH)), dim3(kH), 0, c.stream, params, K, x, batch, y);
    JP_HIP(hipGetLastError());
}

void mlp_grad(const Ctx &c, const float *params, int K, const float *x, const float *target, const float *mask,
              int64_t batch, float *grad, float *loss) {
    JP_CHECK(K >= 1 && K <= 256, JP_EINVAL, "selector outputs must be in [1, 256]");
    c.zero(grad, (size_t)mlp_param_count(K));
    c.zero(loss, 1);
    if (batch <= 0) return;
    hipLaunchKernelGGL(k_mlp_grad, dim3(grid_x(batch, kH)), dim3(kH), 0, c.stream, params, K, x, target, mask, batch,
                       grad, loss);
    JP_HIP(hipGetLastError());
}

void mlp_adam(const Ctx &c, float *params, float *m, float *v, const float *grad, int64_t n, int step, float lr,
              float b1, float b2, float eps) {
    if (n <= 0) return;
    JP_CHECK(step >= 1, JP_EINVAL, "Adam step counts from 1");
    const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(grid_x(ceil_div(n, 256), 256)), dim3(256), 0, c.stream, params, m, v, grad, n, lr,
                       b1, b2, eps, c1, c2);
    JP_HIP(hipGetLastError());
}

// Threshold cells of the selector: Delta1 on 8 geometric points from 2 to the
// largest y degree, Delta2 on 8 geometric points from 1 to the largest x
// degree, and a light-only cell (index 64).  Features 7 / 12 hold
// log(1 + max y degree) in R / S and feature 14 log(1 + max x degree).
void selector_cells(const float *f, int64_t *d1, int64_t *d2) {
    const double maxy = std::max(std::exp((double)f[7]), std::exp((double)f[12])) - 1.0;
    const double maxx = std::exp((double)f[14]) - 1.0;
    const double ylo = 2.0, yhi = std::max(maxy, 2.0), xlo = 1.0, xhi = std::max(maxx, 1.0);
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) {
            const double a = ylo * std::pow(yhi / ylo, i / 7.0);
            const double b = xlo * std::pow(xhi / xlo, j / 7.0);
            d1[i * 8 + j] = std::max<int64_t>(1, (int64_t)std::llround(a));
            d2[i * 8 + j] = std::max<int64_t>(1, (int64_t)std::llround(b));
        }
    d1[64] = d2[64] = JP_DELTA_INF;
}

Thresholds select_thresholds(const Ctx &c, const TwoPathSummary &s, const jp_options &o) {
    jp_calibration cal_default;
    if (!c.cal) default_calibration(&cal_default);
    const jp_calibration &cal = c.cal ? *c.cal : cal_default;
    if (o.strategy != JP_STRATEGY_AUTO_MLP || !c.sel || !c.sel->ready()) {
        jp_options oo = o;
        if (oo.strategy == JP_STRATEGY_AUTO_MLP) oo.strategy = JP_STRATEGY_AUTO_COST;
        return choose_thresholds(s, oo, cal);
    }
    const Selector &sel = *c.sel;
    float f[kFeatures], in[kFeatures];
    features16(s, f);
    for (int i = 0; i < kFeatures; ++i) in[i] = (f[i] - sel.mean[i]) / sel.scale[i];
    DBuf<float> io = c.buf<float>(kFeatures + kSelectorCells);
    c.upload(io.get(), in, sizeof(in));
    mlp_forward(c, sel.params.get(), sel.n_out, io.get(), 1, io.get() + kFeatures);
    float score[kSelectorCells];
    c.load_n(score, io.get() + kFeatures, kSelectorCells);
    int64_t d1[kSelectorCells], d2[kSelectorCells];
    selector_cells(f, d1, d2);
    // Candidates: light only, and every cell whose heavy part alone is
    // estimated below the whole light-only plan (a cell whose product costs
    // more than evaluating everything light cannot win).
    double cost[kSelectorCells];
    int64_t uvw[3 * kSelectorCells];
    plan_costs(s.view(), cal, kSelectorCells, d1, d2, cost, uvw);
    const double light = cost[kSelectorCells - 1];
    int best = kSelectorCells - 1;
    for (int k = 0; k + 1 < kSelectorCells; ++k) {
        if (heavy_cost(cal, uvw[3 * k], uvw[3 * k + 1], uvw[3 * k + 2]) >= light) continue;
        if (score[k] < score[best]) best = k;
    }
    Thresholds th;
    th.d1 = d1[best];
    th.d2 = d2[best];
    th.strategy = JP_STRATEGY_AUTO_MLP;
    return th;
}

}  // namespace jp
