// C ABI of libjoinproject: argument validation, device/stream binding,
// exception-to-status translation and result ownership.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "pipeline.hpp"

struct jp_handle {
    int device = 0;
    hipStream_t stream = nullptr;
    std::shared_ptr<jp::Allocator> alloc;
    int num_cus = 256;
    std::string err;
    jp_calibration cal;
    jp::Selector sel;  // after alloc: its buffer returns to the allocator first
    std::map<uint64_t, int> tune;  // heavy-product kernel per shape class
    std::unique_ptr<jp::PinnedScratch> pinned;  // small read-backs
    jp::StatusPool status_pool;                 // cleared look-back status words
    int64_t lookback_wait = 10000;              // device wall-clock ticks (100 us)
};

// A recorded and captured batched evaluation (jp_two_path_batch_plan).
struct jp_plan {
    int device = 0;
    int32_t n_inst = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    jp::DBuf<uint8_t> arena_own;  // the arena, when the library allocated it
    jp::DBuf<uint8_t> dev_values, dev_uploads;
    jp::DBuf<int> flag;
    jp::DBuf<jp_instance> dev_inst;
    jp::DBuf<unsigned long long> dev_print;
    jp::Replay replay;
    jp::StatusPool pool;
    std::unique_ptr<jp_result> result;  // its columns live in the arena
    unsigned long long print = 0;       // fingerprint of the inputs at plan time
    int64_t nmax = 1;                   // longest input column
    ~jp_plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

namespace {

// Working memory of the no-allocation entry point (jp_two_path_static): a
// fixed device array per GPU, the largest input it takes, and one lock per
// device so that calls in this process never overlap on one array.
constexpr size_t kStaticScratchBytes = size_t(256) << 20;
constexpr int64_t kStaticMaxEdges = int64_t(1) << 19;  // per relation
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

namespace {

struct StaticScratch {
    std::mutex init_mu;
    std::mutex call_mu[kMaxDevices];
    void *ptr[kMaxDevices] = {};       // device address of `scratch` on each device
    hipError_t err[kMaxDevices] = {};  // result of the address query
    bool done[kMaxDevices] = {};
};
StaticScratch g_scratch;

// Looks up the device address of `scratch` once per device, with that device
// current (each GPU holds its own copy of the array).  Host code uses only
// this address: the array's name is a host-side stand-in.
void static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> g(g_scratch.init_mu);
    if (g_scratch.done[device]) return;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) (void)hipGetLastError();
    g_scratch.ptr[device] = e == hipSuccess ? p : nullptr;
    g_scratch.err[device] = e;
    g_scratch.done[device] = true;
}

// Makes the handle's device current for the scope of one call.
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) JP_HIP(hipSetDevice(dev));
    }
    ~DeviceScope() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

jp::Ctx make_ctx(jp_handle *h) {
    jp::Ctx c;
    c.stream = h->stream;
    c.alloc = h->alloc;
    c.device = h->device;
    c.num_cus = h->num_cus;
    c.cal = &h->cal;
    c.sel = &h->sel;
    c.tune = &h->tune;
    c.pinned = h->pinned.get();
    c.status_pool = &h->status_pool;
    c.lookback_wait = h->lookback_wait;
    return c;
}

template <class F>
jp_status guarded(jp_handle *h, F f) {
    try {
        DeviceScope ds(h->device);
        f();
        h->err.clear();
        return JP_OK;
    } catch (const jp::Error &e) {
        h->err = e.msg;
        (void)hipGetLastError();
        return e.st;
    } catch (const std::bad_alloc &) {
        h->err = "host allocation failed";
        return JP_ENOMEM;
    } catch (...) {
        h->err = "unexpected internal error";
        return JP_EINTERNAL;
    }
}

bool bad_col(const void *p, int64_t n) { return n < 0 || (n > 0 && p == nullptr); }

jp_status validate_options(jp_handle *h, const jp_options &o) {
    if (o.strategy < JP_STRATEGY_AUTO_COST || o.strategy > JP_STRATEGY_AUTO_MLP) {
        h->err = "unknown strategy";
        return JP_EINVAL;
    }
    if (o.strategy == JP_STRATEGY_FIXED && (o.delta1 < 1 || o.delta2 < 1)) {
        h->err = "FIXED thresholds must be >= 1";
        return JP_EINVAL;
    }
    if (o.bmm < JP_BMM_AUTO || o.bmm > JP_BMM_F16 || o.y_rule < JP_Y_RULE_MAX ||
        o.y_rule > JP_Y_RULE_R_ONLY || o.dedup < JP_DEDUP_AUTO || o.dedup > JP_DEDUP_SEGMENTED) {
        h->err = "bad option value";
        return JP_EINVAL;
    }
    return JP_OK;
}

// Order-independent 64-bit fingerprint of every instance's four input
// columns: the sum over elements of a mixed (instance, column, index, value).
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
__global__ __launch_bounds__(256) void k_fingerprint(const jp_instance *inst, unsigned long long *out) {
    const jp_instance q = inst[blockIdx.y];
    const unsigned long long salt = (unsigned long long)blockIdx.y << 40;
    unsigned long long h = 0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < q.n_r; e += stride) {
        h += mix64(salt ^ ((unsigned long long)e << 2) ^ ((unsigned long long)(uint32_t)q.r_x[e] << 42));
        h += mix64(salt ^ ((unsigned long long)e << 2 | 1) ^ ((unsigned long long)(uint32_t)q.r_y[e] << 42));
    }
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < q.n_s; e += stride) {
        h += mix64(salt ^ ((unsigned long long)e << 2 | 2) ^ ((unsigned long long)(uint32_t)q.s_z[e] << 42));
        h += mix64(salt ^ ((unsigned long long)e << 2 | 3) ^ ((unsigned long long)(uint32_t)q.s_y[e] << 42));
    }
    for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o);
    if ((threadIdx.x & 63) == 0) atomicAdd(out, h);
}

unsigned long long fingerprint(const jp::Ctx &c, jp_plan *p, int64_t nmax) {
    c.zero(p->dev_print.get(), 1);
    const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(jp::ceil_div(nmax, 256 * 8), 64));
    hipLaunchKernelGGL(k_fingerprint, dim3(gx, (unsigned)p->n_inst), dim3(256), 0, c.stream,
                       (const jp_instance *)p->dev_inst.get(), p->dev_print.get());
    JP_HIP(hipGetLastError());
    return c.load(p->dev_print.get());
}

// Device memory through another allocator, counting the largest amount live
// at once (rounded to 256 bytes, as the arena hands it out).
class PeakAllocator final : public jp::Allocator {
  public:
    explicit PeakAllocator(std::shared_ptr<jp::Allocator> inner) : Allocator(inner->device()), in_(std::move(inner)) {}
    void *alloc(size_t bytes) override {
        void *p = in_->alloc(bytes);
        const size_t r = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
        live_[p] = r;
        cur_ += r;
        peak_ = std::max(peak_, cur_);
        return p;
    }
    void release(void *p) override {
        auto it = live_.find(p);
        if (it != live_.end()) {
            cur_ -= it->second;
            live_.erase(it);
        }
        in_->release(p);
    }
    size_t peak() const { return peak_; }

  private:
    std::shared_ptr<jp::Allocator> in_;
    std::unordered_map<void *, size_t> live_;
    size_t cur_ = 0, peak_ = 0;
};

}  // namespace

// Used by the test hooks (testing.hip).
jp::Ctx jp_handle_ctx(jp_handle *h) { return make_ctx(h); }
void jp_handle_set_lookback_wait(jp_handle *h, int64_t ticks) { h->lookback_wait = ticks; }
jp_status jp_handle_guard(jp_handle *h, void (*fn)(void *), void *arg) {
    return guarded(h, [&] { fn(arg); });
}

extern "C" {

void jp_default_options(jp_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->strategy = JP_STRATEGY_AUTO_COST;
    opt->bmm = JP_BMM_AUTO;
    opt->y_rule = JP_Y_RULE_MAX;
    opt->dedup = JP_DEDUP_AUTO;
    opt->seed = 0x9e3779b97f4a7c15ull;
}

jp_status jp_create(jp_handle **out, int device) {
    if (!out) return JP_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return device < 0 ? JP_EINVAL : JP_EHIP;
    }
    auto h = std::make_unique<jp_handle>();
    h->device = device;
    h->alloc = std::make_shared<jp::PoolAllocator>(device);
    {
        int prev = -1;
        (void)hipGetDevice(&prev);
        if (prev != device) (void)hipSetDevice(device);
        h->pinned = std::make_unique<jp::PinnedScratch>(1 << 20);
        static_scratch_init(device);
        if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
    }
    jp::default_calibration(&h->cal);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        h->num_cus = cus;
    int clock_khz = 0;  // device wall clock, for the 100 us look-back wait
    if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && clock_khz > 0)
        h->lookback_wait = (int64_t)clock_khz / 10;
    (void)hipGetLastError();
    *out = h.release();
    return JP_OK;
}

void jp_destroy(jp_handle *h) {
    if (!h) return;
    {
        int prev = -1;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(h->device);
        (void)hipStreamSynchronize(h->stream);
        h->alloc->release_cached();
        if (prev >= 0) (void)hipSetDevice(prev);
    }
    delete h;
}

jp_status jp_set_stream(jp_handle *h, void *stream) {
    if (!h) return JP_EINVAL;
    return guarded(h, [&] {
        hipStream_t s = (hipStream_t)stream;
        if (s != h->stream) {
            // cached blocks were last used on the old stream
            JP_HIP(hipStreamSynchronize(h->stream));
            h->stream = s;
        }
    });
}

jp_status jp_set_allocator(jp_handle *h, void *(*alloc_fn)(size_t, void *), void (*free_fn)(void *, void *),
                           void *user) {
    if (!h) return JP_EINVAL;
    if ((alloc_fn == nullptr) != (free_fn == nullptr)) {
        h->err = "alloc and free must both be given or both be NULL";
        return JP_EINVAL;
    }
    return guarded(h, [&] {
        // Work queued on the stream may still use blocks of the old source.
        JP_HIP(hipStreamSynchronize(h->stream));
        std::shared_ptr<jp::Allocator> a;
        if (alloc_fn) a = std::make_shared<jp::UserAllocator>(h->device, alloc_fn, free_fn, user);
        else a = std::make_shared<jp::PoolAllocator>(h->device);
        // Buffers the handle keeps between calls come from the new source
        // from now on; live results keep the source they came from.
        h->status_pool.block.reset();
        h->status_pool.used = 0;
        h->alloc->release_cached();
        h->alloc = std::move(a);
        if (h->sel.ready()) {
            const int64_t np = jp::mlp_param_count(h->sel.n_out);
            jp::Ctx c = make_ctx(h);
            jp::DBuf<float> p = c.buf<float>((size_t)np);
            JP_HIP(hipMemcpyAsync(p.get(), h->sel.params.get(), (size_t)np * sizeof(float),
                                  hipMemcpyDeviceToDevice, c.stream));
            c.sync();
            h->sel.params = std::move(p);
        }
    });
}

const char *jp_last_error(const jp_handle *h) { return h ? h->err.c_str() : "null handle"; }

jp_status jp_two_path(jp_handle *h, const int32_t *r_x, const int32_t *r_y, int64_t n_r, const int32_t *s_z,
                      const int32_t *s_y, int64_t n_s, const jp_options *opt, jp_result **out) {
    if (!h) return JP_EINVAL;
    if (!out) {
        h->err = "out is NULL";
        return JP_EINVAL;
    }
    *out = nullptr;
    if (bad_col(r_x, n_r) || bad_col(r_y, n_r) || bad_col(s_z, n_s) || bad_col(s_y, n_s)) {
        h->err = "relation column is NULL or its length is negative";
        return JP_EINVAL;
    }
    jp_options o;
    jp_default_options(&o);
    if (opt) o = *opt;
    jp_status v = validate_options(h, o);
    if (v != JP_OK) return v;
    jp_result *r = nullptr;
    jp_status st = guarded(h, [&] { r = jp::run_two_path(make_ctx(h), r_x, r_y, n_r, s_z, s_y, n_s, o); });
    if (st == JP_OK) *out = r;
    return st;
}

jp_status jp_ssj(jp_handle *h, const int32_t *r_x, const int32_t *r_y, int64_t n_r, const int32_t *s_z,
                 const int32_t *s_y, int64_t n_s, int64_t min_overlap, int32_t order, const jp_options *opt,
                 jp_result **out) {
    if (!h) return JP_EINVAL;
    if (!out) {
        h->err = "out is NULL";
        return JP_EINVAL;
    }
    *out = nullptr;
    if (bad_col(r_x, n_r) || bad_col(r_y, n_r) || bad_col(s_z, n_s) || bad_col(s_y, n_s)) {
        h->err = "relation column is NULL or its length is negative";
        return JP_EINVAL;
    }
    if (min_overlap < 1 || (order != 0 && order != 1)) {
        h->err = "min_overlap must be >= 1 and order 0 or 1";
        return JP_EINVAL;
    }
    jp_options o;
    jp_default_options(&o);
    if (opt) o = *opt;
    jp_status v = validate_options(h, o);
    if (v != JP_OK) return v;
    o.dedup = JP_DEDUP_GLOBAL;  // counts come from one sort of all witnesses
    jp::OverlapSpec spec;
    spec.min_c = min_overlap;
    spec.order = order;
    spec.force_wide = jp::wide_overlap_keys_flag() != 0;
    jp_result *r = nullptr;
    jp_status st = guarded(h, [&] { r = jp::run_two_path(make_ctx(h), r_x, r_y, n_r, s_z, s_y, n_s, o, &spec); });
    if (st == JP_OK) *out = r;
    return st;
}

jp_status jp_bsi(jp_handle *h, const int32_t *r_x, const int32_t *r_y, int64_t n_r, const int32_t *s_z,
                 const int32_t *s_y, int64_t n_s, const int32_t *t_x, const int32_t *t_z, int64_t n_t,
                 const jp_options *opt, uint8_t *answers, jp_stats *stats) {
    if (!h) return JP_EINVAL;
    if (bad_col(r_x, n_r) || bad_col(r_y, n_r) || bad_col(s_z, n_s) || bad_col(s_y, n_s) || bad_col(t_x, n_t) ||
        bad_col(t_z, n_t) || bad_col(answers, n_t)) {
        h->err = "a column or the answer array is NULL, or a length is negative";
        return JP_EINVAL;
    }
    jp_options o;
    jp_default_options(&o);
    if (opt) o = *opt;
    jp_status v = validate_options(h, o);
    if (v != JP_OK) return v;
    return guarded(h, [&] { jp::run_bsi(make_ctx(h), r_x, r_y, n_r, s_z, s_y, n_s, t_x, t_z, n_t, o, answers, stats); });
}

jp_status jp_two_path_static(jp_handle *h, const int32_t *r_x, const int32_t *r_y, int64_t n_r, const int32_t *s_z,
                             const int32_t *s_y, int64_t n_s, const jp_options *opt, int32_t *out_x, int32_t *out_z,
                             int64_t cap, int64_t *n_out, jp_stats *stats) {
    if (!h) return JP_EINVAL;
    if (!n_out || cap < 0 || bad_col(out_x, cap) || bad_col(out_z, cap)) {
        h->err = "n_out is NULL, or an output column is NULL with cap > 0, or cap < 0";
        return JP_EINVAL;
    }
    *n_out = 0;
    if (bad_col(r_x, n_r) || bad_col(r_y, n_r) || bad_col(s_z, n_s) || bad_col(s_y, n_s)) {
        h->err = "relation column is NULL or its length is negative";
        return JP_EINVAL;
    }
    if (n_r > kStaticMaxEdges || n_s > kStaticMaxEdges) {
        h->err = "jp_two_path_static takes at most " + std::to_string(kStaticMaxEdges) +
                 " edges per relation (its working memory is a fixed " + std::to_string(kStaticScratchBytes >> 20) +
                 " MiB device array); use jp_two_path";
        return JP_EINVAL;
    }
    if (h->device >= kMaxDevices || !g_scratch.done[h->device] || !g_scratch.ptr[h->device]) {
        h->err = std::string("static scratch unavailable on this device: ") +
                 (h->device < kMaxDevices && g_scratch.done[h->device] ? hipGetErrorString(g_scratch.err[h->device])
                                                                      : "device index out of range");
        return JP_EHIP;
    }
    jp_options o;
    jp_default_options(&o);
    if (opt) o = *opt;
    jp_status v = validate_options(h, o);
    if (v != JP_OK) return v;
    o.flags &= ~JP_FLAG_TIMING;  // no event objects
    std::lock_guard<std::mutex> lock(g_scratch.call_mu[h->device]);
    int64_t n = 0;
    jp_stats st{};
    jp_status status = guarded(h, [&] {
        jp::Ctx c = make_ctx(h);
        // Every buffer of the call is carved from the device's static array;
        // the look-back status words too (cleared when first handed out).
        auto arena = std::make_shared<jp::ArenaAllocator>(h->device, g_scratch.ptr[h->device], kStaticScratchBytes);
        jp::StatusPool pool;
        c.alloc = arena;
        c.status_pool = &pool;
        c.tune = nullptr;  // kernel by shape: no timed race
        std::unique_ptr<jp_result> r;
        try {
            r.reset(jp::run_two_path(c, r_x, r_y, n_r, s_z, s_y, n_s, o));
            n = r->n;
            st = r->stats;
            if (n > 0 && n <= cap) {
                JP_HIP(hipMemcpyAsync(out_x, r->cols[0].get(), (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                      c.stream));
                JP_HIP(hipMemcpyAsync(out_z, r->cols[1].get(), (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                      c.stream));
            }
            c.sync();
        } catch (...) {
            // the array is reused by the next call: let queued work finish
            (void)hipStreamSynchronize(c.stream);
            (void)hipGetLastError();
            throw;
        }
    });
    if (status != JP_OK) return status;
    *n_out = n;
    if (stats) *stats = st;
    if (n > cap) {
        h->err = "output capacity " + std::to_string(cap) + " is smaller than the " + std::to_string(n) +
                 " distinct pairs (reported in *n_out)";
        return JP_ECAPACITY;
    }
    return JP_OK;
}

jp_status jp_two_path_batch(jp_handle *h, int32_t n_inst, const jp_instance *inst, const jp_options *opt,
                            jp_result **out) {
    if (!h) return JP_EINVAL;
    if (!out) {
        h->err = "out is NULL";
        return JP_EINVAL;
    }
    *out = nullptr;
    if (n_inst < 0 || (n_inst > 0 && !inst)) {
        h->err = "n_inst must be >= 0 and inst non-NULL";
        return JP_EINVAL;
    }
    for (int32_t i = 0; i < n_inst; ++i)
        if (bad_col(inst[i].r_x, inst[i].n_r) || bad_col(inst[i].r_y, inst[i].n_r) ||
            bad_col(inst[i].s_z, inst[i].n_s) || bad_col(inst[i].s_y, inst[i].n_s)) {
            h->err = "instance " + std::to_string(i) + ": relation column is NULL or its length is negative";
            return JP_EINVAL;
        }
    jp_options o;
    jp_default_options(&o);
    if (opt) o = *opt;
    jp_status v = validate_options(h, o);
    if (v != JP_OK) return v;
    jp_result *r = nullptr;
    jp_status st = guarded(h, [&] { r = jp::run_two_path_batch(make_ctx(h), n_inst, inst, o); });
    if (st == JP_OK) *out = r;
    return st;
}

jp_status jp_two_path_batch_plan(jp_handle *h, int32_t n_inst, const jp_instance *inst, const jp_options *opt,
                                 void *arena, int64_t arena_bytes, jp_plan **out, int64_t *arena_needed) {
    if (!h) return JP_EINVAL;
    if (!out || !arena_needed || arena_bytes < 0 || (arena && arena_bytes == 0) || ((uintptr_t)arena % 256) != 0) {
        h->err = "out / arena_needed NULL, arena_bytes negative, or an arena that is empty or not 256-byte aligned";
        return JP_EINVAL;
    }
    *out = nullptr;
    *arena_needed = 0;
    if (n_inst < 1 || n_inst > 65535 || !inst) {
        h->err = "a plan needs 1 to 65535 instances";
        return JP_EINVAL;
    }
    for (int32_t i = 0; i < n_inst; ++i)
        if (bad_col(inst[i].r_x, inst[i].n_r) || bad_col(inst[i].r_y, inst[i].n_r) ||
            bad_col(inst[i].s_z, inst[i].n_s) || bad_col(inst[i].s_y, inst[i].n_s)) {
            h->err = "instance " + std::to_string(i) + ": relation column is NULL or its length is negative";
            return JP_EINVAL;
        }
    jp_options o;
    jp_default_options(&o);
    if (opt) o = *opt;
    jp_status v = validate_options(h, o);
    if (v != JP_OK) return v;
    o.flags &= ~JP_FLAG_TIMING;
    auto plan = std::make_unique<jp_plan>();
    plan->device = h->device;
    plan->n_inst = n_inst;
    int64_t needed = 0;
    jp_status st = guarded(h, [&] {
        jp::Ctx c = make_ctx(h);
        int64_t nmax = 1;
        for (int32_t i = 0; i < n_inst; ++i) nmax = std::max(nmax, std::max(inst[i].n_r, inst[i].n_s));
        plan->dev_inst = c.buf<jp_instance>((size_t)n_inst);
        plan->dev_print = c.buf<unsigned long long>(1);
        plan->flag = c.buf<int>(1);
        JP_HIP(hipMemcpyAsync(plan->dev_inst.get(), inst, (size_t)n_inst * sizeof(jp_instance), hipMemcpyHostToDevice,
                              c.stream));
        plan->nmax = nmax;
        plan->print = fingerprint(c, plan.get(), nmax);
        // 1. the recorded run, measuring its peak working memory
        {
            jp::Ctx rc = c;
            auto peak = std::make_shared<PeakAllocator>(h->alloc);
            jp::StatusPool pool;
            rc.alloc = peak;
            rc.status_pool = &pool;
            plan->replay.mode = jp::Replay::RECORD;
            rc.replay = &plan->replay;
            std::unique_ptr<jp_result> r(jp::run_two_path_batch(rc, n_inst, inst, o));
            r.reset();
            pool.block.reset();
            needed = (int64_t)(peak->peak() + peak->peak() / 8 + (size_t(1) << 20));
        }
        if (arena_bytes < needed) return;  // JP_ECAPACITY below
        uint8_t *base = (uint8_t *)arena;
        if (!base) {
            plan->arena_own = c.buf<uint8_t>((size_t)arena_bytes);
            base = plan->arena_own.get();
        }
        // 2. recorded read-backs and uploads on the device, for the capture
        jp::Replay &rp = plan->replay;
        plan->dev_values = c.buf<uint8_t>(std::max<size_t>(rp.values.size(), 1));
        plan->dev_uploads = c.buf<uint8_t>(std::max<size_t>(rp.uploads.size(), 1));
        if (!rp.values.empty())
            JP_HIP(hipMemcpyAsync(plan->dev_values.get(), rp.values.data(), rp.values.size(), hipMemcpyHostToDevice,
                                  c.stream));
        if (!rp.uploads.empty())
            JP_HIP(hipMemcpyAsync(plan->dev_uploads.get(), rp.uploads.data(), rp.uploads.size(),
                                  hipMemcpyHostToDevice, c.stream));
        c.sync();
        rp.mode = jp::Replay::CAPTURE;
        rp.pos = rp.upos = 0;
        rp.dev_values = plan->dev_values.get();
        rp.dev_uploads = plan->dev_uploads.get();
        rp.flag = plan->flag.get();
        // 3. the capture: the same run on a stream of the plan, every buffer
        // from the arena
        JP_HIP(hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking));
        jp::Ctx cc = c;
        cc.stream = plan->cap_stream;
        cc.alloc = std::make_shared<jp::ArenaAllocator>(h->device, base, (size_t)arena_bytes);
        cc.status_pool = &plan->pool;
        cc.pinned = nullptr;
        cc.replay = &rp;
        JP_HIP(hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeRelaxed));
        try {
            cc.zero(plan->flag.get(), 1);
            plan->result.reset(jp::run_two_path_batch(cc, n_inst, inst, o));
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(plan->cap_stream, &g);
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            throw;
        }
        JP_HIP(hipStreamEndCapture(plan->cap_stream, &plan->graph));
        JP_CHECK(rp.pos == rp.values.size() && rp.upos == rp.uploads.size(), JP_EINTERNAL,
                 "plan capture diverged from the recorded run");
        JP_HIP(hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0));
    });
    if (st == JP_ENOMEM && plan->result == nullptr && arena_bytes >= needed && needed > 0) {
        // the arena's free ranges were too fragmented for the run
        *arena_needed = 2 * needed;
        h->err = "the arena of " + std::to_string(arena_bytes) + " bytes is too small for the plan; about " +
                 std::to_string(2 * needed) + " bytes are needed";
        return JP_ECAPACITY;
    }
    if (st != JP_OK) return st;
    if (arena_bytes < needed) {
        *arena_needed = needed;
        h->err = "the arena of " + std::to_string(arena_bytes) + " bytes is too small for the plan; " +
                 std::to_string(needed) + " bytes are needed";
        return JP_ECAPACITY;
    }
    *arena_needed = needed;
    *out = plan.release();
    return JP_OK;
}

jp_status jp_plan_launch(jp_handle *h, jp_plan *p) {
    if (!h || !p) return JP_EINVAL;
    if (p->device != h->device) {
        h->err = "the plan was made on another device";
        return JP_EINVAL;
    }
    bool changed = false;
    jp_status st = guarded(h, [&] {
        jp::Ctx c = make_ctx(h);
        if (fingerprint(c, p, p->nmax) != p->print) {
            changed = true;
            return;
        }
        JP_HIP(hipGraphLaunch(p->exec, c.stream));
        JP_CHECK(c.load(p->flag.get()) == 0, JP_EINTERNAL, "a replayed read-back differs from the recorded one");
    });
    if (st != JP_OK) return st;
    if (changed) {
        h->err = "the instances' contents changed since the plan was made; make a new plan";
        return JP_ECAPACITY;
    }
    return JP_OK;
}

jp_status jp_plan_result(const jp_plan *p, const int32_t **cols, int64_t *n_tuples, int64_t *offsets) {
    if (!p || !p->result) return JP_EINVAL;
    if (cols) {
        cols[0] = p->result->cols[0].get();
        cols[1] = p->result->cols[1].get();
    }
    if (n_tuples) *n_tuples = p->result->n;
    if (offsets)
        for (size_t i = 0; i < p->result->batch_off.size(); ++i) offsets[i] = p->result->batch_off[i];
    return JP_OK;
}

jp_status jp_plan_copy(jp_handle *h, const jp_plan *p, int32_t *const *cols) {
    if (!h) return JP_EINVAL;
    if (!p || !p->result || !cols || (p->result->n > 0 && (!cols[0] || !cols[1]))) {
        h->err = "plan, its result or a destination column is NULL";
        return JP_EINVAL;
    }
    return guarded(h, [&] {
        const int64_t n = p->result->n;
        for (int i = 0; i < 2; ++i)
            if (n > 0)
                JP_HIP(hipMemcpyAsync(cols[i], p->result->cols[i].get(), (size_t)n * sizeof(int32_t),
                                      hipMemcpyDeviceToDevice, h->stream));
    });
}

void jp_plan_free(jp_plan *p) {
    if (!p) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(p->device);
    if (p->cap_stream) (void)hipStreamSynchronize(p->cap_stream);
    delete p;
    if (prev >= 0) (void)hipSetDevice(prev);
}

jp_status jp_result_batch_offsets(const jp_result *r, int32_t *n_inst, int64_t *offsets) {
    if (!r || !n_inst) return JP_EINVAL;
    *n_inst = r->batch_off.empty() ? 0 : (int32_t)(r->batch_off.size() - 1);
    if (offsets)
        for (size_t i = 0; i < r->batch_off.size(); ++i) offsets[i] = r->batch_off[i];
    return JP_OK;
}

jp_status jp_star(jp_handle *h, int k, const int32_t *const *x, const int32_t *const *y, const int64_t *n,
                  const jp_options *opt, jp_result **out) {
    if (!h) return JP_EINVAL;
    if (!out) {
        h->err = "out is NULL";
        return JP_EINVAL;
    }
    *out = nullptr;
    if (k < 2 || k > 8 || !x || !y || !n) {
        h->err = "k must be in [2, 8] and x, y, n non-NULL";
        return JP_EINVAL;
    }
    for (int i = 0; i < k; ++i)
        if (bad_col(x[i], n[i]) || bad_col(y[i], n[i])) {
            h->err = "relation column is NULL or its length is negative";
            return JP_EINVAL;
        }
    jp_options o;
    jp_default_options(&o);
    if (opt) o = *opt;
    jp_status v = validate_options(h, o);
    if (v != JP_OK) return v;
    jp_result *r = nullptr;
    jp_status st = guarded(h, [&] { r = jp::run_star(make_ctx(h), k, x, y, n, o); });
    if (st == JP_OK) *out = r;
    return st;
}

void jp_default_calibration(jp_calibration *cal) {
    if (cal) jp::default_calibration(cal);
}

jp_status jp_set_calibration(jp_handle *h, const jp_calibration *cal) {
    if (!h) return JP_EINVAL;
    if (!cal || cal->n_mm < 0 || cal->n_mm > 24 || !(cal->t_witness >= 0) || !(cal->t_byte >= 0) ||
        !(cal->t_seq >= 0) || !(cal->t_x >= 0) || !(cal->eps > 0 && cal->eps < 1)) {
        h->err = "bad calibration";
        return JP_EINVAL;
    }
    for (int i = 0; i < cal->n_mm; ++i)
        if (!(cal->mm_p[i] > 0) || !(cal->mm_s[i] >= 0)) {
            h->err = "bad product time table";
            return JP_EINVAL;
        }
    h->cal = *cal;
    return JP_OK;
}

jp_status jp_get_calibration(const jp_handle *h, jp_calibration *cal) {
    if (!h || !cal) return JP_EINVAL;
    *cal = h->cal;
    return JP_OK;
}

static bool bad_index(const jp_degree_index &d, bool need_sum) {
    if (d.n < 0 || (d.n > 0 && (!d.deg || !d.count || (need_sum && !d.sum)))) return true;
    for (int64_t i = 0; i < d.n; ++i)
        if (d.deg[i] < 0 || d.count[i] < 0 || (i > 0 && d.deg[i] <= d.deg[i - 1])) return true;
    return false;
}

jp_status jp_plan_summary(const jp_two_path_summary *s, const jp_calibration *cal, int64_t *delta1, int64_t *delta2,
                          double *cost, double *cost_light_only) {
    if (!s || !delta1 || !delta2) return JP_EINVAL;
    if (s->n_r < 0 || s->n_s < 0 || s->dom_x < 0 || s->dom_y < 0 || s->dom_z < 0 || s->J < 0 ||
        bad_index(s->y, true) || bad_index(s->x, true) || bad_index(s->xcdf, false) || bad_index(s->z, false))
        return JP_EINVAL;
    try {
        jp_calibration c;
        if (cal) c = *cal;
        else jp::default_calibration(&c);
        const jp::PlanResult r = jp::algorithm2(*s, c);
        *delta1 = r.d1;
        *delta2 = r.d2;
        if (cost) *cost = r.cost;
        if (cost_light_only) *cost_light_only = r.cost_light_only;
        return JP_OK;
    } catch (...) {
        return JP_EINTERNAL;
    }
}

jp_status jp_plan_theory(int64_t n, double out, int64_t *delta1, int64_t *delta2) {
    if (!delta1 || !delta2 || !std::isfinite(out)) return JP_EINVAL;
    const jp::Thresholds th = jp::theory_thresholds(n, out);
    *delta1 = th.d1;
    *delta2 = th.d2;
    return JP_OK;
}

double jp_estimate_out(int64_t dom_x, int64_t dom_z, int64_t J, int64_t n) {
    return jp::estimate_out(dom_x, dom_z, J, n);
}

jp_status jp_plan_two_path(jp_handle *h, const int32_t *r_x, const int32_t *r_y, int64_t n_r, const int32_t *s_z,
                           const int32_t *s_y, int64_t n_s, const jp_options *opt, int64_t *delta1,
                           int64_t *delta2, float *features) {
    if (!h) return JP_EINVAL;
    if (!delta1 || !delta2 || bad_col(r_x, n_r) || bad_col(r_y, n_r) || bad_col(s_z, n_s) || bad_col(s_y, n_s)) {
        h->err = "bad argument to jp_plan_two_path";
        return JP_EINVAL;
    }
    jp_options o;
    jp_default_options(&o);
    if (opt) o = *opt;
    jp_status v = validate_options(h, o);
    if (v != JP_OK) return v;
    return guarded(h, [&] { jp::plan_two_path(make_ctx(h), r_x, r_y, n_r, s_z, s_y, n_s, o, delta1, delta2, features); });
}

jp_status jp_plan_cells(jp_handle *h, const int32_t *r_x, const int32_t *r_y, int64_t n_r, const int32_t *s_z,
                        const int32_t *s_y, int64_t n_s, const jp_options *opt, int32_t n_cells,
                        const int64_t *delta1, const int64_t *delta2, double *est_seconds, int64_t *heavy_dims) {
    if (!h) return JP_EINVAL;
    if (n_cells < 0 || (n_cells > 0 && (!delta1 || !delta2)) || bad_col(r_x, n_r) || bad_col(r_y, n_r) ||
        bad_col(s_z, n_s) || bad_col(s_y, n_s)) {
        h->err = "bad argument to jp_plan_cells";
        return JP_EINVAL;
    }
    for (int32_t i = 0; i < n_cells; ++i)
        if (delta1[i] < 1 || delta2[i] < 1) {
            h->err = "thresholds must be >= 1";
            return JP_EINVAL;
        }
    jp_options o;
    jp_default_options(&o);
    if (opt) o = *opt;
    jp_status v = validate_options(h, o);
    if (v != JP_OK) return v;
    return guarded(h, [&] {
        jp::plan_cells(make_ctx(h), r_x, r_y, n_r, s_z, s_y, n_s, o, n_cells, delta1, delta2, est_seconds,
                       heavy_dims);
    });
}

double jp_heavy_cost(const jp_calibration *cal, int64_t u, int64_t v, int64_t w) {
    jp_calibration d;
    if (!cal) jp::default_calibration(&d);
    return jp::heavy_cost(cal ? *cal : d, u, v, w);
}

int32_t jp_selector_cells(const float *features, int64_t *delta1, int64_t *delta2) {
    if (!features || !delta1 || !delta2) return 0;
    jp::selector_cells(features, delta1, delta2);
    return jp::kSelectorCells;
}

int64_t jp_mlp_param_count(int32_t n_out) { return n_out < 1 ? 0 : jp::mlp_param_count(n_out); }

jp_status jp_set_selector(jp_handle *h, const float *params, int32_t n_out, const float *feat_mean,
                          const float *feat_scale) {
    if (!h) return JP_EINVAL;
    if (!params) {
        h->sel.params.reset();
        h->sel.n_out = 0;
        return JP_OK;
    }
    if (n_out != jp::kSelectorCells || !feat_mean || !feat_scale) {
        h->err = "selector needs 65 outputs and the feature mean and scale";
        return JP_EINVAL;
    }
    for (int i = 0; i < jp::kFeatures; ++i)
        if (!(feat_scale[i] > 0) || !std::isfinite(feat_mean[i])) {
            h->err = "feature scale must be positive and the mean finite";
            return JP_EINVAL;
        }
    const int64_t np = jp::mlp_param_count(n_out);
    for (int64_t i = 0; i < np; ++i)
        if (!std::isfinite(params[i])) {
            h->err = "selector weights must be finite";
            return JP_EINVAL;
        }
    return guarded(h, [&] {
        jp::Ctx c = make_ctx(h);
        jp::DBuf<float> p = c.buf<float>((size_t)np);
        JP_HIP(hipMemcpyAsync(p.get(), params, (size_t)np * sizeof(float), hipMemcpyHostToDevice, c.stream));
        c.sync();
        h->sel.params = std::move(p);
        h->sel.n_out = n_out;
        std::memcpy(h->sel.mean, feat_mean, sizeof(h->sel.mean));
        std::memcpy(h->sel.scale, feat_scale, sizeof(h->sel.scale));
    });
}

jp_status jp_mlp_forward(jp_handle *h, const float *params, int32_t n_out, const float *x, int64_t batch,
                         float *y) {
    if (!h) return JP_EINVAL;
    if (n_out < 1 || n_out > 256 || batch < 0 || !params || bad_col(x, batch) || bad_col(y, batch)) {
        h->err = "bad argument to jp_mlp_forward";
        return JP_EINVAL;
    }
    return guarded(h, [&] { jp::mlp_forward(make_ctx(h), params, n_out, x, batch, y); });
}

jp_status jp_mlp_grad(jp_handle *h, const float *params, int32_t n_out, const float *x, const float *target,
                      const float *weight, int64_t batch, float *grad, float *loss) {
    if (!h) return JP_EINVAL;
    if (n_out < 1 || n_out > 256 || batch < 0 || !params || !grad || !loss || bad_col(x, batch) ||
        bad_col(target, batch) || bad_col(weight, batch)) {
        h->err = "bad argument to jp_mlp_grad";
        return JP_EINVAL;
    }
    return guarded(h, [&] { jp::mlp_grad(make_ctx(h), params, n_out, x, target, weight, batch, grad, loss); });
}

jp_status jp_mlp_adam(jp_handle *h, float *params, float *m, float *v, const float *grad, int64_t n, int32_t step,
                      float lr, float beta1, float beta2, float eps) {
    if (!h) return JP_EINVAL;
    if (n < 0 || step < 1 || bad_col(params, n) || bad_col(m, n) || bad_col(v, n) || bad_col(grad, n) ||
        !(lr >= 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0)) {
        h->err = "bad argument to jp_mlp_adam";
        return JP_EINVAL;
    }
    return guarded(h, [&] { jp::mlp_adam(make_ctx(h), params, m, v, grad, n, step, lr, beta1, beta2, eps); });
}

jp_status jp_result_size(const jp_result *r, int64_t *n_tuples, int32_t *arity) {
    if (!r) return JP_EINVAL;
    if (n_tuples) *n_tuples = r->n;
    if (arity) *arity = r->arity;
    return JP_OK;
}

jp_status jp_result_columns(const jp_result *r, const int32_t **cols) {
    if (!r || !cols) return JP_EINVAL;
    for (int i = 0; i < r->arity; ++i) cols[i] = r->cols[i].get();
    return JP_OK;
}

jp_status jp_result_copy(jp_handle *h, const jp_result *r, int32_t *const *cols) {
    if (!h) return JP_EINVAL;
    if (!r || !cols) {
        h->err = "result or column array is NULL";
        return JP_EINVAL;
    }
    for (int i = 0; i < r->arity; ++i)
        if (r->n > 0 && !cols[i]) {
            h->err = "destination column is NULL";
            return JP_EINVAL;
        }
    return guarded(h, [&] {
        for (int i = 0; i < r->arity; ++i)
            if (r->n > 0)
                JP_HIP(hipMemcpyAsync(cols[i], r->cols[i].get(), (size_t)r->n * sizeof(int32_t),
                                      hipMemcpyDeviceToDevice, h->stream));
    });
}

jp_status jp_result_stats(const jp_result *r, jp_stats *s) {
    if (!r || !s) return JP_EINVAL;
    *s = r->stats;
    return JP_OK;
}

void jp_result_free(jp_result *r) { delete r; }

uint64_t jp_product_shape_class(int64_t u, int64_t w, int64_t ld) {
    return (u < 0 || w < 0 || ld < 0) ? 0 : jp::product_shape_class(u, w, ld);
}

jp_status jp_set_product_table(jp_handle *h, int32_t n, const uint64_t *classes, const int32_t *kinds) {
    if (!h) return JP_EINVAL;
    if (n < 0 || (n > 0 && (!classes || !kinds))) {
        h->err = "bad product table";
        return JP_EINVAL;
    }
    for (int32_t i = 0; i < n; ++i)
        if (kinds[i] != JP_BMM_BITPOP && kinds[i] != JP_BMM_I8_T128 && kinds[i] != JP_BMM_I8_T256) {
            h->err = "product table kinds must be JP_BMM_BITPOP, JP_BMM_I8_T128 or JP_BMM_I8_T256";
            return JP_EINVAL;
        }
    // kept as the variant codes of the kernel choice (T128 = 0, T256 = 1, BITPOP = 2)
    for (int32_t i = 0; i < n; ++i)
        h->tune[classes[i]] = kinds[i] == JP_BMM_I8_T128 ? 0 : (kinds[i] == JP_BMM_I8_T256 ? 1 : 2);
    return JP_OK;
}

jp_status jp_bool_matmul(jp_handle *h, const int8_t *A, const int8_t *Bt, int64_t u, int64_t w, int64_t k,
                         int64_t ld, int32_t kind, int32_t *rows, int32_t *cols, int64_t cap, int64_t *nnz,
                         double *ms) {
    if (!h) return JP_EINVAL;
    if (u < 0 || w < 0 || k < 0 || cap < 0 || !nnz || ld < k || ld % jp::kBmmPadK != 0 ||
        bad_col(A, u * ld) || bad_col(Bt, w * ld) || bad_col(rows, cap) || bad_col(cols, cap) ||
        kind < JP_BMM_AUTO || kind > JP_BMM_F16) {
        h->err = "bad argument to jp_bool_matmul (ld must be >= k and a multiple of 128)";
        return JP_EINVAL;
    }
    if (kind == JP_BMM_F16 && ld >= (int64_t(1) << 24)) {
        h->err = "fp16 product: counts may reach 2^24, beyond fp32's exact range";
        return JP_EPRECISION;
    }
    int64_t count = 0;
    double t = 0;
    jp_status st = guarded(h, [&] {
        jp::Ctx c = make_ctx(h);
        jp::DBuf<unsigned long long> cnt = c.buf<unsigned long long>(1);
        jp::EventPair ev;
        JP_HIP(hipEventRecord(ev.a, c.stream));
        jp::bool_matmul_pairs(c, A, Bt, u, w, ld, kind, rows, cols, cap, cnt.get());
        JP_HIP(hipEventRecord(ev.b, c.stream));
        unsigned long long v = c.load(cnt.get());
        float f = 0;
        JP_HIP(hipEventElapsedTime(&f, ev.a, ev.b));
        count = (int64_t)v;
        t = f;
    });
    if (st != JP_OK) return st;
    *nnz = count;
    if (ms) *ms = t;
    if (count > cap) {
        h->err = "capacity too small for the nonzero count";
        return JP_ECAPACITY;
    }
    return JP_OK;
}

}  // extern "C"
