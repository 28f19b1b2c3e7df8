// Host-side infrastructure shared by every translation unit of libjoinproject:
// error propagation, a caching device allocator, RAII device buffers, the
// per-call execution context and device-time phase markers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <initializer_list>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/jp.h"

namespace jp {

// Internal failures travel as exceptions and are turned into a status at the
// C boundary; nothing throws across it.
struct Error {
    jp_status st;
    std::string msg;
};

[[noreturn]] inline void fail(jp_status st, const std::string &msg) { throw Error{st, msg}; }

#define JP_HIP(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            ::jp::fail(JP_EHIP, std::string(#call) + " failed: " + hipGetErrorString(e_)); \
    } while (0)

#define JP_CHECK(cond, st, msg)                       \
    do {                                              \
        if (!(cond)) ::jp::fail((st), (msg));         \
    } while (0)

// Source of every device buffer of a call.  Buffers are used on one stream at
// a time, so a released block may be handed out again at once: later work on
// that stream is ordered after the work that used it.
class Allocator {
  public:
    explicit Allocator(int device) : device_(device) {}
    virtual ~Allocator() = default;
    // Raises JP_ENOMEM when no memory can be had; never returns nullptr.
    virtual void *alloc(size_t bytes) = 0;
    virtual void release(void *p) = 0;
    // Returns cached blocks to the device (no-op where nothing is cached).
    virtual void release_cached() {}
    int device() const { return device_; }

  private:
    int device_;
};

// Built-in caching allocator.  Blocks are rounded (powers of two below 1 MiB,
// 2 MiB multiples above), kept on release, and reused best-fit for requests
// at least 2/3 of their size.  When hipMalloc fails the cache is emptied and
// the request retried once.
class PoolAllocator final : public Allocator {
  public:
    explicit PoolAllocator(int device) : Allocator(device) {}
    ~PoolAllocator() override { release_cached(); }

    void *alloc(size_t bytes) override {
        if (bytes == 0) bytes = 1;
        size_t r = round(bytes);
        std::lock_guard<std::mutex> g(mu_);
        auto it = free_.lower_bound(r);
        if (it != free_.end() && it->first * 2 <= r * 3) {
            void *p = it->second;
            live_[p] = it->first;
            cached_ -= it->first;
            free_.erase(it);
            return p;
        }
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, r);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            release_cached_locked();
            e = hipMalloc(&p, r);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                fail(JP_ENOMEM, "device allocation of " + std::to_string(r) + " bytes failed");
            }
        }
        live_[p] = r;
        return p;
    }

    void release(void *p) override {
        if (!p) return;
        std::lock_guard<std::mutex> g(mu_);
        auto it = live_.find(p);
        if (it == live_.end()) return;
        free_.emplace(it->second, p);
        cached_ += it->second;
        live_.erase(it);
    }

    void release_cached() override {
        std::lock_guard<std::mutex> g(mu_);
        release_cached_locked();
    }

  private:
    static size_t round(size_t b) {
        if (b <= (1u << 20)) {
            size_t r = 256;
            while (r < b) r <<= 1;
            return r;
        }
        const size_t g = 2u << 20;
        return (b + g - 1) / g * g;
    }
    void release_cached_locked() {
        for (auto &kv : free_) (void)hipFree(kv.second);
        free_.clear();
        cached_ = 0;
    }

    std::mutex mu_;
    std::multimap<size_t, void *> free_;
    std::unordered_map<void *, size_t> live_;
    size_t cached_ = 0;
};

// Caller-supplied allocation functions (jp_set_allocator).  Every request goes
// to the caller; a NULL return becomes JP_ENOMEM.  Requests are rounded up to
// 256 bytes so that every buffer keeps the alignment the kernels assume.
class UserAllocator final : public Allocator {
  public:
    using AllocFn = void *(*)(size_t, void *);
    using FreeFn = void (*)(void *, void *);
    UserAllocator(int device, AllocFn a, FreeFn f, void *user) : Allocator(device), a_(a), f_(f), user_(user) {}

    void *alloc(size_t bytes) override {
        const size_t r = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
        void *p = a_(r, user_);
        if (!p) fail(JP_ENOMEM, "the caller's allocator returned NULL for " + std::to_string(r) + " bytes");
        if ((uintptr_t)p % 256 != 0) {
            f_(p, user_);
            fail(JP_EINVAL, "the caller's allocator returned a pointer not aligned to 256 bytes");
        }
        return p;
    }
    void release(void *p) override {
        if (p) f_(p, user_);
    }

  private:
    AllocFn a_;
    FreeFn f_;
    void *user_;
};

// First-fit allocator over one fixed device region (the no-allocation entry
// point).  Free ranges are kept by offset and merged with their neighbours on
// release; a request that fits no free range raises JP_ENOMEM.  Nothing is
// ever taken from the device runtime.
class ArenaAllocator final : public Allocator {
  public:
    ArenaAllocator(int device, void *base, size_t bytes) : Allocator(device), base_((uint8_t *)base), bytes_(bytes) {
        if (bytes_) free_[0] = bytes_;
    }
    void *alloc(size_t bytes) override {
        const size_t r = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < r) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > r) free_[off + r] = len - r;
            live_[off] = r;
            in_use_ += r;
            peak_ = std::max(peak_, in_use_);
            return base_ + off;
        }
        fail(JP_ENOMEM, "the static scratch of " + std::to_string(bytes_ >> 20) + " MiB has no free range of " +
                            std::to_string(r) + " bytes (" + std::to_string(in_use_) + " bytes in use): the input is "
                            "too large for the no-allocation entry point");
    }
    void release(void *p) override {
        if (!p) return;
        const size_t off = (size_t)((uint8_t *)p - base_);
        auto lt = live_.find(off);
        if (lt == live_.end()) return;
        size_t start = off, len = lt->second;
        live_.erase(lt);
        in_use_ -= len;
        auto next = free_.lower_bound(start);
        if (next != free_.end() && next->first == start + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
    }
    size_t peak() const { return peak_; }
    size_t in_use() const { return in_use_; }

  private:
    uint8_t *base_;
    size_t bytes_;
    std::map<size_t, size_t> free_;  // offset -> length
    std::map<size_t, size_t> live_;  // offset -> length
    size_t in_use_ = 0, peak_ = 0;
};

// Owning device buffer of n elements of T from an Allocator.
template <class T>
class DBuf {
  public:
    DBuf() = default;
    DBuf(std::shared_ptr<Allocator> a, size_t n) : a_(std::move(a)), n_(n) {
        p_ = static_cast<T *>(a_->alloc(n * sizeof(T)));
    }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept { swap(o); }
    DBuf &operator=(DBuf &&o) noexcept {
        reset();
        swap(o);
        return *this;
    }
    ~DBuf() { reset(); }
    void reset() {
        if (p_ && a_) a_->release(p_);
        p_ = nullptr;
        n_ = 0;
    }
    T *get() const { return p_; }
    size_t size() const { return n_; }
    T *release_ptr() {
        T *p = p_;
        p_ = nullptr;
        n_ = 0;
        return p;
    }

  private:
    void swap(DBuf &o) {
        std::swap(a_, o.a_);
        std::swap(p_, o.p_);
        std::swap(n_, o.n_);
    }
    std::shared_ptr<Allocator> a_;
    T *p_ = nullptr;
    size_t n_ = 0;
};

struct Selector;

// x dimension of a launch grid.  A dispatch counts its work-items in 32 bits,
// so a grid of 2^32 or more work-items would be cut short: refuse it.
inline unsigned grid_x(int64_t blocks, int threads) {
    if (blocks < 1 || blocks * (int64_t)threads > (int64_t)UINT32_MAX)
        fail(JP_EINVAL, "launch grid of " + std::to_string(blocks) + " workgroups out of range");
    return (unsigned)blocks;
}

// Clearing kernel (used instead of hipMemsetAsync so that a captured stream
// holds only kernel nodes).
template <class W>
__global__ __launch_bounds__(256) void k_zero_words(W *p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) p[i] = W{};
}

// Copies n bytes of device memory to mapped pinned host memory (small
// read-backs: one tiny kernel instead of a staged runtime copy).
template <class B>
__global__ __launch_bounds__(256) void k_to_host(const B *src, B *dst, int64_t n) {
    for (int64_t i = threadIdx.x; i < n; i += 256) dst[i] = src[i];
}

// Gathers up to 8 device scalars into one contiguous block (one read-back).
struct ScalarList {
    const int64_t *p[8];
    int n;
};
template <class T>
__global__ __launch_bounds__(64) void k_gather_scalars(ScalarList l, T *dst) {
    if ((int)threadIdx.x < l.n) dst[threadIdx.x] = *l.p[threadIdx.x];
}

// Pinned, device-mapped host buffer for small read-backs (one per handle).
struct PinnedScratch {
    uint8_t *host = nullptr, *dev = nullptr;
    size_t bytes = 0;
    explicit PinnedScratch(size_t n) {
        void *h = nullptr;
        if (hipHostMalloc(&h, n, hipHostMallocMapped) != hipSuccess) {
            (void)hipGetLastError();
            return;
        }
        void *d = nullptr;
        if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipHostFree(h);
            return;
        }
        host = (uint8_t *)h;
        dev = (uint8_t *)d;
        bytes = n;
    }
    ~PinnedScratch() {
        if (host) (void)hipHostFree(host);
    }
    PinnedScratch(const PinnedScratch &) = delete;
    PinnedScratch &operator=(const PinnedScratch &) = delete;
};

// Cleared status words for the single-pass look-back kernels of one handle.
// One block is cleared by one launch and handed out in consecutive pieces,
// one per pass; when a pass needs more than is left, the whole block is
// cleared again, ordered on the stream after every pass that used it.
struct StatusPool {
    static constexpr size_t kWords = 1u << 16;
    DBuf<uint64_t> block;
    size_t used = 0;
};

// Compares n bytes of live device data with the recorded bytes of a plan and
// raises *flag on any difference (captured-plan replays).
__global__ __launch_bounds__(256) inline void k_replay_check(const uint8_t *live, const uint8_t *rec, int64_t n,
                                                             int *flag) {
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        bad |= live[i] != rec[i];
    if (bad) *flag = 1;
}

// Recording and capture of one pipeline run for a reusable plan (a captured
// HIP graph).  RECORD: the run executes normally and every value the host
// reads back from the device, and every block it uploads, is kept in order.
// CAPTURE: the same host code runs again while the stream is being captured;
// read-backs return the recorded values (no wait) and add a check node that
// compares the live device bytes with them at replay time, and uploads come
// from a device copy of the recorded blocks, so the graph references no host
// memory.  The host decisions of the run (thresholds, grid sizes, buffer
// sizes) are therefore those of the recorded run.
struct Replay {
    enum Mode { RECORD, CAPTURE } mode = RECORD;
    std::vector<uint8_t> values;  // read-back bytes, in order
    size_t pos = 0;
    std::vector<uint8_t> uploads;  // uploaded bytes, in order
    size_t upos = 0;
    const uint8_t *dev_values = nullptr;   // device copies (capture)
    const uint8_t *dev_uploads = nullptr;
    int *flag = nullptr;                   // device: raised by a failed check
};

// Execution context of one call: device, stream, allocator, chip size.
struct Ctx {
    hipStream_t stream = nullptr;
    std::shared_ptr<Allocator> alloc;
    int device = 0;
    int num_cus = 256;
    size_t lds_bytes = 160 * 1024;
    const jp_calibration *cal = nullptr;  // optimizer constants of the handle
    const Selector *sel = nullptr;        // learned threshold selector of the handle (may be empty)
    std::map<uint64_t, int> *tune = nullptr;  // product kernel per shape class, raced once (handle-owned)
    mutable int *bmm_used = nullptr;          // where to report the product kernel used (may be null)
    mutable bool *bmm_sym = nullptr;          // set when a symmetric product ran on half its tiles (may be null)

    template <class T>
    DBuf<T> buf(size_t n) const {
        return DBuf<T>(alloc, n);
    }
    void sync() const {
        if (replay && replay->mode == Replay::CAPTURE) return;  // nothing to wait for while capturing
        JP_HIP(hipStreamSynchronize(stream));
    }
    Replay *replay = nullptr;  // set while a plan is recorded or captured
    bool capturing() const { return replay && replay->mode == Replay::CAPTURE; }
    // Host-to-device copy of n bytes whose source may be released once the
    // call's next wait returns (in a captured plan: a copy of the recorded block).
    void upload(void *dev, const void *host, size_t bytes) const {
        if (!bytes) return;
        if (capturing()) {
            Replay &r = *replay;
            JP_CHECK(r.upos + bytes <= r.uploads.size() && std::memcmp(r.uploads.data() + r.upos, host, bytes) == 0,
                     JP_EINTERNAL, "plan capture diverged from the recorded run (upload)");
            JP_HIP(hipMemcpyAsync(dev, r.dev_uploads + r.upos, bytes, hipMemcpyDeviceToDevice, stream));
            r.upos += bytes;
            return;
        }
        if (replay) replay->uploads.insert(replay->uploads.end(), (const uint8_t *)host, (const uint8_t *)host + bytes);
        JP_HIP(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, stream));
    }
    PinnedScratch *pinned = nullptr;  // small read-backs go through it when set
    StatusPool *status_pool = nullptr;  // handle-owned, see take_status
    // How long a look-back lane waits for a predecessor tile's status before
    // computing that tile's sum itself, in ticks of the device wall clock.
    int64_t lookback_wait = 10000;
    // `words` cleared 64-bit words from the handle's pool, valid for one
    // launch on this stream; nullptr when there is no pool or the request is
    // larger than the pool.
    uint64_t *take_status(size_t words) const {
        if (!status_pool || words > StatusPool::kWords) return nullptr;
        StatusPool &p = *status_pool;
        if (!p.block.get()) {
            p.block = buf<uint64_t>(StatusPool::kWords);
            p.used = StatusPool::kWords;
        }
        if (p.used + words > StatusPool::kWords) {
            zero(p.block.get(), StatusPool::kWords);
            p.used = 0;
        }
        uint64_t *r = p.block.get() + p.used;
        p.used += words;
        return r;
    }
    template <class T>
    T load(const T *dev) const {  // small device-to-host read, waits on the stream
        T v;
        load_n(&v, dev, 1);
        return v;
    }
    // Several device int64 scalars with one wait: out[i] = *ptrs[i].
    void load_scalars(std::initializer_list<const int64_t *> ptrs, int64_t *out) const {
        ScalarList l;
        l.n = 0;
        for (const int64_t *q : ptrs) {
            if (l.n == 8) fail(JP_EINTERNAL, "too many scalars in one read-back");
            l.p[l.n++] = q;
        }
        if (!l.n) return;
        int64_t *tmp = static_cast<int64_t *>(alloc->alloc(8 * sizeof(int64_t)));
        hipLaunchKernelGGL(k_gather_scalars<int64_t>, dim3(1), dim3(64), 0, stream, l, tmp);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) {
            try {
                load_n(out, (const int64_t *)tmp, (size_t)l.n);
            } catch (...) {
                alloc->release(tmp);
                throw;
            }
        }
        alloc->release(tmp);
        if (e != hipSuccess) fail(JP_EHIP, std::string("scalar gather failed: ") + hipGetErrorString(e));
    }
    // unordered: the device holds these values in an order that may differ
    // between runs (appended with atomics), so a captured plan does not
    // compare them byte by byte.
    template <class T>
    void load_n(T *host, const T *dev, size_t n, bool unordered = false) const {
        if (!n) return;
        const size_t bytes = n * sizeof(T);
        if (capturing()) {
            Replay &r = *replay;
            JP_CHECK(r.pos + bytes <= r.values.size(), JP_EINTERNAL, "plan capture diverged from the recorded run");
            const int64_t blocks = std::min<int64_t>(((int64_t)bytes + 255) / 256, 64);
            if (!unordered)
                hipLaunchKernelGGL(k_replay_check, dim3((unsigned)blocks), dim3(256), 0, stream, (const uint8_t *)dev,
                                   r.dev_values + r.pos, (int64_t)bytes, r.flag);
            JP_HIP(hipGetLastError());
            std::memcpy(host, r.values.data() + r.pos, bytes);
            r.pos += bytes;
            return;
        }
        load_n_now(host, dev, n);
        if (replay) replay->values.insert(replay->values.end(), (const uint8_t *)host, (const uint8_t *)host + bytes);
    }
    template <class T>
    void load_n_now(T *host, const T *dev, size_t n) const {
        const size_t bytes = n * sizeof(T);
        if (pinned && pinned->host && bytes <= pinned->bytes && bytes <= 4096) {
            hipLaunchKernelGGL(k_to_host<uint8_t>, dim3(1), dim3(256), 0, stream, (const uint8_t *)dev, pinned->dev,
                               (int64_t)bytes);
            JP_HIP(hipGetLastError());
            sync();
            std::memcpy(host, pinned->host, bytes);
            return;
        }
        JP_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, stream));
        sync();
    }
    template <class T>
    void zero(T *dev, size_t n) const {
        const size_t bytes = n * sizeof(T);
        const uintptr_t a = (uintptr_t)dev;
        if (bytes == 0) return;
        if (a % 16 == 0 && bytes % 16 == 0) zero_words((uint4 *)dev, bytes / 16);
        else if (a % 8 == 0 && bytes % 8 == 0) zero_words((uint64_t *)dev, bytes / 8);
        else if (a % 4 == 0 && bytes % 4 == 0) zero_words((uint32_t *)dev, bytes / 4);
        else zero_words((uint8_t *)dev, bytes);
    }
    template <class W>
    void zero_words(W *p, size_t n) const {
        const int64_t blocks = std::min<int64_t>(((int64_t)n + 255) / 256, (int64_t)num_cus * 8);
        hipLaunchKernelGGL(k_zero_words<W>, dim3(grid_x(blocks, 256)), dim3(256), 0, stream, p, (int64_t)n);
        JP_HIP(hipGetLastError());
    }
};

// Two HIP events destroyed with their owner (also when a call fails between
// their creation and use).
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    EventPair() {
        JP_HIP(hipEventCreate(&a));
        hipError_t e = hipEventCreate(&b);
        if (e != hipSuccess) {
            (void)hipEventDestroy(a);
            fail(JP_EHIP, std::string("hipEventCreate failed: ") + hipGetErrorString(e));
        }
    }
    ~EventPair() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    EventPair(const EventPair &) = delete;
    EventPair &operator=(const EventPair &) = delete;
};

// Device-time phase markers (HIP events on the call's stream).
class Timeline {
  public:
    Timeline(const Ctx &c, bool on) : c_(c), on_(on) {}
    ~Timeline() {
        for (auto e : ev_) (void)hipEventDestroy(e);
    }
    int mark() {
        if (!on_) return -1;
        hipEvent_t e;
        JP_HIP(hipEventCreate(&e));
        JP_HIP(hipEventRecord(e, c_.stream));
        ev_.push_back(e);
        return (int)ev_.size() - 1;
    }
    double ms(int a, int b) const {
        if (!on_ || a < 0 || b < 0) return 0.0;
        JP_HIP(hipEventSynchronize(ev_[b]));
        float t = 0;
        JP_HIP(hipEventElapsedTime(&t, ev_[a], ev_[b]));
        return t;
    }

  private:
    const Ctx &c_;
    bool on_;
    std::vector<hipEvent_t> ev_;
};

inline int bits_for(uint64_t max_value) {  // bits needed to hold values 0..max_value
    int b = 0;
    while (b < 64 && (max_value >> b)) ++b;
    return b;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }


}  // namespace jp
