// Test hooks: the device primitives behind a C entry point each.
#include "../../include/jp_testing.h"
#include "debug.hpp"
#include "pipeline.hpp"
#include "prims.hpp"

jp::Ctx jp_handle_ctx(jp_handle *h);
jp_status jp_handle_guard(jp_handle *h, void (*fn)(void *), void *arg);
void jp_handle_set_lookback_wait(jp_handle *h, int64_t ticks);

namespace {
template <class K>
struct SortArgs {
    jp_handle *h;
    K *keys;
    int64_t n;
    int bits;
};
template <class K>
void do_sort(void *p) {
    auto *a = (SortArgs<K> *)p;
    jp::Ctx c = jp_handle_ctx(a->h);
    jp::DBuf<K> tmp = c.buf<K>((size_t)std::max<int64_t>(a->n, 1));
    K *r = jp::radix_sort(c, a->keys, tmp.get(), a->n, a->bits);
    if (r != a->keys && a->n > 0)
        JP_HIP(hipMemcpyAsync(a->keys, r, a->n * sizeof(K), hipMemcpyDeviceToDevice, c.stream));
    c.sync();
}
struct ScanArgs {
    jp_handle *h;
    const int64_t *in;
    int64_t *out;
    int64_t n;
    int64_t total;
};
void do_scan(void *p) {
    auto *a = (ScanArgs *)p;
    jp::Ctx c = jp_handle_ctx(a->h);
    jp::DBuf<int64_t> t = c.buf<int64_t>(1);
    jp::scan_exclusive(c, a->n, jp::ArrayGet{a->in}, jp::ArrayPut{a->out}, t.get());
    a->total = c.load(t.get());
}
struct UniqArgs {
    jp_handle *h;
    const uint64_t *in;
    uint64_t *out;
    int64_t n;
    int64_t n_out;
};
void do_unique(void *p) {
    auto *a = (UniqArgs *)p;
    jp::Ctx c = jp_handle_ctx(a->h);
    jp::DBuf<int64_t> t = c.buf<int64_t>(1);
    const uint64_t *s = a->in;
    uint64_t *d = a->out;
    jp::compact(
        c, a->n, [=] __device__(int64_t i) { return i == 0 || s[i] != s[i - 1]; },
        [=] __device__(int64_t i, int64_t q) { d[q] = s[i]; }, t.get());
    a->n_out = c.load(t.get());
}
}  // namespace

extern "C" {
jp_status jp_test_radix_sort_u64(jp_handle *h, uint64_t *keys, int64_t n, int32_t bits) {
    if (!h || n < 0 || (n && !keys) || bits < 0 || bits > 64) return JP_EINVAL;
    SortArgs<uint64_t> a{h, keys, n, bits};
    return jp_handle_guard(h, do_sort<uint64_t>, &a);
}
jp_status jp_test_radix_sort_u32(jp_handle *h, uint32_t *keys, int64_t n, int32_t bits) {
    if (!h || n < 0 || (n && !keys) || bits < 0 || bits > 32) return JP_EINVAL;
    SortArgs<uint32_t> a{h, keys, n, bits};
    return jp_handle_guard(h, do_sort<uint32_t>, &a);
}
jp_status jp_test_radix_sort_u128(jp_handle *h, uint64_t *keys, int64_t n, int32_t bits) {
    if (!h || n < 0 || (n && !keys) || bits < 0 || bits > 128 || ((uintptr_t)keys & 15)) return JP_EINVAL;
    SortArgs<unsigned __int128> a{h, (unsigned __int128 *)keys, n, bits};
    return jp_handle_guard(h, do_sort<unsigned __int128>, &a);
}
jp_status jp_test_exclusive_scan(jp_handle *h, const int64_t *in, int64_t *out, int64_t n, int64_t *total) {
    if (!h || n < 0 || (n && (!in || !out)) || !total) return JP_EINVAL;
    ScanArgs a{h, in, out, n, 0};
    jp_status st = jp_handle_guard(h, do_scan, &a);
    *total = a.total;
    return st;
}
jp_status jp_test_set_lookback_wait(jp_handle *h, int64_t ticks) {
    if (!h || ticks < 0) return JP_EINVAL;
    jp_handle_set_lookback_wait(h, ticks);
    return JP_OK;
}
int32_t jp_test_set_checks(int32_t on) {
    const int32_t prev = jp::checks_flag();
    jp::checks_flag() = on ? 1 : 0;
    return prev;
}
int32_t jp_test_set_wide_overlap_keys(int32_t on) {
    const int32_t prev = jp::wide_overlap_keys_flag();
    jp::wide_overlap_keys_flag() = on ? 1 : 0;
    return prev;
}
jp_status jp_test_unique_u64(jp_handle *h, const uint64_t *in, int64_t n, uint64_t *out, int64_t *n_out) {
    if (!h || n < 0 || (n && (!in || !out)) || !n_out) return JP_EINVAL;
    UniqArgs a{h, in, out, n, 0};
    jp_status st = jp_handle_guard(h, do_unique, &a);
    *n_out = a.n_out;
    return st;
}
}
