// Optional run-time validation of intermediate arrays.  With JP_CHECKS set
// in the environment every stage's index arrays are range-checked on the
// device before the next stage uses them, and a violation becomes
// JP_EINTERNAL naming the array (instead of an out-of-range access later).
// With JP_DEBUG_DUMP set, arrays of at most 64 elements are printed.
#pragma once

#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "prims.hpp"

namespace jp {

inline int &checks_flag() {
    static int on = std::getenv("JP_CHECKS") ? 1 : 0;
    return on;
}
inline bool checks_on() { return checks_flag() == 1; }
inline bool dump_on() {
    static int on = -1;
    if (on < 0) on = std::getenv("JP_DEBUG_DUMP") ? 1 : 0;
    return on == 1;
}

// Every a[i] in [lo, hi).
template <class T>
void check_range(const Ctx &c, const char *name, const T *a, int64_t n, int64_t lo, int64_t hi) {
    if (!checks_on() || n <= 0) return;
    DBuf<unsigned long long> bad = c.buf<unsigned long long>(1);
    unsigned long long *b = bad.get();
    c.zero(b, 1);
    for_each(c, n, [=] __device__(int64_t i) {
        int64_t v = (int64_t)a[i];
        if (v < lo || v >= hi) atomicAdd(b, 1ull);
    });
    unsigned long long nb = c.load(b);
    if (nb) fail(JP_EINTERNAL, std::string("check failed: ") + name + " has " + std::to_string(nb) +
                                    " values outside [" + std::to_string(lo) + "," + std::to_string(hi) + ")");
}

// a nondecreasing, a[0] == first, a[n-1] == last (last < 0: not checked).
template <class T>
void check_monotone(const Ctx &c, const char *name, const T *a, int64_t n, int64_t first, int64_t last) {
    if (!checks_on() || n <= 0) return;
    DBuf<unsigned long long> bad = c.buf<unsigned long long>(1);
    unsigned long long *b = bad.get();
    c.zero(b, 1);
    for_each(c, n, [=] __device__(int64_t i) {
        bool ok = (i == 0) ? ((int64_t)a[0] == first) : (a[i - 1] <= a[i]);
        if (i == n - 1 && last >= 0 && (int64_t)a[i] != last) ok = false;
        if (!ok) atomicAdd(b, 1ull);
    });
    unsigned long long nb = c.load(b);
    if (nb) fail(JP_EINTERNAL, std::string("check failed: ") + name + " is not monotone with the expected ends");
}

template <class T>
void dump(const Ctx &c, const char *name, const T *a, int64_t n) {
    if (!dump_on() || n > 64) return;
    std::vector<T> h((size_t)std::max<int64_t>(n, 1));
    c.load_n(h.data(), a, (size_t)n);
    std::fprintf(stderr, "[jp] %s[%lld] =", name, (long long)n);
    for (int64_t i = 0; i < n; ++i) std::fprintf(stderr, " %lld", (long long)h[i]);
    std::fprintf(stderr, "\n");
}

}  // namespace jp
