/*
 * jp_testing.h: test hooks of libjoinproject.  The device-wide primitives
 * that the join-project pipelines are built from, exposed one by one so each
 * can be checked against a plain host computation.  Not part of the stable
 * ABI.  All pointers are device pointers on the handle's device; work is
 * ordered on the handle's stream and the call waits for it.  Status codes as
 * in jp.h.
 */
#ifndef JP_TESTING_H
#define JP_TESTING_H

#include "jp.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Stable LSD radix sort of n keys on their low `bits` bits, in place. */
jp_status jp_test_radix_sort_u64(jp_handle *h, uint64_t *keys, int64_t n, int32_t bits);
jp_status jp_test_radix_sort_u32(jp_handle *h, uint32_t *keys, int64_t n, int32_t bits);
/* 128-bit keys as (low, high) 64-bit word pairs, 16-byte aligned; bits <= 128. */
jp_status jp_test_radix_sort_u128(jp_handle *h, uint64_t *keys, int64_t n, int32_t bits);

/* out[i] = in[0] + ... + in[i-1]; *total (host) = sum of all n values. */
jp_status jp_test_exclusive_scan(jp_handle *h, const int64_t *in, int64_t *out, int64_t n, int64_t *total);

/* Single-pass scans and compactions (every pipeline uses them) let a tile
 * wait for a predecessor tile's published status for at most `ticks` of the
 * device wall clock (hipDeviceAttributeWallClockRate; default 100 us), after
 * which the waiting wave computes that tile's sum from the input itself.
 * ticks = 0 makes every such wait fall back at once, so tests can check the
 * fallback.  Applies to later calls on h; results are the same at any value.
 * JP_EINVAL for a null handle or negative ticks. */
jp_status jp_test_set_lookback_wait(jp_handle *h, int64_t ticks);

/* Stage-by-stage validation of intermediate index arrays (process-wide; the
 * JP_CHECKS environment variable sets the initial value): on = 1 checks every
 * stage's index arrays on the device and turns a violation into
 * JP_EINTERNAL, on = 0 runs the pipelines as shipped.  Returns the previous
 * setting (0 or 1). */
int32_t jp_test_set_checks(int32_t on);

/* jp_ssj builds 64-bit candidate and order keys when the pair ranks and the
 * counts fit in 64 bits, else 128-bit keys.  on = 1 makes later calls use
 * 128-bit keys always (process-wide), so tests reach that path on small
 * inputs.  Returns the previous setting. */
int32_t jp_test_set_wide_overlap_keys(int32_t on);

/* Keeps the first of every run of equal adjacent keys, in order; *n_out (host). */
jp_status jp_test_unique_u64(jp_handle *h, const uint64_t *in, int64_t n, uint64_t *out, int64_t *n_out);

#ifdef __cplusplus
}
#endif
#endif /* JP_TESTING_H */
