// Per-x duplicate removal of light witnesses + heavy nonzeros (dedup.hip).
#pragma once

#include <climits>

#include "common.hpp"

namespace jp {

struct SegDedupIn {
    int64_t dom_x = 0, dom_z = 0;
    int bz = 0;                      // bits of a z rank
    const int64_t *off_x = nullptr;  // R tuples of every x (dom_x + 1)
    const int64_t *eoff = nullptr;   // light candidate offsets of every R tuple (n_e + 1)
    const int64_t *lbase = nullptr;  // list start of every R tuple in zlist
    const int32_t *r_xr = nullptr;   // x rank of every R tuple
    const int32_t *zlist = nullptr;  // concatenated z-rank lists
    int64_t zlist_n = 0;             // their total length (below 2^32)
    const uint64_t *hkeys = nullptr; // sorted heavy nonzeros (x << bz | z)
    int64_t nnz = 0;
    const int32_t *xorig = nullptr, *zorig = nullptr;
    // When every id in [min, max] occurs, rank r is id min + r: the bases
    // replace the table lookups (INT64_MIN: use the tables).
    int64_t x_dense_base = INT64_MIN, z_dense_base = INT64_MIN;
};

struct SegDedupStats {
    int64_t n_units = 0, n_small = 0, n_big = 0, n_cand = 0;
    double ms_kernel = 0;  // the dedup kernel alone (when timed)
};

// Whether z ranks of `bz` bits leave room for the local x index in 32 bits.
bool segmented_dedup_fits(int bz);

// Sorted distinct (x, z) output (original ids) into out_x / out_z.
void segmented_dedup(const Ctx &c, const SegDedupIn &in, DBuf<int32_t> *out_x, DBuf<int32_t> *out_z,
                     int64_t *n_out, SegDedupStats *stats, bool timing = false);

}  // namespace jp
