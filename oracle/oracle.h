/*
 * CPU oracle for the join-project queries.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the package smoke check and the benchmark's CPU
 * baseline leg may load this library.  It shares no code, header, table or
 * helper with the GPU library; it is deliberately plain and slow.
 *
 * What it computes is the plain definition of the query result:
 *   two-path  Q(x,z)      = { (a,c) : exists b, (a,b) in R and (c,b) in S }
 *   star      Q(x1..xk)   = { (a1..ak) : exists b, (ai,b) in Ri for all i }
 *   set similarity (overlap c) and Boolean set intersection (Section 2.1)
 * (paper, Section 2.1 problem definitions; Section 2.2 Boolean-product view),
 * evaluated the way Proposition 1 (Section 2.3) describes: enumerate the full
 * join with a worst-case optimal strategy (here: per y value, all
 * combinations), then project and remove duplicates (here: sort + unique).
 *
 * Inputs are relations given as parallel int32 columns; rows may repeat (set
 * semantics: repeats do not change the result).  Output tuples are distinct
 * and sorted ascending, lexicographically on signed int32.
 *
 * Memory: returned arrays are malloc'ed by the oracle and released with
 * orc_free().  Every function returns 0 on success, -1 on bad arguments and
 * -2 on allocation failure.
 */
#ifndef JP_ORACLE_H
#define JP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Full join size J = sum over y of deg_R(y) * deg_S(y) over the DISTINCT
 * edges of R and S (Section 5, "Indexing relations": computed in the same
 * pass as the index).  Returns J, or -1 on bad arguments. */
int64_t orc_join_size(const int32_t *r_x, const int32_t *r_y, int64_t n_r,
                      const int32_t *s_z, const int32_t *s_y, int64_t n_s);

/* Two-path join-project (Proposition 1 applied to Section 2.1's query). */
int orc_two_path(const int32_t *r_x, const int32_t *r_y, int64_t n_r,
                 const int32_t *s_z, const int32_t *s_y, int64_t n_s,
                 int32_t **out_x, int32_t **out_z, int64_t *n_out);

/* Star join-project with k relations, 1 <= k <= 8.  x[i], y[i] are the
 * columns of relation i with n[i] rows.  *out receives k*n_out int32 values
 * laid out row-major (tuple t occupies out[t*k .. t*k+k-1]). */
int orc_star(int k, const int32_t *const *x, const int32_t *const *y,
             const int64_t *n, int32_t **out, int64_t *n_out);

/* The same results computed by `nthreads` threads (OpenMP), each joining,
 * sorting and deduplicating the tuples of R (of R_1 for the star) in one
 * range of whole first-column values; the per-range results are disjoint
 * and in ascending order, so they are concatenated.  nthreads >= 1. */
int orc_two_path_par(const int32_t *r_x, const int32_t *r_y, int64_t n_r,
                     const int32_t *s_z, const int32_t *s_y, int64_t n_s, int nthreads,
                     int32_t **out_x, int32_t **out_z, int64_t *n_out);
int orc_star_par(int k, const int32_t *const *x, const int32_t *const *y,
                 const int64_t *n, int nthreads, int32_t **out, int64_t *n_out);

/* Set similarity join (Section 2.1): pairs (a, c) with
 * |{b : (a,b) in R} & {b : (c,b) in S}| >= min_c (min_c >= 1), with that
 * overlap in *out_cnt.  order 0: by (a, c); order 1: by overlap descending,
 * then (a, c).  Full join, sort, run lengths. */
int orc_ssj(const int32_t *r_x, const int32_t *r_y, int64_t n_r,
            const int32_t *s_z, const int32_t *s_y, int64_t n_s, int64_t min_c, int order,
            int32_t **out_x, int32_t **out_z, int32_t **out_cnt, int64_t *n_out);

/* Boolean set intersection (Section 2.1): answers[i] = 1 iff the sets of
 * t_x[i] in R and of t_z[i] in S intersect (answers: n_t bytes, caller's). */
int orc_bsi(const int32_t *r_x, const int32_t *r_y, int64_t n_r,
            const int32_t *s_z, const int32_t *s_y, int64_t n_s,
            const int32_t *t_x, const int32_t *t_z, int64_t n_t, uint8_t *answers);

void orc_free(void *p);

#ifdef __cplusplus
}
#endif
#endif
