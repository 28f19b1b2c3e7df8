/*
 * CPU oracle for the join-project queries.  TEST INFRASTRUCTURE ONLY: only
 * tests, the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * Plain C, qsort + binary search, one thread (the *_par variants at the end
 * split the same computation by first-column ranges over OpenMP threads).
 * Nothing here is blocked, fused or reordered beyond the definitions it
 * follows:
 *   - query definitions: paper Section 2.1 (two-path and star queries);
 *   - evaluation: Proposition 1 (Section 2.3): enumerate the full join with a
 *     worst-case optimal strategy, then project and deduplicate.
 * Ids are arbitrary int32 values; ordering is signed int32 order.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    uint32_t y; /* join value, biased so unsigned order == signed order */
    uint32_t v; /* free value (x or z), biased likewise */
} orc_pair;

static uint32_t bias(int32_t v) { return (uint32_t)v ^ 0x80000000u; }
static int32_t unbias(uint32_t u) { return (int32_t)(u ^ 0x80000000u); }

static int cmp_pair(const void *a, const void *b)
{
    const orc_pair *p = (const orc_pair *)a, *q = (const orc_pair *)b;
    if (p->y != q->y) return p->y < q->y ? -1 : 1;
    if (p->v != q->v) return p->v < q->v ? -1 : 1;
    return 0;
}

static int cmp_pair_by_v(const void *a, const void *b);

static int cmp_u64(const void *a, const void *b)
{
    uint64_t p = *(const uint64_t *)a, q = *(const uint64_t *)b;
    return (p > q) - (p < q);
}

/* Relation as distinct (y, v) pairs sorted by y then v: the y-indexed copy
 * of the relation (Section 5, "Indexing relations"). */
static orc_pair *index_by_y(const int32_t *v, const int32_t *y, int64_t n, int64_t *n_distinct)
{
    orc_pair *p = (orc_pair *)malloc((size_t)(n > 0 ? n : 1) * sizeof(orc_pair));
    if (!p) return NULL;
    for (int64_t i = 0; i < n; ++i) {
        p[i].y = bias(y[i]);
        p[i].v = bias(v[i]);
    }
    qsort(p, (size_t)n, sizeof(orc_pair), cmp_pair);
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (m == 0 || cmp_pair(&p[m - 1], &p[i]) != 0) p[m++] = p[i];
    *n_distinct = m;
    return p;
}

/* First index in p[0..n) whose y is >= key. */
static int64_t lower_y(const orc_pair *p, int64_t n, uint32_t key)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (p[mid].y < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

int64_t orc_join_size(const int32_t *r_x, const int32_t *r_y, int64_t n_r,
                      const int32_t *s_z, const int32_t *s_y, int64_t n_s)
{
    if (n_r < 0 || n_s < 0 || (n_r && (!r_x || !r_y)) || (n_s && (!s_z || !s_y))) return -1;
    int64_t nr, ns;
    orc_pair *R = index_by_y(r_x, r_y, n_r, &nr);
    orc_pair *S = index_by_y(s_z, s_y, n_s, &ns);
    if (!R || !S) { free(R); free(S); return -1; }
    int64_t J = 0;
    for (int64_t i = 0; i < nr; ++i) {
        int64_t lo = lower_y(S, ns, R[i].y);
        int64_t hi = lo;
        while (hi < ns && S[hi].y == R[i].y) ++hi;
        J += hi - lo;
    }
    free(R);
    free(S);
    return J;
}

int orc_two_path(const int32_t *r_x, const int32_t *r_y, int64_t n_r,
                 const int32_t *s_z, const int32_t *s_y, int64_t n_s,
                 int32_t **out_x, int32_t **out_z, int64_t *n_out)
{
    if (!out_x || !out_z || !n_out || n_r < 0 || n_s < 0) return -1;
    if ((n_r && (!r_x || !r_y)) || (n_s && (!s_z || !s_y))) return -1;
    *out_x = *out_z = NULL;
    *n_out = 0;

    int64_t nr, ns;
    orc_pair *R = index_by_y(r_x, r_y, n_r, &nr);
    orc_pair *S = index_by_y(s_z, s_y, n_s, &ns);
    if (!R || !S) { free(R); free(S); return -2; }

    /* Full join size first, so the witness buffer is allocated once. */
    int64_t J = 0;
    for (int64_t i = 0; i < nr; ++i) {
        int64_t lo = lower_y(S, ns, R[i].y), hi = lo;
        while (hi < ns && S[hi].y == R[i].y) ++hi;
        J += hi - lo;
    }

    /* Full join: every (a,b) in R meets every (c,b) in S; keep (a,c). */
    uint64_t *key = (uint64_t *)malloc((size_t)(J > 0 ? J : 1) * sizeof(uint64_t));
    if (!key) { free(R); free(S); return -2; }
    int64_t w = 0;
    for (int64_t i = 0; i < nr; ++i) {
        int64_t j = lower_y(S, ns, R[i].y);
        for (; j < ns && S[j].y == R[i].y; ++j)
            key[w++] = ((uint64_t)R[i].v << 32) | (uint64_t)S[j].v;
    }
    free(R);
    free(S);

    /* Projection with duplicate removal: sort, keep first of each run. */
    qsort(key, (size_t)w, sizeof(uint64_t), cmp_u64);
    int64_t m = 0;
    for (int64_t i = 0; i < w; ++i)
        if (m == 0 || key[m - 1] != key[i]) key[m++] = key[i];

    int32_t *ox = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int32_t *oz = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    if (!ox || !oz) { free(ox); free(oz); free(key); return -2; }
    for (int64_t i = 0; i < m; ++i) {
        ox[i] = unbias((uint32_t)(key[i] >> 32));
        oz[i] = unbias((uint32_t)(key[i] & 0xffffffffu));
    }
    free(key);
    *out_x = ox;
    *out_z = oz;
    *n_out = m;
    return 0;
}

/* Tuples of width g_k compared lexicographically (biased uint32 words). */
static int g_k;
static int cmp_tuple(const void *a, const void *b)
{
    const uint32_t *p = (const uint32_t *)a, *q = (const uint32_t *)b;
    for (int i = 0; i < g_k; ++i)
        if (p[i] != q[i]) return p[i] < q[i] ? -1 : 1;
    return 0;
}

int orc_star(int k, const int32_t *const *x, const int32_t *const *y,
             const int64_t *n, int32_t **out, int64_t *n_out)
{
    if (k < 1 || k > 8 || !x || !y || !n || !out || !n_out) return -1;
    for (int i = 0; i < k; ++i)
        if (n[i] < 0 || (n[i] && (!x[i] || !y[i]))) return -1;
    *out = NULL;
    *n_out = 0;

    orc_pair *Rel[8] = {0};
    int64_t nd[8] = {0};
    int rc = 0;
    for (int i = 0; i < k; ++i) {
        Rel[i] = index_by_y(x[i], y[i], n[i], &nd[i]);
        if (!Rel[i]) rc = -2;
    }
    uint32_t *tup = NULL;
    if (rc) goto done;

    /* Per join value b present in every relation, the full join contributes
     * the Cartesian product of the k neighbour lists of b. */
    int64_t J = 0;
    for (int64_t i = 0; i < nd[0];) {
        uint32_t b = Rel[0][i].y;
        int64_t i2 = i;
        while (i2 < nd[0] && Rel[0][i2].y == b) ++i2;
        int64_t prod = i2 - i;
        for (int r = 1; r < k && prod; ++r) {
            int64_t lo = lower_y(Rel[r], nd[r], b), hi = lo;
            while (hi < nd[r] && Rel[r][hi].y == b) ++hi;
            prod *= hi - lo;
        }
        J += prod;
        i = i2;
    }
    tup = (uint32_t *)malloc((size_t)(J > 0 ? J : 1) * (size_t)k * sizeof(uint32_t));
    if (!tup) { rc = -2; goto done; }

    int64_t w = 0;
    for (int64_t i = 0; i < nd[0];) {
        uint32_t b = Rel[0][i].y;
        int64_t lo[8], hi[8];
        lo[0] = i;
        hi[0] = i;
        while (hi[0] < nd[0] && Rel[0][hi[0]].y == b) ++hi[0];
        int empty = 0;
        for (int r = 1; r < k; ++r) {
            lo[r] = lower_y(Rel[r], nd[r], b);
            hi[r] = lo[r];
            while (hi[r] < nd[r] && Rel[r][hi[r]].y == b) ++hi[r];
            if (hi[r] == lo[r]) empty = 1;
        }
        if (!empty) {
            int64_t cur[8];
            for (int r = 0; r < k; ++r) cur[r] = lo[r];
            for (;;) {
                for (int r = 0; r < k; ++r) tup[w * k + r] = Rel[r][cur[r]].v;
                ++w;
                int r = k - 1;
                while (r >= 0 && ++cur[r] == hi[r]) { cur[r] = lo[r]; --r; }
                if (r < 0) break;
            }
        }
        i = hi[0];
    }

    g_k = k;
    qsort(tup, (size_t)w, (size_t)k * sizeof(uint32_t), cmp_tuple);
    int64_t m = 0;
    for (int64_t t = 0; t < w; ++t) {
        if (m == 0 || cmp_tuple(&tup[(m - 1) * k], &tup[t * k]) != 0) {
            if (m != t) memcpy(&tup[m * k], &tup[t * k], (size_t)k * sizeof(uint32_t));
            ++m;
        }
    }
    int32_t *o = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * (size_t)k * sizeof(int32_t));
    if (!o) { rc = -2; goto done; }
    for (int64_t t = 0; t < m * k; ++t) o[t] = unbias(tup[t]);
    *out = o;
    *n_out = m;

done:
    free(tup);
    for (int i = 0; i < k; ++i) free(Rel[i]);
    return rc;
}

/* ------------------------------------------------------------------------
 * Set similarity join (Section 2.1, "Set Similarity"): the pairs (a, c)
 * whose sets N_R(a) = {b : (a,b) in R} and N_S(c) share at least min_c
 * elements, each with its overlap |N_R(a) & N_S(c)|.  Evaluated as the full
 * join followed by sorting: over distinct edges every element b common to
 * both sets is exactly one witness (a, b, c), so the length of the run of
 * the key (a, c) in the sorted witness list is the overlap.  order = 0:
 * pairs ascending by (a, c); order = 1 (the ordered variant): by overlap
 * descending, ties by (a, c) ascending.
 * ------------------------------------------------------------------------ */

typedef struct {
    uint64_t key; /* biased (a, c) */
    int64_t cnt;
} orc_counted;

static int cmp_counted_desc(const void *a, const void *b)
{
    const orc_counted *p = (const orc_counted *)a, *q = (const orc_counted *)b;
    if (p->cnt != q->cnt) return p->cnt > q->cnt ? -1 : 1;
    return (p->key > q->key) - (p->key < q->key);
}

int orc_ssj(const int32_t *r_x, const int32_t *r_y, int64_t n_r,
            const int32_t *s_z, const int32_t *s_y, int64_t n_s, int64_t min_c, int order,
            int32_t **out_x, int32_t **out_z, int32_t **out_cnt, int64_t *n_out)
{
    if (!out_x || !out_z || !out_cnt || !n_out || n_r < 0 || n_s < 0 || min_c < 1) return -1;
    if ((n_r && (!r_x || !r_y)) || (n_s && (!s_z || !s_y)) || (order != 0 && order != 1)) return -1;
    *out_x = *out_z = *out_cnt = NULL;
    *n_out = 0;
    int64_t nr, ns;
    orc_pair *R = index_by_y(r_x, r_y, n_r, &nr);
    orc_pair *S = index_by_y(s_z, s_y, n_s, &ns);
    if (!R || !S) { free(R); free(S); return -2; }
    int64_t J = 0;
    for (int64_t i = 0; i < nr; ++i) {
        int64_t lo = lower_y(S, ns, R[i].y), hi = lo;
        while (hi < ns && S[hi].y == R[i].y) ++hi;
        J += hi - lo;
    }
    uint64_t *key = (uint64_t *)malloc((size_t)(J > 0 ? J : 1) * sizeof(uint64_t));
    if (!key) { free(R); free(S); return -2; }
    int64_t w = 0;
    for (int64_t i = 0; i < nr; ++i)
        for (int64_t j = lower_y(S, ns, R[i].y); j < ns && S[j].y == R[i].y; ++j)
            key[w++] = ((uint64_t)R[i].v << 32) | (uint64_t)S[j].v;
    free(R);
    free(S);
    qsort(key, (size_t)w, sizeof(uint64_t), cmp_u64);

    /* run lengths of equal keys, filtered by the overlap threshold */
    orc_counted *res = (orc_counted *)malloc((size_t)(w > 0 ? w : 1) * sizeof(orc_counted));
    if (!res) { free(key); return -2; }
    int64_t m = 0;
    for (int64_t i = 0; i < w;) {
        int64_t j = i;
        while (j < w && key[j] == key[i]) ++j;
        if (j - i >= min_c) {
            res[m].key = key[i];
            res[m].cnt = j - i;
            ++m;
        }
        i = j;
    }
    free(key);
    if (order == 1) qsort(res, (size_t)m, sizeof(orc_counted), cmp_counted_desc);
    int32_t *ox = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int32_t *oz = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int32_t *oc = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    if (!ox || !oz || !oc) { free(ox); free(oz); free(oc); free(res); return -2; }
    for (int64_t i = 0; i < m; ++i) {
        ox[i] = unbias((uint32_t)(res[i].key >> 32));
        oz[i] = unbias((uint32_t)(res[i].key & 0xffffffffu));
        oc[i] = (int32_t)res[i].cnt;
    }
    free(res);
    *out_x = ox;
    *out_z = oz;
    *out_cnt = oc;
    *n_out = m;
    return 0;
}

/* ------------------------------------------------------------------------
 * Boolean set intersection (Section 2.1, "Boolean Set Intersection"; the
 * batched workload of Section 3.3): for every query i, answers[i] = 1 when
 * the sets N_R(t_x[i]) and N_S(t_z[i]) have a common element, else 0.  Each
 * query is answered on its own by a merge of the two sorted sets.
 * ------------------------------------------------------------------------ */

/* First index in p[0..n) whose v is >= key (p sorted by (v, y)). */
static int64_t lower_v(const orc_pair *p, int64_t n, uint32_t key)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (p[mid].v < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

int orc_bsi(const int32_t *r_x, const int32_t *r_y, int64_t n_r,
            const int32_t *s_z, const int32_t *s_y, int64_t n_s,
            const int32_t *t_x, const int32_t *t_z, int64_t n_t, uint8_t *answers)
{
    if (n_r < 0 || n_s < 0 || n_t < 0 || (n_t && (!t_x || !t_z || !answers))) return -1;
    if ((n_r && (!r_x || !r_y)) || (n_s && (!s_z || !s_y))) return -1;
    /* both relations sorted by their set id, then element */
    orc_pair *R = (orc_pair *)malloc((size_t)(n_r > 0 ? n_r : 1) * sizeof(orc_pair));
    orc_pair *S = (orc_pair *)malloc((size_t)(n_s > 0 ? n_s : 1) * sizeof(orc_pair));
    if (!R || !S) { free(R); free(S); return -2; }
    for (int64_t i = 0; i < n_r; ++i) { R[i].v = bias(r_x[i]); R[i].y = bias(r_y[i]); }
    for (int64_t i = 0; i < n_s; ++i) { S[i].v = bias(s_z[i]); S[i].y = bias(s_y[i]); }
    qsort(R, (size_t)n_r, sizeof(orc_pair), cmp_pair_by_v);
    qsort(S, (size_t)n_s, sizeof(orc_pair), cmp_pair_by_v);
    for (int64_t q = 0; q < n_t; ++q) {
        const uint32_t a = bias(t_x[q]), c = bias(t_z[q]);
        int64_t i = lower_v(R, n_r, a), j = lower_v(S, n_s, c);
        uint8_t hit = 0;
        while (!hit && i < n_r && j < n_s && R[i].v == a && S[j].v == c) {
            if (R[i].y == S[j].y) hit = 1;
            else if (R[i].y < S[j].y) ++i;
            else ++j;
        }
        answers[q] = hit;
    }
    free(R);
    free(S);
    return 0;
}

/* ------------------------------------------------------------------------
 * Multi-threaded variants (timed CPU baseline, and the check of full-size
 * outputs).  The result is the same set, computed the same way, split by the
 * value of the first output column: R (R_1 for the star) is sorted by that
 * value, cut into ranges of whole values, and each range is joined, sorted
 * and deduplicated on its own by one OpenMP thread.  Output tuples with
 * different first values never coincide and the ranges are in ascending
 * order, so concatenating the per-range results gives the sorted distinct
 * output (Section 2.1: an output tuple's first value comes from R).
 * ------------------------------------------------------------------------ */

static int cmp_pair_by_v(const void *a, const void *b)
{
    const orc_pair *p = (const orc_pair *)a, *q = (const orc_pair *)b;
    if (p->v != q->v) return p->v < q->v ? -1 : 1;
    if (p->y != q->y) return p->y < q->y ? -1 : 1;
    return 0;
}

/* Distinct rows of a relation sorted by (v, y); cut points of `nchunk`
 * ranges of whole v values into cut[0..nchunk]. */
static orc_pair *by_value_chunks(const int32_t *v, const int32_t *y, int64_t n, int64_t *nd, int nchunk,
                                 int64_t *cut)
{
    orc_pair *p = (orc_pair *)malloc((size_t)(n > 0 ? n : 1) * sizeof(orc_pair));
    if (!p) return NULL;
    for (int64_t i = 0; i < n; ++i) {
        p[i].y = bias(y[i]);
        p[i].v = bias(v[i]);
    }
    qsort(p, (size_t)n, sizeof(orc_pair), cmp_pair_by_v);
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (m == 0 || cmp_pair_by_v(&p[m - 1], &p[i]) != 0) p[m++] = p[i];
    *nd = m;
    cut[0] = 0;
    for (int c = 1; c < nchunk; ++c) {
        int64_t at = m * c / nchunk;
        if (at < cut[c - 1]) at = cut[c - 1];
        while (at > cut[c - 1] && at < m && p[at].v == p[at - 1].v) ++at;
        cut[c] = at;
    }
    cut[nchunk] = m;
    return p;
}

static int chunks_for(int nthreads) { return nthreads > 1 ? 8 * nthreads : 1; }

int orc_two_path_par(const int32_t *r_x, const int32_t *r_y, int64_t n_r,
                     const int32_t *s_z, const int32_t *s_y, int64_t n_s, int nthreads,
                     int32_t **out_x, int32_t **out_z, int64_t *n_out)
{
    if (!out_x || !out_z || !n_out || n_r < 0 || n_s < 0 || nthreads < 1) return -1;
    if ((n_r && (!r_x || !r_y)) || (n_s && (!s_z || !s_y))) return -1;
    *out_x = *out_z = NULL;
    *n_out = 0;
    const int nchunk = chunks_for(nthreads);
    int64_t *cut = (int64_t *)malloc((size_t)(nchunk + 1) * sizeof(int64_t));
    uint64_t **ck = (uint64_t **)calloc((size_t)nchunk, sizeof(uint64_t *));
    int64_t *cm = (int64_t *)calloc((size_t)nchunk + 1, sizeof(int64_t));
    int64_t nr, ns;
    orc_pair *R = NULL, *S = NULL;
    int rc = 0;
    if (!cut || !ck || !cm) { rc = -2; goto done; }
    R = by_value_chunks(r_x, r_y, n_r, &nr, nchunk, cut);
    S = index_by_y(s_z, s_y, n_s, &ns);
    if (!R || !S) { rc = -2; goto done; }

#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int c = 0; c < nchunk; ++c) {
        int64_t J = 0;
        for (int64_t i = cut[c]; i < cut[c + 1]; ++i) {
            int64_t lo = lower_y(S, ns, R[i].y), hi = lo;
            while (hi < ns && S[hi].y == R[i].y) ++hi;
            J += hi - lo;
        }
        uint64_t *key = (uint64_t *)malloc((size_t)(J > 0 ? J : 1) * sizeof(uint64_t));
        if (!key) { cm[c] = -1; continue; }
        int64_t w = 0;
        for (int64_t i = cut[c]; i < cut[c + 1]; ++i)
            for (int64_t j = lower_y(S, ns, R[i].y); j < ns && S[j].y == R[i].y; ++j)
                key[w++] = ((uint64_t)R[i].v << 32) | (uint64_t)S[j].v;
        qsort(key, (size_t)w, sizeof(uint64_t), cmp_u64);
        int64_t m = 0;
        for (int64_t i = 0; i < w; ++i)
            if (m == 0 || key[m - 1] != key[i]) key[m++] = key[i];
        ck[c] = key;
        cm[c] = m;
    }

    int64_t total = 0;
    for (int c = 0; c < nchunk; ++c) {
        if (cm[c] < 0) { rc = -2; goto done; }
        total += cm[c];
    }
    int32_t *ox = (int32_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
    int32_t *oz = (int32_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
    if (!ox || !oz) { free(ox); free(oz); rc = -2; goto done; }
    int64_t at = 0;
    for (int c = 0; c < nchunk; ++c)
        for (int64_t i = 0; i < cm[c]; ++i, ++at) {
            ox[at] = unbias((uint32_t)(ck[c][i] >> 32));
            oz[at] = unbias((uint32_t)(ck[c][i] & 0xffffffffu));
        }
    *out_x = ox;
    *out_z = oz;
    *n_out = total;

done:
    if (ck)
        for (int c = 0; c < nchunk; ++c) free(ck[c]);
    free(ck);
    free(cm);
    free(cut);
    free(R);
    free(S);
    return rc;
}

int orc_star_par(int k, const int32_t *const *x, const int32_t *const *y,
                 const int64_t *n, int nthreads, int32_t **out, int64_t *n_out)
{
    if (k < 1 || k > 8 || !x || !y || !n || !out || !n_out || nthreads < 1) return -1;
    for (int i = 0; i < k; ++i)
        if (n[i] < 0 || (n[i] && (!x[i] || !y[i]))) return -1;
    *out = NULL;
    *n_out = 0;
    const int nchunk = chunks_for(nthreads);
    int64_t *cut = (int64_t *)malloc((size_t)(nchunk + 1) * sizeof(int64_t));
    uint32_t **ck = (uint32_t **)calloc((size_t)nchunk, sizeof(uint32_t *));
    int64_t *cm = (int64_t *)calloc((size_t)nchunk + 1, sizeof(int64_t));
    orc_pair *Rel[8] = {0};
    int64_t nd[8] = {0};
    int rc = 0;
    if (!cut || !ck || !cm) { rc = -2; goto done; }
    /* relation 1 by its free value (chunked), the others by y */
    Rel[0] = by_value_chunks(x[0], y[0], n[0], &nd[0], nchunk, cut);
    if (!Rel[0]) rc = -2;
    for (int i = 1; i < k; ++i) {
        Rel[i] = index_by_y(x[i], y[i], n[i], &nd[i]);
        if (!Rel[i]) rc = -2;
    }
    if (rc) goto done;
    g_k = k; /* read-only below */

#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int c = 0; c < nchunk; ++c) {
        /* Per tuple (a, b) of relation 1, every combination of the other
         * relations' neighbour lists of b. */
        int64_t J = 0;
        for (int64_t i = cut[c]; i < cut[c + 1]; ++i) {
            int64_t prod = 1;
            for (int r = 1; r < k && prod; ++r) {
                int64_t lo = lower_y(Rel[r], nd[r], Rel[0][i].y), hi = lo;
                while (hi < nd[r] && Rel[r][hi].y == Rel[0][i].y) ++hi;
                prod *= hi - lo;
            }
            J += prod;
        }
        uint32_t *tup = (uint32_t *)malloc((size_t)(J > 0 ? J : 1) * (size_t)k * sizeof(uint32_t));
        if (!tup) { cm[c] = -1; continue; }
        int64_t w = 0;
        for (int64_t i = cut[c]; i < cut[c + 1]; ++i) {
            const uint32_t b = Rel[0][i].y;
            int64_t lo[8], hi[8], cur[8];
            int empty = 0;
            for (int r = 1; r < k; ++r) {
                lo[r] = lower_y(Rel[r], nd[r], b);
                hi[r] = lo[r];
                while (hi[r] < nd[r] && Rel[r][hi[r]].y == b) ++hi[r];
                if (hi[r] == lo[r]) empty = 1;
                cur[r] = lo[r];
            }
            if (empty) continue;
            for (;;) {
                tup[w * k] = Rel[0][i].v;
                for (int r = 1; r < k; ++r) tup[w * k + r] = Rel[r][cur[r]].v;
                ++w;
                int r = k - 1;
                while (r >= 1 && ++cur[r] == hi[r]) { cur[r] = lo[r]; --r; }
                if (r < 1) break;
            }
        }
        qsort(tup, (size_t)w, (size_t)k * sizeof(uint32_t), cmp_tuple);
        int64_t m = 0;
        for (int64_t t = 0; t < w; ++t) {
            if (m == 0 || cmp_tuple(&tup[(m - 1) * k], &tup[t * k]) != 0) {
                if (m != t) memcpy(&tup[m * k], &tup[t * k], (size_t)k * sizeof(uint32_t));
                ++m;
            }
        }
        ck[c] = tup;
        cm[c] = m;
    }

    int64_t total = 0;
    for (int c = 0; c < nchunk; ++c) {
        if (cm[c] < 0) { rc = -2; goto done; }
        total += cm[c];
    }
    int32_t *o = (int32_t *)malloc((size_t)(total > 0 ? total : 1) * (size_t)k * sizeof(int32_t));
    if (!o) { rc = -2; goto done; }
    int64_t at = 0;
    for (int c = 0; c < nchunk; ++c)
        for (int64_t t = 0; t < cm[c] * k; ++t) o[at++] = unbias(ck[c][t]);
    *out = o;
    *n_out = total;

done:
    if (ck)
        for (int c = 0; c < nchunk; ++c) free(ck[c]);
    free(ck);
    free(cm);
    free(cut);
    for (int i = 0; i < k; ++i) free(Rel[i]);
    return rc;
}

void orc_free(void *p) { free(p); }
