/*
 * CPU oracle for the join-project queries.  TEST INFRASTRUCTURE ONLY: only
 * tests, the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * Plain C, single thread, qsort + binary search.  Nothing here is blocked,
 * fused or reordered beyond the definitions it follows:
 *   - query definitions: paper Section 2.1 (two-path and star queries);
 *   - evaluation: Proposition 1 (Section 2.3): enumerate the full join with a
 *     worst-case optimal strategy, then project and deduplicate.
 * Ids are arbitrary int32 values; ordering is signed int32 order.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

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

void orc_free(void *p) { free(p); }
