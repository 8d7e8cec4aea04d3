/*
 * C oracle for the exact RNG / GRNG at large N -- TEST INFRASTRUCTURE ONLY.
 * Loaded by tests/ and by bench.py's cpu_baseline leg through ctypes; never
 * linked into or called by the product library, and shares no code with it.
 *
 * Inputs are integer grid coordinates (int32, |k| < 2^24) so squared
 * distances are exact int64 values and every comparison is the exact one.
 *
 * RNG (Section 1, the RNG definition equation): u, v linked iff no other z has
 * max(d(u,z), d(v,z)) < d(u,v).  The row of a point x is decided by brute
 * force over the definition: any witness z of the pair (x, y) satisfies
 * d(x,z) < d(x,y), so after sorting all points by their distance to x the
 * witnesses of (x, y) all lie in the prefix of points strictly closer to x
 * than y.  Each pair scans that whole prefix (stopping at the first witness),
 * so nothing is pruned beyond what the definition itself excludes.
 *
 * GRNG (Section 2, Definition 1): pivots i, j linked iff no pivot k has
 * d(k,i) < d(i,j) - (2 r_i + r_j) and d(k,j) < d(i,j) - (r_i + 2 r_j),
 * decided exactly with 128-bit integers.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t d2;
    int64_t idx;
} okey;

static int okey_cmp(const void *a, const void *b)
{
    const okey *x = (const okey *)a, *y = (const okey *)b;
    if (x->d2 != y->d2) return x->d2 < y->d2 ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

static int i64_cmp(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

static int64_t sqd(const int32_t *a, const int32_t *b, int d)
{
    int64_t s = 0;
    for (int t = 0; t < d; ++t) {
        int64_t df = (int64_t)a[t] - (int64_t)b[t];
        s += df * df;
    }
    return s;
}

/* RNG neighbours of the point with coordinates c among the n points of K,
 * ignoring index `self` (the point itself, or -1 for an external query).
 * Only candidates y with y > min_y are decided.  Writes ids ascending. */
static int64_t row_neighbours(const int32_t *K, int64_t n, int d, const int32_t *c,
                              int64_t self, int64_t min_y, okey *keys, int64_t *out)
{
    int64_t cnt = 0, len = 0;
    for (int64_t z = 0; z < n; ++z) {
        if (z == self) continue;
        keys[len].d2 = sqd(c, K + z * d, d);
        keys[len].idx = z;
        ++len;
    }
    qsort(keys, (size_t)len, sizeof(okey), okey_cmp);
    for (int64_t m = 0; m < len; ++m) {
        int64_t y = keys[m].idx, dy = keys[m].d2;
        if (y <= min_y) continue;
        int alive = 1;
        for (int64_t l = 0; l < m && keys[l].d2 < dy; ++l) {
            if (sqd(K + y * d, K + keys[l].idx * d, d) < dy) { alive = 0; break; }
        }
        if (alive) out[cnt++] = y;
    }
    qsort(out, (size_t)cnt, sizeof(int64_t), i64_cmp);
    return cnt;
}

void oracle_free(void *p) { free(p); }

int64_t oracle_rng_row(const int32_t *K, int64_t n, int32_t d, int64_t x, int64_t *out)
{
    okey *keys = (okey *)malloc(sizeof(okey) * (size_t)(n > 0 ? n : 1));
    if (!keys) return -1;
    int64_t c = row_neighbours(K, n, d, K + x * d, x, -1, keys, out);
    free(keys);
    return c;
}

int64_t oracle_query_row(const int32_t *K, int64_t n, int32_t d, const int32_t *qk, int64_t *out)
{
    okey *keys = (okey *)malloc(sizeof(okey) * (size_t)(n > 0 ? n : 1));
    if (!keys) return -1;
    int64_t c = row_neighbours(K, n, d, qk, -1, -1, keys, out);
    free(keys);
    return c;
}

/* Rows of several points in parallel: out is nx*n int64, counts[i] written. */
int64_t oracle_rng_rows(const int32_t *K, int64_t n, int32_t d, const int64_t *xs, int64_t nx,
                        int32_t nthreads, int64_t *counts, int64_t *out)
{
    int64_t err = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        okey *keys = (okey *)malloc(sizeof(okey) * (size_t)(n > 0 ? n : 1));
        if (!keys) {
#pragma omp atomic write
            err = -1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t i = 0; i < nx; ++i)
                counts[i] = row_neighbours(K, n, d, K + xs[i] * d, xs[i], -1, keys, out + i * n);
            free(keys);
        }
    }
    return err;
}

/* Rows of several points in parallel into a caller buffer of `cap` ids per
 * row: out is nx*cap int64.  counts[i] = the row's neighbour count; a row
 * with more than cap neighbours is not written and gets counts[i] = -count.
 * upper != 0 decides only the neighbours y > x of each row (the share of a
 * row that the full build decides), else every y. */
int64_t oracle_rng_rows_cap(const int32_t *K, int64_t n, int32_t d, const int64_t *xs, int64_t nx,
                            int32_t nthreads, int32_t upper, int64_t cap, int64_t *counts, int64_t *out)
{
    int64_t err = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        okey *keys = (okey *)malloc(sizeof(okey) * (size_t)(n > 0 ? n : 1));
        int64_t *buf = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        if (!keys || !buf) {
#pragma omp atomic write
            err = -1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t c = row_neighbours(K, n, d, K + xs[i] * d, xs[i], upper ? xs[i] : -1, keys, buf);
                if (c <= cap) {
                    memcpy(out + i * cap, buf, sizeof(int64_t) * (size_t)c);
                    counts[i] = c;
                } else {
                    counts[i] = -c;
                }
            }
        }
        free(keys);
        free(buf);
    }
    return err;
}

/* All RNG edges (u < v), sorted; *out_uv receives a malloc'd array of 2E int64. */
int64_t oracle_rng_edges(const int32_t *K, int64_t n, int32_t d, int32_t nthreads, int64_t **out_uv)
{
    int64_t **rows = (int64_t **)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t *));
    int64_t *cnt = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    int64_t err = 0;
    if (!rows || !cnt) { free(rows); free(cnt); return -1; }
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        okey *keys = (okey *)malloc(sizeof(okey) * (size_t)(n > 0 ? n : 1));
        int64_t *buf = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        if (!keys || !buf) {
#pragma omp atomic write
            err = -1;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (int64_t x = 0; x < n; ++x) {
                int64_t c = row_neighbours(K, n, d, K + x * d, x, x, keys, buf);
                cnt[x] = c;
                rows[x] = (int64_t *)malloc(sizeof(int64_t) * (size_t)(c > 0 ? c : 1));
                if (!rows[x]) {
#pragma omp atomic write
                    err = -1;
                } else {
                    memcpy(rows[x], buf, sizeof(int64_t) * (size_t)c);
                }
            }
        }
        free(keys);
        free(buf);
    }
    int64_t total = 0;
    for (int64_t x = 0; x < n; ++x) total += cnt[x];
    int64_t *uv = err ? NULL : (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * total + 2));
    if (uv) {
        int64_t e = 0;
        for (int64_t x = 0; x < n; ++x)
            for (int64_t t = 0; t < cnt[x]; ++t) { uv[2 * e] = x; uv[2 * e + 1] = rows[x][t]; ++e; }
    }
    for (int64_t x = 0; x < n; ++x) free(rows[x]);
    free(rows);
    free(cnt);
    if (!uv) return -1;
    *out_uv = uv;
    return total;
}

/* Exact truth of sqrt(a) + c < sqrt(b) for a, b, c >= 0 (integers):
 * needs c^2 < b, then T = b + c^2 - a > 0 and 4 c^2 b < T^2. */
static int sqrt_plus_lt(int64_t a, int64_t c, int64_t b)
{
    __int128 cc = (__int128)c * c;
    if (cc >= (__int128)b) return 0;
    __int128 t = (__int128)b + cc - (__int128)a;
    if (t <= 0) return 0;
    return (__int128)4 * cc * (__int128)b < t * t;
}

int32_t oracle_sqrt_plus_lt(int64_t a, int64_t c, int64_t b) { return sqrt_plus_lt(a, c, b); }

/* GRNG over m pivots with coordinates Kp (m x d) and radii R (grid ints). */
int64_t oracle_grng_edges(const int32_t *Kp, int64_t m, int32_t d, const int64_t *R,
                          int32_t nthreads, int64_t **out_ij)
{
    int64_t *D = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m * m > 0 ? m * m : 1));
    unsigned char *link = (unsigned char *)calloc((size_t)(m * m > 0 ? m * m : 1), 1);
    if (!D || !link) { free(D); free(link); return -1; }
#pragma omp parallel for num_threads(nthreads > 0 ? nthreads : 1) schedule(static)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < m; ++j) D[i * m + j] = sqd(Kp + i * d, Kp + j * d, d);
#pragma omp parallel for num_threads(nthreads > 0 ? nthreads : 1) schedule(dynamic, 4)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = i + 1; j < m; ++j) {
            int64_t dij = D[i * m + j];
            int64_t c1 = 2 * R[i] + R[j], c2 = R[i] + 2 * R[j];
            int blocked = 0;
            for (int64_t k = 0; k < m && !blocked; ++k) {
                if (k == i || k == j) continue;
                blocked = sqrt_plus_lt(D[k * m + i], c1, dij) && sqrt_plus_lt(D[k * m + j], c2, dij);
            }
            link[i * m + j] = (unsigned char)!blocked;
        }
    }
    int64_t total = 0;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = i + 1; j < m; ++j) total += link[i * m + j];
    int64_t *ij = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * total + 2));
    if (ij) {
        int64_t e = 0;
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = i + 1; j < m; ++j)
                if (link[i * m + j]) { ij[2 * e] = i; ij[2 * e + 1] = j; ++e; }
    }
    free(D);
    free(link);
    if (!ij) return -1;
    *out_ij = ij;
    return total;
}
