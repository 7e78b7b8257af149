/*
 * Local NBNN oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU statement of what local NBNN
 * computes (McCann & Lowe, "Local Naive Bayes Nearest Neighbor for Image
 * Classification", Sec. 5, Algorithm 2) and of the original NBNN rule it is
 * derived from (Sec. 1, Algorithm 1; Sec. 3, Eq. for the NBNN rule).
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header or table with the GPU
 * library; both only read the same generated input arrays.
 *
 * Conventions (readings of points the paper leaves open):
 *   - distance is the squared Euclidean distance, no square root
 *     (Algorithm 2 and Algorithm 1 both use ||d - p||^2);
 *   - the k+1 nearest neighbours are the k+1 smallest (distance, index)
 *     pairs in lexicographic order, so equal distances go to the lower
 *     reference index;
 *   - totals start at 0 for every class; argmin ties go to the lowest class;
 *   - integer (u8) descriptors use exact int64 arithmetic; float descriptors
 *     are widened to double and use the direct form sum_t (q_t - r_t)^2.
 *
 * Parallelism: OpenMP over query descriptors (or blocks of them) for the
 * distance scans only;
 * every reduction into per-image totals runs serially per image in
 * descriptor order, then neighbour order, so float totals are reproducible.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* distances                                                           */
/* ------------------------------------------------------------------ */

/* Squared Euclidean distance ||a - b||^2 of two u8 descriptors, exact in
 * int64 (Algorithm 2, the dist_B and dist_C lines; Algorithm 1's update). */
int64_t or_sqdist_u8(const uint8_t *a, const uint8_t *b, int32_t dim)
{
    int64_t s = 0;
    for (int32_t t = 0; t < dim; ++t) {
        int64_t d = (int64_t)a[t] - (int64_t)b[t];
        s += d * d;
    }
    return s;
}

/* The same distance by the expanded identity ||a||^2 + ||b||^2 - 2 a.b,
 * also exact in int64.  Used only to pin or_sqdist_u8 by a second route. */
int64_t or_sqdist_u8_expanded(const uint8_t *a, const uint8_t *b, int32_t dim)
{
    int64_t aa = 0, bb = 0, ab = 0;
    for (int32_t t = 0; t < dim; ++t) {
        aa += (int64_t)a[t] * a[t];
        bb += (int64_t)b[t] * b[t];
        ab += (int64_t)a[t] * b[t];
    }
    return aa + bb - 2 * ab;
}

/* Squared Euclidean distance of two float descriptors, widened to double,
 * direct form, summed in dimension order. */
double or_sqdist_f32(const float *a, const float *b, int32_t dim)
{
    double s = 0.0;
    for (int32_t t = 0; t < dim; ++t) {
        double d = (double)a[t] - (double)b[t];
        s += d * d;
    }
    return s;
}

/* ------------------------------------------------------------------ */
/* k+1 nearest neighbours: NN(d_i, k+1) of Algorithm 2                 */
/* ------------------------------------------------------------------ */

typedef struct { int64_t d; int64_t idx; } pair_i64;
typedef struct { double d; int64_t idx; } pair_f64;

static int cmp_pair_i64(const void *x, const void *y)
{
    const pair_i64 *a = (const pair_i64 *)x, *b = (const pair_i64 *)y;
    if (a->d != b->d) return a->d < b->d ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

static int cmp_pair_f64(const void *x, const void *y)
{
    const pair_f64 *a = (const pair_f64 *)x, *b = (const pair_f64 *)y;
    if (a->d != b->d) return a->d < b->d ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

/* Route "sort": all N distances, full sort by (distance, index), keep the
 * first kp.  Memory O(N) per thread; meant for small N.  Returns 0, or -1 if
 * kp > N or an allocation failed. */
int or_knn_u8_sort(const uint8_t *Q, int64_t n, const uint8_t *R, int64_t N,
                   int32_t dim, int32_t kp, int32_t *out_idx, int64_t *out_dist)
{
    if (kp < 1 || kp > N) return -1;
    int err = 0;
#pragma omp parallel
    {
        pair_i64 *all = (pair_i64 *)malloc(sizeof(pair_i64) * (size_t)N);
        if (!all) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < n; ++i) {
            if (!all) continue;
            const uint8_t *q = Q + i * dim;
            for (int64_t j = 0; j < N; ++j) {
                all[j].d = or_sqdist_u8(q, R + j * dim, dim);
                all[j].idx = j;
            }
            qsort(all, (size_t)N, sizeof(pair_i64), cmp_pair_i64);
            for (int32_t p = 0; p < kp; ++p) {
                out_idx[i * kp + p] = (int32_t)all[p].idx;
                out_dist[i * kp + p] = all[p].d;
            }
        }
        free(all);
    }
    return err;
}

/* Route "scan": one pass over the references in index order, keeping a
 * sorted list of the kp best (distance, index) pairs.  A reference enters
 * only if it is strictly better in the (distance, index) order than the
 * current kp-th entry.  Same result as the sort route; O(kp) memory. */
int or_knn_u8_scan(const uint8_t *Q, int64_t n, const uint8_t *R, int64_t N,
                   int32_t dim, int32_t kp, int32_t *out_idx, int64_t *out_dist)
{
    if (kp < 1 || kp > N) return -1;
    int err = 0;
#pragma omp parallel
    {
        pair_i64 *best = (pair_i64 *)malloc(sizeof(pair_i64) * (size_t)kp);
        if (!best) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < n; ++i) {
            if (!best) continue;
            const uint8_t *q = Q + i * dim;
            int32_t filled = 0;
            for (int64_t j = 0; j < N; ++j) {
                pair_i64 c = { or_sqdist_u8(q, R + j * dim, dim), j };
                if (filled == kp && cmp_pair_i64(&c, &best[kp - 1]) >= 0)
                    continue;
                int32_t pos = filled < kp ? filled : kp - 1;
                while (pos > 0 && cmp_pair_i64(&c, &best[pos - 1]) < 0) {
                    best[pos] = best[pos - 1];
                    --pos;
                }
                best[pos] = c;
                if (filled < kp) ++filled;
            }
            for (int32_t p = 0; p < kp; ++p) {
                out_idx[i * kp + p] = (int32_t)best[p].idx;
                out_dist[i * kp + p] = best[p].d;
            }
        }
        free(best);
    }
    return err;
}

/* Float descriptors: same two routes with double distances. */
int or_knn_f32_sort(const float *Q, int64_t n, const float *R, int64_t N,
                    int32_t dim, int32_t kp, int32_t *out_idx, double *out_dist)
{
    if (kp < 1 || kp > N) return -1;
    int err = 0;
#pragma omp parallel
    {
        pair_f64 *all = (pair_f64 *)malloc(sizeof(pair_f64) * (size_t)N);
        if (!all) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < n; ++i) {
            if (!all) continue;
            const float *q = Q + i * dim;
            for (int64_t j = 0; j < N; ++j) {
                all[j].d = or_sqdist_f32(q, R + j * dim, dim);
                all[j].idx = j;
            }
            qsort(all, (size_t)N, sizeof(pair_f64), cmp_pair_f64);
            for (int32_t p = 0; p < kp; ++p) {
                out_idx[i * kp + p] = (int32_t)all[p].idx;
                out_dist[i * kp + p] = all[p].d;
            }
        }
        free(all);
    }
    return err;
}

int or_knn_f32_scan(const float *Q, int64_t n, const float *R, int64_t N,
                    int32_t dim, int32_t kp, int32_t *out_idx, double *out_dist)
{
    if (kp < 1 || kp > N) return -1;
    int err = 0;
#pragma omp parallel
    {
        pair_f64 *best = (pair_f64 *)malloc(sizeof(pair_f64) * (size_t)kp);
        if (!best) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < n; ++i) {
            if (!best) continue;
            const float *q = Q + i * dim;
            int32_t filled = 0;
            for (int64_t j = 0; j < N; ++j) {
                pair_f64 c = { or_sqdist_f32(q, R + j * dim, dim), j };
                if (filled == kp && cmp_pair_f64(&c, &best[kp - 1]) >= 0)
                    continue;
                int32_t pos = filled < kp ? filled : kp - 1;
                while (pos > 0 && cmp_pair_f64(&c, &best[pos - 1]) < 0) {
                    best[pos] = best[pos - 1];
                    --pos;
                }
                best[pos] = c;
                if (filled < kp) ++filled;
            }
            for (int32_t p = 0; p < kp; ++p) {
                out_idx[i * kp + p] = (int32_t)best[p].idx;
                out_dist[i * kp + p] = best[p].d;
            }
        }
        free(best);
    }
    return err;
}

/* ------------------------------------------------------------------ */
/* Route "block": the scan route, tiled for the cache                  */
/* ------------------------------------------------------------------ */
/*
 * Same per-pair arithmetic as or_sqdist_u8 / or_sqdist_f32 (direct form,
 * summed in dimension order) and the same insertion rule as the scan
 * route, so the lists are identical to the scan and sort routes'.  Only
 * the loop order differs: a thread takes a block of OR_QB queries and
 * walks the references in groups of OR_JB; each group is widened and
 * transposed once into a small buffer and then compared with every query
 * of the block, OR_JB references at a time, so a group is read from memory
 * once per block instead of once per query.  The per-reference distances of
 * a group are independent sums, so each vector lane carries one reference's
 * sum and no sum is reordered.
 *
 * u8 data is summed in int32: a squared difference is at most 255^2 and a
 * row of at most 256 elements sums to less than 2^31, so the sums are exact
 * (the same integers as the int64 routes).
 */
#define OR_QB 64   /* queries per block (a multiple of OR_NQ) */
#define OR_JB 16   /* references per group */
#define OR_NQ 4    /* queries that share each load of a group's column */

typedef double or_vd8 __attribute__((vector_size(64)));     /* 8 doubles */
typedef int32_t or_vi16 __attribute__((vector_size(64)));   /* 16 int32 */

/* acc[i][jj] = sum over t = 0..dim-1, in that order, of (q_i[t] - r_jj[t])^2
 * for the queries of a block (rows of qb; nq rounded up to OR_NQ, the extra
 * rows are zeros) and the OR_JB references of a group, stored transposed:
 * rt[t * OR_JB + jj].  Each vector lane holds one reference's running sum,
 * so every sum is the sequential sum of or_sqdist_f32. */
__attribute__((target_clones("avx512f", "avx2", "default")))
static void group_f64(const double *qb, int32_t nq, const double *rt, int32_t dim,
                      double *acc)
{
    for (int32_t i0 = 0; i0 < nq; i0 += OR_NQ) {
        or_vd8 s[OR_NQ][2];
        memset(s, 0, sizeof s);
        for (int32_t t = 0; t < dim; ++t) {
            or_vd8 r0, r1;
            memcpy(&r0, rt + (int64_t)t * OR_JB, sizeof r0);
            memcpy(&r1, rt + (int64_t)t * OR_JB + 8, sizeof r1);
            for (int32_t u = 0; u < OR_NQ; ++u) {
                const double qt = qb[(int64_t)(i0 + u) * dim + t];
                or_vd8 d0 = qt - r0, d1 = qt - r1;
                s[u][0] += d0 * d0;
                s[u][1] += d1 * d1;
            }
        }
        memcpy(acc + (int64_t)i0 * OR_JB, s, sizeof s);
    }
}

/* The same for u8 data widened to int32 (exact: see above). */
__attribute__((target_clones("avx512f", "avx2", "default")))
static void group_i32(const int32_t *qb, int32_t nq, const int32_t *rt, int32_t dim,
                      int32_t *acc)
{
    for (int32_t i0 = 0; i0 < nq; i0 += OR_NQ) {
        or_vi16 s[OR_NQ];
        memset(s, 0, sizeof s);
        for (int32_t t = 0; t < dim; ++t) {
            or_vi16 r;
            memcpy(&r, rt + (int64_t)t * OR_JB, sizeof r);
            for (int32_t u = 0; u < OR_NQ; ++u) {
                or_vi16 d = qb[(int64_t)(i0 + u) * dim + t] - r;
                s[u] += d * d;
            }
        }
        memcpy(acc + (int64_t)i0 * OR_JB, s, sizeof s);
    }
}

/* Insert candidate c into the sorted list best[0..filled) of capacity kp,
 * exactly as the scan route does (strictly better than the kp-th entry). */
static void list_insert_i64(pair_i64 *best, int32_t *filled, int32_t kp, pair_i64 c)
{
    if (*filled == kp && cmp_pair_i64(&c, &best[kp - 1]) >= 0) return;
    int32_t pos = *filled < kp ? *filled : kp - 1;
    while (pos > 0 && cmp_pair_i64(&c, &best[pos - 1]) < 0) {
        best[pos] = best[pos - 1];
        --pos;
    }
    best[pos] = c;
    if (*filled < kp) ++*filled;
}

static void list_insert_f64(pair_f64 *best, int32_t *filled, int32_t kp, pair_f64 c)
{
    if (*filled == kp && cmp_pair_f64(&c, &best[kp - 1]) >= 0) return;
    int32_t pos = *filled < kp ? *filled : kp - 1;
    while (pos > 0 && cmp_pair_f64(&c, &best[pos - 1]) < 0) {
        best[pos] = best[pos - 1];
        --pos;
    }
    best[pos] = c;
    if (*filled < kp) ++*filled;
}

/* u8 descriptors.  Either output may be left out:
 *   out_idx/out_dist (both or neither): the kp nearest (distance, index)
 *     pairs of every query, as or_knn_u8_scan;
 *   D (with labels, n_classes): per-class nearest distance of every query,
 *     as or_class_nn_u8 (INT64_MAX for a class with no reference).
 * Returns 0, or -1 on bad arguments or a failed allocation. */
int or_knn_u8_block(const uint8_t *Q, int64_t n, const uint8_t *R, int64_t N,
                    int32_t dim, int32_t kp, const int32_t *labels, int32_t n_classes,
                    int32_t *out_idx, int64_t *out_dist, int64_t *D)
{
    const int want_list = out_idx != NULL;
    if (want_list && (kp < 1 || kp > N || out_dist == NULL)) return -1;
    if (dim < 1 || dim > 256) return -1;
    if (D != NULL) {
        if (labels == NULL || n_classes < 1) return -1;
        for (int64_t j = 0; j < N; ++j)
            if (labels[j] < 0 || labels[j] >= n_classes) return -1;
    }
    const int64_t nblk = (n + OR_QB - 1) / OR_QB;
    int err = 0;
#pragma omp parallel
    {
        int32_t *qb = (int32_t *)malloc(sizeof(int32_t) * OR_QB * (size_t)dim);
        int32_t *rt = (int32_t *)malloc(sizeof(int32_t) * OR_JB * (size_t)dim);
        int32_t *acc = (int32_t *)malloc(sizeof(int32_t) * OR_QB * OR_JB);
        pair_i64 *best = (pair_i64 *)malloc(sizeof(pair_i64) * OR_QB * (size_t)(kp > 0 ? kp : 1));
        int32_t filled[OR_QB];
        int ok = qb && rt && acc && best;
        if (!ok) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t b = 0; b < nblk; ++b) {
            if (!ok) continue;
            const int64_t i0 = b * OR_QB;
            const int32_t nq = (int32_t)(n - i0 < OR_QB ? n - i0 : OR_QB);
            for (int32_t i = nq; i < OR_QB; ++i)
                for (int32_t t = 0; t < dim; ++t) qb[i * dim + t] = 0;
            for (int32_t i = 0; i < nq; ++i) {
                for (int32_t t = 0; t < dim; ++t) qb[i * dim + t] = Q[(i0 + i) * dim + t];
                filled[i] = 0;
                if (D != NULL)
                    for (int32_t c = 0; c < n_classes; ++c) D[(i0 + i) * n_classes + c] = INT64_MAX;
            }
            for (int64_t j0 = 0; j0 < N; j0 += OR_JB) {
                const int32_t jb = (int32_t)(N - j0 < OR_JB ? N - j0 : OR_JB);
                for (int32_t t = 0; t < dim; ++t)
                    for (int32_t jj = 0; jj < OR_JB; ++jj)
                        rt[t * OR_JB + jj] = jj < jb ? R[(j0 + jj) * dim + t] : 0;
                group_i32(qb, nq, rt, dim, acc);
                for (int32_t i = 0; i < nq; ++i)
                    for (int32_t jj = 0; jj < jb; ++jj) {
                        int64_t d = acc[i * OR_JB + jj];
                        if (want_list) {
                            pair_i64 c = { d, j0 + jj };
                            list_insert_i64(best + (int64_t)i * kp, &filled[i], kp, c);
                        }
                        if (D != NULL) {
                            int64_t *Dc = D + (i0 + i) * n_classes + labels[j0 + jj];
                            if (d < *Dc) *Dc = d;
                        }
                    }
            }
            if (want_list)
                for (int32_t i = 0; i < nq; ++i)
                    for (int32_t p = 0; p < kp; ++p) {
                        out_idx[(i0 + i) * kp + p] = (int32_t)best[i * kp + p].idx;
                        out_dist[(i0 + i) * kp + p] = best[i * kp + p].d;
                    }
        }
        free(qb);
        free(rt);
        free(acc);
        free(best);
    }
    return err;
}

/* Float descriptors: the kp nearest (distance, index) pairs, double
 * distances, as or_knn_f32_scan. */
int or_knn_f32_block(const float *Q, int64_t n, const float *R, int64_t N,
                     int32_t dim, int32_t kp, int32_t *out_idx, double *out_dist)
{
    if (kp < 1 || kp > N || dim < 1) return -1;
    const int64_t nblk = (n + OR_QB - 1) / OR_QB;
    int err = 0;
#pragma omp parallel
    {
        double *qb = (double *)malloc(sizeof(double) * OR_QB * (size_t)dim);
        double *rt = (double *)malloc(sizeof(double) * OR_JB * (size_t)dim);
        double *acc = (double *)malloc(sizeof(double) * OR_QB * OR_JB);
        pair_f64 *best = (pair_f64 *)malloc(sizeof(pair_f64) * OR_QB * (size_t)kp);
        int32_t filled[OR_QB];
        int ok = qb && rt && acc && best;
        if (!ok) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t b = 0; b < nblk; ++b) {
            if (!ok) continue;
            const int64_t i0 = b * OR_QB;
            const int32_t nq = (int32_t)(n - i0 < OR_QB ? n - i0 : OR_QB);
            for (int32_t i = nq; i < OR_QB; ++i)
                for (int32_t t = 0; t < dim; ++t) qb[i * dim + t] = 0.0;
            for (int32_t i = 0; i < nq; ++i) {
                for (int32_t t = 0; t < dim; ++t) qb[i * dim + t] = (double)Q[(i0 + i) * dim + t];
                filled[i] = 0;
            }
            for (int64_t j0 = 0; j0 < N; j0 += OR_JB) {
                const int32_t jb = (int32_t)(N - j0 < OR_JB ? N - j0 : OR_JB);
                for (int32_t t = 0; t < dim; ++t)
                    for (int32_t jj = 0; jj < OR_JB; ++jj)
                        rt[t * OR_JB + jj] = jj < jb ? (double)R[(j0 + jj) * dim + t] : 0.0;
                group_f64(qb, nq, rt, dim, acc);
                for (int32_t i = 0; i < nq; ++i)
                    for (int32_t jj = 0; jj < jb; ++jj) {
                        pair_f64 c = { acc[i * OR_JB + jj], j0 + jj };
                        list_insert_f64(best + (int64_t)i * kp, &filled[i], kp, c);
                    }
            }
            for (int32_t i = 0; i < nq; ++i)
                for (int32_t p = 0; p < kp; ++p) {
                    out_idx[(i0 + i) * kp + p] = (int32_t)best[i * kp + p].idx;
                    out_dist[(i0 + i) * kp + p] = best[i * kp + p].d;
                }
        }
        free(qb);
        free(rt);
        free(acc);
        free(best);
    }
    return err;
}

/* ------------------------------------------------------------------ */
/* Algorithm 2 scoring, given each descriptor's k+1 nearest neighbours */
/* ------------------------------------------------------------------ */

static int check_offsets(const int64_t *offsets, int32_t n_img, int64_t n)
{
    if (n_img < 0 || offsets[0] != 0) return -1;
    for (int32_t m = 0; m < n_img; ++m)
        if (offsets[m + 1] < offsets[m]) return -1;
    if (offsets[n_img] != n) return -1;
    return 0;
}

/* argmin_C totals[C], lowest class on ties (Algorithm 2, return line). */
static int32_t argmin_i64(const int64_t *t, int32_t nc)
{
    int32_t b = 0;
    for (int32_t c = 1; c < nc; ++c)
        if (t[c] < t[b]) b = c;
    return b;
}

static int32_t argmin_f64(const double *t, int32_t nc)
{
    int32_t b = 0;
    for (int32_t c = 1; c < nc; ++c)
        if (t[c] < t[b]) b = c;
    return b;
}

/* Algorithm 2 as printed, for one image at a time.
 *   nbr_idx/nbr_dist: [n, k+1], the k+1 nearest neighbours of every
 *   descriptor in (distance, index) order.
 * For each descriptor: dist_B is the distance of the (k+1)-th neighbour;
 * for every class C found among the first k neighbours,
 * dist_C = min over all retrieved p_j of class C of ||d - p_j||^2, and
 * totals[C] += dist_C - dist_B.  Returns argmin per image.
 * Integer distances: totals are exact int64. */
int or_local_nbnn_i64(const int32_t *nbr_idx, const int64_t *nbr_dist, int64_t n,
                      int32_t k, const int32_t *labels, int32_t n_classes,
                      const int64_t *offsets, int32_t n_img,
                      int64_t *totals, int32_t *out_class)
{
    if (k < 1 || n_classes < 1 || check_offsets(offsets, n_img, n)) return -1;
    const int32_t kp = k + 1;
    for (int32_t m = 0; m < n_img; ++m) {
        int64_t *T = totals + (int64_t)m * n_classes;
        for (int32_t c = 0; c < n_classes; ++c) T[c] = 0;
        for (int64_t i = offsets[m]; i < offsets[m + 1]; ++i) {
            const int32_t *pi = nbr_idx + i * kp;
            const int64_t *pd = nbr_dist + i * kp;
            int64_t dist_b = pd[k];
            for (int32_t j = 0; j < k; ++j) {
                int32_t C = labels[pi[j]];
                /* each class found in the k nearest is adjusted once */
                int seen = 0;
                for (int32_t jj = 0; jj < j; ++jj)
                    if (labels[pi[jj]] == C) seen = 1;
                if (seen) continue;
                int64_t dist_c = INT64_MAX;
                for (int32_t jj = 0; jj < kp; ++jj)
                    if (labels[pi[jj]] == C && pd[jj] < dist_c) dist_c = pd[jj];
                T[C] += dist_c - dist_b;
            }
        }
        out_class[m] = argmin_i64(T, n_classes);
    }
    return 0;
}

/* Same with double distances; totals summed in descriptor order, then in
 * neighbour order. */
int or_local_nbnn_f64(const int32_t *nbr_idx, const double *nbr_dist, int64_t n,
                      int32_t k, const int32_t *labels, int32_t n_classes,
                      const int64_t *offsets, int32_t n_img,
                      double *totals, int32_t *out_class)
{
    if (k < 1 || n_classes < 1 || check_offsets(offsets, n_img, n)) return -1;
    const int32_t kp = k + 1;
    for (int32_t m = 0; m < n_img; ++m) {
        double *T = totals + (int64_t)m * n_classes;
        for (int32_t c = 0; c < n_classes; ++c) T[c] = 0.0;
        for (int64_t i = offsets[m]; i < offsets[m + 1]; ++i) {
            const int32_t *pi = nbr_idx + i * kp;
            const double *pd = nbr_dist + i * kp;
            double dist_b = pd[k];
            for (int32_t j = 0; j < k; ++j) {
                int32_t C = labels[pi[j]];
                int seen = 0;
                for (int32_t jj = 0; jj < j; ++jj)
                    if (labels[pi[jj]] == C) seen = 1;
                if (seen) continue;
                double dist_c = INFINITY;
                for (int32_t jj = 0; jj < kp; ++jj)
                    if (labels[pi[jj]] == C && pd[jj] < dist_c) dist_c = pd[jj];
                T[C] += dist_c - dist_b;
            }
        }
        out_class[m] = argmin_f64(T, n_classes);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Per-class nearest distances, Algorithm 1 (original NBNN), and the   */
/* closed form of Algorithm 2's totals                                 */
/* ------------------------------------------------------------------ */

/* D[i][C] = min over references of class C of ||d_i - r||^2, i.e.
 * ||d_i - NN_C(d_i)||^2 of Algorithm 1; INT64_MAX for a class with no
 * reference.  Also returns, per descriptor, the (k+1)-th smallest distance
 * of the whole merged set (the multiset order statistic, tie-free). */
int or_class_nn_u8(const uint8_t *Q, int64_t n, const uint8_t *R, int64_t N,
                   int32_t dim, const int32_t *labels, int32_t n_classes,
                   int32_t k, int64_t *D, int64_t *kth)
{
    if (n_classes < 1 || k < 0 || k + 1 > N) return -1;
    for (int64_t j = 0; j < N; ++j)
        if (labels[j] < 0 || labels[j] >= n_classes) return -1;
    const int32_t kp = k + 1;
    int err = 0;
#pragma omp parallel
    {
        int64_t *best = (int64_t *)malloc(sizeof(int64_t) * (size_t)kp);
        if (!best) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < n; ++i) {
            if (!best) continue;
            int64_t *Di = D + i * n_classes;
            for (int32_t c = 0; c < n_classes; ++c) Di[c] = INT64_MAX;
            int32_t filled = 0;
            for (int64_t j = 0; j < N; ++j) {
                int64_t d = or_sqdist_u8(Q + i * dim, R + j * dim, dim);
                if (d < Di[labels[j]]) Di[labels[j]] = d;
                /* k+1 smallest values of the multiset, sorted */
                if (filled == kp && d >= best[kp - 1]) continue;
                int32_t pos = filled < kp ? filled : kp - 1;
                while (pos > 0 && d < best[pos - 1]) {
                    best[pos] = best[pos - 1];
                    --pos;
                }
                best[pos] = d;
                if (filled < kp) ++filled;
            }
            kth[i] = best[kp - 1];
        }
        free(best);
    }
    return err;
}

/* Closed form of Algorithm 2's totals:
 *   totals[m][C] = sum over d in image m of min(0, D_C(d) - delta_(k+1)(d)).
 * A class whose nearest reference is closer than the (k+1)-th distance is
 * necessarily among the k nearest with that distance as its first
 * occurrence; otherwise its update is 0.  Classes with no reference get 0. */
int or_closed_form_i64(const int64_t *D, const int64_t *kth, int64_t n,
                       int32_t n_classes, const int64_t *offsets, int32_t n_img,
                       int64_t *totals, int32_t *out_class)
{
    if (n_classes < 1 || check_offsets(offsets, n_img, n)) return -1;
    for (int32_t m = 0; m < n_img; ++m) {
        int64_t *T = totals + (int64_t)m * n_classes;
        for (int32_t c = 0; c < n_classes; ++c) T[c] = 0;
        for (int64_t i = offsets[m]; i < offsets[m + 1]; ++i)
            for (int32_t c = 0; c < n_classes; ++c) {
                int64_t dc = D[i * n_classes + c];
                if (dc != INT64_MAX && dc < kth[i]) T[c] += dc - kth[i];
            }
        out_class[m] = argmin_i64(T, n_classes);
    }
    return 0;
}

/* Algorithm 1 (original NBNN): totals[m][C] = sum over d of D_C(d), argmin.
 * Every class must own at least one reference. */
int or_nbnn_i64(const int64_t *D, int64_t n, int32_t n_classes,
                const int64_t *offsets, int32_t n_img,
                int64_t *totals, int32_t *out_class)
{
    if (n_classes < 1 || check_offsets(offsets, n_img, n)) return -1;
    for (int64_t i = 0; i < n * n_classes; ++i)
        if (D[i] == INT64_MAX) return -1;
    for (int32_t m = 0; m < n_img; ++m) {
        int64_t *T = totals + (int64_t)m * n_classes;
        for (int32_t c = 0; c < n_classes; ++c) T[c] = 0;
        for (int64_t i = offsets[m]; i < offsets[m + 1]; ++i)
            for (int32_t c = 0; c < n_classes; ++c) T[c] += D[i * n_classes + c];
        out_class[m] = argmin_i64(T, n_classes);
    }
    return 0;
}

/* Number of OpenMP threads a parallel region would use (1 without OpenMP). */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
