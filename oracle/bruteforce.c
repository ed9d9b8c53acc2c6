/*
 * CPU brute-force oracle for the geometric-search hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code with the HIP library.
 *
 * What it computes is the plain definition of each query the paper's search
 * index answers (Section 2.1, "Original interface" and "New interface";
 * Section 2.2 for callbacks): for every query, every value is tested, so the
 * result is the exact answer a hierarchy must reproduce.
 *
 *   - values: points [n][dim], or boxes [n][2][dim] (lo row then hi row);
 *   - spatial (radius) query: the closed ball of radius r around a point;
 *     result = indices of matching values, ascending, in CSR form (offsets +
 *     indices, the compressed-sparse-row layout of Section 2.1);
 *   - intersects(box) query: closed overlap of the query box with the value;
 *   - nearest query: the k values closest to the query point, ordered by
 *     (squared distance, index), padded with (+inf, -1) when k > n;
 *   - pure-callback queries (Section 2.2, query form (1)): per-query COUNT, and
 *     COUNT plus a fixed-point sum of distances, nothing stored per match;
 *   - the early-terminating count of Section 2.2: a query stops once it has
 *     counted n_max matches, so its result is min(count, n_max);
 *   - the callback-with-output form (Section 2.1, query call (2)) as the
 *     squared distance of each match of a CSR result;
 *   - search for pairs of objects (Section 2.6): the self-join of a point set
 *     with a radius, as per-point pair counts and upper-triangle CSR rows;
 *   - density-based clustering over the radius search (Section 2.4, DBSCAN):
 *     core points, their eps-connected components and border points;
 *   - ray predicates (Section 2.5): the values a ray meets, counted, listed
 *     (intersect), listed in the order met (ordered intersect), and the k met
 *     first, ordered by (entry parameter, index);
 *   - Chamfer loss of nearest-neighbour pairs and its gradient, in float64.
 *
 * Floating-point contract (the paper fixes none; this follows the exactness
 * requirement of the hot path): squared distances in float32, one rounding per
 * operation, summed over dimensions from 0 upwards starting at 0, no fused
 * multiply-add (build with -ffp-contract=off), IEEE denormals, comparisons
 * d2 <= fl(r*r).  Ties in nearest search go to the smaller index.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { KIND_POINTS = 0, KIND_BOXES = 1 };
enum { RED_COUNT = 0, RED_COUNT_SUMDIST = 1 };

/* Squared distance between two points: t_d = q_d - p_d, acc = acc + t_d*t_d. */
static float dist2_point(const float *q, const float *p, int dim)
{
    float acc = 0.0f;
    for (int d = 0; d < dim; ++d) {
        float t = q[d] - p[d];
        float s = t * t;
        acc = acc + s;
    }
    return acc;
}

/* Squared distance from a point to a closed box: per dimension the gap to the
 * nearer face (0 inside), accumulated as for two points. */
static float dist2_box(const float *q, const float *lo, const float *hi, int dim)
{
    float acc = 0.0f;
    for (int d = 0; d < dim; ++d) {
        float t = 0.0f;
        if (q[d] < lo[d])
            t = lo[d] - q[d];
        else if (q[d] > hi[d])
            t = q[d] - hi[d];
        float s = t * t;
        acc = acc + s;
    }
    return acc;
}

/* Distance from query point q to value j. */
static float dist2_value(const float *values, int64_t j, int dim, int kind, const float *q)
{
    if (kind == KIND_POINTS)
        return dist2_point(q, values + j * dim, dim);
    const float *lo = values + j * 2 * dim;
    return dist2_box(q, lo, lo + dim, dim);
}

/* Closed overlap of query box [qlo,qhi] with value j. */
static int overlaps_value(const float *values, int64_t j, int dim, int kind, const float *qlo, const float *qhi)
{
    const float *lo, *hi;
    if (kind == KIND_POINTS) {
        lo = hi = values + j * dim;
    } else {
        lo = values + j * 2 * dim;
        hi = lo + dim;
    }
    for (int d = 0; d < dim; ++d)
        if (!(lo[d] <= qhi[d] && qlo[d] <= hi[d]))
            return 0;
    return 1;
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* spatial (radius) search                                              */
/* ------------------------------------------------------------------ */

int oracle_spatial_count(const float *values, int64_t n, int dim, int kind, const float *queries, int64_t m,
                         float radius, int32_t *counts)
{
    const float r2 = radius * radius;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        const float *q = queries + i * dim;
        int32_t c = 0;
        for (int64_t j = 0; j < n; ++j)
            if (dist2_value(values, j, dim, kind, q) <= r2)
                ++c;
        counts[i] = c;
    }
    return 0;
}

/* offsets[m+1] must hold the CSR offsets of the counts above. */
int oracle_spatial_fill(const float *values, int64_t n, int dim, int kind, const float *queries, int64_t m,
                        float radius, const int64_t *offsets, int32_t *indices)
{
    const float r2 = radius * radius;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        const float *q = queries + i * dim;
        int64_t o = offsets[i];
        for (int64_t j = 0; j < n; ++j)
            if (dist2_value(values, j, dim, kind, q) <= r2)
                indices[o++] = (int32_t)j;
    }
    return 0;
}

/* Query boxes are [m][2][dim]. */
int oracle_intersects_count(const float *values, int64_t n, int dim, int kind, const float *qboxes, int64_t m,
                            int32_t *counts)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        const float *qlo = qboxes + i * 2 * dim;
        int32_t c = 0;
        for (int64_t j = 0; j < n; ++j)
            c += overlaps_value(values, j, dim, kind, qlo, qlo + dim);
        counts[i] = c;
    }
    return 0;
}

int oracle_intersects_fill(const float *values, int64_t n, int dim, int kind, const float *qboxes, int64_t m,
                           const int64_t *offsets, int32_t *indices)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        const float *qlo = qboxes + i * 2 * dim;
        int64_t o = offsets[i];
        for (int64_t j = 0; j < n; ++j)
            if (overlaps_value(values, j, dim, kind, qlo, qlo + dim))
                indices[o++] = (int32_t)j;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* pure-callback reductions                                             */
/* ------------------------------------------------------------------ */

/* COUNT: number of matches.  COUNT_SUMDIST: also the sum over matches of
 * trunc(sqrtf(d2) * 2^scale_bits) as a 64-bit integer, which makes the sum
 * independent of the order in which matches are visited. */
int oracle_reduce(const float *values, int64_t n, int dim, int kind, const float *queries, int64_t m,
                  float radius, int op, int scale_bits, int32_t *counts, int64_t *sum_fixed)
{
    const float r2 = radius * radius;
    const float scale = ldexpf(1.0f, scale_bits);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        const float *q = queries + i * dim;
        int32_t c = 0;
        int64_t s = 0;
        for (int64_t j = 0; j < n; ++j) {
            float d2 = dist2_value(values, j, dim, kind, q);
            if (d2 <= r2) {
                ++c;
                if (op == RED_COUNT_SUMDIST) {
                    float dist = sqrtf(d2);
                    float scaled = dist * scale;
                    s += (int64_t)scaled;
                }
            }
        }
        counts[i] = c;
        if (op == RED_COUNT_SUMDIST)
            sum_fixed[i] = s;
    }
    return 0;
}

/* A ray o + t*dir (t >= 0) against the closed box [lo, hi] (Section 2.5, ray
 * predicates), by slabs: in each dimension with dir != 0 the parameters
 * t1 = (lo - o) / dir and t2 = (hi - o) / dir (float32, correctly rounded
 * division); a dimension with dir == 0 admits every t when lo <= o <= hi and
 * none otherwise.  Starting from tmin = 0 and tmax = +inf and taking the
 * dimensions in order, tmin = max(tmin, min(t1, t2)) and
 * tmax = min(tmax, max(t1, t2)); the ray meets the box iff tmin <= tmax, and
 * tmin is then its entry parameter. */
static int ray_box(const float *o, const float *dir, const float *lo, const float *hi, int dim, float *t_entry)
{
    float tmin = 0.0f, tmax = INFINITY;
    for (int k = 0; k < dim; ++k) {
        if (dir[k] == 0.0f) {
            if (o[k] < lo[k] || o[k] > hi[k])
                return 0;
            continue;
        }
        const float t1 = (lo[k] - o[k]) / dir[k];
        const float t2 = (hi[k] - o[k]) / dir[k];
        const float tn = t1 < t2 ? t1 : t2, tf = t1 < t2 ? t2 : t1;
        if (tn > tmin)
            tmin = tn;
        if (tf < tmax)
            tmax = tf;
    }
    if (tmin > tmax)
        return 0;
    *t_entry = tmin;
    return 1;
}

static int ray_value(const float *values, int64_t j, int dim, int kind, const float *ray, float *t)
{
    const float *lo = values + j * (kind == KIND_BOXES ? 2 * dim : dim);
    const float *hi = kind == KIND_BOXES ? lo + dim : lo;
    return ray_box(ray, ray + dim, lo, hi, dim, t);
}

/* Rays are [m][2][dim]: the origin row, then the direction row. */
int oracle_ray_count(const float *values, int64_t n, int dim, int kind, const float *rays, int64_t m, int32_t *counts)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        int32_t c = 0;
        float t;
        for (int64_t j = 0; j < n; ++j)
            c += ray_value(values, j, dim, kind, rays + i * 2 * dim, &t);
        counts[i] = c;
    }
    return 0;
}

/* The k values a ray meets first, in the order (entry parameter, index),
 * padded with (+inf, -1). */
int oracle_ray_nearest(const float *values, int64_t n, int dim, int kind, const float *rays, int64_t m, int k,
                       float *t_out, int32_t *idx_out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        float *bt = t_out + i * k;
        int32_t *bi = idx_out + i * k;
        for (int s = 0; s < k; ++s) {
            bt[s] = INFINITY;
            bi[s] = -1;
        }
        for (int64_t j = 0; j < n; ++j) {
            float t;
            if (!ray_value(values, j, dim, kind, rays + i * 2 * dim, &t))
                continue;
            if (bi[k - 1] >= 0 && !(t < bt[k - 1]))  /* equal t: the earlier (smaller) index stays */
                continue;
            int s = k - 1;
            while (s > 0 && (bi[s - 1] < 0 || t < bt[s - 1])) {
                bt[s] = bt[s - 1];
                bi[s] = bi[s - 1];
                --s;
            }
            bt[s] = t;
            bi[s] = (int32_t)j;
        }
    }
    return 0;
}

/* Ray intersect (Section 2.5): every value the ray meets, as CSR rows with
 * ascending indices (offsets[m+1] from the counts; indices == NULL fills the
 * offsets only). */
int oracle_ray_intersect(const float *values, int64_t n, int dim, int kind, const float *rays, int64_t m,
                         int64_t *offsets, int32_t *indices)
{
    int32_t *counts = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    if (!counts)
        return -1;
    oracle_ray_count(values, n, dim, kind, rays, m, counts);
    offsets[0] = 0;
    for (int64_t i = 0; i < m; ++i)
        offsets[i + 1] = offsets[i] + counts[i];
    free(counts);
    if (!indices)
        return 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        int64_t at = offsets[i];
        float t;
        for (int64_t j = 0; j < n; ++j)
            if (ray_value(values, j, dim, kind, rays + i * 2 * dim, &t))
                indices[at++] = (int32_t)j;
    }
    return 0;
}

/* Ray ordered intersect (Section 2.5: the hits in the order a physical ray
 * meets them): each CSR row of oracle_ray_intersect reordered by (entry
 * parameter, index), with the entry parameters in t_out.  Insertion sort: a
 * hit moves before every earlier hit with a larger entry parameter, so equal
 * parameters keep ascending indices. */
int oracle_ray_ordered_intersect(const float *values, int64_t n, int dim, int kind, const float *rays, int64_t m,
                                 const int64_t *offsets, int32_t *indices, float *t_out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        const int64_t o = offsets[i];
        int64_t len = 0;
        for (int64_t j = 0; j < n; ++j) {
            float t;
            if (!ray_value(values, j, dim, kind, rays + i * 2 * dim, &t))
                continue;
            int64_t s = len++;
            while (s > 0 && t_out[o + s - 1] > t) {
                t_out[o + s] = t_out[o + s - 1];
                indices[o + s] = indices[o + s - 1];
                --s;
            }
            t_out[o + s] = t;
            indices[o + s] = (int32_t)j;
        }
    }
    return 0;
}

/* DBSCAN (Section 2.4) by its definition, brute force: a point is core when
 * at least min_pts points (itself included) lie within eps (d2 <= fl(eps^2));
 * core points within eps of each other are connected, and each connected
 * component of core points is a cluster labelled by its smallest index; a
 * non-core point with a core point within eps is a border point and takes the
 * label of its smallest-index core neighbour; every other point is noise (-1).
 * Labelling by smallest indices makes the answer unique.  O(n^2). */
int oracle_dbscan(const float *points, int64_t n, int dim, float eps, int32_t min_pts, int32_t *labels)
{
    const float r2 = eps * eps;
    unsigned char *core = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!core || !queue) {
        free(core);
        free(queue);
        return -1;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j)
            if (dist2_point(points + i * dim, points + j * dim, dim) <= r2)
                ++c;
        core[i] = c >= min_pts;
        labels[i] = -1;
    }
    for (int64_t i = 0; i < n; ++i) {  /* components of core points, in index order */
        if (!core[i] || labels[i] >= 0)
            continue;
        int64_t head = 0, tail = 0;
        queue[tail++] = i;
        labels[i] = (int32_t)i;
        while (head < tail) {
            const int64_t a = queue[head++];
            for (int64_t b = 0; b < n; ++b)
                if (core[b] && labels[b] < 0 && dist2_point(points + a * dim, points + b * dim, dim) <= r2) {
                    labels[b] = (int32_t)i;
                    queue[tail++] = b;
                }
        }
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < n; ++j) {  /* border points: the smallest-index core neighbour */
        if (core[j])
            continue;
        for (int64_t b = 0; b < n; ++b)
            if (core[b] && dist2_point(points + j * dim, points + b * dim, dim) <= r2) {
                labels[j] = labels[b];
                break;
            }
    }
    free(core);
    free(queue);
    return 0;
}

/* Callback with output (Section 2.1, query call (2)): for every match of a
 * CSR result (row i of offsets/indices belongs to query i), the squared
 * distance between query i and the matched value, as in the search itself. */
int oracle_match_distances(const float *values, int64_t n, int dim, int kind, const float *queries, int64_t m,
                           const int64_t *offsets, const int32_t *indices, float *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = offsets[i]; p < offsets[i + 1]; ++p)
            out[p] = (indices[p] >= 0 && indices[p] < n) ? dist2_value(values, indices[p], dim, kind, queries + i * dim)
                                                         : NAN;
    return 0;
}

/* Early-terminating count (Section 2.2, the callback that stops a query's
 * search once it has seen n_max matches): values are tested in index order
 * and the count stops growing, and the scan ends, at n_max.  The paper's
 * listing compares after a post-increment, which would let the count reach
 * n_max + 1; the intended result, and this one, is min(count, n_max). */
int oracle_count_up_to(const float *values, int64_t n, int dim, int kind, const float *queries, int64_t m,
                       float radius, int32_t n_max, int32_t *counts)
{
    const float r2 = radius * radius;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        const float *q = queries + i * dim;
        int32_t c = 0;
        for (int64_t j = 0; j < n && c < n_max; ++j)
            if (dist2_value(values, j, dim, kind, q) <= r2)
                ++c;
        counts[i] = c;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* pair search (self-join)                                              */
/* ------------------------------------------------------------------ */

/* Search for pairs of objects (Section 2.6 names a dedicated traversal for
 * it; DBSCAN of Section 2.4 is built on it), read as the self-join of a point
 * set with a radius: the unordered pairs {i, j}, i != j, whose squared distance
 * is at most fl(r*r).  degree[i] = the number of j != i paired with i. */
int oracle_self_join_degree(const float *points, int64_t n, int dim, float radius, int32_t *degree)
{
    const float r2 = radius * radius;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = 0;
        for (int64_t j = 0; j < n; ++j)
            if (j != i && dist2_point(points + i * dim, points + j * dim, dim) <= r2)
                ++c;
        degree[i] = c;
    }
    return 0;
}

/* The same pairs as CSR rows of the upper triangle: row i lists the j > i
 * paired with i, ascending; offsets[n] is the number of pairs.  Call with
 * indices == NULL to get the offsets only. */
int oracle_self_join_pairs(const float *points, int64_t n, int dim, float radius, int64_t *offsets, int32_t *indices)
{
    const float r2 = radius * radius;
    offsets[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int64_t j = i + 1; j < n; ++j)
            if (dist2_point(points + i * dim, points + j * dim, dim) <= r2) {
                if (indices)
                    indices[offsets[i] + c] = (int32_t)j;
                ++c;
            }
        offsets[i + 1] = offsets[i] + c;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* nearest (kNN)                                                        */
/* ------------------------------------------------------------------ */

/* (da, ia) < (db, ib) in the order (squared distance, then index). */
static int pair_less(float da, int32_t ia, float db, int32_t ib)
{
    return da < db || (da == db && ia < ib);
}

/* The first min(k, n) values in the order (d2, index), ascending; remaining
 * slots (+inf, -1).  A sorted list of the best k so far is kept and each value
 * is inserted where it belongs, which yields the first k of the full order. */
int oracle_knn(const float *values, int64_t n, int dim, int kind, const float *queries, int64_t m, int k,
               float *dist2, int32_t *indices)
{
    if (k <= 0)
        return 1;
#pragma omp parallel
    {
        float *bd = (float *)malloc(sizeof(float) * (size_t)k);
        int32_t *bi = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < m; ++i) {
            const float *q = queries + i * dim;
            int have = 0;
            for (int64_t j = 0; j < n; ++j) {
                float d = dist2_value(values, j, dim, kind, q);
                int32_t jj = (int32_t)j;
                if (have == k && !pair_less(d, jj, bd[k - 1], bi[k - 1]))
                    continue;
                int pos = have < k ? have : k - 1;
                while (pos > 0 && pair_less(d, jj, bd[pos - 1], bi[pos - 1])) {
                    bd[pos] = bd[pos - 1];
                    bi[pos] = bi[pos - 1];
                    --pos;
                }
                bd[pos] = d;
                bi[pos] = jj;
                if (have < k)
                    ++have;
            }
            for (int s = 0; s < k; ++s) {
                dist2[i * k + s] = s < have ? bd[s] : INFINITY;
                indices[i * k + s] = s < have ? bi[s] : -1;
            }
        }
        free(bd);
        free(bi);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Chamfer loss of nearest-neighbour pairs (float64 reference)          */
/* ------------------------------------------------------------------ */

/* Nearest neighbour (k = 1, ties to the smaller index) of each point of one
 * cloud within another; -1 if the other cloud is empty. */
static void nn_cloud(const float *src, int64_t ns, const float *dst, int64_t nd, int32_t *nn, float *d2out)
{
    for (int64_t i = 0; i < ns; ++i) {
        float best = INFINITY;
        int32_t bi = -1;
        for (int64_t j = 0; j < nd; ++j) {
            float d = dist2_point(src + i * 3, dst + j * 3, 3);
            if (bi < 0 || pair_less(d, (int32_t)j, best, bi)) {
                best = d;
                bi = (int32_t)j;
            }
        }
        nn[i] = bi;
        d2out[i] = best;
    }
}

/* Pair p holds a[a_off[p]..a_off[p+1]) and b[b_off[p]..b_off[p+1]) (3D).
 * nn_ab[i] = local index in B_p of the nearest point to a_i; nn_ba likewise.
 * loss[p] = sum_i d2(a_i, B_p) + sum_j d2(b_j, A_p), float32 terms summed in
 * float64 in ascending point order (all of A_p, then all of B_p). */
int oracle_chamfer_forward(const float *a, const int64_t *a_off, const float *b, const int64_t *b_off, int P,
                           double *loss, int32_t *nn_ab, int32_t *nn_ba)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int p = 0; p < P; ++p) {
        int64_t na = a_off[p + 1] - a_off[p], nb = b_off[p + 1] - b_off[p];
        const float *ap = a + a_off[p] * 3, *bp = b + b_off[p] * 3;
        float *da = (float *)malloc(sizeof(float) * (size_t)(na > 0 ? na : 1));
        float *db = (float *)malloc(sizeof(float) * (size_t)(nb > 0 ? nb : 1));
        nn_cloud(ap, na, bp, nb, nn_ab + a_off[p], da);
        nn_cloud(bp, nb, ap, na, nn_ba + b_off[p], db);
        double s = 0.0;
        if (nb > 0)
            for (int64_t i = 0; i < na; ++i)
                s += (double)da[i];
        if (na > 0)
            for (int64_t j = 0; j < nb; ++j)
                s += (double)db[j];
        loss[p] = s;
        free(da);
        free(db);
    }
    return 0;
}

/* Gradient of loss[p] = sum_i |a_i - b_nn(i)|^2 + sum_j |b_j - a_nn(j)|^2 with
 * the neighbour assignment held fixed, times grad_loss[p]:
 *   dL/da_i = 2(a_i - b_nn(i)) + sum_{j : nn_ba(j) = i} 2(a_i - b_j)
 * and symmetrically for b.  Computed in float64 from float32 coordinates. */
int oracle_chamfer_backward(const float *a, const int64_t *a_off, const float *b, const int64_t *b_off, int P,
                            const int32_t *nn_ab, const int32_t *nn_ba, const double *grad_loss, double *grad_a,
                            double *grad_b)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int p = 0; p < P; ++p) {
        int64_t a0 = a_off[p], na = a_off[p + 1] - a0, b0 = b_off[p], nb = b_off[p + 1] - b0;
        double g = grad_loss[p];
        for (int64_t i = 0; i < na * 3; ++i)
            grad_a[a0 * 3 + i] = 0.0;
        for (int64_t j = 0; j < nb * 3; ++j)
            grad_b[b0 * 3 + j] = 0.0;
        for (int64_t i = 0; i < na; ++i) {
            int32_t j = nn_ab[a0 + i];
            if (j < 0)
                continue;
            for (int d = 0; d < 3; ++d) {
                double diff = (double)a[(a0 + i) * 3 + d] - (double)b[(b0 + j) * 3 + d];
                grad_a[(a0 + i) * 3 + d] += 2.0 * g * diff;
                grad_b[(b0 + j) * 3 + d] -= 2.0 * g * diff;
            }
        }
        for (int64_t j = 0; j < nb; ++j) {
            int32_t i = nn_ba[b0 + j];
            if (i < 0)
                continue;
            for (int d = 0; d < 3; ++d) {
                double diff = (double)b[(b0 + j) * 3 + d] - (double)a[(a0 + i) * 3 + d];
                grad_b[(b0 + j) * 3 + d] += 2.0 * g * diff;
                grad_a[(a0 + i) * 3 + d] -= 2.0 * g * diff;
            }
        }
    }
    return 0;
}
