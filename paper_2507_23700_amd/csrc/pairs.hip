// Search for pairs of objects (Section 2.6: a dedicated traversal for it) and
// density-based clustering on top of it (Section 2.4: DBSCAN on the index).
//
// The self-join of a tree's own points: thread p takes the leaf at sorted
// position p (its coordinates and value index come from the leaf record, so
// the threads of a wavefront hold Morton neighbours without any query
// ordering) and walks only the subtrees after its own leaf, so every
// unordered pair within the radius is met exactly once.  Per-pair results go
// to arrays indexed by sorted position: a pair's two positions are close in
// Morton order most of the time, so the atomics of one wavefront land in a
// few cache lines; a last pass moves them to input order.
//
// DBSCAN, three passes over the pairs, all in sorted-position space:
//   1. pair counts: a point is core when its pairs plus itself reach min_pts;
//   2. one pair walk: core-core pairs are united in a lock-free union-find
//      whose links always go from the larger root to the smaller, and each
//      non-core point keeps the smallest index among its core partners
//      (atomic minimum, from whichever side of the pair meets it);
//   3. labels: a cluster takes the smallest value index among its core
//      points, a non-core point the label of its smallest-index core partner,
//      or -1 (noise).
// Labelling by smallest indices makes the result unique, so it is compared
// with a brute-force definition element by element.
#include "device_util.hpp"
#include "geometry.hpp"
#include "internal.hpp"
#include "profile.hpp"
#include "traverse.hpp"

namespace ax {
namespace {

// Coordinates and value index of the point leaf at sorted position p.
template <int D>
__device__ __forceinline__ int load_point_leaf(const float *__restrict__ leaves, int64_t p, float (&c)[D])
{
    constexpr int F = leaf_floats(D, ARBORX_POINTS);
    const float4 *r = reinterpret_cast<const float4 *>(leaves + p * F);
    float v[F];
#pragma unroll
    for (int k = 0; k < F / 4; ++k) {
        const float4 x = r[k];
        v[4 * k] = x.x;
        v[4 * k + 1] = x.y;
        v[4 * k + 2] = x.z;
        v[4 * k + 3] = x.w;
    }
#pragma unroll
    for (int d = 0; d < D; ++d)
        c[d] = v[d];
    return __float_as_int(v[D]);
}

template <int D>
__device__ __forceinline__ int leaf_index(const float *__restrict__ leaves, int64_t p)
{
    return __float_as_int(leaves[p * leaf_floats(D, ARBORX_POINTS) + D]);
}

// Pass 1: deg[q] = partners of the point at sorted position q.
template <int D>
__global__ void k_pair_degree(const Node<D> *__restrict__ nodes, const float *__restrict__ leaves, int64_t n,
                              float r2, int32_t *__restrict__ deg)
{
    const int64_t p = xcd_block() * blockDim.x + threadIdx.x;
    if (p >= n - 1)  // the last position has no later partner
        return;
    Sphere<D> pred;
    load_point_leaf<D>(leaves, p, pred.c);
    pred.r2 = r2;
    int c = 0;
    auto f = [&](int q, int, float) {
        ++c;
        atomicAdd(deg + q, 1);
    };
    traverse_pairs_after<D>(nodes, (int)(n - 1), (int)p, (int)(n - 1), pred, f);
    if (c)
        atomicAdd(deg + p, c);
}

// out[index of the leaf at q] = by_pos[q].
template <int D>
__global__ void k_to_input_order(const int32_t *__restrict__ by_pos, const float *__restrict__ leaves, int64_t n,
                                 int32_t *__restrict__ out)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int id = leaf_index<D>(leaves, q);
        if (id >= 0 && id < n)
            out[id] = by_pos[q];
    }
}

__device__ __forceinline__ int32_t load_parent(const int32_t *parent, int32_t x)
{
    return __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x.  Every link points to a smaller position (unions link the larger
// root to the smaller; shortcuts below point a node at a smaller member of its
// own chain), so a chain strictly decreases and ends at a root.  The nodes
// above the root found are then pointed at it: they are not roots (and never
// become roots again), and the root is a smaller member of the same
// component, so the links still decrease.  Another thread may have shortcut a
// node past r meanwhile; the walk stops at the first node not above r, so it
// never points a smaller node at a larger one.
__device__ __forceinline__ int32_t find_root(int32_t *parent, int32_t x)
{
    int32_t r = x, p = load_parent(parent, r);
    while (p != r) {
        r = p;
        p = load_parent(parent, r);
    }
    while (x > r) {
        const int32_t next = load_parent(parent, x);
        if (next != r)
            __hip_atomic_store(parent + x, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = next;
    }
    return r;
}

// Link the components of a and b: the larger root is pointed at the smaller.
// A failed exchange means another thread linked that root meanwhile, which can
// happen at most n - 1 times in all, so the bounded loop always finishes.
__device__ __forceinline__ void unite(int32_t *parent, int32_t a, int32_t b, int64_t n)
{
    for (int64_t iter = 0; iter <= n; ++iter) {
        a = find_root(parent, a);
        b = find_root(parent, b);
        if (a == b)
            return;
        if (a < b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(parent + a, a, b) == a)
            return;
    }
}

__global__ void k_dbscan_init(int32_t *__restrict__ parent, int32_t *__restrict__ border,
                              int32_t *__restrict__ cmin, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        parent[i] = (int32_t)i;
        border[i] = INT32_MAX;
        cmin[i] = INT32_MAX;
    }
}

// Pass 2: one pair walk per position.
template <int D>
__global__ void k_dbscan_pairs(const Node<D> *__restrict__ nodes, const float *__restrict__ leaves, int64_t n,
                               float r2, int min_pts, const int32_t *__restrict__ deg, int32_t *__restrict__ parent,
                               int32_t *__restrict__ border)
{
    const int64_t p = xcd_block() * blockDim.x + threadIdx.x;
    if (p >= n - 1)
        return;
    Sphere<D> pred;
    const int id = load_point_leaf<D>(leaves, p, pred.c);
    pred.r2 = r2;
    const bool core_p = deg[p] + 1 >= min_pts;
    int best = INT32_MAX;
    auto f = [&](int q, int qid, float) {
        const bool core_q = deg[q] + 1 >= min_pts;
        if (core_p && core_q)
            unite(parent, (int32_t)p, q, n);
        else if (core_p)
            atomicMin(border + q, id);
        else if (core_q)
            best = qid < best ? qid : best;
    };
    traverse_pairs_after<D>(nodes, (int)(n - 1), (int)p, (int)(n - 1), pred, f);
    if (best != INT32_MAX)
        atomicMin(border + p, best);
}

// Pass 3a: the smallest value index of each cluster, kept at its root.
template <int D>
__global__ void k_dbscan_cluster_min(int32_t *__restrict__ parent, const int32_t *__restrict__ deg, int64_t n,
                                     int min_pts, const float *__restrict__ leaves, int32_t *__restrict__ cmin)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        if (deg[q] + 1 >= min_pts)
            atomicMin(cmin + find_root(parent, (int32_t)q), leaf_index<D>(leaves, q));
}

// Pass 3b: labels of core points.
template <int D>
__global__ void k_dbscan_core_labels(int32_t *__restrict__ parent, const int32_t *__restrict__ deg, int64_t n,
                                     int min_pts, const float *__restrict__ leaves,
                                     const int32_t *__restrict__ cmin, int32_t *__restrict__ labels)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        if (deg[q] + 1 >= min_pts) {
            const int id = leaf_index<D>(leaves, q);
            if (id >= 0 && id < n)
                labels[id] = cmin[find_root(parent, (int32_t)q)];
        }
}

// Pass 3c: labels of the other points, from their smallest-index core
// partner (labelled in pass 3b), else noise.
template <int D>
__global__ void k_dbscan_border_labels(const int32_t *__restrict__ deg, const int32_t *__restrict__ border, int64_t n,
                                       int min_pts, const float *__restrict__ leaves, int32_t *__restrict__ labels)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        if (deg[q] + 1 < min_pts) {
            const int id = leaf_index<D>(leaves, q);
            const int b = border[q];
            if (id >= 0 && id < n)
                labels[id] = (b >= 0 && b < n) ? labels[b] : -1;
        }
}

constexpr int kPairBlock = 256;

template <int D>
arborx_status degree_by_position(const TreeDev &t, float r2, int32_t *deg, hipStream_t s)
{
    const int64_t n = t.n;
    fill_kernel<int32_t><<<grid_for(n, 256, 65536), 256, 0, s>>>(deg, n, 0);
    if (n > 1) {
        ProfScope ps("pair_degree", s);
        k_pair_degree<D><<<grid_for(n - 1, kPairBlock, INT32_MAX), kPairBlock, 0, s>>>(
            static_cast<const Node<D> *>(t.nodes), t.leaves, n, r2, deg);
    }
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

template <int D>
arborx_status self_join_degree_impl(const TreeDev &t, float r2, int32_t *degree, Temps &tmp, hipStream_t s)
{
    int32_t *deg;
    arborx_status st = tmp.get(&deg, t.n);
    if (st != ARBORX_OK || (st = degree_by_position<D>(t, r2, deg, s)) != ARBORX_OK)
        return st;
    k_to_input_order<D><<<grid_for(t.n, 256, 65536), 256, 0, s>>>(deg, t.leaves, t.n, degree);
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

template <int D>
arborx_status dbscan_impl(const TreeDev &t, float eps, int min_pts, int32_t *labels, Temps &tmp, hipStream_t s)
{
    const int64_t n = t.n;
    const float r2 = eps * eps;
    int32_t *deg, *parent, *border, *cmin;
    arborx_status st;
    if ((st = tmp.get(&deg, n)) != ARBORX_OK || (st = tmp.get(&parent, n)) != ARBORX_OK ||
        (st = tmp.get(&border, n)) != ARBORX_OK || (st = tmp.get(&cmin, n)) != ARBORX_OK)
        return st;
    if ((st = degree_by_position<D>(t, r2, deg, s)) != ARBORX_OK)
        return st;
    ProfScope ps("dbscan", s);
    const unsigned g = grid_for(n, 256, 65536);
    k_dbscan_init<<<g, 256, 0, s>>>(parent, border, cmin, n);
    if (n > 1)
        k_dbscan_pairs<D><<<grid_for(n - 1, kPairBlock, INT32_MAX), kPairBlock, 0, s>>>(
            static_cast<const Node<D> *>(t.nodes), t.leaves, n, r2, min_pts, deg, parent, border);
    k_dbscan_cluster_min<D><<<g, 256, 0, s>>>(parent, deg, n, min_pts, t.leaves, cmin);
    k_dbscan_core_labels<D><<<g, 256, 0, s>>>(parent, deg, n, min_pts, t.leaves, cmin, labels);
    k_dbscan_border_labels<D><<<g, 256, 0, s>>>(deg, border, n, min_pts, t.leaves, labels);
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

}  // namespace

arborx_status self_join_degree(const TreeDev &t, float radius, int32_t *degree, hipStream_t s)
{
    if (t.n == 0)
        return ARBORX_OK;
    Temps tmp(s);
    const float r2 = radius * radius;
    switch (t.dim) {
    case 2: return self_join_degree_impl<2>(t, r2, degree, tmp, s);
    case 3: return self_join_degree_impl<3>(t, r2, degree, tmp, s);
    case 6: return self_join_degree_impl<6>(t, r2, degree, tmp, s);
    default: return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in");
    }
}

arborx_status dbscan(const TreeDev &t, float eps, int min_pts, int32_t *labels, hipStream_t s)
{
    if (t.n == 0)
        return ARBORX_OK;
    Temps tmp(s);
    switch (t.dim) {
    case 2: return dbscan_impl<2>(t, eps, min_pts, labels, tmp, s);
    case 3: return dbscan_impl<3>(t, eps, min_pts, labels, tmp, s);
    case 6: return dbscan_impl<6>(t, eps, min_pts, labels, tmp, s);
    default: return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in");
    }
}

}  // namespace ax
