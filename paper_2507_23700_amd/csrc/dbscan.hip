// Density-based clustering on top of the radius search (Section 2.4: DBSCAN
// built on the index's fused queries).  Three passes over the tree:
//   1. core points: a fused COUNT of the points within eps of each point
//      (itself included), core when at least min_pts;
//   2. clusters: every core point walks its eps-ball and unites itself with the
//      core neighbours of larger index in a lock-free union-find whose links
//      always go from the larger root to the smaller, so each component's root
//      ends as its smallest index, whatever the order of the unions;
//   3. labels: core points take their root; a non-core point takes the label of
//      its smallest-index core neighbour, or -1 (noise).
// Labelling by smallest indices makes the result unique, so it is compared
// with a brute-force definition element by element.
#include "device_util.hpp"
#include "geometry.hpp"
#include "internal.hpp"
#include "profile.hpp"
#include "traverse.hpp"

namespace ax {
namespace {

__device__ __forceinline__ int32_t load_parent(const int32_t *parent, int32_t x)
{
    return __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x: parents only ever point to smaller indices, so the chain is
// strictly decreasing and ends.
__device__ __forceinline__ int32_t find_root(const int32_t *parent, int32_t x)
{
    int32_t p = load_parent(parent, x);
    while (p != x) {
        x = p;
        p = load_parent(parent, x);
    }
    return x;
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

__global__ void k_dbscan_init(int32_t *__restrict__ parent, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        parent[i] = (int32_t)i;
}

// Pass 2: thread t handles point perm[t] (Morton order keeps walks coherent).
template <int D>
__global__ void k_dbscan_union(const Node<D> *__restrict__ nodes, const TreeHeader *__restrict__ hdr,
                               const float *__restrict__ points, int64_t n, float r2, int min_pts,
                               const int32_t *__restrict__ counts, const uint32_t *__restrict__ perm,
                               int32_t *__restrict__ parent, int stack_cap)
{
    extern __shared__ int s_stack[];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n)
        return;
    const int64_t i = perm ? (int64_t)perm[t] : t;
    if (i < 0 || i >= n || counts[i] < min_pts)
        return;
    Sphere<D> pred;
    pred.load(points, i, r2);
    int spill[kSpill];
    ShortStack<int> st(s_stack + threadIdx.x, blockDim.x, stack_cap, spill);
    auto f = [&](int j, float) {
        if (j > i && j < n && counts[j] >= min_pts)
            unite(parent, (int32_t)i, j, n);
    };
    traverse_spatial<D>(nodes, hdr->root, hdr->n > 1 ? hdr->n - 1 : 1, pred, st, f);
}

__global__ void k_dbscan_core_labels(const int32_t *__restrict__ parent, const int32_t *__restrict__ counts,
                                     int64_t n, int min_pts, int32_t *__restrict__ labels)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        labels[i] = counts[i] >= min_pts ? find_root(parent, (int32_t)i) : -1;
}

// Pass 3 for non-core points: the label of the smallest-index core neighbour.
template <int D>
__global__ void k_dbscan_border(const Node<D> *__restrict__ nodes, const TreeHeader *__restrict__ hdr,
                                const float *__restrict__ points, int64_t n, float r2, int min_pts,
                                const int32_t *__restrict__ counts, const uint32_t *__restrict__ perm,
                                int32_t *__restrict__ labels, int stack_cap)
{
    extern __shared__ int s_stack[];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n)
        return;
    const int64_t i = perm ? (int64_t)perm[t] : t;
    if (i < 0 || i >= n || counts[i] >= min_pts)
        return;
    Sphere<D> pred;
    pred.load(points, i, r2);
    int spill[kSpill];
    ShortStack<int> st(s_stack + threadIdx.x, blockDim.x, stack_cap, spill);
    int best = INT32_MAX;
    auto f = [&](int j, float) {
        if (j < best && j < n && counts[j] >= min_pts)
            best = j;
    };
    traverse_spatial<D>(nodes, hdr->root, hdr->n > 1 ? hdr->n - 1 : 1, pred, st, f);
    labels[i] = best == INT32_MAX ? -1 : labels[best];
}

template <int D>
arborx_status dbscan_impl(const TreeDev &t, const float *points, float eps, int min_pts, const uint32_t *perm,
                          int32_t *counts, int32_t *parent, int32_t *labels, hipStream_t s)
{
    const int64_t n = t.n;
    const float r2 = eps * eps;
    const Tuning &tu = tuning(OP_REDUCE);
    const int block = tu.block;
    int cap = tu.stack;
    while (cap > 1 && (size_t)cap * block * sizeof(int) > 65536)
        cap >>= 1;
    const size_t lds = (size_t)cap * block * sizeof(int);
    const unsigned grid = (unsigned)((n + block - 1) / block);
    const Node<D> *nodes = static_cast<const Node<D> *>(t.nodes);
    ProfScope ps("dbscan", s);
    k_dbscan_init<<<grid_for(n, 256, 65536), 256, 0, s>>>(parent, n);
    k_dbscan_union<D><<<grid, block, lds, s>>>(nodes, t.hdr, points, n, r2, min_pts, counts, perm, parent, cap);
    k_dbscan_core_labels<<<grid_for(n, 256, 65536), 256, 0, s>>>(parent, counts, n, min_pts, labels);
    k_dbscan_border<D><<<grid, block, lds, s>>>(nodes, t.hdr, points, n, r2, min_pts, counts, perm, labels, cap);
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

}  // namespace

arborx_status dbscan(const TreeDev &t, const float *points, float eps, int min_pts, const uint32_t *perm,
                     int32_t *counts, int32_t *parent, int32_t *labels, hipStream_t s)
{
    if (t.n == 0)
        return ARBORX_OK;
    switch (t.dim) {
    case 2: return dbscan_impl<2>(t, points, eps, min_pts, perm, counts, parent, labels, s);
    case 3: return dbscan_impl<3>(t, points, eps, min_pts, perm, counts, parent, labels, s);
    case 6: return dbscan_impl<6>(t, points, eps, min_pts, perm, counts, parent, labels, s);
    default: return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in");
    }
}

}  // namespace ax
