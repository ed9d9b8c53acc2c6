// Search for pairs of objects (Section 2.6: a dedicated traversal for it) and
// density-based clustering on top of it (Section 2.4: DBSCAN on the index).
//
// The self-join of a tree's own points: a thread takes consecutive leaves in
// sorted order (coordinates and value indices come from the leaf records, so
// the threads of a wavefront hold Morton neighbours without any query
// ordering) and visits only the subtrees after its own leaves, so every
// unordered pair within the radius is met exactly once.  Two walks give the
// same pairs: a top-down packet walk over several leaves per thread (the
// default) and the stackless walk from each leaf's own rope (schedule 2).
// Pair counts go to an array indexed by sorted position: a pair's two
// positions are close in Morton order most of the time, so the atomics of one
// wavefront land in a few cache lines; a last pass moves them to input order.
//
// DBSCAN, two passes over the pairs:
//   1. pair counts: a point is core when its pairs plus itself reach min_pts;
//   2. one pair walk: core-core pairs are united in a lock-free union-find
//      over value indices whose links always go from the larger root to the
//      smaller, so each cluster's root ends as its smallest core index (over
//      sorted positions instead, the lanes of a wavefront, Morton neighbours,
//      contend for the same few roots: eight times slower at 10^7 points); each
//      non-core point keeps the smallest index among its core partners
//      (atomic minimum, from whichever side of the pair meets it);
// then labels: a core point takes its root, a non-core point the label of its
// smallest-index core partner, or -1 (noise).  Labelling by smallest indices
// makes the result unique, so it is compared with a brute-force definition
// element by element.
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

// Pass 1: deg[q] = partners of the point at sorted position q.  NQ leaves per
// thread over the packet walk, or (NQ = 0) one leaf per thread over its rope;
// Q: one leaf per thread over the quantized nodes.
template <int D, int NQ, bool Q = false>
__global__ void k_pair_degree(const Node<D> *__restrict__ nodes, const QNode<D> *__restrict__ qnodes,
                              const TreeHeader *__restrict__ hdr,
                              const float *__restrict__ leaves, int64_t n, float r2, int32_t *__restrict__ deg,
                              int stack_cap)
{
    extern __shared__ int s_stack[];
    constexpr int W = NQ ? NQ : 1;
    const int64_t p0 = (xcd_block() * blockDim.x + threadIdx.x) * W;
    if (p0 >= n - 1)  // the last position has no later partner
        return;
    Sphere<D> pred[W];
    int c[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        c[j] = 0;
        if (p0 + j < n - 1) {
            load_point_leaf<D>(leaves, p0 + j, pred[j].c);
            pred[j].r2 = r2;
        } else {
            pred[j].dead();
        }
    }
    if constexpr (NQ == 0) {
        auto f = [&](int q, int, float) {
            ++c[0];
            atomicAdd(deg + q, 1);
        };
        traverse_pairs_after<D>(nodes, (int)(n - 1), (int)p0, (int)(n - 1), pred[0], f);
    } else {
        int spill[kSpill];
        ShortStack<int> st(s_stack + threadIdx.x, blockDim.x, stack_cap, spill);
        auto f = [&](int j, int q, int, float) {
#pragma unroll
            for (int jj = 0; jj < W; ++jj)
                if (jj == j)
                    ++c[jj];
            atomicAdd(deg + q, 1);
        };
        if constexpr (Q) {
            auto f1 = [&](int q, int qid, float d) { f(0, q, qid, d); };
            traverse_pairs_q<D>(qnodes, *hdr, (int)(n - 1), (int)p0, pred[0], st, f1);
        } else {
            traverse_pairs_packet<D, W>(nodes, hdr->root, (int)(n - 1), (int)p0, pred, st, f);
        }
    }
#pragma unroll
    for (int j = 0; j < W; ++j)
        if (c[j])
            atomicAdd(deg + p0 + j, c[j]);
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

// Parent links are read and shortened with workgroup-scope accesses, which
// the per-XCD L2 serves, so another XCD's recent link may not be visible yet.
// That is safe: links only ever go from a value to a smaller value of the same
// component and are never undone, so a stale parent is still an ancestor, and
// a stale root is caught by the exchange in unite, which is device-wide and
// returns the true parent.
__device__ __forceinline__ int32_t load_parent(const int32_t *parent, int32_t x)
{
    return __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Root of x.  Every link points to a smaller index (unions link the larger
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
            __hip_atomic_store(parent + x, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        x = next;
    }
    return r;
}

// Link the components of a and b: the larger root is pointed at the smaller
// by a device-wide exchange.  When it fails, the value it returns is that
// root's true parent, smaller than it, and the walk goes on from there; so
// every failure moves one of the two ends to a smaller index, and at most 2n
// rounds finish.  Returns the root the merged component had when the link
// was made: an ancestor of both a and b from then on (links are never
// undone), so a caller may start its next find there instead of at a.
__device__ __forceinline__ int32_t unite(int32_t *parent, int32_t a, int32_t b, int64_t n)
{
    a = find_root(parent, a);
    b = find_root(parent, b);
    for (int64_t iter = 0; iter <= 2 * n + 1; ++iter) {
        if (a == b)
            return a;
        if (a < b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        const int32_t old = atomicCAS(parent + a, a, b);
        if (old == a)
            return b;
        a = find_root(parent, old);
        b = find_root(parent, b);
    }
    return b;
}

__global__ void k_dbscan_init(int32_t *__restrict__ parent, int32_t *__restrict__ border, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        parent[i] = (int32_t)i;
        border[i] = INT32_MAX;
    }
}

// Pass 2: one pair walk, NQ leaves per thread (NQ = 0: the rope walk; Q: one
// leaf per thread over the quantized nodes).  parent is indexed by value
// index, deg and border by sorted position.
template <int D, int NQ, bool Q = false>
__global__ void k_dbscan_pairs(const Node<D> *__restrict__ nodes, const QNode<D> *__restrict__ qnodes,
                               const TreeHeader *__restrict__ hdr,
                               const float *__restrict__ leaves, int64_t n, float r2, int min_pts,
                               const int32_t *__restrict__ deg, int32_t *__restrict__ parent,
                               int32_t *__restrict__ border, int stack_cap)
{
    extern __shared__ int s_stack[];
    constexpr int W = NQ ? NQ : 1;
    const int64_t p0 = (xcd_block() * blockDim.x + threadIdx.x) * W;
    if (p0 >= n - 1)
        return;
    Sphere<D> pred[W];
    int id[W], best[W], root[W];  // root: an ancestor of id in the union-find forest, where finds start
    bool core[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        best[j] = INT32_MAX;
        core[j] = false;
        id[j] = -1;
        if (p0 + j < n - 1) {
            id[j] = load_point_leaf<D>(leaves, p0 + j, pred[j].c);
            pred[j].r2 = r2;
            core[j] = deg[p0 + j] + 1 >= min_pts;
        } else {
            pred[j].dead();
        }
    }
#pragma unroll
    for (int j = 0; j < W; ++j)
        root[j] = id[j];
    auto pair = [&](int j, int q, int qid) {
        const bool core_q = deg[q] + 1 >= min_pts;
#pragma unroll
        for (int jj = 0; jj < W; ++jj)
            if (jj == j) {
                if (core[jj] && core_q)
                    root[jj] = unite(parent, root[jj], qid, n);
                else if (core[jj])
                    atomicMin(border + q, id[jj]);
                else if (core_q)
                    best[jj] = qid < best[jj] ? qid : best[jj];
            }
    };
    if constexpr (NQ == 0) {
        auto f = [&](int q, int qid, float) { pair(0, q, qid); };
        traverse_pairs_after<D>(nodes, (int)(n - 1), (int)p0, (int)(n - 1), pred[0], f);
    } else {
        int spill[kSpill];
        ShortStack<int> st(s_stack + threadIdx.x, blockDim.x, stack_cap, spill);
        auto f = [&](int j, int q, int qid, float) { pair(j, q, qid); };
        if constexpr (Q) {
            auto f1 = [&](int q, int qid, float) { pair(0, q, qid); };
            traverse_pairs_q<D>(qnodes, *hdr, (int)(n - 1), (int)p0, pred[0], st, f1);
        } else {
            traverse_pairs_packet<D, W>(nodes, hdr->root, (int)(n - 1), (int)p0, pred, st, f);
        }
    }
#pragma unroll
    for (int j = 0; j < W; ++j)
        if (best[j] != INT32_MAX)
            atomicMin(border + p0 + j, best[j]);
}

// Labels of core points: the root of their value index, the cluster's
// smallest core index.
template <int D>
__global__ void k_dbscan_core_labels(int32_t *__restrict__ parent, const int32_t *__restrict__ deg, int64_t n,
                                     int min_pts, const float *__restrict__ leaves, int32_t *__restrict__ labels)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        if (deg[q] + 1 >= min_pts) {
            const int id = leaf_index<D>(leaves, q);
            if (id >= 0 && id < n)
                labels[id] = find_root(parent, id);
        }
}

// Labels of the other points, from their smallest-index core partner
// (labelled by the previous pass), else noise.
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

// Launch shape of the pair walks: the reductions' tuning (block, stack; the
// rope walk for schedule 2), with NQ leaves per thread over the packet walk
// (queries_per_thread, else 2 up to 3D and 1 in 6D: at 10^7 points in 3D, two
// leaves per thread ran DBSCAN's pair pass fastest and the pair count as fast
// as four, on float nodes).  On quantized nodes the default is one leaf per
// thread over them: at 10^7 points in 3D the pair count took 2.22 ms against
// 2.44 ms for two leaves per thread on float nodes, DBSCAN 8.3 against 9.2 ms.
struct PairLaunch {
    int nq, block, cap;
    bool q;  // one leaf per thread over the quantized nodes
    unsigned grid;
    size_t lds;
};

// The pair walks follow the reductions' tuning (schedule, queries per thread,
// node format, launch shape).
PairLaunch pair_launch(const TreeDev &t)
{
    const int64_t n = t.n;
    const int dim = t.dim;
    const Tuning &tu = tuning(OP_REDUCE);
    PairLaunch L;
    const bool qf = tree_format(OP_REDUCE, t) == 1 && t.qnodes;
    L.nq = tu.schedule == 2 ? 0 : (tu.packet ? tu.packet : (dim <= 3 && !qf ? 2 : 1));
    L.q = L.nq == 1 && qf;
    launch_shape(OP_REDUCE, dim, L.block, L.cap);
    while (L.cap > 1 && (size_t)L.cap * L.block * sizeof(int) > 65536)
        L.cap >>= 1;
    L.lds = L.nq ? (size_t)L.cap * L.block * sizeof(int) : 0;
    const int64_t per = L.nq ? L.nq : 1;
    L.grid = grid_for((n - 1 + per - 1) / per, L.block, INT32_MAX);
    return L;
}

template <int D>
arborx_status degree_by_position(const TreeDev &t, float r2, int32_t *deg, hipStream_t s)
{
    const int64_t n = t.n;
    fill_kernel<int32_t><<<grid_for(n, 256, 65536), 256, 0, s>>>(deg, n, 0);
    if (n > 1) {
        const PairLaunch L = pair_launch(t);
        const Node<D> *nodes = static_cast<const Node<D> *>(t.nodes);
        ProfScope ps("pair_degree", s);
        const QNode<D> *qnodes = static_cast<const QNode<D> *>(t.qnodes);
#define AX_PD(NQ, QF) \
    k_pair_degree<D, NQ, QF><<<L.grid, L.block, L.lds, s>>>(nodes, qnodes, t.hdr, t.leaves, n, r2, deg, L.cap)
        if (L.nq == 0)
            AX_PD(0, false);
        else if (L.q)
            AX_PD(1, true);
        else if (L.nq == 1)
            AX_PD(1, false);
        else if (L.nq == 2)
            AX_PD(2, false);
        else
            AX_PD(4, false);
#undef AX_PD
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
    int32_t *deg, *parent, *border;
    arborx_status st;
    if ((st = tmp.get(&deg, n)) != ARBORX_OK || (st = tmp.get(&parent, n)) != ARBORX_OK ||
        (st = tmp.get(&border, n)) != ARBORX_OK)
        return st;
    if ((st = degree_by_position<D>(t, r2, deg, s)) != ARBORX_OK)
        return st;
    ProfScope ps("dbscan", s);
    const unsigned g = grid_for(n, 256, 65536);
    k_dbscan_init<<<g, 256, 0, s>>>(parent, border, n);
    if (n > 1) {
        const PairLaunch L = pair_launch(t);
        const Node<D> *nodes = static_cast<const Node<D> *>(t.nodes);
        const QNode<D> *qnodes = static_cast<const QNode<D> *>(t.qnodes);
#define AX_DP(NQ, QF)                                                                                             \
    k_dbscan_pairs<D, NQ, QF><<<L.grid, L.block, L.lds, s>>>(nodes, qnodes, t.hdr, t.leaves, n, r2, min_pts, deg, \
                                                             parent, border, L.cap)
        if (L.nq == 0)
            AX_DP(0, false);
        else if (L.q)
            AX_DP(1, true);
        else if (L.nq == 1)
            AX_DP(1, false);
        else if (L.nq == 2)
            AX_DP(2, false);
        else
            AX_DP(4, false);
#undef AX_DP
    }
    k_dbscan_core_labels<D><<<g, 256, 0, s>>>(parent, deg, n, min_pts, t.leaves, labels);
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
