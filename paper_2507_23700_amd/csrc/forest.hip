// Forest queries: B batches of queries, batch b = queries [boff[b], boff[b+1])
// searched in tree btree[b] of a forest (radius btree-specific for reductions).
//
// 1. ordering: each query gets the key (batch << mbits) | Morton code of the
//    query inside its target tree's box, and one radix sort orders all
//    queries by batch, then along the curve inside the batch;
// 2. one persistent launch: a grid sized to fill the GPU once, each
//    workgroup repeatedly takes the next block of sorted queries from an
//    atomic counter until none are left, so uneven batches and uneven
//    per-query work balance dynamically.  Each lane answers one query against
//    its batch's tree.
// The query path allocates nothing once the forest's workspace is reserved, and
// never synchronises, so it can be captured in a hipGraph.  Results use indices
// local to the target tree (value index minus the tree's first value), the
// same as querying that tree built on its own.
#include <algorithm>

#include "device_util.hpp"
#include "geometry.hpp"
#include "internal.hpp"
#include "profile.hpp"
#include "traverse.hpp"

namespace ax {
namespace {

constexpr int kForestBlock = 256;

__device__ __forceinline__ int batch_of(const int64_t *__restrict__ boff, int B, int64_t i)
{
    int lo = 0, hi = B;  // last b with boff[b] <= i
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (boff[mid] <= i)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

template <int D, typename K>
__global__ void k_forest_codes(const float *__restrict__ q, int64_t m, const int64_t *__restrict__ boff, int B,
                               const int32_t *__restrict__ btree, int T, const TreeHeader *__restrict__ hdrs,
                               int mbits, K *__restrict__ codes, uint32_t *__restrict__ ids)
{
    const int bits = mbits / D;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int b = batch_of(boff, B, i);
        const int t = btree[b];
        uint32_t c[D];
        if (t >= 0 && t < T && hdrs[t].n > 0) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const float lo = hdrs[t].lo[d], ext = hdrs[t].hi[d] - lo;
                c[d] = quantise(q[i * D + d], lo, ext > 0.0f ? 1.0f / ext : 0.0f, bits);
            }
        } else {
#pragma unroll
            for (int d = 0; d < D; ++d)
                c[d] = 0;
        }
        codes[i] = ((K)b << mbits) | (K)interleave<D>(c, bits);
        ids[i] = (uint32_t)i;
    }
}

// Next block of `span` sorted positions for this workgroup (one per thread by
// default), or -1 when all are taken.
__device__ __forceinline__ int64_t next_block(unsigned long long *counter, int64_t m, int64_t span = 0)
{
    __shared__ int64_t s_start;
    if (threadIdx.x == 0) {
        const unsigned long long c = atomicAdd(counter, 1ull);
        s_start = (int64_t)c * (span > 0 ? span : (int64_t)blockDim.x);
    }
    __syncthreads();
    const int64_t start = s_start;
    __syncthreads();
    return start < m ? start : -1;
}

template <int D, bool SUMDIST, int FMT>
__global__ __launch_bounds__(kForestBlock) void k_forest_reduce(
    const Node<D> *__restrict__ nodes, const QNode<D> *__restrict__ qnodes, const Node4<D> *__restrict__ wnodes,
    const float *__restrict__ leaves, int kind,
    int n_nodes, const TreeHeader *__restrict__ hdrs, int T,
    const float *__restrict__ queries, int64_t m, const uint32_t *__restrict__ perm, const int64_t *__restrict__ boff,
    int B, const int32_t *__restrict__ btree, const float *__restrict__ bradius, float scale, int32_t *__restrict__ counts,
    int64_t *__restrict__ sums, unsigned long long *counter, int stack_cap)
{
    extern __shared__ int s_stack[];
    int spill[kSpill];
    for (int64_t start; (start = next_block(counter, m)) >= 0;) {
        const int64_t t = start + threadIdx.x;
        if (t >= m)
            continue;
        const int64_t qi = perm[t];
        if (qi < 0 || qi >= m)
            continue;
        const int b = batch_of(boff, B, qi);
        const int tr = btree[b];
        int c = 0;
        long long s = 0;
        if (tr >= 0 && tr < T) {
            const float r = bradius[b];
            Sphere<D> pred;
            pred.load(queries, qi, r * r);
            ShortStack<int> st(s_stack + threadIdx.x, blockDim.x, stack_cap, spill);
            auto f = [&](int, float d2) {
                ++c;
                if (SUMDIST)
                    s += fixed_term(d2, scale);
            };
            if (FMT == 1)
                traverse_spatial_q<D>(qnodes, hdrs[tr], n_nodes, leaves, kind, pred, st, f);
            else if (FMT == 2)
                traverse_spatial4<D>(wnodes, hdrs[tr].root, n_nodes, pred, st, f);
            else
                traverse_spatial<D>(nodes, hdrs[tr].root, n_nodes, pred, st, f);
        }
        counts[qi] = c;
        if (SUMDIST)
            sums[qi] = s;
    }
}

// Packet form of the forest reduction (binary nodes): thread t of a block
// takes NQ consecutive sorted positions.  Sorting is by (batch, Morton code),
// so they usually share a batch and tree and are walked together; a packet
// that straddles trees is walked one query at a time.
template <int D, bool SUMDIST, int NQ>
__global__ __launch_bounds__(kForestBlock) void k_forest_reduce_packet(
    const Node<D> *__restrict__ nodes, int n_nodes, const TreeHeader *__restrict__ hdrs, int T,
    const float *__restrict__ queries, int64_t m, const uint32_t *__restrict__ perm, const int64_t *__restrict__ boff,
    int B, const int32_t *__restrict__ btree, const float *__restrict__ bradius, float scale, int32_t *__restrict__ counts,
    int64_t *__restrict__ sums, unsigned long long *counter, int stack_cap)
{
    extern __shared__ int s_stack[];
    int spill[kSpill];
    for (int64_t start; (start = next_block(counter, m, (int64_t)kForestBlock * NQ)) >= 0;) {
        int64_t qi[NQ];
        int tr[NQ];
        Sphere<D> pred[NQ];
        bool same = true;
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            const int64_t p = start + (int64_t)threadIdx.x * NQ + j;
            qi[j] = p < m ? (int64_t)perm[p] : -1;
            tr[j] = -1;
            if (qi[j] >= 0 && qi[j] < m) {
                const int b = batch_of(boff, B, qi[j]);
                tr[j] = btree[b] >= 0 && btree[b] < T ? btree[b] : -1;
                const float r = bradius[b];
                pred[j].load(queries, qi[j], r * r);
            } else {
                qi[j] = -1;
                pred[j].dead();
            }
            if (qi[j] >= 0 && tr[j] != tr[0])
                same = false;
        }
        int c[NQ];
        long long s[NQ];
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            c[j] = 0;
            s[j] = 0;
        }
        ShortStack<int> st(s_stack + threadIdx.x, blockDim.x, stack_cap, spill);
        if (same && tr[0] >= 0) {
            auto f = [&](int j, int, float d2) {
#pragma unroll
                for (int jj = 0; jj < NQ; ++jj)
                    if (jj == j) {
                        ++c[jj];
                        if (SUMDIST)
                            s[jj] += fixed_term(d2, scale);
                    }
            };
            traverse_spatial_packet<D, NQ>(nodes, hdrs[tr[0]].root, n_nodes, pred, st, f);
        } else {
#pragma unroll
            for (int j = 0; j < NQ; ++j)
                if (qi[j] >= 0 && tr[j] >= 0) {
                    st.clear();
                    auto f = [&](int, float d2) {
                        ++c[j];
                        if (SUMDIST)
                            s[j] += fixed_term(d2, scale);
                    };
                    traverse_spatial<D>(nodes, hdrs[tr[j]].root, n_nodes, pred[j], st, f);
                }
        }
#pragma unroll
        for (int j = 0; j < NQ; ++j)
            if (qi[j] >= 0) {
                counts[qi[j]] = c[j];
                if (SUMDIST)
                    sums[qi[j]] = s[j];
            }
    }
}

template <int D, int K, int FMT>
__global__ __launch_bounds__(kForestBlock) void k_forest_knn(
    const Node<D> *__restrict__ nodes, const QNode<D> *__restrict__ qnodes, const Node4<D> *__restrict__ wnodes,
    int n_nodes,
    const float *__restrict__ leaves, int kind,
    const TreeHeader *__restrict__ hdrs, int T, const float *__restrict__ queries, int64_t m,
    const uint32_t *__restrict__ perm, const int64_t *__restrict__ boff, int B, const int32_t *__restrict__ btree,
    int k_out, float *__restrict__ out_d2, int32_t *__restrict__ out_idx, unsigned long long *counter, int stack_cap,
    int seed, const uint64_t *__restrict__ keys, int mbits)
{
    extern __shared__ int s_stack[];
    KnnEntry spill[kSpill];
    for (int64_t start; (start = next_block(counter, m)) >= 0;) {
        const int64_t t = start + threadIdx.x;
        if (t >= m)
            continue;
        const int64_t qi = perm[t];
        if (qi < 0 || qi >= m)
            continue;
        const int b = batch_of(boff, B, qi);
        const int tr = btree[b];
        TopK<K> best;
        TreeHeader h;
        if (tr >= 0 && tr < T) {
            h = hdrs[tr];
        } else {
            h.n = 0;
            h.root = -1;
            h.start = 0;
        }
        float q[D];
#pragma unroll
        for (int d = 0; d < D; ++d)
            q[d] = queries[qi * D + d];
        ShortStack<KnnEntry> st(reinterpret_cast<KnnEntry *>(s_stack) + threadIdx.x, blockDim.x, stack_cap, spill);
        // the seed searches this tree's segment of the forest's sorted build keys
        const SeedKeys sk{keys, tr >= 0 && tr < T ? (uint64_t)tr << mbits : 0, mbits / D};
        if (FMT == 1)
            knn_search_q<D, K>(qnodes, n_nodes, leaves, kind, h, q, best, st, seed, sk);
        else if (FMT == 2)
            knn_search4<D, K>(nodes, wnodes, n_nodes, leaves, kind, h, q, best, st, seed, sk);
        else
            knn_search<D, K>(nodes, n_nodes, leaves, kind, h, q, best, st, seed, sk);
        best.store(k_out, out_d2 + qi * k_out, out_idx + qi * k_out, h.start);  // indices local to the tree
    }
}

// Local indices for reductions are not needed (no indices are output); kNN
// converts above.  Workspace layout for m queries:
//   codes[2][m] (K), ids[2][m] (u32), radix workspace, counter.
template <typename K>
size_t forest_ws_bytes(int64_t m)
{
    const int64_t mm = m > 0 ? m : 1;
    return 2 * mm * sizeof(K) + 2 * mm * sizeof(uint32_t) + radix_workspace_bytes(mm) + 1024;
}

arborx_status reserve_ws(ForestDev &f, int64_t m, hipStream_t s)
{
    const size_t need = std::max(forest_ws_bytes<uint64_t>(m), forest_ws_bytes<uint32_t>(m));
    if (f.ws_bytes >= need)
        return ARBORX_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return fail(ARBORX_E_NOMEM, "forest workspace too small during graph capture: call arborx_forest_reserve first");
    if (f.ws)
        dfree(f.ws, s);
    f.ws = nullptr;
    f.ws_bytes = 0;
    arborx_status st = dalloc(&f.ws, need, s);
    if (st == ARBORX_OK)
        f.ws_bytes = need;
    return st;
}

// Sorted permutation of the queries (by batch, then Morton inside the batch).
template <int D, typename K>
arborx_status forest_order(const ForestDev &f, const float *q, int64_t m, const int64_t *boff, int B,
                           const int32_t *btree, uint32_t **perm, unsigned long long **counter, hipStream_t s)
{
    const int64_t mm = m > 0 ? m : 1;
    uint8_t *p = static_cast<uint8_t *>(f.ws);
    K *codes = reinterpret_cast<K *>(p);
    K *codes2 = codes + mm;
    uint32_t *ids = reinterpret_cast<uint32_t *>(codes2 + mm);
    uint32_t *ids2 = ids + mm;
    uint8_t *rws = reinterpret_cast<uint8_t *>(ids2 + mm);
    rws = reinterpret_cast<uint8_t *>((reinterpret_cast<uintptr_t>(rws) + 255) & ~uintptr_t(255));
    *counter = reinterpret_cast<unsigned long long *>(rws + radix_workspace_bytes(mm));
    int bb = 1;
    while ((1 << bb) < B)
        ++bb;
    const int kbits = (int)sizeof(K) * 8 - (sizeof(K) == 8 ? 1 : 0);
    int mbits = (kbits - bb) / D * D;
    if (mbits > 8 * D)
        mbits = 8 * D;  // 8 bits per dimension order the queries of one batch well enough
    ProfScope ps("forest_order", s);
    k_forest_codes<D, K><<<grid_for(m, 256, 65536), 256, 0, s>>>(q, m, boff, B, btree, f.T, f.hdrs, mbits, codes,
                                                                 ids);
    bool alt = false;
    AX_HIP(radix_sort_pairs<K>(codes, ids, codes2, ids2, m, 0, mbits + bb, rws, s, &alt));
    *perm = alt ? ids2 : ids;
    return ARBORX_OK;
}

int persistent_grid(const void *kernel, int block, size_t lds)
{
    int dev = 0, cus = 256, per = 1;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, block, lds) != hipSuccess || per < 1)
        per = 1;
    return cus * per;
}

template <int D>
arborx_status forest_reduce_impl(ForestDev &f, const float *q, int64_t m, const int64_t *boff, const int32_t *btree,
                                 const float *brad, int B, int op, int scale_bits, int32_t *counts, int64_t *sums,
                                 hipStream_t s)
{
    uint32_t *perm;
    unsigned long long *counter;
    int bb = 1;
    while ((1 << bb) < B)
        ++bb;
    arborx_status st = bb <= 20 ? forest_order<D, uint32_t>(f, q, m, boff, B, btree, &perm, &counter, s)
                                : forest_order<D, uint64_t>(f, q, m, boff, B, btree, &perm, &counter, s);
    if (st != ARBORX_OK)
        return st;
    fill_kernel<unsigned long long><<<1, 64, 0, s>>>(counter, 1, 0ull);
    const Tuning &tu = tuning(OP_REDUCE);
    int block_unused = 0, cap = 0;
    launch_shape(OP_REDUCE, D, block_unused, cap);
    while (cap > 1 && (size_t)cap * kForestBlock * sizeof(int) > 65536)
        cap >>= 1;
    const size_t lds = (size_t)cap * kForestBlock * sizeof(int);
    const float scale = ldexpf(1.0f, scale_bits);
    ProfScope ps(op == ARBORX_COUNT_SUMDIST ? "forest_reduce_sumdist" : "forest_reduce_count", s);
    const Node<D> *nodes = static_cast<const Node<D> *>(f.nodes);
    const QNode<D> *qnodes = static_cast<const QNode<D> *>(f.qnodes);
    const Node4<D> *wnodes = static_cast<const Node4<D> *>(f.wnodes);
    const int nn = (int)(f.n > 0 ? f.n : 1);
    const int fmt = node_format(OP_REDUCE, D, f.kind, true);
    const int nq = tu.packet ? tu.packet : (D <= 3 ? 4 : 1);
    if (fmt == 0 && nq > 1) {
#define AX_FRP(SD, N)                                                                                            \
    do {                                                                                                         \
        const int grid = persistent_grid((const void *)k_forest_reduce_packet<D, SD, N>, kForestBlock, lds);    \
        k_forest_reduce_packet<D, SD, N><<<grid, kForestBlock, lds, s>>>(nodes, nn, f.hdrs, f.T, q, m, perm, boff, B, \
                                                                         btree, brad, scale, counts, sums, counter, cap); \
    } while (0)
        if (op == ARBORX_COUNT_SUMDIST) {
            if (nq == 2)
                AX_FRP(true, 2);
            else
                AX_FRP(true, 4);
        } else {
            if (nq == 2)
                AX_FRP(false, 2);
            else
                AX_FRP(false, 4);
        }
#undef AX_FRP
        AX_HIP(hipGetLastError());
        return ARBORX_OK;
    }
#define AX_FREDUCE(SD, F)                                                                                        \
    do {                                                                                                         \
        const int grid = persistent_grid((const void *)k_forest_reduce<D, SD, F>, kForestBlock, lds);           \
        k_forest_reduce<D, SD, F><<<grid, kForestBlock, lds, s>>>(nodes, qnodes, wnodes, f.leaves, f.kind, nn, f.hdrs, \
                                                                  f.T, q, m, perm, boff, B, btree, brad, scale,  \
                                                                  counts, sums, counter, cap);                 \
    } while (0)
    if (op == ARBORX_COUNT_SUMDIST) {
        if (fmt == 1)
            AX_FREDUCE(true, 1);
        else if (fmt == 2)
            AX_FREDUCE(true, 2);
        else
            AX_FREDUCE(true, 0);
    } else {
        if (fmt == 1)
            AX_FREDUCE(false, 1);
        else if (fmt == 2)
            AX_FREDUCE(false, 2);
        else
            AX_FREDUCE(false, 0);
    }
#undef AX_FREDUCE
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

template <int D, int K>
arborx_status forest_knn_launch(ForestDev &f, const float *q, int64_t m, const int64_t *boff, const int32_t *btree,
                                int B, int k, float *d2, int32_t *idx, hipStream_t s)
{
    uint32_t *perm;
    unsigned long long *counter;
    int bb = 1;
    while ((1 << bb) < B)
        ++bb;
    arborx_status st = bb <= 20 ? forest_order<D, uint32_t>(f, q, m, boff, B, btree, &perm, &counter, s)
                                : forest_order<D, uint64_t>(f, q, m, boff, B, btree, &perm, &counter, s);
    if (st != ARBORX_OK)
        return st;
    fill_kernel<unsigned long long><<<1, 64, 0, s>>>(counter, 1, 0ull);
    const Tuning &tu = tuning(OP_KNN);
    const int fmt = node_format(OP_KNN, D, f.kind, true);
    int block_unused = 0, cap = 0;
    launch_shape(OP_KNN, D, block_unused, cap);
    while (cap > 1 && (size_t)cap * kForestBlock * sizeof(KnnEntry) > 65536)
        cap >>= 1;
    const size_t lds = (size_t)cap * kForestBlock * sizeof(KnnEntry);
    ProfScope ps("forest_knn", s);
#define AX_FKNN(F)                                                                                                 \
    do {                                                                                                           \
        const int grid = persistent_grid((const void *)k_forest_knn<D, K, F>, kForestBlock, lds);                 \
        k_forest_knn<D, K, F><<<grid, kForestBlock, lds, s>>>(                                                    \
            static_cast<const Node<D> *>(f.nodes), static_cast<const QNode<D> *>(f.qnodes),                        \
            static_cast<const Node4<D> *>(f.wnodes), (int)(f.n > 0 ? f.n : 1), f.leaves, f.kind, f.hdrs, f.T, q, m, \
            perm, boff, B, btree, k, d2, idx, counter, cap, tu.seed, f.keys, f.mbits);                             \
    } while (0)
    if (fmt == 1)
        AX_FKNN(1);
    else if (fmt == 2)
        AX_FKNN(2);
    else
        AX_FKNN(0);
#undef AX_FKNN
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

template <int D>
arborx_status forest_knn_impl(ForestDev &f, const float *q, int64_t m, const int64_t *boff, const int32_t *btree,
                              int B, int k, float *d2, int32_t *idx, hipStream_t s)
{
    if (k <= 1)
        return forest_knn_launch<D, 1>(f, q, m, boff, btree, B, k, d2, idx, s);
    if (k <= 4)
        return forest_knn_launch<D, 4>(f, q, m, boff, btree, B, k, d2, idx, s);
    if (k <= 8)
        return forest_knn_launch<D, 8>(f, q, m, boff, btree, B, k, d2, idx, s);
    if (k <= 16)
        return forest_knn_launch<D, 16>(f, q, m, boff, btree, B, k, d2, idx, s);
    if (k <= 32)
        return forest_knn_launch<D, 32>(f, q, m, boff, btree, B, k, d2, idx, s);
    return forest_knn_launch<D, 64>(f, q, m, boff, btree, B, k, d2, idx, s);
}

}  // namespace

arborx_status forest_reserve(ForestDev &f, int64_t m, hipStream_t s) { return reserve_ws(f, m, s); }

arborx_status forest_query_reduce(ForestDev &f, const float *q, int64_t m, const int64_t *boff, const int32_t *btree,
                                  const float *brad, int B, int op, int scale_bits, int32_t *counts, int64_t *sums,
                                  hipStream_t s)
{
    if (m == 0)
        return ARBORX_OK;
    arborx_status st = check_nodes(f.qnodes, f.wnodes, f.n, node_format(OP_REDUCE, f.dim, f.kind, true));
    if (st == ARBORX_OK)
        st = reserve_ws(f, m, s);
    if (st != ARBORX_OK)
        return st;
    switch (f.dim) {
    case 2: return forest_reduce_impl<2>(f, q, m, boff, btree, brad, B, op, scale_bits, counts, sums, s);
    case 3: return forest_reduce_impl<3>(f, q, m, boff, btree, brad, B, op, scale_bits, counts, sums, s);
    case 6: return forest_reduce_impl<6>(f, q, m, boff, btree, brad, B, op, scale_bits, counts, sums, s);
    default: return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in");
    }
}

arborx_status forest_query_knn(ForestDev &f, const float *q, int64_t m, const int64_t *boff, const int32_t *btree,
                               int B, int k, float *d2, int32_t *idx, hipStream_t s)
{
    if (m == 0)
        return ARBORX_OK;
    arborx_status st = check_nodes(f.qnodes, f.wnodes, f.n, node_format(OP_KNN, f.dim, f.kind, true));
    if (st == ARBORX_OK)
        st = reserve_ws(f, m, s);
    if (st != ARBORX_OK)
        return st;
    switch (f.dim) {
    case 2: return forest_knn_impl<2>(f, q, m, boff, btree, B, k, d2, idx, s);
    case 3: return forest_knn_impl<3>(f, q, m, boff, btree, B, k, d2, idx, s);
    case 6: return forest_knn_impl<6>(f, q, m, boff, btree, B, k, d2, idx, s);
    default: return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in");
    }
}

}  // namespace ax
