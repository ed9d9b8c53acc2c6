// Host-side internals shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/arborx.h"

namespace ax {

constexpr int kMaxDim = 10;

// Device-resident tree header written by the build kernels.
// Device-resident tree header written by the build kernels (one per tree of
// a forest).
struct TreeHeader {
    int32_t root;    // index of the root node (-1 when the tree is empty)
    int32_t height;  // edges on the longest root-to-leaf path
    int32_t n;       // values in the tree
    int32_t start;   // position of the tree's first leaf in the sorted leaf array
    float lo[kMaxDim];
    float hi[kMaxDim];
    float qscale[kMaxDim];  // quantized-node frame: coordinate = lo + code * qscale
};

// Device-resident per-call header of a CSR query, written by the scan.
struct QueryHeader {
    unsigned long long total;      // offsets[m]
    unsigned long long big_rows;   // rows with stash_regs(dim) < len <= kRowSortBlock
    unsigned long long huge_rows;  // rows with len > kRowSortBlock
    unsigned long long pad;
};

struct Tuning {
    int block = 256;
    int order = 1;
    int stack = 16;
    int schedule = 0;
    int build = 0;
    int seed = 0;   // kNN starting bound: 0 k-th of 2k nearby leaves, 1 none, 2 farthest of k nearby leaves
    int nodes = 0;  // 0: binary float, 1: binary with quantized 16-bit child boxes (exact leaf tests), 2: four-wide
    int packet = 0; // radius walks on binary nodes: queries per thread (1, 2 or 4) walked together; 0 = by
                    // operation, dimension and format (up to 3D, where neighbouring paths overlap most: for
                    // the fused reductions 4 on float nodes, 2 on quantized ones; 2 for the CSR count; 1 in
                    // 6D)
    bool by_dim = false;  // the library's defaults: block and stack also follow the dimension (launch_shape)
};
// Block size and short-stack depth a launch of `op` in dimension `dim` uses:
// the tuning's, except that the library's defaults in 6D take the shapes
// measured best on the 6D Gaussian mixture at 2*10^6 points over quantized
// nodes (kNN: 64-thread blocks, 16-entry ring, 7.4 -> 6.7 ms; CSR count:
// 64-thread blocks, 10.8 -> 10.2 ms; reductions keep the 3D shape).
void launch_shape(int op, int dim, int &block, int &stack);
// Tuning is kept per operation kind so the autotuner can pick each separately.
enum Op { OP_SPATIAL = 0, OP_REDUCE = 1, OP_KNN = 2, OP_KINDS = 3 };
const Tuning &tuning(int op = OP_SPATIAL);
void set_tuning_op(int op, const Tuning &t);
// Node format the thread schedule of `op` walks on a tree (or forest) of
// dimension `dim` over values of `kind`: the tuning's; under the library's
// defaults 1 for the radius walks over points and for kNN over points in 6D,
// and 0 for every other walk (kNN up to 3D, box values, forests).
int node_format(int op, int dim, int kind, bool forest);
int node_format_of(const Tuning &t, int op, int dim, int kind, bool forest);
// Quantized (1) and four-wide (2) nodes are built only while some operation
// asks for that format on a structure of this dimension, kind and form.
bool format_requested(int format, int dim, int kind, bool forest);
// Node format a single-tree walk of `op` uses: node_format for the thread
// schedule (kNN: any schedule but the wavefront packet), else binary.
int walk_format(int op, int dim, int kind);
// ARBORX_E_INVALID unless the structure holds the nodes of format `fmt`.
arborx_status check_nodes(const void *qnodes, const void *wnodes, int64_t n, int fmt);
bool tree_has_format(arborx_tree tree, int format);
bool forest_has_format(arborx_forest forest, int format);


// Error reporting: thread-local last message.
void set_error(const std::string &msg);
arborx_status fail(arborx_status st, const std::string &msg);
arborx_status hip_fail(hipError_t e, const char *what);

#define AX_HIP(call)                                                       \
    do {                                                                   \
        hipError_t _e = (call);                                            \
        if (_e != hipSuccess)                                              \
            return ::ax::hip_fail(_e, #call);                              \
    } while (0)

// Stream-ordered device allocation; returns ARBORX_E_NOMEM on failure.
arborx_status dalloc(void **p, size_t bytes, hipStream_t s);
void dfree(void *p, hipStream_t s);

// Scoped set of stream-ordered temporaries, freed on destruction.
struct Temps {
    hipStream_t s;
    void *ptrs[32];
    int n = 0;
    explicit Temps(hipStream_t st) : s(st) {}
    ~Temps()
    {
        for (int i = 0; i < n; ++i)
            dfree(ptrs[i], s);
    }
    template <typename T>
    arborx_status get(T **p, size_t count)
    {
        if (n == (int)(sizeof(ptrs) / sizeof(ptrs[0])))
            return fail(ARBORX_E_NOMEM, "too many temporaries in one call");
        void *q = nullptr;
        arborx_status st = dalloc(&q, count * sizeof(T) + 256, s);
        if (st != ARBORX_OK)
            return st;
        ptrs[n++] = q;
        *p = static_cast<T *>(q);
        return ARBORX_OK;
    }
};

inline unsigned grid_for(int64_t n, int block, int64_t cap = 1 << 20)
{
    int64_t g = (n + block - 1) / block;
    if (g < 1)
        g = 1;
    if (g > cap)
        g = cap;
    return (unsigned)g;
}

// ---- radix sort (sort.hip) ------------------------------------------------
// Workspace bytes for sorting n pairs.
size_t radix_workspace_bytes(int64_t n);
// Stable LSD sort of (keys, vals) by bits [begin, end).  Uses keys_alt/vals_alt
// as the ping-pong buffers; on return *in_alt tells which buffer holds the result.
template <typename K>
hipError_t radix_sort_pairs(K *keys, uint32_t *vals, K *keys_alt, uint32_t *vals_alt, int64_t n, int begin, int end,
                            void *workspace, hipStream_t s, bool *in_alt);

// ---- scan (scan.hip) ----------------------------------------------------
size_t scan_workspace_bytes(int64_t n);
// offsets[0..m] = exclusive scan of counts; also writes offsets[m] to *total_dev.
hipError_t csr_offsets(const int32_t *counts, int64_t m, int64_t *offsets, int64_t *total_dev, void *workspace,
                       hipStream_t s);
// As csr_offsets, and also lists the rows longer than `regs` (big_list,
// up to kRowSortBlock) and longer than kRowSortBlock (huge_list); totals go to
// *qh.  With `order` (position -> row, e.g. the traversal order of the
// queries) and ordered_counts[i] = counts[order[i]], the lists follow that
// order, so a second walk over them stays coherent; else row order.  Lists
// need room for m entries.
hipError_t csr_offsets_lists(const int32_t *counts, const int32_t *ordered_counts, const uint32_t *order, int64_t m,
                             int regs, int64_t *offsets, int32_t *big_list, int32_t *huge_list, QueryHeader *qh,
                             void *workspace, hipStream_t s);

// ---- build (build.hip) ----------------------------------------------------
struct TreeDev {
    int64_t n = 0;
    int dim = 0;
    int kind = 0;
    void *nodes = nullptr;  // Node<dim>[max(n-1, 1)]
    void *qnodes = nullptr; // QNode<dim>[max(n-1, 1)]: the same tree, 16-bit internal boxes, exact point leaves
    void *wnodes = nullptr; // Node4<dim>[max(n-1, 1)]: the same tree two levels per node
    uint64_t *codes = nullptr;  // [n] sorted Morton codes of the leaves (the build's sort keys)
    float *leaves = nullptr; // n leaf records in sorted order (see leaf_floats)
    TreeHeader *hdr = nullptr;
};
// Node format a walk of `op` takes on tree t: walk_format's, except that the
// library's defaults fall back to float nodes on a tree built without the
// quantized ones (a request the caller made for a missing format is an error).
int tree_format(int op, const TreeDev &t);
size_t node_bytes(int dim);
// Number of node slots allocated for a tree of n values.
inline int tree_nodes(const TreeDev &t) { return t.n > 1 ? (int)(t.n - 1) : 1; }
arborx_status build_tree(const float *values, int64_t n, int dim, int kind, TreeDev &t, hipStream_t s);
hipError_t morton64_points(const float *pts, int64_t n, int dim, const float *bounds, uint64_t *codes,
                           hipStream_t s);

// Forest: T trees over one packed value array; tree t = values [seg[t], seg[t+1]).
struct ForestDev {
    int64_t n = 0;
    int dim = 0, kind = 0, T = 0;
    void *nodes = nullptr;     // Node<dim>[n]: one slot per split plus a spare for a last one-value tree
    void *qnodes = nullptr;    // QNode<dim>[n]
    void *wnodes = nullptr;    // Node4<dim>[n]
    float *leaves = nullptr;   // n leaf records, sorted inside each tree
    uint64_t *keys = nullptr;  // [n] sorted build keys (tree << mbits | tree-local Morton code), in the build workspace
    int mbits = 0;             // bits of the tree-local code in a key
    TreeHeader *hdrs = nullptr;  // [T]
    int64_t *seg = nullptr;    // [T+1] device copy of the tree offsets
    void *ws = nullptr;        // query workspace, grown on demand (reserve before graph capture)
    size_t ws_bytes = 0;
    void *bws = nullptr;       // build workspace, sized at allocation for n values in T trees
    size_t bws_bytes = 0;
    int max_tiles = 0;         // upper bound of the build's per-tree tiles: n / tile + T + 1
};
arborx_status build_forest(const float *values, const int64_t *seg_host, int T, int dim, int kind, ForestDev &f,
                           hipStream_t s);
// Every allocation of a forest of n values in T trees (structure and build
// workspace), then rebuilds from device values and device offsets [T+1] that
// launch kernels only: capturable in a graph.
arborx_status forest_alloc(int64_t n, int T, int dim, int kind, ForestDev &f, hipStream_t s);
arborx_status forest_rebuild(const float *values, const int64_t *tree_offsets, ForestDev &f, hipStream_t s);
void forest_release(ForestDev &f, hipStream_t s);
// Grow the query workspace to serve m queries without allocating.
arborx_status forest_reserve(ForestDev &f, int64_t m, hipStream_t s);
arborx_status forest_query_reduce(ForestDev &f, const float *q, int64_t m, const int64_t *boff, const int32_t *btree,
                                  const float *brad, int B, int op, int scale_bits, int32_t *counts, int64_t *sums,
                                  hipStream_t s);
arborx_status forest_query_knn(ForestDev &f, const float *q, int64_t m, const int64_t *boff, const int32_t *btree,
                               int B, int k, float *d2, int32_t *idx, hipStream_t s);

// ---- Chamfer (chamfer.hip); offsets are host arrays -----------------------
arborx_status chamfer_forward(const float *a, const int64_t *a_off, const float *b, const int64_t *b_off, int P,
                              float *loss, int32_t *nn_ab, int32_t *nn_ba, hipStream_t s);
arborx_status chamfer_backward(const float *a, const int64_t *a_off, const float *b, const int64_t *b_off, int P,
                               const int32_t *nn_ab, const int32_t *nn_ba, const float *grad_loss, float *grad_a,
                               float *grad_b, hipStream_t s);

// ---- queries (query.hip) --------------------------------------------------
enum class Pred { Sphere, Box, Ray };
// Per-match value kept by a CSR query: none; the walk's float (squared
// distance, or a ray's entry parameter) with rows sorted by index; or that
// float with rows sorted by (value, index) (a ray's hits in the order met).
enum ValueMode { VALUES_NONE = 0, VALUES_BY_INDEX = 1, VALUES_ORDERED = 2 };
arborx_status query_order(const TreeDev &t, const float *queries, int64_t m, Pred pred, int op, uint32_t **perm,
                          Temps &tmp, hipStream_t s);
// Matches of a CSR count walk beyond a query's stash row, kept in chained
// chunks of kChunk ints (the last int of a full chunk is the index of the
// next chunk) taken from kOvfPools sub-pools, each with its own allocation
// counter, chosen by workgroup so that allocations rarely contend.  A row
// whose chunks would not fit, or that grows past kRowSortBlock, is marked for
// a second walk instead.
constexpr int kChunk = 32;
constexpr int kOvfPools = 256;
struct OverflowPool {
    int32_t *head;                 // [m] first chunk of each row longer than the stash; -2: walk it again
    int32_t *pool;                 // kOvfPools sub-pools of `per` ints each
    float *dpool;                  // NULL, or the match distances, slot for slot beside pool
    unsigned long long *ctr;       // kOvfPools counters, one per 64 bytes (stride 8), zero before the walk
    int32_t per;                   // ints per sub-pool, a multiple of kChunk
};
// Ints of the overflow pool for m queries (factor times as many as the stash
// rows, at most 2^31 - 1 in all, at least one chunk per sub-pool).
int64_t overflow_pool_ints(int64_t m, int dim, int factor = 1);
// Pool factor by predicate: rays meet far more values than a radius query
// aimed at about ten (48 on average against 2*10^6 small boxes), and a row
// whose chunks do not fit is walked a second time.
inline int overflow_factor(Pred pred) { return pred == Pred::Ray ? 4 : 1; }
// Count pass; also stores each query's first stash_regs(dim) matches in
// stash[query][stash_regs(dim)], further matches in ovf, and (with perm)
// ordered_counts[t] = counts[perm[t]].
// With stash_d2 (and ovf.dpool), each match's squared distance is kept beside
// its index: stash_d2[query][stash_regs(dim)] and the parallel pool.
arborx_status spatial_count(const TreeDev &t, Pred pred, const float *queries, int64_t m, float radius,
                            const uint32_t *perm, int32_t *counts, int32_t *ordered_counts, int32_t *stash,
                            float *stash_d2, const OverflowPool &ovf, hipStream_t s);
// Fill pass: stash rows are copied, listed longer rows are copied from the
// stash and their overflow chunks, and the rest (huge rows, rows whose chunks
// did not fit) are walked again.
// With dist, each match's value is written beside its index, rows sorted as
// `mode` says (VALUES_BY_INDEX or VALUES_ORDERED).  sorted = false (indices
// only) leaves the stash rows in the order the walk found their matches, and
// the caller then skips the row sorts.
arborx_status spatial_fill(const TreeDev &t, Pred pred, const float *queries, int64_t m, float radius,
                           const int32_t *counts, const int32_t *stash, const float *stash_d2,
                           const OverflowPool &ovf, const int64_t *offsets, const int32_t *big_list, int64_t nbig,
                           const int32_t *huge_list, int64_t nhuge, int32_t *indices, float *dist, int mode,
                           hipStream_t s, bool sorted = true);
// Row sorts; with dist, each value moves with its index, rows sorted by
// index or (mode VALUES_ORDERED) by (value, index).
arborx_status sort_big_rows(const int64_t *offsets, int32_t *indices, float *dist, int mode, const int32_t *big_list,
                            int64_t nbig, hipStream_t s);
arborx_status sort_huge_rows(int64_t n_values, const int64_t *offsets, int32_t *indices, float *dist, int mode,
                             const int32_t *huge_list, int64_t h, Temps &tmp, hipStream_t s);
arborx_status spatial_reduce(const TreeDev &t, const float *queries, int64_t m, float radius, int op,
                             int scale_bits, const uint32_t *perm, int32_t *counts, int64_t *sums, hipStream_t s);
// out[p] = squared distance of match p (CSR row i = query i) from the build input.
arborx_status match_distances(const TreeDev &t, const float *values, const float *queries, int64_t m,
                              const int64_t *offsets, const int32_t *indices, float *out, hipStream_t s);
// Ray predicates (ray.hip); rays are [m][2][dim] (origin row, direction row).
// perm: traversal order of the rays (may be NULL).
arborx_status ray_count(const TreeDev &t, const float *rays, int64_t m, const uint32_t *perm, int32_t *counts,
                        hipStream_t s);
arborx_status ray_nearest(const TreeDev &t, const float *rays, int64_t m, const uint32_t *perm, int k, float *t_out,
                          int32_t *idx_out,
                          hipStream_t s);
// Pair search over the tree's own points (pairs.hip): degree[i] = number of
// values j != i within radius of value i (input order).
arborx_status self_join_degree(const TreeDev &t, float radius, int32_t *degree, hipStream_t s);
// DBSCAN over the tree's own points (pairs.hip), labels[n] in input order.
arborx_status dbscan(const TreeDev &t, float eps, int min_pts, int32_t *labels, hipStream_t s);
// Early-terminating count: counts[i] = min(matches of query i, n_max).
arborx_status spatial_count_up_to(const TreeDev &t, const float *queries, int64_t m, float radius, int n_max,
                                  const uint32_t *perm, int32_t *counts, hipStream_t s);
arborx_status knn_query(const TreeDev &t, const float *queries, int64_t m, int k, const uint32_t *perm,
                        float *dist2, int32_t *indices, hipStream_t s);
// Node fetches per query of the one-query-per-thread radius walk (op 0) or
// kNN walk (op 1, k = 1..64, after seeding).
arborx_status debug_node_visits(const TreeDev &t, const float *queries, int64_t m, float radius, int op, int k,
                                int32_t *visits, hipStream_t s);
// kNN whose query ordering runs in the library's static per-device scratch
// (at most ARBORX_NOALLOC_MAX_QUERIES queries): no device allocation.
arborx_status knn_query_noalloc(const TreeDev &t, const float *queries, int64_t m, int k, float *dist2,
                                int32_t *indices, hipStream_t s);

// Matches a CSR count walk keeps per query (its stash row), sorted in
// registers when copied out; longer rows are walked again.  32 in 6D, where
// radius rows run longer for the same selectivity.
__host__ __device__ constexpr int stash_regs(int dim) { return dim >= 6 ? 32 : 16; }
constexpr int kMaxStashRegs = 32;
constexpr int kRowSortBlock = 4096;   // rows up to this length are sorted by one workgroup

}  // namespace ax
