/*
 * arborx.h — C ABI of an MI355X (gfx950) linear-BVH geometric search library.
 *
 * The operations follow the search index of the ArborX 2.0 paper (arXiv
 * 2507.23700): a bounding volume hierarchy built from an array of values
 * (Section 2.1, "New interface": the index constructor), queried with arrays of
 * predicates in three forms (Section 2.1, query calls (1)-(3)): a storage query
 * returning compressed-sparse-row offsets plus indices (Section 2.1, original
 * interface and its footnote on the CSR format), and pure-callback queries that
 * reduce per match without storing anything (Section 2.2).  Every call takes a
 * stream, the counterpart of the paper's execution-space argument (Section
 * 2.1, "Lack of execution spaces").  size/empty/bounds are `arborx_bvh_info`.
 *
 * Conventions shared by every entry point:
 *   - Pointers are DEVICE pointers unless marked [host].  Coordinates are
 *     float32, row-major: points [n][dim]; boxes [n][2][dim] (the lo row, then
 *     the hi row).  Result indices are int32 indices into the build input.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls are stream-ordered and asynchronous unless they return a [host]
 *     value, in which case they synchronise `stream` before returning.
 *   - The caller owns inputs and outputs and keeps them alive until `stream`
 *     has passed the call.  Trees and forests own their device memory.
 *   - Errors are status codes; nothing throws across the ABI.  Arguments are
 *     validated on the host before any device work, and on error no output is
 *     written.  arborx_last_error() returns a thread-local message.
 *   - Distances are squared Euclidean distances computed in float32 with one
 *     rounding per operation, dimensions summed from 0 upwards, no fused
 *     multiply-add.  A radius r matches values with d2 <= fl(r*r) (closed ball).
 *     For box values d2 is the distance to the nearest point of the box.
 *   - Coordinates must be finite; results for NaN or infinite inputs are
 *     unspecified (never a fault).
 *   - Supported dimensions: 2, 3 and 6.  Other dim in 1..10 returns
 *     ARBORX_E_UNSUPPORTED; dim outside 1..10 returns ARBORX_E_INVALID.
 */
#ifndef ARBORX355_ARBORX_H
#define ARBORX355_ARBORX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct arborx_tree_s *arborx_tree;     /* opaque; immutable after build */
typedef struct arborx_forest_s *arborx_forest; /* opaque; many trees in one structure */

typedef enum {
    ARBORX_OK = 0,
    ARBORX_E_INVALID = 1,     /* bad argument (null pointer, negative size, NaN radius, ...) */
    ARBORX_E_UNSUPPORTED = 2, /* valid but not compiled in (e.g. dim 4) */
    ARBORX_E_NOMEM = 3,       /* device allocation failed */
    ARBORX_E_CAPACITY = 4,    /* output buffer too small; *total says how much is needed */
    ARBORX_E_DEVICE = 5       /* no usable GPU, or a HIP runtime error */
} arborx_status;

typedef enum { ARBORX_POINTS = 0, ARBORX_BOXES = 1 } arborx_kind;

/* Pure-callback reducers (Section 2.2, query form (1)).
 * COUNT:         counts[i] = number of values within the radius of query i.
 * COUNT_SUMDIST: also sum_fixed[i] = sum over matches of trunc(sqrtf(d2) * 2^S),
 *                an integer sum that does not depend on visiting order. */
typedef enum { ARBORX_COUNT = 0, ARBORX_COUNT_SUMDIST = 1 } arborx_reducer;

/* Traversal schedule knobs; every schedule returns identical results. */
typedef struct arborx_tuning {
    int32_t block;        /* threads per workgroup for traversal kernels: 64, 128, 256 (0 = default) */
    int32_t order;        /* sort queries along the Morton curve before traversal: 1 = on a 24-bit grid (three
                             sort passes), 2 = on a 16-bit grid (two passes); 0 = input order */
    int32_t stack;        /* LDS short-stack entries per thread: 4..64 (0 = default); deeper trees spill */
    int32_t schedule;     /* 0 = thread per query with a short stack; 1 = wavefront packet (64 queries share
                             node fetches); 2 = thread per query, stackless with ropes (radius / intersects
                             only; kNN uses the short stack) */
    int32_t build;        /* hierarchy handoff: 0 = chunked (LDS inside chunks), 1 = single pass (device scope);
                             both give the identical tree */
    int32_t seed_mode;    /* kNN starting bound: 0 = the k-th smallest distance among the 2k leaves around the
                             query's Morton position (default), 1 = none (+inf), 2 = the largest distance
                             among the k leaves around it */
    int32_t node_format;  /* node layout walked by the thread schedule (schedule 0): 0 = binary nodes with float
                             child boxes; 1 = binary nodes with internal child boxes as 16-bit codes rounded
                             outward (32 bytes in 3D), a point tree's leaf children stored exactly in the node
                             and a box tree's decided on their exact records; 2 = four-wide nodes (two levels
                             per fetch).  Every format gives identical results.  Formats 1 and 2 are built only
                             while some operation asks for them when the tree is built; asking later is
                             ARBORX_E_INVALID.  The defaults (arborx_set_tuning(NULL)): 1 for ARBORX_OP_SPATIAL
                             and ARBORX_OP_REDUCE, 0 for ARBORX_OP_KNN, over trees of points; under them a 6D
                             kNN over points also walks format 1, while trees of boxes, forests and a tree built
                             without format 1 are walked on format 0 */
    int32_t queries_per_thread; /* radius searches (CSR count pass of sphere queries, fused reductions) with
                                   the thread schedule on binary nodes: 1, 2 or 4 Morton-neighbouring queries
                                   answered by one thread in one walk over the union of their paths; 0 = by
                                   operation, dimension and format (up to 3D: 2 for CSR; for reductions 4 on
                                   format 0, 2 on format 1; 1 in 6D).  Defaults: 1 for ARBORX_OP_SPATIAL, 0
                                   otherwise */
} arborx_tuning;

/* Operation kinds that carry their own tuning. */
typedef enum { ARBORX_OP_SPATIAL = 0, ARBORX_OP_REDUCE = 1, ARBORX_OP_KNN = 2 } arborx_op;

/* Library version string, e.g. "arborx355 0.1". [host] */
const char *arborx_version(void);

/* Thread-local message describing the last error of this thread ("" if none). [host] */
const char *arborx_last_error(void);

/*
 * Device memory hook.  The library takes all of its device memory (tree and
 * forest storage, per-call temporaries, CSR plans) from alloc_fn and returns it
 * to free_fn, for example to share a framework's caching allocator; by
 * default it uses stream-ordered allocations from the device's pool.
 *   alloc_fn(bytes, stream, ctx) returns device memory for work queued on
 *     `stream`, or NULL (the call then fails with ARBORX_E_NOMEM).
 *   free_fn(ptr, stream, ctx) hands a block back.  `stream` is the stream the
 *     block was allocated for, and every use of the block by the library was
 *     queued on that stream before the call or has already completed: the
 *     block may be given at once to later work on that stream, and to other
 *     streams once that stream has passed this point (the contract of a
 *     per-stream caching allocator).  Blocks that work on other streams used
 *     (a destroyed tree that queries on several streams read, a replaced
 *     query order) are handed back only after that work has completed; the
 *     library checks for that at its later allocations and in this call.
 *   ctx is passed through unchanged.
 * Both NULL restores the default.  Allowed only while the library holds no
 * device memory of the previous allocator (no live tree, forest or plan);
 * blocks still waiting for other streams are waited for here.  Otherwise
 * ARBORX_E_INVALID.  Not to be called concurrently with other library calls.  [host]
 */
typedef void *(*arborx_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*arborx_free_fn)(void *ptr, void *stream, void *ctx);
arborx_status arborx_set_allocator(arborx_alloc_fn alloc_fn, arborx_free_fn free_fn, void *ctx);

/* Set the traversal schedule used by later queries; NULL restores the defaults.  [host] */
arborx_status arborx_set_tuning(const arborx_tuning *tuning);

/* Current traversal schedule (of ARBORX_OP_SPATIAL). [host] */
arborx_status arborx_get_tuning(arborx_tuning *tuning);

/* Per-operation forms: op is an arborx_op; NULL restores that operation's defaults. [host] */
arborx_status arborx_set_tuning_op(int32_t op, const arborx_tuning *tuning);
arborx_status arborx_get_tuning_op(int32_t op, arborx_tuning *tuning);

/*
 * Pick the fastest schedule for one operation on the caller's own queries:
 * every candidate (block size, short-stack depth, thread or wavefront-packet
 * schedule, query ordering, kNN seeding) runs on `queries`; all must produce
 * identical outputs (checked with a device hash, else ARBORX_E_DEVICE); the
 * fastest by event timing on `stream` (median of three runs) becomes the
 * tuning of `op`, unless the tuning in force is within 3% of it.  radius is
 * used for ARBORX_OP_SPATIAL / ARBORX_OP_REDUCE, k for ARBORX_OP_KNN.  If the
 * environment variable ARBORX_TUNING_CACHE names a file, a choice recorded
 * there for the same operation, dimension, kind, k and size classes is reused
 * (*best_ms = -1) and new choices are appended.  Synchronises.
 *   best [host, may be NULL] receives the chosen schedule; best_ms [host, may be NULL] its time.
 */
arborx_status arborx_autotune(arborx_tree tree, int32_t op, const float *queries, int64_t m, float radius, int32_t k,
                              arborx_tuning *best, double *best_ms, void *stream);

/*
 * The same for forest queries (op ARBORX_OP_REDUCE, timed with COUNT_SUMDIST,
 * or ARBORX_OP_KNN with k): the candidates are what a forest walk honours
 * (stack depth, queries per thread of the reduction, node formats the forest
 * holds, kNN seeding); every candidate must give the same outputs; the one in
 * force is kept unless another is at least 3% faster (median of three timed
 * runs).  Arguments as arborx_forest_query_reduce / _knn.  Synchronises.
 */
arborx_status arborx_autotune_forest(arborx_forest forest, int32_t op, const float *queries, int64_t m,
                                     const int64_t *batch_offsets, const int32_t *batch_tree,
                                     const float *batch_radius, int32_t B, int32_t k, arborx_tuning *best,
                                     double *best_ms, void *stream);

/*
 * Build a BVH over n values (Section 2.1, index constructor; Section 2.6: 64-bit
 * Morton codes and a bottom-up hierarchy construction).
 *   values  [n][dim] points or [n][2][dim] boxes (kind), device, read during the call only
 *   n       0 <= n < 2^31-1; n = 0 gives an empty tree (queries return nothing)
 *   out     [host] receives the tree handle; destroy with arborx_bvh_destroy
 * Work is queued on `stream`; the tree may be queried on any stream afterwards
 * (queries on other streams wait for the build).  Returns ARBORX_E_NOMEM if
 * device memory runs out.
 */
arborx_status arborx_bvh_build(const float *values, int64_t n, int32_t dim, int32_t kind, void *stream,
                               arborx_tree *out);

/* Release a tree.  Waits for outstanding work on the tree.  NULL is allowed. [host] */
arborx_status arborx_bvh_destroy(arborx_tree tree);

/*
 * Tree metadata (Section 2.1: size(), empty(), bounds()).  Synchronises with the build.
 *   n       [host] number of values (0 = empty)
 *   dim     [host] dimension;  kind [host] ARBORX_POINTS or ARBORX_BOXES
 *   bounds  [host] 2*dim floats: lo then hi of the scene box (+inf/-inf when empty); may be NULL
 *   height  [host] edges on the longest root-to-leaf path; may be NULL
 */
arborx_status arborx_bvh_info(arborx_tree tree, int64_t *n, int32_t *dim, int32_t *kind, float *bounds,
                              int32_t *height);

/*
 * Radius (sphere) search with CSR output (Section 2.1, storage query (3)).
 *   queries   [m][dim] query points
 *   radius    >= 0 (may be +inf); NaN is ARBORX_E_INVALID
 *   offsets   [m+1] int64, caller-allocated: offsets[0] = 0, offsets[i+1]-offsets[i] = matches of query i
 *   indices   int32 matches, row i at [offsets[i], offsets[i+1]), ascending within each row
 *   capacity  number of int32 slots in indices
 *   total     [host] receives offsets[m]
 * Two-phase protocol: if indices is NULL or capacity < total, offsets and
 * *total are filled and ARBORX_E_CAPACITY is returned; call again with a
 * large enough buffer.  Synchronises `stream` (to read the total).
 * Temporary device memory: about 4*(2*S + 5)*m bytes plus the query order,
 * where S is the per-query register stash (16 matches; 32 in 6D): the stash
 * rows and an overflow pool of the same size that keeps longer rows.
 */
arborx_status arborx_query_spatial(arborx_tree tree, const float *queries, int64_t m, float radius, int64_t *offsets,
                                   int32_t *indices, int64_t capacity, int64_t *total, void *stream);

/*
 * The same radius search in two calls, so that a caller can size `indices`
 * from the count without a second counting walk:
 *   arborx_query_spatial_begin  orders the queries, counts the matches, fills
 *     offsets[m+1] and *total [host], and returns a plan (synchronises);
 *   arborx_query_finish         writes the indices (capacity >= *total, else
 *     ARBORX_E_CAPACITY and the plan stays usable); asynchronous;
 *   arborx_plan_destroy         releases the plan's device memory.
 * queries and offsets must stay unchanged until the plan is destroyed, and
 * every call of a plan uses the stream given to begin.
 */
typedef struct arborx_plan_s *arborx_plan;
arborx_status arborx_query_spatial_begin(arborx_tree tree, const float *queries, int64_t m, float radius,
                                         int64_t *offsets, int64_t *total, arborx_plan *plan, void *stream);
arborx_status arborx_query_intersects_begin(arborx_tree tree, const float *qboxes, int64_t m, int64_t *offsets,
                                            int64_t *total, arborx_plan *plan, void *stream);
arborx_status arborx_query_finish(arborx_plan plan, int32_t *indices, int64_t capacity);
arborx_status arborx_plan_destroy(arborx_plan plan);

/*
 * Storage query without the canonical row order (Section 2.1, query call (3),
 * whose results come in the order the search meets them): as
 * arborx_query_finish, but each row holds its matches in the order the walk
 * found them (a row longer than the per-query register stash: the stash part,
 * then the rest as found) instead of ascending, which saves the row sorts.
 * The set of indices in every row, offsets and total are those of the sorted
 * form; the order inside a row may change from call to call.  Indices only:
 * a plan begun with distances writes its indices and no distances; a plan of
 * arborx_query_ray_ordered_intersect is ARBORX_E_INVALID.  Asynchronous.
 */
arborx_status arborx_query_finish_unsorted(arborx_plan plan, int32_t *indices, int64_t capacity);

/*
 * Box-overlap search with CSR output (Section 2.1, intersects predicate).
 *   qboxes  [m][2][dim] query boxes; a value matches if its box (a point is a
 *           degenerate box) overlaps the closed query box in every dimension.
 * Everything else as arborx_query_spatial.
 */
arborx_status arborx_query_intersects(arborx_tree tree, const float *qboxes, int64_t m, int64_t *offsets,
                                      int32_t *indices, int64_t capacity, int64_t *total, void *stream);

/*
 * k-nearest search (Section 2.1, nearest predicate: a point and a number of
 * neighbours).  Row i of the [m][k] outputs holds the min(k, n) values nearest
 * to query i in ascending (d2, index) order (ties go to the smaller index);
 * the rest of the row is (+inf, -1).
 *   k       1..64
 *   dist2   [m][k] float32 squared distances;  indices [m][k] int32
 * Does not synchronise.
 */
arborx_status arborx_query_knn(arborx_tree tree, const float *queries, int64_t m, int32_t k, float *dist2,
                               int32_t *indices, void *stream);

/*
 * Allocation-free k-nearest search, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments and the same results, bit for bit, as
 * arborx_query_knn, but the call allocates nothing: the Morton ordering of the
 * queries runs in a static scratch area that the library holds once per GPU
 * (ARBORX_NOALLOC_MAX_QUERIES x 16 bytes + 1 MiB, about 33 MiB, reserved with
 * the library's code on that GPU until the process ends), and the order is not
 * cached on the tree.
 *   m       0..ARBORX_NOALLOC_MAX_QUERIES; larger m returns ARBORX_E_CAPACITY
 *           before any device work.
 * Every call on one GPU uses that GPU's one scratch area: calls that overlap
 * in time on the same GPU (on different streams, or from different threads
 * without ordering) race and give undefined results.  Calls ordered on one
 * stream are safe; nothing has to be cleared between them.  While `stream` is
 * being captured the call does not wait on the tree's build event (the
 * caller orders the build before the capture).  Does not synchronise.
 */
#define ARBORX_NOALLOC_MAX_QUERIES 2097152
arborx_status arborx_query_knn_noalloc(arborx_tree tree, const float *queries, int64_t m, int32_t k, float *dist2,
                                       int32_t *indices, void *stream);

/*
 * Radius search fused with a per-query reduction; nothing is stored per match
 * (Section 2.2, pure callback).
 *   op          ARBORX_COUNT or ARBORX_COUNT_SUMDIST
 *   counts      [m] int32
 *   sum_fixed   [m] int64, required for COUNT_SUMDIST (ignored, may be NULL, for COUNT)
 *   scale_bits  S in 0..40 for COUNT_SUMDIST; each match adds trunc(sqrtf(d2) * 2^S);
 *               the sum is unspecified unless every term and the sum stay below 2^63
 * Does not synchronise.
 */
arborx_status arborx_query_spatial_reduce(arborx_tree tree, const float *queries, int64_t m, float radius,
                                          int32_t op, int32_t *counts, int64_t *sum_fixed, int32_t scale_bits,
                                          void *stream);

/*
 * Early-terminating count (Section 2.2: a callback may end a query's search
 * once it has what it needs, here after n_max matches; the paper's example
 * counts up to a limit).  counts[i] = min(number of values within radius of
 * query i, n_max), exactly.  The walk of each query stops at its n_max-th
 * match, so small limits are cheaper than a full COUNT.
 *   queries  [m][dim] query points;  radius >= 0 (may be +inf), NaN is ARBORX_E_INVALID
 *   n_max    >= 0 (0 gives all zeros without a walk)
 *   counts   [m] int32 output
 * Uses the thread walk over binary nodes with the block size, stack depth and
 * query order of ARBORX_OP_REDUCE.  Asynchronous.
 */
arborx_status arborx_query_spatial_count_up_to(arborx_tree tree, const float *queries, int64_t m, float radius,
                                               int32_t n_max, int32_t *counts, void *stream);

/*
 * Callback with output (Section 2.1, query call (2); Section 2.2): a radius
 * search whose callback emits one output per match, here the match's float32
 * squared distance as the walk computed it, stored in CSR form beside the
 * indices.  The walk keeps each distance with its index (in the register
 * stash, the overflow chunks, and a second walk for rows that need one), and
 * the row sorts move it along, so no pass after the search reads the values
 * again.  Same arguments, protocol and results as arborx_query_spatial, plus
 *   distances [capacity] float32 output: distances[p] is the squared distance
 *             between query i and value indices[p], for p in row i
 * If indices or distances is NULL, or capacity < total, offsets and *total are
 * filled and ARBORX_E_CAPACITY is returned.  Temporary device memory twice
 * that of arborx_query_spatial.  Synchronises `stream` (to read the total).
 * The plan form: arborx_query_spatial_with_distances_begin, then
 * arborx_query_finish_with_distances (distances must not be NULL when the
 * total is not 0; arborx_query_finish on such a plan writes indices only).
 */
arborx_status arborx_query_spatial_with_distances(arborx_tree tree, const float *queries, int64_t m, float radius,
                                                  int64_t *offsets, int32_t *indices, float *distances,
                                                  int64_t capacity, int64_t *total, void *stream);
arborx_status arborx_query_spatial_with_distances_begin(arborx_tree tree, const float *queries, int64_t m, float radius,
                                                        int64_t *offsets, int64_t *total, arborx_plan *plan,
                                                        void *stream);
arborx_status arborx_query_finish_with_distances(arborx_plan plan, int32_t *indices, float *distances,
                                                 int64_t capacity);

/*
 * The same per-match output computed after a search instead: the float32
 * squared distance of every match of any radius CSR result (for example one
 * produced earlier by arborx_query_spatial), evaluated exactly as in the search.
 *   values    the array the tree was built from (unchanged since the build)
 *   queries   [m][dim] the radius query's points;  offsets [m+1], indices [total] its result
 *   distances [total] float32 output aligned with indices (NaN for an index outside the tree)
 * Asynchronous; stream-ordered after the search when issued on its stream.
 */
arborx_status arborx_query_match_distances(arborx_tree tree, const float *values, const float *queries, int64_t m,
                                           const int64_t *offsets, const int32_t *indices, float *distances,
                                           void *stream);

/*
 * DBSCAN over the tree's own points (Section 2.4: density-based clustering
 * built on the index's radius search).  A point is core when at least min_pts
 * points, itself included, lie within eps (closed ball, d2 <= fl(eps*eps)); core
 * points within eps of each other share a cluster.  labels[i]:
 *   core point    the smallest index among the core points of its cluster;
 *   border point  (not core, some core point within eps) the label of its
 *                 smallest-index core neighbour;
 *   noise         -1.
 * These tie rules make the result unique.  Built on the pair search of
 * arborx_self_join_degree: every pair of points within eps is met once.
 *   points  the [n][dim] array the tree was built from (a tree of points); the
 *           walks read the same coordinates from the tree's leaf records
 *   eps >= 0 (NaN is ARBORX_E_INVALID);  min_pts >= 0 (0 or 1: every point is core)
 *   labels  [n] int32 output
 * Asynchronous; temporary memory 16 bytes per point.
 */
arborx_status arborx_dbscan(arborx_tree tree, const float *points, float eps, int32_t min_pts, int32_t *labels,
                            void *stream);

/*
 * Search for pairs of objects (Section 2.6: a dedicated traversal for it), as
 * the self-join of the tree's own points with a radius: the unordered pairs
 * {i, j}, i != j, with d2(p_i, p_j) <= fl(radius*radius) (closed ball).  Each
 * leaf walks only the part of the tree after its own sorted position, so every
 * pair is found exactly once.
 *   radius >= 0 (NaN is ARBORX_E_INVALID); +inf pairs everything
 *   degree [n] int32 output, input order: degree[i] = number of j != i paired
 *          with i (the number of pairs is half the sum)
 * A tree of boxes is ARBORX_E_INVALID.  Asynchronous; temporary memory 4 bytes
 * per point.
 */
arborx_status arborx_self_join_degree(arborx_tree tree, float radius, int32_t *degree, void *stream);

/*
 * Ray intersect (Section 2.5, the intersect predicate: every value a ray
 * meets, as if the objects were transparent), with CSR output.
 *   rays      [m][2][dim]: origin row, then direction row (any length, zero
 *             components allowed); hits as in arborx_query_ray_count
 *   offsets, indices, capacity, total: as arborx_query_spatial; rows ascending
 * Rays are ordered by the Morton code of their origins before the walk.
 * Temporary device memory: as arborx_query_spatial, with an overflow pool four
 * times larger (rays meet many more values than a radius query).
 * Synchronises `stream` (to read the total).  Plan form:
 * arborx_query_ray_intersect_begin, then arborx_query_finish.
 */
arborx_status arborx_query_ray_intersect(arborx_tree tree, const float *rays, int64_t m, int64_t *offsets,
                                        int32_t *indices, int64_t capacity, int64_t *total, void *stream);
arborx_status arborx_query_ray_intersect_begin(arborx_tree tree, const float *rays, int64_t m, int64_t *offsets,
                                              int64_t *total, arborx_plan *plan, void *stream);

/*
 * Ray ordered intersect (Section 2.5, ordered_intersect: the values a ray
 * meets, in the order a physical ray meets them), with CSR output: each row
 * ordered by (entry parameter, index), and the entry parameters beside the
 * indices.  The first k entries of a row are arborx_query_ray_nearest's.
 *   t_entry   [capacity] float32 output: the ray parameter t >= 0 at which it
 *             enters the value's box (0 when the origin is inside)
 * If indices or t_entry is NULL, or capacity < total, offsets and *total are
 * filled and ARBORX_E_CAPACITY is returned.  Synchronises `stream`.  Plan form:
 * arborx_query_ray_ordered_intersect_begin, then
 * arborx_query_finish_with_distances (its `distances` receive the entry
 * parameters) or arborx_query_finish (indices only, still in order).
 */
arborx_status arborx_query_ray_ordered_intersect(arborx_tree tree, const float *rays, int64_t m, int64_t *offsets,
                                                int32_t *indices, float *t_entry, int64_t capacity, int64_t *total,
                                                void *stream);
arborx_status arborx_query_ray_ordered_intersect_begin(arborx_tree tree, const float *rays, int64_t m,
                                                      int64_t *offsets, int64_t *total, arborx_plan *plan,
                                                      void *stream);

/*
 * Ray predicates (Section 2.5: rays traced against the index's values).  Ray i
 * is rays[i] = {origin[dim], direction[dim]} ([m][2][dim]) and covers
 * o + t*dir for t >= 0.  It meets a value's closed box (a point is a degenerate
 * box) when, taking the dimensions in order from tmin = 0, tmax = +inf, with
 * t1 = (lo - o) / dir and t2 = (hi - o) / dir in float32 for dir != 0,
 * tmin = max(tmin, min(t1, t2)) and tmax = min(tmax, max(t1, t2)) end with
 * tmin <= tmax (a dimension with dir == 0 needs lo <= o <= hi); tmin is the
 * entry parameter.
 *   arborx_query_ray_count    counts[m]: number of values each ray meets;
 *   arborx_query_ray_nearest  the k values met first: t_entry[m][k] and
 *                             indices[m][k] ordered by (entry t, index),
 *                             padded with (+inf, -1); 1 <= k <= 64.
 * Asynchronous.
 */
arborx_status arborx_query_ray_count(arborx_tree tree, const float *rays, int64_t m, int32_t *counts, void *stream);
arborx_status arborx_query_ray_nearest(arborx_tree tree, const float *rays, int64_t m, int32_t k, float *t_entry,
                                       int32_t *indices, void *stream);

/* ------------------------------------------------------------------------ */
/* Forest: many independent trees in one structure, queried in one launch.  */
/* ------------------------------------------------------------------------ */

/*
 * Build T trees at once.  Tree t holds values [tree_offsets[t], tree_offsets[t+1])
 * of the packed array `values` (points [n][dim] or boxes [n][2][dim]); trees may
 * be empty.  tree_offsets [host] has T+1 nondecreasing entries starting at 0.
 * Each tree is the tree arborx_bvh_build would give for its values alone.
 */
arborx_status arborx_forest_build(const float *values, const int64_t *tree_offsets, int32_t T, int32_t dim,
                                  int32_t kind, void *stream, arborx_forest *out);
arborx_status arborx_forest_destroy(arborx_forest forest);
/*
 * A forest that can be rebuilt inside a captured graph (Section 2.1: an index
 * built from arrays of values; here many trees, refilled in place).
 * arborx_forest_create makes every device allocation for n values in T trees
 * of dimension dim (the structure and the build's workspace) and builds
 * nothing; its trees are empty until the first rebuild.
 * arborx_forest_rebuild builds the trees from device arrays:
 *   values        [n][dim] points or [n][2][dim] boxes (device)
 *   tree_offsets  [T+1] int64 (DEVICE): tree t holds values
 *                 [tree_offsets[t], tree_offsets[t+1]); expected nondecreasing
 *                 from 0 to n.  Not read on the host: an array that is not
 *                 is made so on the device (offsets clamped to [0, n], each at
 *                 least the one before, the last n), never read out of range.
 * The rebuild launches kernels only: no allocation, no host read, no copy, no
 * synchronisation, so it can be captured in a hipGraph together with forest
 * queries (after arborx_forest_reserve) and replayed with new values, offsets
 * and queries of the same sizes; the result equals arborx_forest_build's.
 * While `stream` is being captured the rebuild neither waits for earlier uses
 * of the forest nor records its completion: the caller orders them.
 * arborx_forest_build is create + a copy of host offsets + rebuild.
 */
arborx_status arborx_forest_create(int64_t n, int32_t T, int32_t dim, int32_t kind, void *stream,
                                   arborx_forest *out);
arborx_status arborx_forest_rebuild(arborx_forest forest, const float *values, const int64_t *tree_offsets,
                                    void *stream);


/* Forest metadata [host]: T, total values, dim, and per-tree root and height
 * arrays of T entries (roots/heights may be NULL; -1 root = empty tree). */
arborx_status arborx_forest_info(arborx_forest forest, int32_t *T, int64_t *n, int32_t *dim, int32_t *roots,
                                 int32_t *heights);

/* Grow the query workspace so that forest queries of up to m queries allocate
 * nothing (required before capturing them in a hipGraph). */
arborx_status arborx_forest_reserve(arborx_forest forest, int64_t m, void *stream);

/*
 * Batched queries: batch b is queries [batch_offsets[b], batch_offsets[b+1]) of
 * the packed query array, searched in tree batch_tree[b] only.  batch_offsets
 * ([B+1], int64), batch_tree ([B], int32) and batch_radius ([B], float) are
 * DEVICE arrays; m [host] must equal batch_offsets[B].  Queries of a batch
 * whose tree index is out of range match nothing.  Results are per query, in
 * input order, with indices LOCAL to the target tree (identical to querying
 * that tree built alone).  All batches run in one persistent launch that takes
 * Morton-ordered blocks of queries from a work counter; nothing synchronises,
 * and after arborx_forest_reserve nothing allocates (graph-capturable; while
 * capturing, the call does not wait for the build: order it before capture).
 */
arborx_status arborx_forest_query_reduce(arborx_forest forest, const float *queries, int64_t m,
                                         const int64_t *batch_offsets, const int32_t *batch_tree,
                                         const float *batch_radius, int32_t B, int32_t op, int32_t *counts,
                                         int64_t *sum_fixed, int32_t scale_bits, void *stream);
arborx_status arborx_forest_query_knn(arborx_forest forest, const float *queries, int64_t m,
                                      const int64_t *batch_offsets, const int32_t *batch_tree, int32_t B, int32_t k,
                                      float *dist2, int32_t *indices, void *stream);

/* ------------------------------------------------------------------------ */
/* Chamfer loss of nearest neighbours between paired 3D point clouds.        */
/* ------------------------------------------------------------------------ */

/*
 * Pair p holds clouds a[a_off[p]..a_off[p+1]) and b[b_off[p]..b_off[p+1]) (3D
 * points, device); a_off, b_off are [P+1] HOST offsets.  nn_ab[i] receives the
 * index, local to B_p, of the nearest point of B_p to a_i (the k = 1 nearest
 * query of Section 2.1, ties to the smaller index; -1 if B_p is empty), nn_ba
 * likewise; loss[p] (device float) = sum of those float32 squared distances
 * over both directions, accumulated in float64.
 */
arborx_status arborx_chamfer_forward(const float *a, const int64_t *a_off, const float *b, const int64_t *b_off,
                                     int32_t P, float *loss, int32_t *nn_ab, int32_t *nn_ba, void *stream);

/*
 * Gradient of sum_p grad_loss[p] * loss[p] with the neighbour indices of the
 * forward pass held fixed: dL/da_i = 2(a_i - b_nn(i)) + sum_{j: nn(j)=i} 2(a_i - b_j)
 * (symmetrically for b), evaluated in float64 and rounded once to float32.
 * grad_loss [P], grad_a [na][3], grad_b [nb][3] are device arrays.
 */
arborx_status arborx_chamfer_backward(const float *a, const int64_t *a_off, const float *b, const int64_t *b_off,
                                      int32_t P, const int32_t *nn_ab, const int32_t *nn_ba, const float *grad_loss,
                                      float *grad_a, float *grad_b, void *stream);

/* ------------------------------------------------------------------------ */
/* Diagnostics: building blocks exposed for component tests.                */
/* ------------------------------------------------------------------------ */

/*
 * Stable LSD radix sort of (key, value) pairs by key bits [begin_bit, end_bit),
 * in place.  keys: uint64 when key_bits == 64, uint32 when key_bits == 32.
 * Equal keys keep their input order.  Does not synchronise.
 */
arborx_status arborx_debug_radix_sort(void *keys, uint32_t *values, int64_t n, int32_t key_bits, int32_t begin_bit,
                                      int32_t end_bit, void *stream);

/*
 * 64-bit Morton codes of n points [n][dim] normalised by the box bounds [2][dim]
 * (device, lo row then hi row): b = floor(63/dim) bits per dimension, cell
 * q_d = clamp(floor((x_d - lo_d) / (hi_d - lo_d) * 2^b), 0, 2^b - 1) (0 when
 * hi_d == lo_d), bits interleaved from the most significant down with
 * dimension 0 first within each group.  Does not synchronise.
 */
arborx_status arborx_debug_morton64(const float *points, int64_t n, int32_t dim, const float *bounds, uint64_t *codes,
                                    void *stream);

/* Walk statistics for the touched-bytes measurement: visits[i] = node fetches
 * of query i in the one-query-per-thread depth-first radius walk over binary
 * nodes (op 0, radius) or in the kNN walk after its seeding (op 1, k 1..64).
 * Touched bytes = fetches x the node size (64 B in 3D).  Asynchronous. */
arborx_status arborx_debug_node_visits(arborx_tree tree, const float *queries, int64_t m, float radius, int32_t op,
                                       int32_t k, int32_t *visits, void *stream);

/*
 * Copy the tree's nodes to host memory for invariant checks.  Synchronises.
 *   child   [host] [n-1][2] int32: >= 0 internal node, < 0 leaf holding value ~child
 *   lo, hi  [host] [n-1][2][dim] float32 boxes of the two children
 *   root    [host] index of the root node
 * For n == 1 the single node holds the leaf and an empty slot (INT32_MIN).
 */
arborx_status arborx_debug_tree_nodes(arborx_tree tree, int32_t *child, float *lo, float *hi, int32_t *root);

/*
 * Vector-ALU issue probe for counter calibration: `blocks` workgroups of 256
 * threads each run `iters` rounds of eight independent float32 FMA chains
 * (8 * iters VALU instructions per wavefront in the loop) and write one float
 * per thread to out [device, blocks * 256 floats] so the work is kept.  Its
 * SQ_INSTS_VALU / SQ_BUSY_CYCLES is the achievable issue rate that kernel
 * counter readings are compared with.  blocks in 1..2^20, iters in 1..2^20.
 * Does not synchronise.
 */
arborx_status arborx_debug_valu_probe(float *out, int32_t blocks, int32_t iters, void *stream);

/* ------------------------------------------------------------------------ */
/* Profiling: per-phase GPU time measured with events on the launch stream.  */
/* ------------------------------------------------------------------------ */

/* Enable (1) or disable (0) phase timing for later calls.  [host] */
arborx_status arborx_profile_enable(int32_t on);

/*
 * Wait for the recorded phases, then report and reset them, one entry per phase
 * name: names [host] char[cap][32] (NUL-terminated), ms [host] total
 * milliseconds, launches [host] number of timed phase instances, *count [host]
 * entries written (at most cap).
 */
arborx_status arborx_profile_collect(char *names, double *ms, int64_t *launches, int32_t cap, int32_t *count);

#ifdef __cplusplus
}
#endif

#endif /* ARBORX355_ARBORX_H */
