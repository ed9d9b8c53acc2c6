// extern "C" entry points declared in include/arborx.h: argument validation,
// stream handling, temporaries, and dispatch to the kernels.
#include <cmath>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "device_util.hpp"
#include "internal.hpp"
#include "profile.hpp"

// Streams that have read a structure, each with an event recorded after its
// latest use, so that destroying the structure can order the release of its
// memory after every use without synchronising the device.
struct StreamUses {
    std::mutex mu;
    std::vector<std::pair<hipStream_t, hipEvent_t>> ev;

    void note(hipStream_t s)
    {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
            return;  // a captured graph's lifetime is the caller's to order
        std::lock_guard<std::mutex> lock(mu);
        hipEvent_t e = nullptr;
        for (auto &u : ev)
            if (u.first == s)
                e = u.second;
        if (!e) {
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                (void)hipStreamSynchronize(s);  // cannot track: finish the use now
                return;
            }
            ev.emplace_back(s, e);
        }
        if (hipEventRecord(e, s) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipStreamSynchronize(s);
        }
    }
    // Make `to` wait for every recorded use so far.
    void wait(hipStream_t to)
    {
        std::lock_guard<std::mutex> lock(mu);
        for (auto &u : ev)
            (void)hipStreamWaitEvent(to, u.second, 0);
    }
    // Make `to` wait for every recorded use, then drop the events.
    void wait_all(hipStream_t to)
    {
        std::lock_guard<std::mutex> lock(mu);
        for (auto &u : ev) {
            (void)hipStreamWaitEvent(to, u.second, 0);
            (void)hipEventDestroy(u.second);
        }
        ev.clear();
    }
};

// Records a use on scope exit, so that error paths after a launch are covered too.
struct NoteUse {
    StreamUses &u;
    hipStream_t s;
    ~NoteUse() { u.note(s); }
};

// The traversal order of the last query array a tree was asked about,
// identified by its address, length, predicate kind and order mode.  A
// repeated call reuses it; a changed array under the same address only makes
// the reused order less coherent, never the results different, because any
// permutation of the queries is a valid traversal order.
struct OrderCache {
    std::mutex mu;
    const float *queries = nullptr;
    int64_t m = -1;
    int pred = -1, mode = 0;
    uint32_t *perm = nullptr;
    hipEvent_t ready = nullptr;
};

struct arborx_tree_s {
    ax::TreeDev dev;
    hipEvent_t ready = nullptr;
    StreamUses uses;
    OrderCache order;
};

struct arborx_forest_s {
    ax::ForestDev dev;
    hipEvent_t ready = nullptr;
    StreamUses uses;
};

// State carried from the count call of a CSR query to its fill call.
struct arborx_plan_s {
    arborx_tree tree;
    ax::Pred pred;
    const float *queries;
    int64_t m;
    float radius;
    int64_t *offsets;
    hipStream_t stream;
    ax::Temps tmp;
    uint32_t *perm = nullptr;
    int32_t *counts = nullptr, *ordered_counts = nullptr, *stash = nullptr, *big_list = nullptr, *huge_list = nullptr;
    float *stash_d2 = nullptr;  // with per-match values (distances, or a ray's entry parameters)
    int mode = ax::VALUES_NONE; // how rows are sorted and whether values are kept
    ax::OverflowPool ovf{};
    ax::QueryHeader h{};
    arborx_plan_s(hipStream_t s) : tmp(s) {}
};

namespace ax {

static thread_local std::string g_error;
// Defaults measured on MI355X at 10^7 points: 256-thread blocks for the radius
// walks; 64-thread blocks and an 8-entry LDS ring for kNN (its 8-byte stack
// entries and larger register set).  Over trees of points the radius walks
// run over quantized nodes (half the node loads; a point's leaf is exact in
// its parent), the CSR count one query per thread; kNN over float nodes up to
// 3D, where its top-k insertions rather than node loads bound it
// (node_format_of below).
static Tuning default_tuning(int op)
{
    Tuning t;
    if (op == OP_KNN) {
        t.block = 64;
        t.stack = 8;
    } else {
        t.nodes = 1;
    }
    if (op == OP_SPATIAL)
        t.packet = 1;
    t.by_dim = true;
    return t;
}

void launch_shape(int op, int dim, int &block, int &stack)
{
    const Tuning &t = tuning(op);
    block = t.block;
    stack = t.stack;
    if (t.by_dim && dim >= 6) {
        if (op == OP_KNN) {
            block = 64;
            stack = 16;
        } else if (op == OP_SPATIAL) {
            block = 64;
        }
    }
}
static Tuning g_tuning[OP_KINDS] = {default_tuning(OP_SPATIAL), default_tuning(OP_REDUCE), default_tuning(OP_KNN)};
static std::mutex g_pool_mutex;
static bool g_pool_ready[64] = {};

const Tuning &tuning(int op) { return g_tuning[op >= 0 && op < OP_KINDS ? op : 0]; }

int node_format_of(const Tuning &t, int op, int dim, int kind, bool forest)
{
    if (!t.by_dim)
        return t.nodes;
    if (forest || kind == ARBORX_BOXES)  // a box leaf is not exact in the node: its record is fetched again
        return 0;
    return op == OP_KNN && dim >= 6 ? 1 : t.nodes;
}

int node_format(int op, int dim, int kind, bool forest) { return node_format_of(tuning(op), op, dim, kind, forest); }

bool format_requested(int format, int dim, int kind, bool forest)
{
    for (int op = 0; op < OP_KINDS; ++op)
        if (node_format(op, dim, kind, forest) == format)
            return true;
    return false;
}

bool tree_has_format(arborx_tree tree, int format)
{
    return tree && (format == 0 || (format == 1 && tree->dev.qnodes) || (format == 2 && tree->dev.wnodes));
}

bool forest_has_format(arborx_forest forest, int format)
{
    return forest && (format == 0 || (format == 1 && forest->dev.qnodes) || (format == 2 && forest->dev.wnodes));
}

int walk_format(int op, int dim, int kind)
{
    const Tuning &t = tuning(op);
    const bool thread_walk = op == OP_KNN ? t.schedule != 1 : t.schedule == 0;  // kNN has no rope walk
    return thread_walk ? node_format(op, dim, kind, false) : 0;
}

int tree_format(int op, const TreeDev &t)
{
    const int f = walk_format(op, t.dim, t.kind);
    return (f == 1 && !t.qnodes && tuning(op).by_dim) ? 0 : f;
}

arborx_status check_nodes(const void *qnodes, const void *wnodes, int64_t n, int fmt)
{
    if (n > 0 && ((fmt == 1 && !qnodes) || (fmt == 2 && !wnodes)))
        return fail(ARBORX_E_INVALID, "node_format asks for nodes the structure was built without; "
                                      "set it before building");
    return ARBORX_OK;
}

void set_tuning_op(int op, const Tuning &t)
{
    if (op >= 0 && op < OP_KINDS)
        g_tuning[op] = t;
}

void set_error(const std::string &msg) { g_error = msg; }

arborx_status fail(arborx_status st, const std::string &msg)
{
    set_error(msg);
    return st;
}

arborx_status hip_fail(hipError_t e, const char *what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? ARBORX_E_NOMEM : ARBORX_E_DEVICE;
}

// Keep freed stream-ordered memory in the device pool for reuse.
static void ensure_pool()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return;
    std::lock_guard<std::mutex> lock(g_pool_mutex);
    if (g_pool_ready[dev])
        return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t threshold = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold);
    }
    g_pool_ready[dev] = true;
}

// Caller-supplied allocator (arborx_set_allocator).  Each block taken from
// it is remembered with the stream it was allocated for; a block released on
// another stream (after work there that may still be running) waits in
// `pending` with an event until that work has completed.  The user's
// functions are never called with the mutex held: they may run arbitrary code.
struct UserAllocator {
    arborx_alloc_fn alloc = nullptr;
    arborx_free_fn free_ = nullptr;
    void *ctx = nullptr;
};
struct PendingFree {
    void *p;
    hipStream_t owner;
    hipEvent_t done;
};
static std::mutex g_alloc_mu;
static UserAllocator g_user;
static std::unordered_map<void *, hipStream_t> g_user_blocks;
static std::vector<PendingFree> g_pending;
static std::atomic<int64_t> g_default_live{0};

// Hand back the pending blocks whose event has completed (all of them, after
// waiting, if `wait`).
static void drain_pending(bool wait)
{
    std::vector<PendingFree> ready;
    UserAllocator u;
    {
        std::lock_guard<std::mutex> lock(g_alloc_mu);
        u = g_user;
        for (size_t i = 0; i < g_pending.size();) {
            if (wait)
                (void)hipEventSynchronize(g_pending[i].done);
            const hipError_t q = hipEventQuery(g_pending[i].done);
            if (q == hipSuccess || wait) {
                ready.push_back(g_pending[i]);
                g_pending[i] = g_pending.back();
                g_pending.pop_back();
            } else {
                (void)hipGetLastError();  // "not ready" must not surface as a later call's error
                ++i;
            }
        }
    }
    for (const PendingFree &f : ready) {
        (void)hipEventDestroy(f.done);
        if (u.free_)
            u.free_(f.p, f.owner, u.ctx);
    }
}

arborx_status dalloc(void **p, size_t bytes, hipStream_t s)
{
    *p = nullptr;
    UserAllocator u;
    bool pending = false;
    {
        std::lock_guard<std::mutex> lock(g_alloc_mu);
        u = g_user;
        pending = !g_pending.empty();
    }
    if (u.alloc) {
        if (pending)
            drain_pending(false);
        void *q = u.alloc(bytes ? bytes : 1, static_cast<void *>(s), u.ctx);
        if (!q)
            return fail(ARBORX_E_NOMEM, "the caller's allocator returned no memory for " + std::to_string(bytes) +
                                            " bytes");
        std::lock_guard<std::mutex> lock(g_alloc_mu);
        g_user_blocks[q] = s;
        *p = q;
        return ARBORX_OK;
    }
    ensure_pool();
    hipError_t e = hipMallocAsync(p, bytes ? bytes : 1, s);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(ARBORX_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    ++g_default_live;
    return ARBORX_OK;
}

// Release p after the work queued on s so far.
void dfree(void *p, hipStream_t s)
{
    if (!p)
        return;
    UserAllocator u;
    hipStream_t owner = nullptr;
    bool user = false;
    {
        std::lock_guard<std::mutex> lock(g_alloc_mu);
        auto it = g_user_blocks.find(p);
        if (it != g_user_blocks.end()) {
            user = true;
            owner = it->second;
            g_user_blocks.erase(it);
            u = g_user;
        }
    }
    if (!user) {
        (void)hipFreeAsync(p, s);
        --g_default_live;
        return;
    }
    if (s != owner) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess && hipEventRecord(e, s) == hipSuccess) {
            std::lock_guard<std::mutex> lock(g_alloc_mu);
            g_pending.push_back(PendingFree{p, owner, e});
            return;
        }
        (void)hipGetLastError();
        if (e)
            (void)hipEventDestroy(e);
        (void)hipStreamSynchronize(s);
    }
    if (u.free_)
        u.free_(p, static_cast<void *>(owner), u.ctx);
}

static arborx_status check_device()
{
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return fail(ARBORX_E_DEVICE, "no usable GPU");
    }
    return ARBORX_OK;
}

static bool dim_valid(int dim) { return dim >= 1 && dim <= kMaxDim; }
static bool dim_compiled(int dim) { return dim == 2 || dim == 3 || dim == 6; }

static arborx_status check_tree(arborx_tree t)
{
    if (!t)
        return fail(ARBORX_E_INVALID, "tree is NULL");
    return ARBORX_OK;
}

// Stream of the calling device on which destroyed structures release their
// memory, after waiting for the build and every recorded use.
static hipStream_t release_stream()
{
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        streams[dev] = nullptr;
    }
    return streams[dev];
}

static void release_tree(arborx_tree t)
{
    if (!t)
        return;
    hipStream_t rs = release_stream();
    if (t->ready)
        (void)hipStreamWaitEvent(rs, t->ready, 0);
    t->uses.wait_all(rs);
    if (!rs)
        (void)hipDeviceSynchronize();
    dfree(t->dev.nodes, rs);
    dfree(t->dev.qnodes, rs);
    dfree(t->dev.wnodes, rs);
    dfree(t->dev.codes, rs);
    dfree(t->dev.leaves, rs);
    dfree(t->dev.hdr, rs);
    if (t->order.ready)
        (void)hipStreamWaitEvent(rs, t->order.ready, 0);
    dfree(t->order.perm, rs);
    if (t->order.ready)
        (void)hipEventDestroy(t->order.ready);
    if (t->ready)
        (void)hipEventDestroy(t->ready);
    delete t;
}

// Traversal order for a query call on tree t: the cached one when the call
// repeats the last query array, else a new one that replaces it.
static arborx_status tree_order(arborx_tree t, const float *queries, int64_t m, Pred pred, int op, uint32_t **perm,
                                Temps &tmp, hipStream_t s)
{
    *perm = nullptr;
    const int mode = tuning(op).order;
    if (!mode || t->dev.n == 0 || m <= 1)
        return ARBORX_OK;
    OrderCache &oc = t->order;
    std::lock_guard<std::mutex> lock(oc.mu);
    if (oc.perm && oc.queries == queries && oc.m == m && oc.pred == (int)pred && oc.mode == mode) {
        AX_HIP(hipStreamWaitEvent(s, oc.ready, 0));
        *perm = oc.perm;
        return ARBORX_OK;
    }
    uint32_t *fresh = nullptr, *keep = nullptr;
    arborx_status st = query_order(t->dev, queries, m, pred, op, &fresh, tmp, s);
    if (st != ARBORX_OK || !fresh)
        return st;
    if ((st = dalloc((void **)&keep, (size_t)m * sizeof(uint32_t), s)) != ARBORX_OK)
        return st;
    AX_HIP(hipMemcpyAsync(keep, fresh, (size_t)m * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    if (!oc.ready)
        AX_HIP(hipEventCreateWithFlags(&oc.ready, hipEventDisableTiming));
    if (oc.perm) {  // release the old order after every use of the tree so far
        hipStream_t rs = release_stream();
        (void)hipStreamWaitEvent(rs, oc.ready, 0);
        t->uses.wait(rs);
        dfree(oc.perm, rs);
    }
    AX_HIP(hipEventRecord(oc.ready, s));
    oc.queries = queries;
    oc.m = m;
    oc.pred = (int)pred;
    oc.mode = mode;
    oc.perm = keep;
    *perm = keep;
    return ARBORX_OK;
}

static arborx_status wait_tree(arborx_tree t, hipStream_t s)
{
    AX_HIP(hipStreamWaitEvent(s, t->ready, 0));
    return ARBORX_OK;
}

}  // namespace ax

using namespace ax;

extern "C" {

const char *arborx_version(void) { return "arborx355 0.1"; }

const char *arborx_last_error(void) { return g_error.c_str(); }

static arborx_status to_tuning(const arborx_tuning *t, const Tuning &base, Tuning &n)
{
    n = base;
    n.by_dim = false;  // a caller's tuning is used as given
    if (t->block) {
        if (t->block != 64 && t->block != 128 && t->block != 256)
            return fail(ARBORX_E_INVALID, "block must be 64, 128 or 256");
        n.block = t->block;
    }
    if (t->order < 0 || t->order > 2)
        return fail(ARBORX_E_INVALID, "order must be 0 (none), 1 (24-bit Morton) or 2 (16-bit Morton)");
    n.order = t->order;
    if (t->stack) {
        if (t->stack < 1 || t->stack > 64 || (t->stack & (t->stack - 1)))
            return fail(ARBORX_E_INVALID, "stack must be a power of two in 1..64");
        n.stack = t->stack;
    }
    if (t->schedule < 0 || t->schedule > 2)
        return fail(ARBORX_E_INVALID, "schedule must be 0 (thread, short stack), 1 (wavefront packet) or 2 (ropes)");
    n.schedule = t->schedule;
    if (t->build != 0 && t->build != 1)
        return fail(ARBORX_E_INVALID, "build must be 0 or 1");
    n.build = t->build;
    if (t->seed_mode < 0 || t->seed_mode > 2)
        return fail(ARBORX_E_INVALID, "seed_mode must be 0, 1 or 2");
    n.seed = t->seed_mode;
    if (t->node_format < 0 || t->node_format > 2)
        return fail(ARBORX_E_INVALID, "node_format must be 0 (binary), 1 (binary, 16-bit boxes) or 2 (four-wide)");
    n.nodes = t->node_format;
    if (t->queries_per_thread != 0 && t->queries_per_thread != 1 && t->queries_per_thread != 2 &&
        t->queries_per_thread != 4)
        return fail(ARBORX_E_INVALID, "queries_per_thread must be 0 (default), 1, 2 or 4");
    n.packet = t->queries_per_thread;
    return ARBORX_OK;
}

static void from_tuning(const Tuning &g, arborx_tuning *t)
{
    t->block = g.block;
    t->order = g.order;
    t->stack = g.stack;
    t->schedule = g.schedule;
    t->build = g.build;
    t->seed_mode = g.seed;
    t->node_format = g.nodes;
    t->queries_per_thread = g.packet;
}

arborx_status arborx_set_allocator(arborx_alloc_fn alloc_fn, arborx_free_fn free_fn, void *ctx)
{
    if (!alloc_fn != !free_fn)
        return fail(ARBORX_E_INVALID, "alloc_fn and free_fn must both be given or both be NULL");
    drain_pending(true);
    std::lock_guard<std::mutex> lock(g_alloc_mu);
    if (!g_user_blocks.empty() || !g_pending.empty() || g_default_live.load() != 0)
        return fail(ARBORX_E_INVALID, "the library still holds device memory (a live tree, forest or plan)");
    g_user.alloc = alloc_fn;
    g_user.free_ = free_fn;
    g_user.ctx = alloc_fn ? ctx : nullptr;
    return ARBORX_OK;
}

arborx_status arborx_set_tuning(const arborx_tuning *t)
{
    if (!t) {
        for (int op = 0; op < OP_KINDS; ++op)
            g_tuning[op] = default_tuning(op);
        return ARBORX_OK;
    }
    Tuning n;
    arborx_status st = to_tuning(t, g_tuning[0], n);
    if (st != ARBORX_OK)
        return st;
    for (auto &g : g_tuning)
        g = n;
    return ARBORX_OK;
}

arborx_status arborx_set_tuning_op(int32_t op, const arborx_tuning *t)
{
    if (op < 0 || op >= OP_KINDS)
        return fail(ARBORX_E_INVALID, "unknown operation");
    if (!t) {
        g_tuning[op] = default_tuning(op);
        return ARBORX_OK;
    }
    Tuning n;
    arborx_status st = to_tuning(t, g_tuning[op], n);
    if (st == ARBORX_OK)
        g_tuning[op] = n;
    return st;
}

arborx_status arborx_get_tuning(arborx_tuning *t)
{
    if (!t)
        return fail(ARBORX_E_INVALID, "tuning is NULL");
    from_tuning(g_tuning[0], t);
    return ARBORX_OK;
}

arborx_status arborx_get_tuning_op(int32_t op, arborx_tuning *t)
{
    if (!t)
        return fail(ARBORX_E_INVALID, "tuning is NULL");
    if (op < 0 || op >= OP_KINDS)
        return fail(ARBORX_E_INVALID, "unknown operation");
    from_tuning(g_tuning[op], t);
    return ARBORX_OK;
}

arborx_status arborx_bvh_build(const float *values, int64_t n, int32_t dim, int32_t kind, void *stream,
                               arborx_tree *out)
{
    if (!out)
        return fail(ARBORX_E_INVALID, "out is NULL");
    if (n < 0 || n >= INT32_MAX)
        return fail(ARBORX_E_INVALID, "n must be in [0, 2^31-1)");
    if (!dim_valid(dim))
        return fail(ARBORX_E_INVALID, "dim must be in 1..10");
    if (kind != ARBORX_POINTS && kind != ARBORX_BOXES)
        return fail(ARBORX_E_INVALID, "kind must be ARBORX_POINTS or ARBORX_BOXES");
    if (n > 0 && !values)
        return fail(ARBORX_E_INVALID, "values is NULL");
    if (!dim_compiled(dim))
        return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in (2, 3 and 6 are)");
    arborx_status st = check_device();
    if (st != ARBORX_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    arborx_tree t = new arborx_tree_s();
    st = build_tree(values, n, dim, kind, t->dev, s);
    if (st == ARBORX_OK) {
        hipError_t e = hipEventCreateWithFlags(&t->ready, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventRecord(t->ready, s);
        if (e != hipSuccess)
            st = hip_fail(e, "hipEventRecord");
    }
    if (st != ARBORX_OK) {
        std::string msg = g_error;
        (void)hipStreamSynchronize(s);
        release_tree(t);
        set_error(msg);
        return st;
    }
    *out = t;
    return ARBORX_OK;
}

arborx_status arborx_bvh_destroy(arborx_tree t)
{
    release_tree(t);
    return ARBORX_OK;
}

arborx_status arborx_bvh_info(arborx_tree t, int64_t *n, int32_t *dim, int32_t *kind, float *bounds, int32_t *height)
{
    arborx_status st = check_tree(t);
    if (st != ARBORX_OK)
        return st;
    AX_HIP(hipEventSynchronize(t->ready));
    TreeHeader h;
    AX_HIP(hipMemcpy(&h, t->dev.hdr, sizeof(h), hipMemcpyDeviceToHost));
    if (n)
        *n = t->dev.n;
    if (dim)
        *dim = t->dev.dim;
    if (kind)
        *kind = t->dev.kind;
    if (bounds)
        for (int d = 0; d < t->dev.dim; ++d) {
            bounds[d] = h.lo[d];
            bounds[t->dev.dim + d] = h.hi[d];
        }
    if (height)
        *height = h.height;
    return ARBORX_OK;
}

static arborx_status csr_begin(arborx_tree t, Pred pred, const float *queries, int64_t m, float radius,
                               int64_t *offsets, int64_t *total, arborx_plan *out, void *stream,
                               int mode = VALUES_NONE)
{
    const bool with_dist = mode != VALUES_NONE;
    arborx_status st = check_tree(t);
    if (st != ARBORX_OK)
        return st;
    if (!out)
        return fail(ARBORX_E_INVALID, "plan is NULL");
    if (m < 0 || m >= INT32_MAX)
        return fail(ARBORX_E_INVALID, "m must be in [0, 2^31-1)");
    if (m > 0 && !queries)
        return fail(ARBORX_E_INVALID, "queries is NULL");
    if (!offsets)
        return fail(ARBORX_E_INVALID, "offsets is NULL");
    if (!total)
        return fail(ARBORX_E_INVALID, "total is NULL");
    if (pred == Pred::Sphere && (std::isnan(radius) || radius < 0.0f))
        return fail(ARBORX_E_INVALID, "radius must be >= 0 and not NaN");
    if ((st = check_device()) != ARBORX_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = wait_tree(t, s)) != ARBORX_OK)
        return st;
    NoteUse note_use{t->uses, s};
    arborx_plan p = new arborx_plan_s(s);
    p->tree = t;
    p->pred = pred;
    p->queries = queries;
    p->m = m;
    p->radius = radius;
    p->offsets = offsets;
    p->stream = s;
    p->mode = mode;
    auto bail = [&](arborx_status e) {
        std::string msg = g_error;
        delete p;
        set_error(msg);
        return e;
    };
    QueryHeader *qh;
    uint8_t *sws;
    const int64_t mm = m > 0 ? m : 1;
    if ((st = p->tmp.get(&qh, 1)) != ARBORX_OK || (st = p->tmp.get(&p->counts, mm)) != ARBORX_OK ||
        (st = p->tmp.get(&p->ordered_counts, mm)) != ARBORX_OK ||
        (st = p->tmp.get(&p->stash, mm * stash_regs(t->dev.dim))) != ARBORX_OK ||
        (st = p->tmp.get(&p->ovf.head, mm)) != ARBORX_OK ||
        (st = p->tmp.get(&p->ovf.pool, overflow_pool_ints(mm, t->dev.dim, overflow_factor(pred)))) != ARBORX_OK ||
        (st = p->tmp.get(&p->ovf.ctr, (size_t)kOvfPools * 8)) != ARBORX_OK ||
        (st = p->tmp.get(&p->big_list, mm)) != ARBORX_OK || (st = p->tmp.get(&p->huge_list, mm)) != ARBORX_OK ||
        (st = p->tmp.get(&sws, scan_workspace_bytes(m))) != ARBORX_OK)
        return bail(st);
    p->ovf.dpool = nullptr;
    if (with_dist && ((st = p->tmp.get(&p->stash_d2, mm * stash_regs(t->dev.dim))) != ARBORX_OK ||
                      (st = p->tmp.get(&p->ovf.dpool, overflow_pool_ints(mm, t->dev.dim, overflow_factor(pred)))) !=
                          ARBORX_OK))
        return bail(st);
    if ((st = tree_order(t, queries, m, pred, OP_SPATIAL, &p->perm, p->tmp, s)) != ARBORX_OK)
        return bail(st);
    p->ovf.per = (int32_t)(overflow_pool_ints(mm, t->dev.dim, overflow_factor(pred)) / kOvfPools);
    if ((st = spatial_count(t->dev, pred, queries, m, radius, p->perm, p->counts, p->ordered_counts, p->stash,
                            p->stash_d2, p->ovf, s)) != ARBORX_OK)
        return bail(st);
    {
        ProfScope ps("scan", s);
        hipError_t e = csr_offsets_lists(p->counts, p->ordered_counts, p->perm, m, stash_regs(t->dev.dim), offsets,
                                         p->big_list, p->huge_list,
                                         qh, sws, s);
        if (e != hipSuccess)
            return bail(hip_fail(e, "csr_offsets_lists"));
    }
    hipError_t e = hipMemcpyAsync(&p->h, qh, sizeof(p->h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return bail(hip_fail(e, "reading the match total"));
    *total = (int64_t)p->h.total;
    p->perm = nullptr;  // the tree's cached order may be replaced once this call returns
    *out = p;
    return ARBORX_OK;
}

static arborx_status csr_finish(arborx_plan p, int32_t *indices, int64_t capacity, float *dist = nullptr,
                                bool sorted = true)
{
    if (!p)
        return fail(ARBORX_E_INVALID, "plan is NULL");
    if (!sorted && p->mode == VALUES_ORDERED)
        return fail(ARBORX_E_INVALID, "rows of an ordered plan are always ordered by their values");
    if (capacity < 0)
        return fail(ARBORX_E_INVALID, "capacity must be >= 0");
    if (dist && !p->stash_d2)
        return fail(ARBORX_E_INVALID, "distances asked of a plan begun without them");
    if (!indices || capacity < (int64_t)p->h.total)
        return fail(ARBORX_E_CAPACITY, "indices capacity " + std::to_string(capacity) + " < total " +
                                           std::to_string((long long)p->h.total));
    if (p->h.total == 0)
        return ARBORX_OK;
    arborx_status st;
    if (!dist && p->mode == VALUES_ORDERED &&  // rows ordered by value need the values even when not returned
        (st = p->tmp.get(&dist, (size_t)p->h.total)) != ARBORX_OK)
        return st;
    NoteUse note_use{p->tree->uses, p->stream};
    st = spatial_fill(p->tree->dev, p->pred, p->queries, p->m, p->radius, p->counts, p->stash, p->stash_d2, p->ovf,
                      p->offsets, p->big_list, (int64_t)p->h.big_rows, p->huge_list, (int64_t)p->h.huge_rows,
                      indices, dist, p->mode, p->stream, sorted);
    if (st != ARBORX_OK || !sorted)
        return st;
    if ((st = sort_big_rows(p->offsets, indices, dist, p->mode, p->big_list, (int64_t)p->h.big_rows, p->stream)) !=
        ARBORX_OK)
        return st;
    return sort_huge_rows(p->tree->dev.n, p->offsets, indices, dist, p->mode, p->huge_list, (int64_t)p->h.huge_rows,
                          p->tmp, p->stream);
}

static arborx_status csr_query(arborx_tree t, Pred pred, const float *queries, int64_t m, float radius,
                               int64_t *offsets, int32_t *indices, int64_t capacity, int64_t *total, void *stream,
                               int mode = VALUES_NONE, float *dist = nullptr)
{
    if (capacity < 0)
        return fail(ARBORX_E_INVALID, "capacity must be >= 0");
    const bool with_dist = mode != VALUES_NONE;
    arborx_plan p = nullptr;
    arborx_status st = csr_begin(t, pred, queries, m, radius, offsets, total, &p, stream, mode);
    if (st != ARBORX_OK)
        return st;
    st = (with_dist && p->h.total > 0 && !dist) ? fail(ARBORX_E_CAPACITY, "the per-match value output is NULL")
                                                 : csr_finish(p, indices, capacity, p->h.total > 0 ? dist : nullptr);
    std::string msg = g_error;
    delete p;
    set_error(msg);
    return st;
}

arborx_status arborx_query_spatial_begin(arborx_tree t, const float *queries, int64_t m, float radius,
                                         int64_t *offsets, int64_t *total, arborx_plan *plan, void *stream)
{
    return csr_begin(t, Pred::Sphere, queries, m, radius, offsets, total, plan, stream);
}

arborx_status arborx_query_intersects_begin(arborx_tree t, const float *qboxes, int64_t m, int64_t *offsets,
                                            int64_t *total, arborx_plan *plan, void *stream)
{
    return csr_begin(t, Pred::Box, qboxes, m, 0.0f, offsets, total, plan, stream);
}

arborx_status arborx_query_finish(arborx_plan plan, int32_t *indices, int64_t capacity)
{
    return csr_finish(plan, indices, capacity);
}

arborx_status arborx_query_finish_unsorted(arborx_plan plan, int32_t *indices, int64_t capacity)
{
    return csr_finish(plan, indices, capacity, nullptr, false);
}

arborx_status arborx_query_spatial_with_distances_begin(arborx_tree t, const float *queries, int64_t m, float radius,
                                                        int64_t *offsets, int64_t *total, arborx_plan *plan,
                                                        void *stream)
{
    return csr_begin(t, Pred::Sphere, queries, m, radius, offsets, total, plan, stream, VALUES_BY_INDEX);
}

arborx_status arborx_query_finish_with_distances(arborx_plan plan, int32_t *indices, float *distances,
                                                 int64_t capacity)
{
    if (plan && plan->h.total > 0 && !distances)
        return fail(ARBORX_E_INVALID, "distances is NULL");
    if (plan && plan->h.total == 0)
        return csr_finish(plan, indices, capacity);
    return csr_finish(plan, indices, capacity, distances);
}

arborx_status arborx_query_spatial_with_distances(arborx_tree t, const float *queries, int64_t m, float radius,
                                                  int64_t *offsets, int32_t *indices, float *distances,
                                                  int64_t capacity, int64_t *total, void *stream)
{
    return csr_query(t, Pred::Sphere, queries, m, radius, offsets, indices, capacity, total, stream, VALUES_BY_INDEX,
                     distances);
}

arborx_status arborx_plan_destroy(arborx_plan plan)
{
    delete plan;
    return ARBORX_OK;
}

arborx_status arborx_query_spatial(arborx_tree t, const float *queries, int64_t m, float radius, int64_t *offsets,
                                   int32_t *indices, int64_t capacity, int64_t *total, void *stream)
{
    return csr_query(t, Pred::Sphere, queries, m, radius, offsets, indices, capacity, total, stream);
}

arborx_status arborx_query_intersects(arborx_tree t, const float *qboxes, int64_t m, int64_t *offsets,
                                      int32_t *indices, int64_t capacity, int64_t *total, void *stream)
{
    return csr_query(t, Pred::Box, qboxes, m, 0.0f, offsets, indices, capacity, total, stream);
}

arborx_status arborx_query_knn(arborx_tree t, const float *queries, int64_t m, int32_t k, float *dist2,
                               int32_t *indices, void *stream)
{
    arborx_status st = check_tree(t);
    if (st != ARBORX_OK)
        return st;
    if (m < 0)
        return fail(ARBORX_E_INVALID, "m must be >= 0");
    if (k < 1 || k > 64)
        return fail(ARBORX_E_INVALID, "k must be in 1..64");
    if (m > 0 && (!queries || !dist2 || !indices))
        return fail(ARBORX_E_INVALID, "queries, dist2 and indices must not be NULL");
    if ((st = check_device()) != ARBORX_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = wait_tree(t, s)) != ARBORX_OK)
        return st;
    NoteUse note_use{t->uses, s};
    Temps tmp(s);
    uint32_t *perm = nullptr;
    if ((st = tree_order(t, queries, m, Pred::Sphere, OP_KNN, &perm, tmp, s)) != ARBORX_OK)
        return st;
    return knn_query(t->dev, queries, m, k, perm, dist2, indices, s);
}

arborx_status arborx_query_knn_noalloc(arborx_tree t, const float *queries, int64_t m, int32_t k, float *dist2,
                                       int32_t *indices, void *stream)
{
    arborx_status st = check_tree(t);
    if (st != ARBORX_OK)
        return st;
    if (m < 0)
        return fail(ARBORX_E_INVALID, "m must be >= 0");
    if (k < 1 || k > 64)
        return fail(ARBORX_E_INVALID, "k must be in 1..64");
    if (m > 0 && (!queries || !dist2 || !indices))
        return fail(ARBORX_E_INVALID, "queries, dist2 and indices must not be NULL");
    if (m > ARBORX_NOALLOC_MAX_QUERIES)
        return fail(ARBORX_E_CAPACITY, "m = " + std::to_string((long long)m) +
                                           " exceeds ARBORX_NOALLOC_MAX_QUERIES = " +
                                           std::to_string(ARBORX_NOALLOC_MAX_QUERIES));
    if ((st = check_device()) != ARBORX_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    AX_HIP(hipStreamIsCapturing(s, &cs));
    if (cs == hipStreamCaptureStatusNone && (st = wait_tree(t, s)) != ARBORX_OK)
        return st;
    NoteUse note_use{t->uses, s};
    return knn_query_noalloc(t->dev, queries, m, k, dist2, indices, s);
}

arborx_status arborx_query_spatial_reduce(arborx_tree t, const float *queries, int64_t m, float radius, int32_t op,
                                          int32_t *counts, int64_t *sum_fixed, int32_t scale_bits, void *stream)
{
    arborx_status st = check_tree(t);
    if (st != ARBORX_OK)
        return st;
    if (m < 0)
        return fail(ARBORX_E_INVALID, "m must be >= 0");
    if (op != ARBORX_COUNT && op != ARBORX_COUNT_SUMDIST)
        return fail(ARBORX_E_INVALID, "unknown reducer");
    if (std::isnan(radius) || radius < 0.0f)
        return fail(ARBORX_E_INVALID, "radius must be >= 0 and not NaN");
    if (op == ARBORX_COUNT_SUMDIST && (scale_bits < 0 || scale_bits > 40))
        return fail(ARBORX_E_INVALID, "scale_bits must be in 0..40");
    if (m > 0 && (!queries || !counts || (op == ARBORX_COUNT_SUMDIST && !sum_fixed)))
        return fail(ARBORX_E_INVALID, "queries, counts (and sum_fixed for COUNT_SUMDIST) must not be NULL");
    if ((st = check_device()) != ARBORX_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = wait_tree(t, s)) != ARBORX_OK)
        return st;
    NoteUse note_use{t->uses, s};
    Temps tmp(s);
    uint32_t *perm = nullptr;
    if ((st = tree_order(t, queries, m, Pred::Sphere, OP_REDUCE, &perm, tmp, s)) != ARBORX_OK)
        return st;
    return spatial_reduce(t->dev, queries, m, radius, op, scale_bits, perm, counts, sum_fixed, s);
}

static arborx_status ray_args(arborx_tree t, const float *rays, int64_t m, const void *out1, const void *out2)
{
    arborx_status st = check_tree(t);
    if (st != ARBORX_OK)
        return st;
    if (m < 0 || m >= INT32_MAX)
        return fail(ARBORX_E_INVALID, "m must be in [0, 2^31-1)");
    if (m > 0 && (!rays || !out1 || !out2))
        return fail(ARBORX_E_INVALID, "rays and outputs must not be NULL");
    return check_device();
}

arborx_status arborx_query_ray_intersect_begin(arborx_tree t, const float *rays, int64_t m, int64_t *offsets,
                                              int64_t *total, arborx_plan *plan, void *stream)
{
    return csr_begin(t, Pred::Ray, rays, m, 0.0f, offsets, total, plan, stream, VALUES_NONE);
}

arborx_status arborx_query_ray_intersect(arborx_tree t, const float *rays, int64_t m, int64_t *offsets,
                                        int32_t *indices, int64_t capacity, int64_t *total, void *stream)
{
    return csr_query(t, Pred::Ray, rays, m, 0.0f, offsets, indices, capacity, total, stream);
}

arborx_status arborx_query_ray_ordered_intersect_begin(arborx_tree t, const float *rays, int64_t m,
                                                      int64_t *offsets, int64_t *total, arborx_plan *plan,
                                                      void *stream)
{
    return csr_begin(t, Pred::Ray, rays, m, 0.0f, offsets, total, plan, stream, VALUES_ORDERED);
}

arborx_status arborx_query_ray_ordered_intersect(arborx_tree t, const float *rays, int64_t m, int64_t *offsets,
                                                int32_t *indices, float *t_entry, int64_t capacity, int64_t *total,
                                                void *stream)
{
    return csr_query(t, Pred::Ray, rays, m, 0.0f, offsets, indices, capacity, total, stream, VALUES_ORDERED,
                     t_entry);
}

arborx_status arborx_query_ray_count(arborx_tree t, const float *rays, int64_t m, int32_t *counts, void *stream)
{
    arborx_status st = ray_args(t, rays, m, counts, counts);
    if (st != ARBORX_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = wait_tree(t, s)) != ARBORX_OK)
        return st;
    NoteUse note_use{t->uses, s};
    Temps tmp(s);
    uint32_t *perm = nullptr;
    if ((st = tree_order(t, rays, m, Pred::Ray, OP_REDUCE, &perm, tmp, s)) != ARBORX_OK)
        return st;
    return ray_count(t->dev, rays, m, perm, counts, s);
}

arborx_status arborx_query_ray_nearest(arborx_tree t, const float *rays, int64_t m, int32_t k, float *t_entry,
                                       int32_t *indices, void *stream)
{
    if (k < 1 || k > 64)
        return fail(ARBORX_E_INVALID, "k must be in 1..64");
    arborx_status st = ray_args(t, rays, m, t_entry, indices);
    if (st != ARBORX_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = wait_tree(t, s)) != ARBORX_OK)
        return st;
    NoteUse note_use{t->uses, s};
    Temps tmp(s);
    uint32_t *perm = nullptr;
    if ((st = tree_order(t, rays, m, Pred::Ray, OP_KNN, &perm, tmp, s)) != ARBORX_OK)
        return st;
    return ray_nearest(t->dev, rays, m, perm, k, t_entry, indices, s);
}

arborx_status arborx_dbscan(arborx_tree t, const float *points, float eps, int32_t min_pts, int32_t *labels,
                            void *stream)
{
    arborx_status st = check_tree(t);
    if (st != ARBORX_OK)
        return st;
    if (t->dev.kind != ARBORX_POINTS)
        return fail(ARBORX_E_INVALID, "DBSCAN clusters a tree built from points");
    if (std::isnan(eps) || eps < 0.0f)
        return fail(ARBORX_E_INVALID, "eps must be >= 0 and not NaN");
    if (min_pts < 0)
        return fail(ARBORX_E_INVALID, "min_pts must be >= 0");
    const int64_t n = t->dev.n;
    if (n > 0 && (!points || !labels))
        return fail(ARBORX_E_INVALID, "points and labels must not be NULL");
    if ((st = check_device()) != ARBORX_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = wait_tree(t, s)) != ARBORX_OK)
        return st;
    if (n == 0)
        return ARBORX_OK;
    NoteUse note_use{t->uses, s};
    return dbscan(t->dev, eps, min_pts, labels, s);
}

arborx_status arborx_self_join_degree(arborx_tree t, float radius, int32_t *degree, void *stream)
{
    arborx_status st = check_tree(t);
    if (st != ARBORX_OK)
        return st;
    if (t->dev.kind != ARBORX_POINTS)
        return fail(ARBORX_E_INVALID, "the self-join pairs the points of a tree built from points");
    if (std::isnan(radius) || radius < 0.0f)
        return fail(ARBORX_E_INVALID, "radius must be >= 0 and not NaN");
    if (t->dev.n > 0 && !degree)
        return fail(ARBORX_E_INVALID, "degree must not be NULL");
    if ((st = check_device()) != ARBORX_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = wait_tree(t, s)) != ARBORX_OK)
        return st;
    if (t->dev.n == 0)
        return ARBORX_OK;
    NoteUse note_use{t->uses, s};
    return self_join_degree(t->dev, radius, degree, s);
}

arborx_status arborx_query_match_distances(arborx_tree t, const float *values, const float *queries, int64_t m,
                                           const int64_t *offsets, const int32_t *indices, float *distances,
                                           void *stream)
{
    arborx_status st = check_tree(t);
    if (st != ARBORX_OK)
        return st;
    if (m < 0)
        return fail(ARBORX_E_INVALID, "m must be >= 0");
    if (m > 0 && (!queries || !offsets || (t->dev.n > 0 && (!values || !indices || !distances))))
        return fail(ARBORX_E_INVALID, "values, queries, offsets, indices and distances must not be NULL");
    if ((st = check_device()) != ARBORX_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = wait_tree(t, s)) != ARBORX_OK)
        return st;
    return match_distances(t->dev, values, queries, m, offsets, indices, distances, s);
}

arborx_status arborx_query_spatial_count_up_to(arborx_tree t, const float *queries, int64_t m, float radius,
                                               int32_t n_max, int32_t *counts, void *stream)
{
    arborx_status st = check_tree(t);
    if (st != ARBORX_OK)
        return st;
    if (m < 0)
        return fail(ARBORX_E_INVALID, "m must be >= 0");
    if (std::isnan(radius) || radius < 0.0f)
        return fail(ARBORX_E_INVALID, "radius must be >= 0 and not NaN");
    if (n_max < 0)
        return fail(ARBORX_E_INVALID, "n_max must be >= 0");
    if (m > 0 && (!queries || !counts))
        return fail(ARBORX_E_INVALID, "queries and counts must not be NULL");
    if ((st = check_device()) != ARBORX_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = wait_tree(t, s)) != ARBORX_OK)
        return st;
    NoteUse note_use{t->uses, s};
    Temps tmp(s);
    uint32_t *perm = nullptr;
    if (n_max > 0 && (st = tree_order(t, queries, m, Pred::Sphere, OP_REDUCE, &perm, tmp, s)) != ARBORX_OK)
        return st;
    return spatial_count_up_to(t->dev, queries, m, radius, n_max, perm, counts, s);
}

// ---------------------------------------------------------------------------
// forest
// ---------------------------------------------------------------------------

static arborx_status forest_wait(arborx_forest f, hipStream_t s)
{
    // A graph being captured cannot wait on an event recorded outside it; the
    // caller orders the build before the capture in that case.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return ARBORX_OK;
    AX_HIP(hipStreamWaitEvent(s, f->ready, 0));
    return ARBORX_OK;
}

arborx_status arborx_forest_build(const float *values, const int64_t *tree_offsets, int32_t T, int32_t dim,
                                  int32_t kind, void *stream, arborx_forest *out)
{
    if (!out)
        return fail(ARBORX_E_INVALID, "out is NULL");
    if (T < 1)
        return fail(ARBORX_E_INVALID, "T must be >= 1");
    if (!tree_offsets)
        return fail(ARBORX_E_INVALID, "tree_offsets is NULL");
    if (tree_offsets[0] != 0)
        return fail(ARBORX_E_INVALID, "tree_offsets[0] must be 0");
    for (int t = 0; t < T; ++t)
        if (tree_offsets[t + 1] < tree_offsets[t])
            return fail(ARBORX_E_INVALID, "tree_offsets must be nondecreasing");
    if (tree_offsets[T] >= INT32_MAX)
        return fail(ARBORX_E_INVALID, "too many values");
    if ((int64_t)T + tree_offsets[T] / 4096 + 1 >= INT32_MAX)
        return fail(ARBORX_E_INVALID, "too many trees");
    if (!dim_valid(dim))
        return fail(ARBORX_E_INVALID, "dim must be in 1..10");
    if (kind != ARBORX_POINTS && kind != ARBORX_BOXES)
        return fail(ARBORX_E_INVALID, "kind must be ARBORX_POINTS or ARBORX_BOXES");
    if (tree_offsets[T] > 0 && !values)
        return fail(ARBORX_E_INVALID, "values is NULL");
    if (!dim_compiled(dim))
        return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in (2, 3 and 6 are)");
    arborx_status st = check_device();
    if (st != ARBORX_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    arborx_forest f = new arborx_forest_s();
    st = build_forest(values, tree_offsets, T, dim, kind, f->dev, s);
    if (st == ARBORX_OK) {
        hipError_t e = hipEventCreateWithFlags(&f->ready, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventRecord(f->ready, s);
        if (e != hipSuccess)
            st = hip_fail(e, "hipEventRecord");
    }
    if (st != ARBORX_OK) {
        std::string msg = g_error;
        (void)hipStreamSynchronize(s);
        forest_release(f->dev, s);
        (void)hipStreamSynchronize(s);
        if (f->ready)
            (void)hipEventDestroy(f->ready);
        delete f;
        set_error(msg);
        return st;
    }
    *out = f;
    return ARBORX_OK;
}

arborx_status arborx_forest_create(int64_t n, int32_t T, int32_t dim, int32_t kind, void *stream, arborx_forest *out)
{
    if (!out)
        return fail(ARBORX_E_INVALID, "out is NULL");
    if (T < 1)
        return fail(ARBORX_E_INVALID, "T must be >= 1");
    if (n < 0 || n >= INT32_MAX)
        return fail(ARBORX_E_INVALID, "n must be in [0, 2^31-1)");
    if ((int64_t)T + n / 4096 + 1 >= INT32_MAX)
        return fail(ARBORX_E_INVALID, "too many trees");
    if (!dim_valid(dim))
        return fail(ARBORX_E_INVALID, "dim must be in 1..10");
    if (kind != ARBORX_POINTS && kind != ARBORX_BOXES)
        return fail(ARBORX_E_INVALID, "kind must be ARBORX_POINTS or ARBORX_BOXES");
    if (!dim_compiled(dim))
        return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in (2, 3 and 6 are)");
    arborx_status st = check_device();
    if (st != ARBORX_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    arborx_forest f = new arborx_forest_s();
    st = forest_alloc(n, T, dim, kind, f->dev, s);
    if (st == ARBORX_OK) {
        hipError_t e = hipEventCreateWithFlags(&f->ready, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventRecord(f->ready, s);
        if (e != hipSuccess)
            st = hip_fail(e, "hipEventRecord");
    }
    if (st != ARBORX_OK) {
        std::string msg = g_error;
        (void)hipStreamSynchronize(s);
        forest_release(f->dev, s);
        (void)hipStreamSynchronize(s);
        if (f->ready)
            (void)hipEventDestroy(f->ready);
        delete f;
        set_error(msg);
        return st;
    }
    *out = f;
    return ARBORX_OK;
}

arborx_status arborx_forest_rebuild(arborx_forest f, const float *values, const int64_t *tree_offsets, void *stream)
{
    if (!f)
        return fail(ARBORX_E_INVALID, "forest is NULL");
    if (!tree_offsets)
        return fail(ARBORX_E_INVALID, "tree_offsets is NULL");
    if (f->dev.n > 0 && !values)
        return fail(ARBORX_E_INVALID, "values is NULL");
    arborx_status st = check_device();
    if (st != ARBORX_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    AX_HIP(hipStreamIsCapturing(s, &cs));
    const bool capturing = cs != hipStreamCaptureStatusNone;
    if (!capturing) {  // queries of the old contents on other streams finish first
        AX_HIP(hipStreamWaitEvent(s, f->ready, 0));
        f->uses.wait(s);
    }
    if ((st = forest_rebuild(values, tree_offsets, f->dev, s)) != ARBORX_OK)
        return st;
    if (!capturing)
        AX_HIP(hipEventRecord(f->ready, s));
    return ARBORX_OK;
}

arborx_status arborx_forest_destroy(arborx_forest f)
{
    if (!f)
        return ARBORX_OK;
    hipStream_t rs = release_stream();
    if (f->ready)
        (void)hipStreamWaitEvent(rs, f->ready, 0);
    f->uses.wait_all(rs);
    if (!rs)
        (void)hipDeviceSynchronize();
    forest_release(f->dev, rs);
    if (f->ready)
        (void)hipEventDestroy(f->ready);
    delete f;
    return ARBORX_OK;
}

arborx_status arborx_forest_info(arborx_forest f, int32_t *T, int64_t *n, int32_t *dim, int32_t *roots,
                                 int32_t *heights)
{
    if (!f)
        return fail(ARBORX_E_INVALID, "forest is NULL");
    if (T)
        *T = f->dev.T;
    if (n)
        *n = f->dev.n;
    if (dim)
        *dim = f->dev.dim;
    if (roots || heights) {
        AX_HIP(hipEventSynchronize(f->ready));
        std::vector<TreeHeader> h(f->dev.T);
        AX_HIP(hipMemcpy(h.data(), f->dev.hdrs, sizeof(TreeHeader) * f->dev.T, hipMemcpyDeviceToHost));
        for (int t = 0; t < f->dev.T; ++t) {
            if (roots)
                roots[t] = h[t].root;
            if (heights)
                heights[t] = h[t].height;
        }
    }
    return ARBORX_OK;
}

arborx_status arborx_forest_reserve(arborx_forest f, int64_t m, void *stream)
{
    if (!f)
        return fail(ARBORX_E_INVALID, "forest is NULL");
    if (m < 0 || m >= INT32_MAX)
        return fail(ARBORX_E_INVALID, "m must be in [0, 2^31-1)");
    arborx_status st = check_device();
    if (st != ARBORX_OK)
        return st;
    return forest_reserve(f->dev, m, static_cast<hipStream_t>(stream));
}

static arborx_status forest_query_args(arborx_forest f, const float *queries, int64_t m, const int64_t *boff,
                                       const int32_t *btree, int32_t B)
{
    if (!f)
        return fail(ARBORX_E_INVALID, "forest is NULL");
    if (m < 0 || m >= INT32_MAX)
        return fail(ARBORX_E_INVALID, "m must be in [0, 2^31-1)");
    if (B < 1)
        return fail(ARBORX_E_INVALID, "B must be >= 1");
    if (m > 0 && (!queries || !boff || !btree))
        return fail(ARBORX_E_INVALID, "queries, batch_offsets and batch_tree must not be NULL");
    return check_device();
}

arborx_status arborx_forest_query_reduce(arborx_forest f, const float *queries, int64_t m,
                                         const int64_t *batch_offsets, const int32_t *batch_tree,
                                         const float *batch_radius, int32_t B, int32_t op, int32_t *counts,
                                         int64_t *sum_fixed, int32_t scale_bits, void *stream)
{
    arborx_status st = forest_query_args(f, queries, m, batch_offsets, batch_tree, B);
    if (st != ARBORX_OK)
        return st;
    if (op != ARBORX_COUNT && op != ARBORX_COUNT_SUMDIST)
        return fail(ARBORX_E_INVALID, "unknown reducer");
    if (op == ARBORX_COUNT_SUMDIST && (scale_bits < 0 || scale_bits > 40))
        return fail(ARBORX_E_INVALID, "scale_bits must be in 0..40");
    if (m > 0 && (!batch_radius || !counts || (op == ARBORX_COUNT_SUMDIST && !sum_fixed)))
        return fail(ARBORX_E_INVALID, "batch_radius, counts (and sum_fixed) must not be NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = forest_wait(f, s)) != ARBORX_OK)
        return st;
    NoteUse note_use{f->uses, s};
    return forest_query_reduce(f->dev, queries, m, batch_offsets, batch_tree, batch_radius, B, op, scale_bits, counts,
                               sum_fixed, s);
}

arborx_status arborx_forest_query_knn(arborx_forest f, const float *queries, int64_t m, const int64_t *batch_offsets,
                                      const int32_t *batch_tree, int32_t B, int32_t k, float *dist2, int32_t *indices,
                                      void *stream)
{
    arborx_status st = forest_query_args(f, queries, m, batch_offsets, batch_tree, B);
    if (st != ARBORX_OK)
        return st;
    if (k < 1 || k > 64)
        return fail(ARBORX_E_INVALID, "k must be in 1..64");
    if (m > 0 && (!dist2 || !indices))
        return fail(ARBORX_E_INVALID, "dist2 and indices must not be NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = forest_wait(f, s)) != ARBORX_OK)
        return st;
    NoteUse note_use{f->uses, s};
    return forest_query_knn(f->dev, queries, m, batch_offsets, batch_tree, B, k, dist2, indices, s);
}

// ---------------------------------------------------------------------------
// Chamfer
// ---------------------------------------------------------------------------

static arborx_status chamfer_args(const float *a, const int64_t *a_off, const float *b, const int64_t *b_off, int P)
{
    if (P < 1)
        return fail(ARBORX_E_INVALID, "P must be >= 1");
    if (!a_off || !b_off)
        return fail(ARBORX_E_INVALID, "offsets must not be NULL");
    if (a_off[0] != 0 || b_off[0] != 0)
        return fail(ARBORX_E_INVALID, "offsets must start at 0");
    for (int p = 0; p < P; ++p)
        if (a_off[p + 1] < a_off[p] || b_off[p + 1] < b_off[p])
            return fail(ARBORX_E_INVALID, "offsets must be nondecreasing");
    if (a_off[P] + b_off[P] >= INT32_MAX)
        return fail(ARBORX_E_INVALID, "too many points");
    if ((a_off[P] > 0 && !a) || (b_off[P] > 0 && !b))
        return fail(ARBORX_E_INVALID, "point arrays must not be NULL");
    return check_device();
}

arborx_status arborx_chamfer_forward(const float *a, const int64_t *a_off, const float *b, const int64_t *b_off,
                                     int32_t P, float *loss, int32_t *nn_ab, int32_t *nn_ba, void *stream)
{
    arborx_status st = chamfer_args(a, a_off, b, b_off, P);
    if (st != ARBORX_OK)
        return st;
    if (!loss || (a_off[P] > 0 && !nn_ab) || (b_off[P] > 0 && !nn_ba))
        return fail(ARBORX_E_INVALID, "outputs must not be NULL");
    return chamfer_forward(a, a_off, b, b_off, P, loss, nn_ab, nn_ba, static_cast<hipStream_t>(stream));
}

arborx_status arborx_chamfer_backward(const float *a, const int64_t *a_off, const float *b, const int64_t *b_off,
                                      int32_t P, const int32_t *nn_ab, const int32_t *nn_ba, const float *grad_loss,
                                      float *grad_a, float *grad_b, void *stream)
{
    arborx_status st = chamfer_args(a, a_off, b, b_off, P);
    if (st != ARBORX_OK)
        return st;
    if (!grad_loss || (a_off[P] > 0 && (!nn_ab || !grad_a)) || (b_off[P] > 0 && (!nn_ba || !grad_b)))
        return fail(ARBORX_E_INVALID, "inputs and outputs must not be NULL");
    return chamfer_backward(a, a_off, b, b_off, P, nn_ab, nn_ba, grad_loss, grad_a, grad_b,
                            static_cast<hipStream_t>(stream));
}

arborx_status arborx_debug_radix_sort(void *keys, uint32_t *values, int64_t n, int32_t key_bits, int32_t begin_bit,
                                      int32_t end_bit, void *stream)
{
    if (n < 0 || n > (int64_t)UINT32_MAX)
        return fail(ARBORX_E_INVALID, "n out of range");
    if (key_bits != 32 && key_bits != 64)
        return fail(ARBORX_E_INVALID, "key_bits must be 32 or 64");
    if (begin_bit < 0 || end_bit > key_bits || begin_bit > end_bit || end_bit - begin_bit > 64)
        return fail(ARBORX_E_INVALID, "bad bit range");
    if (n > 0 && (!keys || !values))
        return fail(ARBORX_E_INVALID, "keys and values must not be NULL");
    arborx_status st = check_device();
    if (st != ARBORX_OK)
        return st;
    if (n <= 1)
        return ARBORX_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Temps tmp(s);
    uint32_t *v2;
    uint8_t *ws;
    bool alt = false;
    if ((st = tmp.get(&v2, n)) != ARBORX_OK || (st = tmp.get(&ws, radix_workspace_bytes(n))) != ARBORX_OK)
        return st;
    if (key_bits == 64) {
        uint64_t *k2;
        if ((st = tmp.get(&k2, n)) != ARBORX_OK)
            return st;
        AX_HIP(radix_sort_pairs<uint64_t>(static_cast<uint64_t *>(keys), values, k2, v2, n, begin_bit, end_bit, ws, s,
                                          &alt));
        if (alt)
            AX_HIP(hipMemcpyAsync(keys, k2, n * 8, hipMemcpyDeviceToDevice, s));
    } else {
        uint32_t *k2;
        if ((st = tmp.get(&k2, n)) != ARBORX_OK)
            return st;
        AX_HIP(radix_sort_pairs<uint32_t>(static_cast<uint32_t *>(keys), values, k2, v2, n, begin_bit, end_bit, ws, s,
                                          &alt));
        if (alt)
            AX_HIP(hipMemcpyAsync(keys, k2, n * 4, hipMemcpyDeviceToDevice, s));
    }
    if (alt)
        AX_HIP(hipMemcpyAsync(values, v2, n * 4, hipMemcpyDeviceToDevice, s));
    return ARBORX_OK;
}

arborx_status arborx_debug_morton64(const float *points, int64_t n, int32_t dim, const float *bounds, uint64_t *codes,
                                    void *stream)
{
    if (n < 0)
        return fail(ARBORX_E_INVALID, "n must be >= 0");
    if (!dim_valid(dim))
        return fail(ARBORX_E_INVALID, "dim must be in 1..10");
    if (!dim_compiled(dim))
        return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in");
    if (n > 0 && (!points || !bounds || !codes))
        return fail(ARBORX_E_INVALID, "NULL pointer");
    arborx_status st = check_device();
    if (st != ARBORX_OK)
        return st;
    AX_HIP(morton64_points(points, n, dim, bounds, codes, static_cast<hipStream_t>(stream)));
    return ARBORX_OK;
}

namespace ax {
namespace {
// Eight independent FMA chains per thread: the loop body is VALU work only.
__global__ __launch_bounds__(256) void k_valu_probe(float *__restrict__ out, int iters)
{
    const float x = (float)threadIdx.x * 0x1p-10f;
    float a0 = x, a1 = x + 1.0f, a2 = x + 2.0f, a3 = x + 3.0f, a4 = x + 4.0f, a5 = x + 5.0f, a6 = x + 6.0f,
          a7 = x + 7.0f;
    for (int i = 0; i < iters; ++i) {
        a0 = fmaf(a0, 0.999f, 0.25f);
        a1 = fmaf(a1, 0.999f, 0.25f);
        a2 = fmaf(a2, 0.999f, 0.25f);
        a3 = fmaf(a3, 0.999f, 0.25f);
        a4 = fmaf(a4, 0.999f, 0.25f);
        a5 = fmaf(a5, 0.999f, 0.25f);
        a6 = fmaf(a6, 0.999f, 0.25f);
        a7 = fmaf(a7, 0.999f, 0.25f);
    }
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
}
}  // namespace
}  // namespace ax

arborx_status arborx_debug_valu_probe(float *out, int32_t blocks, int32_t iters, void *stream)
{
    if (!out)
        return fail(ARBORX_E_INVALID, "out is NULL");
    if (blocks < 1 || blocks > (1 << 20) || iters < 1 || iters > (1 << 20))
        return fail(ARBORX_E_INVALID, "blocks and iters must be in 1..2^20");
    arborx_status st = check_device();
    if (st != ARBORX_OK)
        return st;
    k_valu_probe<<<blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(out, iters);
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

arborx_status arborx_debug_node_visits(arborx_tree t, const float *queries, int64_t m, float radius, int32_t op,
                                       int32_t k, int32_t *visits, void *stream)
{
    arborx_status st = check_tree(t);
    if (st != ARBORX_OK)
        return st;
    if (m < 0 || m >= INT32_MAX)
        return fail(ARBORX_E_INVALID, "m must be in [0, 2^31-1)");
    if (op != 0 && op != 1)
        return fail(ARBORX_E_INVALID, "op must be 0 (radius walk) or 1 (kNN walk)");
    if (op == 1 && (k < 1 || k > 64))
        return fail(ARBORX_E_INVALID, "k must be in 1..64");
    if (op == 0 && (std::isnan(radius) || radius < 0.0f))
        return fail(ARBORX_E_INVALID, "radius must be >= 0 and not NaN");
    if (m > 0 && (!queries || !visits))
        return fail(ARBORX_E_INVALID, "queries and visits must not be NULL");
    if ((st = check_device()) != ARBORX_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = wait_tree(t, s)) != ARBORX_OK)
        return st;
    NoteUse note_use{t->uses, s};
    return debug_node_visits(t->dev, queries, m, radius, op, k, visits, s);
}

arborx_status arborx_debug_tree_nodes(arborx_tree t, int32_t *child, float *lo, float *hi, int32_t *root)
{
    arborx_status st = check_tree(t);
    if (st != ARBORX_OK)
        return st;
    if (!child || !lo || !hi || !root)
        return fail(ARBORX_E_INVALID, "NULL pointer");
    AX_HIP(hipEventSynchronize(t->ready));
    TreeHeader h;
    AX_HIP(hipMemcpy(&h, t->dev.hdr, sizeof(h), hipMemcpyDeviceToHost));
    *root = h.root;
    const int64_t nn = t->dev.n > 1 ? t->dev.n - 1 : (t->dev.n == 1 ? 1 : 0);
    if (nn == 0)
        return ARBORX_OK;
    const int D = t->dev.dim;
    const size_t nb = node_bytes(D);
    std::string buf(nn * nb, '\0');
    AX_HIP(hipMemcpy(&buf[0], t->dev.nodes, nn * nb, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < nn; ++i) {
        const char *p = buf.data() + i * nb;
        const float *flo = reinterpret_cast<const float *>(p);
        const float *fhi = flo + 2 * D;
        const int32_t *ch = reinterpret_cast<const int32_t *>(fhi + 2 * D);
        for (int s2 = 0; s2 < 2; ++s2) {
            child[i * 2 + s2] = ch[s2];
            for (int d = 0; d < D; ++d) {
                lo[(i * 2 + s2) * D + d] = flo[s2 * D + d];
                hi[(i * 2 + s2) * D + d] = fhi[s2 * D + d];
            }
        }
    }
    return ARBORX_OK;
}

}  // extern "C"
