// Schedule autotuner.  For one operation kind (radius CSR, radius reduce, kNN)
// it runs the caller's own queries under each candidate schedule, checks that
// every candidate produced the same outputs (an order-independent 64-bit hash
// of the output words, computed on the device), times each with events on the
// caller's stream, and installs the fastest as that operation's tuning.
// Choices can be cached in a JSON-lines file named by ARBORX_TUNING_CACHE,
// keyed by operation, dimension, kind, k and the size classes of n and m.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "device_util.hpp"
#include "internal.hpp"

namespace ax {
namespace {

__device__ __forceinline__ unsigned long long mix64(unsigned long long x)
{
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

// Sum over i of mix(word_i, i): equal inputs give equal hashes whatever the
// summation order.
__global__ void k_hash(const uint32_t *__restrict__ w, int64_t n, unsigned long long salt,
                       unsigned long long *__restrict__ out)
{
    unsigned long long h = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        h += mix64(((unsigned long long)w[i] << 32) ^ (unsigned long long)i ^ salt);
    h = wave_sum(h);
    if (lane_id() == 0)
        atomicAdd(out, h);
}

struct Candidate {
    Tuning t;
    double ms = 0;
};

// Median of three timed runs, in milliseconds, with events on the caller's
// stream.  Short launches vary by several percent between runs; the median
// of three is far steadier than the best of two.
template <class Run>
double median_ms(Run &run, hipEvent_t e0, hipEvent_t e1, hipStream_t s, arborx_status &st)
{
    float t[3] = {0, 0, 0};
    for (int rep = 0; rep < 3 && st == ARBORX_OK; ++rep) {
        (void)hipEventRecord(e0, s);
        st = run();
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&t[rep], e0, e1);
    }
    const float lo = fminf(t[0], fminf(t[1], t[2])), hi = fmaxf(t[0], fmaxf(t[1], t[2]));
    return (double)(t[0] + t[1] + t[2] - lo - hi);
}

// Candidate 0 is the tuning in force; another wins only when at least 3%
// faster, so timing noise on short launches does not flip the choice.
int keep_unless_faster(const std::vector<Candidate> &c, int besti)
{
    return c[besti].ms < 0.97 * c[0].ms ? besti : 0;
}

std::string cache_key(int op, int dim, int kind, int k, int64_t n, int64_t m)
{
    char buf[160];
    std::snprintf(buf, sizeof(buf), "op=%d dim=%d kind=%d k=%d logn=%d logm=%d", op, dim, kind, op == OP_KNN ? k : 0,
                  n > 0 ? (int)std::floor(std::log2((double)n)) : -1, m > 0 ? (int)std::floor(std::log2((double)m)) : -1);
    return buf;
}

bool cache_lookup(const std::string &key, Tuning &t)
{
    const char *path = std::getenv("ARBORX_TUNING_CACHE");
    if (!path || !*path)
        return false;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        char k[200];
        int block, order, stack, schedule, seed, nodes, packet;
        if (std::sscanf(line, "{\"key\": \"%199[^\"]\", \"block\": %d, \"order\": %d, \"stack\": %d, \"schedule\": %d, "
                              "\"seed\": %d, \"nodes\": %d, \"packet\": %d",
                        k, &block, &order, &stack, &schedule, &seed, &nodes, &packet) == 8 &&
            key == k) {
            t.block = block;
            t.order = order;
            t.stack = stack;
            t.schedule = schedule;
            t.seed = seed;
            t.nodes = nodes;
            t.packet = packet;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const std::string &key, const Tuning &t, double ms)
{
    const char *path = std::getenv("ARBORX_TUNING_CACHE");
    if (!path || !*path)
        return;
    FILE *f = std::fopen(path, "a");
    if (!f)
        return;
    std::fprintf(f,
                 "{\"key\": \"%s\", \"block\": %d, \"order\": %d, \"stack\": %d, \"schedule\": %d, \"seed\": %d, "
                 "\"nodes\": %d, \"packet\": %d, \"ms\": %.4f}\n",
                 key.c_str(), t.block, t.order, t.stack, t.schedule, t.seed, t.nodes, t.packet, ms);
    std::fclose(f);
}

}  // namespace
}  // namespace ax

using namespace ax;

extern "C" arborx_status arborx_autotune(arborx_tree tree, int32_t op, const float *queries, int64_t m, float radius,
                                         int32_t k, arborx_tuning *best, double *best_ms, void *stream)
{
    if (!tree)
        return fail(ARBORX_E_INVALID, "tree is NULL");
    if (op < 0 || op >= OP_KINDS)
        return fail(ARBORX_E_INVALID, "unknown operation");
    if (m <= 0 || !queries)
        return fail(ARBORX_E_INVALID, "autotuning needs queries");
    if (op == OP_KNN && (k < 1 || k > 64))
        return fail(ARBORX_E_INVALID, "k must be in 1..64");
    if (op != OP_KNN && (std::isnan(radius) || radius < 0.0f))
        return fail(ARBORX_E_INVALID, "radius must be >= 0 and not NaN");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int64_t n = 0;
    int32_t dim = 0, kind = 0;
    arborx_status st = arborx_bvh_info(tree, &n, &dim, &kind, nullptr, nullptr);
    if (st != ARBORX_OK)
        return st;
    const std::string key = cache_key(op, dim, kind, k, n, m);
    Tuning cached = tuning(op);
    if (cache_lookup(key, cached)) {
        set_tuning_op(op, cached);
        if (best) {
            best->block = cached.block;
            best->order = cached.order;
            best->stack = cached.stack;
            best->schedule = cached.schedule;
            best->build = cached.build;
            best->seed_mode = cached.seed;
            best->queries_per_thread = cached.packet;
            best->node_format = node_format_of(cached, op, dim, kind, false);
        }
        if (best_ms)
            *best_ms = -1.0;
        return ARBORX_OK;
    }

    const Tuning base = tuning(op);
    std::vector<Candidate> cands;
    cands.push_back(Candidate{base, 0});  // the tuning in force: kept unless another is clearly faster
    for (int block : {64, 128, 256})
        for (int stack : {8, 16, 32}) {
            Candidate c;
            c.t = base;
            c.t.block = block;
            c.t.stack = stack;
            c.t.schedule = 0;
            c.t.nodes = 0;
            c.t.order = 1;
            cands.push_back(c);
        }
    for (int block : {64, 128, 256}) {
        Candidate c;
        c.t = base;
        c.t.block = block;
        c.t.schedule = 1;
        c.t.order = 1;
        cands.push_back(c);
    }
    for (int format : {1, 2})  // other node formats, when the tree holds them
        for (int block : {64, 256}) {
            if (!tree_has_format(tree, format))
                break;
            Candidate c;
            c.t = base;
            c.t.block = block;
            c.t.schedule = 0;
            c.t.nodes = format;
            c.t.order = 1;
            cands.push_back(c);
        }
    if (op != OP_KNN)
        for (int format : {0, 1})
            for (int nq : {1, 2, 4}) {  // queries per thread of the radius walks
                if (!tree_has_format(tree, format))
                    break;
                Candidate c;
                c.t = base;
                c.t.schedule = 0;
                c.t.nodes = format;
                c.t.packet = nq;
                cands.push_back(c);
            }
    if (op != OP_KNN)
        for (int block : {64, 256}) {
            Candidate c;
            c.t = base;
            c.t.block = block;
            c.t.schedule = 2;
            c.t.order = 1;
            cands.push_back(c);
        }
    {
        Candidate c;
        c.t = base;
        c.t.order = 0;
        c.t.schedule = 0;
        cands.push_back(c);
    }
    if (op == OP_KNN) {
        const size_t nbase = cands.size();
        for (size_t i = 1; i < nbase; i += 4)
            for (int mode = 0; mode < 3; ++mode)
                if (mode != cands[i].t.seed) {
                    Candidate c = cands[i];
                    c.t.seed = mode;
                    cands.push_back(c);
                }
    }

    for (size_t i = 1; i < cands.size(); ++i)  // candidates are used exactly as listed
        cands[i].t.by_dim = false;
    Temps tmp(s);
    unsigned long long *hash;
    int32_t *o1 = nullptr;
    int64_t *o2 = nullptr, *offsets = nullptr;
    float *d2 = nullptr;
    int32_t *indices = nullptr;
    int64_t total = 0;
    if ((st = tmp.get(&hash, 1)) != ARBORX_OK)
        return st;
    if (op == OP_KNN) {
        if ((st = tmp.get(&d2, m * k)) != ARBORX_OK || (st = tmp.get(&o1, m * k)) != ARBORX_OK)
            return st;
    } else if (op == OP_REDUCE) {
        if ((st = tmp.get(&o1, m)) != ARBORX_OK || (st = tmp.get(&o2, m)) != ARBORX_OK)
            return st;
    } else {
        if ((st = tmp.get(&offsets, m + 1)) != ARBORX_OK)
            return st;
        arborx_plan plan = nullptr;
        if ((st = arborx_query_spatial_begin(tree, queries, m, radius, offsets, &total, &plan, stream)) != ARBORX_OK)
            return st;
        arborx_plan_destroy(plan);
        if ((st = tmp.get(&indices, total > 0 ? total : 1)) != ARBORX_OK)
            return st;
    }
    auto run = [&]() -> arborx_status {
        if (op == OP_KNN)
            return arborx_query_knn(tree, queries, m, k, d2, o1, stream);
        if (op == OP_REDUCE)
            return arborx_query_spatial_reduce(tree, queries, m, radius, ARBORX_COUNT_SUMDIST, o1, o2, 32, stream);
        int64_t tot = 0;
        return arborx_query_spatial(tree, queries, m, radius, offsets, indices, total > 0 ? total : 1, &tot, stream);
    };
    auto digest = [&](unsigned long long *h) -> arborx_status {
        fill_kernel<unsigned long long><<<1, 64, 0, s>>>(hash, 1, 0ull);
        auto add = [&](const void *p, int64_t words, unsigned long long salt) {
            if (words > 0)
                k_hash<<<grid_for(words, 256, 4096), 256, 0, s>>>(static_cast<const uint32_t *>(p), words, salt, hash);
        };
        if (op == OP_KNN) {
            add(d2, m * k, 1);
            add(o1, m * k, 2);
        } else if (op == OP_REDUCE) {
            add(o1, m, 3);
            add(o2, 2 * m, 4);
        } else {
            add(offsets, 2 * (m + 1), 5);
            add(indices, total, 6);
        }
        AX_HIP(hipMemcpyAsync(h, hash, 8, hipMemcpyDeviceToHost, s));
        AX_HIP(hipStreamSynchronize(s));
        return ARBORX_OK;
    };
    hipEvent_t e0, e1;
    AX_HIP(hipEventCreate(&e0));
    AX_HIP(hipEventCreate(&e1));
    unsigned long long ref = 0;
    int besti = -1;
    for (size_t i = 0; i < cands.size() && st == ARBORX_OK; ++i) {
        set_tuning_op(op, cands[i].t);
        if ((st = run()) != ARBORX_OK)
            break;
        unsigned long long h = 0;
        if ((st = digest(&h)) != ARBORX_OK)
            break;
        if (i == 0)
            ref = h;
        else if (h != ref)
            st = fail(ARBORX_E_DEVICE, "schedule candidate " + std::to_string(i) + " changed the results");
        if (st != ARBORX_OK)
            break;
        cands[i].ms = median_ms(run, e0, e1, s, st);
        if (besti < 0 || cands[i].ms < cands[besti].ms)
            besti = (int)i;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != ARBORX_OK || besti < 0) {
        set_tuning_op(op, base);
        return st != ARBORX_OK ? st : fail(ARBORX_E_DEVICE, "no candidate ran");
    }
    besti = keep_unless_faster(cands, besti);
    const Tuning &b = cands[besti].t;
    set_tuning_op(op, b);
    cache_store(key, b, cands[besti].ms);
    if (best) {
        best->block = b.block;
        best->order = b.order;
        best->stack = b.stack;
        best->schedule = b.schedule;
        best->build = b.build;
        best->seed_mode = b.seed;
        best->queries_per_thread = b.packet;
        best->node_format = node_format_of(b, op, dim, kind, false);
    }
    if (best_ms)
        *best_ms = cands[besti].ms;
    return ARBORX_OK;
}

// Forest queries: the same search over the candidates a forest walk honours
// (stack depth, queries per thread of the reductions, node format, kNN seed;
// the forest's work queue fixes block size and query order).
extern "C" arborx_status arborx_autotune_forest(arborx_forest forest, int32_t op, const float *queries, int64_t m,
                                                const int64_t *batch_offsets, const int32_t *batch_tree,
                                                const float *batch_radius, int32_t B, int32_t k, arborx_tuning *best,
                                                double *best_ms, void *stream)
{
    if (!forest)
        return fail(ARBORX_E_INVALID, "forest is NULL");
    if (op != OP_REDUCE && op != OP_KNN)
        return fail(ARBORX_E_INVALID, "forest queries are ARBORX_OP_REDUCE or ARBORX_OP_KNN");
    if (m <= 0 || !queries || !batch_offsets || !batch_tree || B < 1)
        return fail(ARBORX_E_INVALID, "autotuning needs queries and batches");
    if (op == OP_KNN && (k < 1 || k > 64))
        return fail(ARBORX_E_INVALID, "k must be in 1..64");
    if (op == OP_REDUCE && !batch_radius)
        return fail(ARBORX_E_INVALID, "batch_radius is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t T = 0, dim = 0;
    int64_t n = 0;
    arborx_status st = arborx_forest_info(forest, &T, &n, &dim, nullptr, nullptr);
    if (st != ARBORX_OK)
        return st;
    const std::string key = "forest " + cache_key(op, dim, 0, k, n, m);
    const int fkind = ARBORX_POINTS;  // under the defaults every forest walks format 0, whatever its values
    const Tuning base = tuning(op);
    Tuning cached = base;
    if (cache_lookup(key, cached)) {
        set_tuning_op(op, cached);
        if (best) {
            best->block = cached.block;
            best->order = cached.order;
            best->stack = cached.stack;
            best->schedule = cached.schedule;
            best->build = cached.build;
            best->seed_mode = cached.seed;
            best->queries_per_thread = cached.packet;
            best->node_format = node_format_of(cached, op, dim, fkind, true);
        }
        if (best_ms)
            *best_ms = -1.0;
        return ARBORX_OK;
    }
    std::vector<Candidate> cands;
    cands.push_back(Candidate{base, 0});
    Tuning fbase = base;  // the others start from the node format the forest walks under the tuning in force
    fbase.nodes = node_format_of(base, op, dim, fkind, true);
    for (int stack : {4, 8, 16, 32}) {
        Candidate c{fbase, 0};
        c.t.stack = stack;
        c.t.nodes = 0;
        cands.push_back(c);
    }
    if (op == OP_REDUCE)
        for (int nq : {1, 2, 4})
            for (int stack : {8, 16}) {
                Candidate c{fbase, 0};
                c.t.nodes = 0;
                c.t.packet = nq;
                c.t.stack = stack;
                cands.push_back(c);
            }
    for (int format : {1, 2})
        if (forest_has_format(forest, format)) {
            Candidate c{fbase, 0};
            c.t.nodes = format;
            cands.push_back(c);
        }
    if (op == OP_KNN)
        for (int mode = 0; mode < 3; ++mode)
            if (mode != base.seed) {
                Candidate c{fbase, 0};
                c.t.seed = mode;
                cands.push_back(c);
            }

    for (size_t i = 1; i < cands.size(); ++i)
        cands[i].t.by_dim = false;
    Temps tmp(s);
    unsigned long long *hash;
    int32_t *o1 = nullptr;
    int64_t *o2 = nullptr;
    float *d2 = nullptr;
    if ((st = tmp.get(&hash, 1)) != ARBORX_OK)
        return st;
    if (op == OP_KNN) {
        if ((st = tmp.get(&d2, m * k)) != ARBORX_OK || (st = tmp.get(&o1, m * k)) != ARBORX_OK)
            return st;
    } else if ((st = tmp.get(&o1, m)) != ARBORX_OK || (st = tmp.get(&o2, m)) != ARBORX_OK) {
        return st;
    }
    if ((st = arborx_forest_reserve(forest, m, stream)) != ARBORX_OK)
        return st;
    auto run = [&]() -> arborx_status {
        if (op == OP_KNN)
            return arborx_forest_query_knn(forest, queries, m, batch_offsets, batch_tree, B, k, d2, o1, stream);
        return arborx_forest_query_reduce(forest, queries, m, batch_offsets, batch_tree, batch_radius, B,
                                          ARBORX_COUNT_SUMDIST, o1, o2, 32, stream);
    };
    auto digest = [&](unsigned long long *h) -> arborx_status {
        fill_kernel<unsigned long long><<<1, 64, 0, s>>>(hash, 1, 0ull);
        auto add = [&](const void *p, int64_t words, unsigned long long salt) {
            if (words > 0)
                k_hash<<<grid_for(words, 256, 4096), 256, 0, s>>>(static_cast<const uint32_t *>(p), words, salt, hash);
        };
        if (op == OP_KNN) {
            add(d2, m * k, 1);
            add(o1, m * k, 2);
        } else {
            add(o1, m, 3);
            add(o2, 2 * m, 4);
        }
        AX_HIP(hipMemcpyAsync(h, hash, 8, hipMemcpyDeviceToHost, s));
        AX_HIP(hipStreamSynchronize(s));
        return ARBORX_OK;
    };
    hipEvent_t e0, e1;
    AX_HIP(hipEventCreate(&e0));
    AX_HIP(hipEventCreate(&e1));
    unsigned long long ref = 0;
    int besti = -1;
    for (size_t i = 0; i < cands.size() && st == ARBORX_OK; ++i) {
        set_tuning_op(op, cands[i].t);
        if ((st = run()) != ARBORX_OK)
            break;
        unsigned long long h = 0;
        if ((st = digest(&h)) != ARBORX_OK)
            break;
        if (i == 0)
            ref = h;
        else if (h != ref)
            st = fail(ARBORX_E_DEVICE, "forest schedule candidate " + std::to_string(i) + " changed the results");
        if (st != ARBORX_OK)
            break;
        cands[i].ms = median_ms(run, e0, e1, s, st);
        if (besti < 0 || cands[i].ms < cands[besti].ms)
            besti = (int)i;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != ARBORX_OK || besti < 0) {
        set_tuning_op(op, base);
        return st != ARBORX_OK ? st : fail(ARBORX_E_DEVICE, "no candidate ran");
    }
    besti = keep_unless_faster(cands, besti);
    const Tuning &b = cands[besti].t;
    set_tuning_op(op, b);
    cache_store(key, b, cands[besti].ms);
    if (best) {
        best->block = b.block;
        best->order = b.order;
        best->stack = b.stack;
        best->schedule = b.schedule;
        best->build = b.build;
        best->seed_mode = b.seed;
        best->queries_per_thread = b.packet;
        best->node_format = node_format_of(b, op, dim, fkind, true);
    }
    if (best_ms)
        *best_ms = cands[besti].ms;
    return ARBORX_OK;
}
