// Batched queries over a built BVH (Section 2.1: spatial and nearest
// predicates; storage query with CSR output; Section 2.2: pure callbacks).
//
// Queries are first put in Morton order (Section 2.6: sorting is used in
// search as well as construction) so that the 64 lanes of a wavefront walk
// neighbouring paths and share node fetches.  Each thread then answers one
// query with a depth-first walk whose deferred subtrees sit on a short stack:
// the newest entries in a per-thread column of LDS, older ones spilled to
// private memory when the LDS ring is full, so any tree height is handled.
//
// Every node holds the boxes of both children, so one fetch tests two
// children.  A child that is a leaf is decided from the slot box alone: for
// point values the box is the point, and the box distance equals the point
// distance bit for bit.
#include <mutex>
#include <string>
#include <type_traits>

#include "device_util.hpp"
#include "geometry.hpp"
#include "internal.hpp"
#include "profile.hpp"
#include "traverse.hpp"

namespace ax {
namespace {

// Node slots of a single tree (one-value trees still have one node).
__device__ __forceinline__ int node_count(const TreeHeader *hdr) { return hdr->n > 1 ? hdr->n - 1 : 1; }

// Match number c (c >= R, counted from 0) of query qi, past its stash row of
// R: stored in the query's overflow chain, whose current chunk is `cur` (one
// register per query; -2 once the row is given up).  Chunks come from the
// sub-pool of this workgroup as the row grows; the first one is recorded as
// the row's head, each later one in the last slot of its predecessor.
template <int R, bool OUT>
__device__ __forceinline__ void overflow_add(const OverflowPool &o, int64_t qi, int c, int idx, float d2,
                                             int32_t &cur)
{
    if (cur == -2)
        return;
    const int k = c - R;
    const int pos = k % (kChunk - 1);
    if (c >= kRowSortBlock) {  // a huge row: walked again and sorted apart
        cur = -2;
        o.head[qi] = -2;
        return;
    }
    if (pos == 0) {
        const int sub = (int)(blockIdx.x % kOvfPools);
        const unsigned long long b = atomicAdd(&o.ctr[sub * 8], (unsigned long long)kChunk);
        if (b + kChunk > (unsigned long long)o.per) {  // pool exhausted: walk this row again
            cur = -2;
            o.head[qi] = -2;
            return;
        }
        const int32_t next = sub * o.per + (int32_t)b;
        if (k == 0)
            o.head[qi] = next;
        else
            o.pool[cur + kChunk - 1] = next;
        cur = next;
    }
    o.pool[cur + pos] = idx;
    if (OUT)
        o.dpool[cur + pos] = d2;  // the callback's output, in the parallel pool
}

// Stash row writer of the count walks.  Matches gather in a four-entry
// register group that is stored into the query's stash row (one 16-byte
// store, and one for the values) each time it fills, and once more for a
// partial last group, so a match costs a four-way select instead of one over
// the whole row.  Row entries past the count stay unwritten: every reader
// masks the row by its count.
template <bool OUT>
struct StashGroup {
    int g[4];
    float dg[OUT ? 4 : 1];
    __device__ __forceinline__ void add(int c, int idx, float d2, int32_t *row, float *drow)
    {
        const int k = c & 3;
        append_at<4>(g, k, idx);
        if constexpr (OUT)
            append_at<4>(dg, k, d2);
        if (k == 3)
            flush(c - 3, row, drow);
    }
    __device__ __forceinline__ void flush(int base, int32_t *row, float *drow) const
    {
        *reinterpret_cast<int4 *>(row + base) = make_int4(g[0], g[1], g[2], g[3]);
        if constexpr (OUT)
            *reinterpret_cast<float4 *>(drow + base) = make_float4(dg[0], dg[1], dg[2], dg[3]);
    }
    // after the walk, for a row of c matches with a stash row of R
    __device__ __forceinline__ void finish(int c, int R, int32_t *row, float *drow) const
    {
        if (c < R && (c & 3) != 0)
            flush(c & ~3, row, drow);
    }
};

// The other row writer, with the interface of StashGroup: the whole stash row
// of R in registers, stored once after the walk.  The packet walk over float
// nodes measured faster with it; the walks over quantized nodes and the
// one-query walks, with the groups.
template <int R, bool OUT>
struct StashRegs {
    int g[R];
    float dg[OUT ? R : 1];
    __device__ __forceinline__ StashRegs()
    {
#pragma unroll
        for (int k = 0; k < R; ++k)
            g[k] = 0;
#pragma unroll
        for (int k = 0; k < (OUT ? R : 1); ++k)
            dg[k] = 0.0f;
    }
    __device__ __forceinline__ void add(int c, int idx, float d2, int32_t *, float *)
    {
        append_at<R>(g, c, idx);
        if constexpr (OUT)
            append_at<R>(dg, c, d2);
    }
    __device__ __forceinline__ void finish(int, int, int32_t *row, float *drow) const
    {
#pragma unroll
        for (int k = 0; k < R / 4; ++k)
            reinterpret_cast<int4 *>(row)[k] = make_int4(g[4 * k], g[4 * k + 1], g[4 * k + 2], g[4 * k + 3]);
        if constexpr (OUT) {
#pragma unroll
            for (int k = 0; k < R / 4; ++k)
                reinterpret_cast<float4 *>(drow)[k] = make_float4(dg[4 * k], dg[4 * k + 1], dg[4 * k + 2], dg[4 * k + 3]);
        }
    }
};

// Count pass of a CSR query.  With a stash, each query also keeps its first
// stash_regs(D) matches in registers, in the order found, and stores them in
// the stash row of its input position (one aligned 64-byte segment per
// thread), so that the copy into the CSR array later streams rows, counts and
// offsets in input order and sorts each row there; rows that fit need no
// second walk.  With OUT (the callback-with-output form), each match's
// squared distance, as the walk computed it, travels beside its index in a
// parallel register row, stash row and overflow pool.
template <int D, class P, bool STASH, int SCHED, bool OUT = false>
__global__ void k_spatial_count(const Node<D> *__restrict__ nodes, const QNode<D> *__restrict__ qnodes,
                                const Node4<D> *__restrict__ wnodes,
                                const float *__restrict__ leaves, int kind, const TreeHeader *__restrict__ hdr,
                                const float *__restrict__ queries, int64_t m, float r2,
                                const uint32_t *__restrict__ perm, int32_t *__restrict__ counts,
                                int32_t *__restrict__ ordered_counts, int32_t *__restrict__ stash,
                                float *__restrict__ stash_d2, OverflowPool ovf, int stack_cap)
{
    extern __shared__ int s_stack[];
    const int64_t t = xcd_block() * blockDim.x + threadIdx.x;
    if (SCHED != 1 && t >= m)
        return;
    int64_t qi = t < m ? (perm ? (int64_t)perm[t] : t) : m;
    const bool active = qi < m;
    if (SCHED != 1 && !active)
        return;
    P pred;
    if (active)
        pred.load(queries, qi, r2);
    else
        pred.dead();
    int spill[kSpill];
    ShortStack<int> st(s_stack + threadIdx.x, blockDim.x, stack_cap, spill);
    int *wstack = s_stack + wave_id() * kWaveStack;
    constexpr int R = stash_regs(D);
    int c = 0;
    StashGroup<OUT> grp;
    int32_t *row = STASH ? stash + qi * R : nullptr;
    float *drow = OUT ? stash_d2 + qi * R : nullptr;
    int32_t ov = -1;
    auto f = [&](int idx, float d2) {
        if (STASH) {
            if (c < R)
                grp.add(c, idx, d2, row, drow);
            else
                overflow_add<R, OUT>(ovf, qi, c, idx, d2, ov);
        }
        ++c;
    };
    if (SCHED == 1)
        traverse_spatial_wave<D>(nodes, hdr->root, node_count(hdr), pred, wstack, f);
    else if (SCHED == 2)
        traverse_spatial_rope<D>(nodes, hdr->root, node_count(hdr), hdr->start + hdr->n - 1, pred, f);
    else if (SCHED == 3)
        traverse_spatial_q<D>(qnodes, *hdr, node_count(hdr), leaves, kind, pred, st, f);
    else if (SCHED == 4)
        traverse_spatial4<D>(wnodes, hdr->root, node_count(hdr), pred, st, f);
    else
        traverse_spatial<D>(nodes, hdr->root, node_count(hdr), pred, st, f);
    if (!active)
        return;
    if (STASH)
        grp.finish(c, R, row, drow);
    counts[qi] = c;
    if (ordered_counts)
        ordered_counts[t] = c;
}

// Packet form of the CSR count walk (sphere queries, binary nodes, float or
// quantized): thread t answers the NQ queries at sorted positions
// NQ*t .. NQ*t + NQ - 1 in one walk, each with its own register stash row.
template <int D, int NQ, bool OUT = false, bool Q = false>
__global__ __attribute__((amdgpu_waves_per_eu(NQ == 2 && D <= 3 && !OUT ? 6 : 1))) void k_spatial_count_packet(
    const Node<D> *__restrict__ nodes, const QNode<D> *__restrict__ qnodes, const float *__restrict__ leaves,
    int kind, const TreeHeader *__restrict__ hdr, const float *__restrict__ queries,
    int64_t m, float r2, const uint32_t *__restrict__ perm, int32_t *__restrict__ counts,
    int32_t *__restrict__ ordered_counts, int32_t *__restrict__ stash, float *__restrict__ stash_d2,
    OverflowPool ovf, int stack_cap)
{
    extern __shared__ int s_stack[];
    constexpr int R = stash_regs(D);
    const int64_t t = xcd_block() * blockDim.x + threadIdx.x;
    if (t * NQ >= m)
        return;
    Sphere<D> pred[NQ];
    int64_t qi[NQ];
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
        const int64_t p = t * NQ + j;
        qi[j] = p < m ? (perm ? (int64_t)perm[p] : p) : m;
        if (qi[j] < m)
            pred[j].load(queries, qi[j], r2);
        else
            pred[j].dead();
    }
    int spill[kSpill];
    ShortStack<int> st(s_stack + threadIdx.x, blockDim.x, stack_cap, spill);
    int c[NQ];
    using Row = typename std::conditional<Q, StashGroup<OUT>, StashRegs<R, OUT>>::type;
    Row grp[NQ];
    int32_t *row[NQ];
    float *drow[NQ];
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
        c[j] = 0;
        row[j] = stash + qi[j] * R;
        drow[j] = OUT ? stash_d2 + qi[j] * R : nullptr;
    }
    int32_t ov[NQ];
#pragma unroll
    for (int j = 0; j < NQ; ++j)
        ov[j] = -1;
    auto f = [&](int j, int idx, float d2) {
#pragma unroll
        for (int jj = 0; jj < NQ; ++jj)
            if (jj == j) {
                if (c[jj] < R)
                    grp[jj].add(c[jj], idx, d2, row[jj], drow[jj]);
                else
                    overflow_add<R, OUT>(ovf, qi[jj], c[jj], idx, d2, ov[jj]);
                ++c[jj];
            }
    };
    if (Q)
        traverse_spatial_packet_q<D, NQ>(qnodes, *hdr, node_count(hdr), leaves, kind, pred, st, f);
    else
        traverse_spatial_packet<D, NQ>(nodes, hdr->root, node_count(hdr), pred, st, f);
#pragma unroll
    for (int j = 0; j < NQ; ++j)
        if (qi[j] < m) {
            grp[j].finish(c[j], R, row[j], drow[j]);
            counts[qi[j]] = c[j];
            if (ordered_counts)
                ordered_counts[t * NQ + j] = c[j];
        }
}

// An index and its float value (>= 0: a squared distance or a ray's entry
// parameter) as one word.  MODE 1 orders the word like the index, so rows
// sort by index with the value travelling along; MODE 2 orders it by (value,
// index): the bits of a float >= 0 order like the float.
template <int MODE>
__device__ __forceinline__ uint64_t pack_match(int idx, float v)
{
    return MODE == 2 ? (((uint64_t)__float_as_uint(v) << 32) | (uint32_t)idx)
                     : (((uint64_t)(uint32_t)idx << 32) | __float_as_uint(v));
}
template <int MODE>
__device__ __forceinline__ int match_index(uint64_t w)
{
    return (int)(uint32_t)(MODE == 2 ? w : w >> 32);
}
template <int MODE>
__device__ __forceinline__ float match_value(uint64_t w)
{
    return __uint_as_float((uint32_t)(MODE == 2 ? w >> 32 : w));
}

// Rows of at most R matches: sort the stash row in registers (a bitonic
// network, empty slots padded to sort last) and copy it to the CSR slot.
// Thread i handles query i, so consecutive lanes fill adjacent rows.  With a
// value mode, the stashed values are sorted along with the indices (packed
// with them into one word) and copied to the same slots of dist.  Without
// SORT (index rows only) the row is copied in the order the walk found it.
template <int R, int MODE, bool SORT = true>
__global__ void k_copy_stash(const int32_t *__restrict__ stash, const float *__restrict__ stash_d2, int64_t m,
                             const int32_t *__restrict__ counts, const int64_t *__restrict__ offsets,
                             int32_t *__restrict__ indices, float *__restrict__ dist)
{
    const int64_t qi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (qi >= m)
        return;
    const int c = counts[qi];
    if (c > R)
        return;
    const int4 *row = reinterpret_cast<const int4 *>(stash + qi * R);
    const int64_t o = offsets[qi];
    int v[R];
#pragma unroll
    for (int k = 0; k < R / 4; ++k) {
        const int4 x = row[k];
        v[4 * k] = x.x;
        v[4 * k + 1] = x.y;
        v[4 * k + 2] = x.z;
        v[4 * k + 3] = x.w;
    }
    if constexpr (MODE != 0) {
        const float4 *drow = reinterpret_cast<const float4 *>(stash_d2 + qi * R);
        uint64_t w[R];
#pragma unroll
        for (int k = 0; k < R / 4; ++k) {
            const float4 x = drow[k];
            w[4 * k] = pack_match<MODE>(v[4 * k], x.x);
            w[4 * k + 1] = pack_match<MODE>(v[4 * k + 1], x.y);
            w[4 * k + 2] = pack_match<MODE>(v[4 * k + 2], x.z);
            w[4 * k + 3] = pack_match<MODE>(v[4 * k + 3], x.w);
        }
#pragma unroll
        for (int k = 0; k < R; ++k)
            w[k] = k < c ? w[k] : ~0ull;
        sort_network<R>(w);
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (k < c) {
                indices[o + k] = match_index<MODE>(w[k]);
                dist[o + k] = match_value<MODE>(w[k]);
            }
    } else {
        if constexpr (SORT) {
#pragma unroll
            for (int k = 0; k < R; ++k)
                v[k] = k < c ? v[k] : INT32_MAX;
            sort_network<R>(v);
        }
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (k < c)
                indices[o + k] = v[k];
    }
}

// Listed rows (longer than the stash, at most kRowSortBlock) whose overflow
// chunks all fit: one wavefront per row copies the stash row, then the chunks
// in chain order, into the row's CSR slot, in the order found; the rows are
// sorted afterwards like walked ones.
__global__ __launch_bounds__(256) void k_copy_overflow(const int32_t *__restrict__ stash,
                                                       const float *__restrict__ stash_d2, int R, OverflowPool ovf,
                                                       const int32_t *__restrict__ counts,
                                                       const int64_t *__restrict__ offsets,
                                                       const int32_t *__restrict__ list, int64_t nb,
                                                       int32_t *__restrict__ indices, float *__restrict__ dist)
{
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t b = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id(); b < nb; b += waves) {
        const int64_t row = list[b];
        const int c = counts[row];
        if (c <= R || c > kRowSortBlock)
            continue;
        int32_t cur = ovf.head[row];
        if (cur < 0)
            continue;
        const int64_t o = offsets[row];
        if (lane < R) {
            indices[o + lane] = stash[row * R + lane];
            if (dist)
                dist[o + lane] = stash_d2[row * R + lane];
        }
        for (int done = R; done < c; done += kChunk - 1) {
            const int n = c - done < kChunk - 1 ? c - done : kChunk - 1;
            if (lane < n) {
                indices[o + done + lane] = ovf.pool[cur + lane];
                if (dist)
                    dist[o + done + lane] = ovf.dpool[cur + lane];
            }
            if (done + n < c)
                cur = ovf.pool[cur + kChunk - 1];
        }
    }
}

// Second walk for listed rows (longer than the stash) that were not kept in
// overflow chunks: matches written in traversal order, sorted afterwards.
template <int D, class P, int FMT>
__global__ void k_spatial_fill_rows(const Node<D> *__restrict__ nodes, const QNode<D> *__restrict__ qnodes,
                                    const Node4<D> *__restrict__ wnodes,
                                    const float *__restrict__ leaves, int kind, const TreeHeader *__restrict__ hdr,
                                    const float *__restrict__ queries, int64_t m, float r2,
                                    const int32_t *__restrict__ rows, int64_t nrows, const int32_t *__restrict__ head,
                                    const int64_t *__restrict__ offsets, int32_t *__restrict__ indices,
                                    float *__restrict__ dist, int stack_cap)
{
    extern __shared__ int s_stack[];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nrows)
        return;
    const int64_t qi = rows[j];
    if (qi < 0 || qi >= m)
        return;
    if (head && head[qi] >= 0)  // copied from its overflow chunks
        return;
    P pred;
    pred.load(queries, qi, r2);
    int spill[kSpill];
    ShortStack<int> st(s_stack + threadIdx.x, blockDim.x, stack_cap, spill);
    const int64_t o = offsets[qi];
    const int64_t len = offsets[qi + 1] - o;
    int64_t k = 0;
    auto f = [&](int idx, float d2) {
        if (k < len) {
            indices[o + k] = idx;
            if (dist)
                dist[o + k] = d2;
        }
        ++k;
    };
    if (FMT == 1)
        traverse_spatial_q<D>(qnodes, *hdr, node_count(hdr), leaves, kind, pred, st, f);
    else if (FMT == 2)
        traverse_spatial4<D>(wnodes, hdr->root, node_count(hdr), pred, st, f);
    else
        traverse_spatial<D>(nodes, hdr->root, node_count(hdr), pred, st, f);
}

// Listed rows of at most one wavefront (kWave entries): one wavefront per row,
// a bitonic network across the lanes with shuffles, padding sorting last.
// With a value mode, each index travels with its value (packed into one word).
template <int MODE>
__global__ __launch_bounds__(256) void k_sort_rows_wave(const int64_t *__restrict__ offsets,
                                                        int32_t *__restrict__ indices, float *__restrict__ dist,
                                                        const int32_t *__restrict__ list, int64_t nb)
{
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t b = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id(); b < nb; b += waves) {
        const int64_t row = list[b];
        const int64_t o = offsets[row];
        const int64_t len = offsets[row + 1] - o;
        if (len > kWave)
            continue;
        uint64_t v = MODE ? ~0ull : (0xffffffffull << 32);
        if (lane < len)
            v = MODE ? pack_match<MODE>(indices[o + lane], dist[o + lane])
                     : ((uint64_t)(uint32_t)indices[o + lane] << 32);
#pragma unroll
        for (int k = 2; k <= kWave; k <<= 1)
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), j, kWave);
                const uint32_t lo = MODE ? __shfl_xor((uint32_t)v, j, kWave) : 0u;
                const uint64_t other = ((uint64_t)hi << 32) | lo;
                const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
                v = keep_min ? (v < other ? v : other) : (v < other ? other : v);
            }
        if (lane < len) {
            if (MODE) {
                indices[o + lane] = match_index<MODE>(v);
                dist[o + lane] = match_value<MODE>(v);
            } else {
                indices[o + lane] = (int32_t)(v >> 32);
            }
        }
    }
}

// One workgroup per listed row of kWave < len <= kRowSortBlock entries:
// bitonic sort in LDS (with a value mode the values move with their indices;
// mode 2 sorts by (value, index)).
template <int MODE>
__global__ __launch_bounds__(256) void k_sort_rows(const int64_t *__restrict__ offsets, int32_t *__restrict__ indices,
                                                   float *__restrict__ dist, const int32_t *__restrict__ list,
                                                   int64_t nb)
{
    constexpr bool OUT = MODE != 0;
    __shared__ int32_t s[kRowSortBlock];
    __shared__ float sd[OUT ? kRowSortBlock : 1];
    for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const int64_t row = list[b];
        const int64_t o = offsets[row];
        const int64_t len64 = offsets[row + 1] - o;
        if (len64 <= kWave || len64 > kRowSortBlock)
            continue;
        const int len = (int)len64;
        int p2 = 1;
        while (p2 < len)
            p2 <<= 1;
        for (int i = threadIdx.x; i < p2; i += blockDim.x) {
            s[i] = i < len ? indices[o + i] : INT32_MAX;
            if (OUT)
                sd[i] = i < len ? dist[o + i] : INFINITY;
        }
        __syncthreads();
        for (int kk = 2; kk <= p2; kk <<= 1) {
            for (int j = kk >> 1; j > 0; j >>= 1) {
                for (int i = threadIdx.x; i < p2; i += blockDim.x) {
                    const int ixj = i ^ j;
                    if (ixj > i) {
                        const int a = s[i], c = s[ixj];
                        const bool up = (i & kk) == 0;
                        bool greater = a > c;
                        if (MODE == 2) {
                            const float va = sd[i], vc = sd[ixj];
                            greater = va > vc || (va == vc && a > c);
                        }
                        if (greater == up) {
                            s[i] = c;
                            s[ixj] = a;
                            if (OUT) {
                                const float t = sd[i];
                                sd[i] = sd[ixj];
                                sd[ixj] = t;
                            }
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int i = threadIdx.x; i < len; i += blockDim.x) {
            indices[o + i] = s[i];
            if (OUT)
                dist[o + i] = sd[i];
        }
        __syncthreads();
    }
}

// Rows longer than a workgroup can sort: gather as (row rank, index) keys,
// radix sort, scatter back.
__global__ void k_huge_lengths(const int64_t *__restrict__ offsets, const int32_t *__restrict__ list, int64_t h,
                               int32_t *__restrict__ lens)
{
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < h; b += (int64_t)gridDim.x * blockDim.x)
        lens[b] = (int32_t)(offsets[list[b] + 1] - offsets[list[b]]);
}

__global__ void k_huge_gather(const int64_t *__restrict__ offsets, const int32_t *__restrict__ indices,
                              const float *__restrict__ dist, const int32_t *__restrict__ list, int64_t h,
                              const int64_t *__restrict__ starts, int ib, uint64_t *__restrict__ keys,
                              uint32_t *__restrict__ vals)
{
    for (int64_t b = blockIdx.x; b < h; b += gridDim.x) {
        const int64_t o = offsets[list[b]], len = offsets[list[b] + 1] - o, st = starts[b];
        for (int64_t j = threadIdx.x; j < len; j += blockDim.x) {
            keys[st + j] = ((uint64_t)b << ib) | (uint32_t)indices[o + j];
            vals[st + j] = dist ? __float_as_uint(dist[o + j]) : 0u;
        }
    }
}

__global__ void k_huge_scatter(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals, int64_t total,
                               int ib, int64_t h, const int64_t *__restrict__ offsets,
                               const int32_t *__restrict__ list, const int64_t *__restrict__ starts,
                               int32_t *__restrict__ indices, float *__restrict__ dist)
{
    const uint64_t lowmask = (1ull << ib) - 1ull;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = keys[p];
        const int64_t b = (int64_t)(key >> ib);
        if (b < h) {
            const int64_t at = offsets[list[b]] + (p - starts[b]);
            indices[at] = (int32_t)(key & lowmask);
            if (dist)
                dist[at] = __uint_as_float(vals[p]);
        }
    }
}

// Mode 2 for huge rows: after the sort by (row rank, index), re-key every
// entry as (row rank, value bits) with its index as payload; a stable sort by
// that key then orders each row by (value, index).
__global__ void k_huge_by_value(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals, int64_t total,
                                int ib, uint64_t *__restrict__ keys2, uint32_t *__restrict__ vals2)
{
    const uint64_t lowmask = (1ull << ib) - 1ull;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = keys[p];
        keys2[p] = ((key >> ib) << 32) | vals[p];
        vals2[p] = (uint32_t)(key & lowmask);
    }
}

__global__ void k_huge_scatter_by_value(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                                        int64_t total, int64_t h, const int64_t *__restrict__ offsets,
                                        const int32_t *__restrict__ list, const int64_t *__restrict__ starts,
                                        int32_t *__restrict__ indices, float *__restrict__ dist)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = keys[p];
        const int64_t b = (int64_t)(key >> 32);
        if (b < h) {
            const int64_t at = offsets[list[b]] + (p - starts[b]);
            indices[at] = (int32_t)vals[p];
            dist[at] = __uint_as_float((uint32_t)key);
        }
    }
}

template <int D, bool SUMDIST, int SCHED>
__global__ void k_spatial_reduce(const Node<D> *__restrict__ nodes, const QNode<D> *__restrict__ qnodes,
                                 const Node4<D> *__restrict__ wnodes,
                                 const float *__restrict__ leaves, int kind, const TreeHeader *__restrict__ hdr,
                                 const float *__restrict__ queries, int64_t m, float r2, float scale,
                                 const uint32_t *__restrict__ perm, int32_t *__restrict__ counts,
                                 int64_t *__restrict__ sums, int stack_cap)
{
    extern __shared__ int s_stack[];
    const int64_t t = xcd_block() * blockDim.x + threadIdx.x;
    if (SCHED != 1 && t >= m)
        return;
    const int64_t qi = t < m ? (perm ? (int64_t)perm[t] : t) : m;
    const bool active = qi < m;
    if (SCHED != 1 && !active)
        return;
    Sphere<D> pred;
    if (active)
        pred.load(queries, qi, r2);
    else
        pred.dead();
    int spill[kSpill];
    ShortStack<int> st(s_stack + threadIdx.x, blockDim.x, stack_cap, spill);
    int *wstack = s_stack + wave_id() * kWaveStack;
    int c = 0;
    long long s = 0;
    auto f = [&](int, float d2) {
        ++c;
        if (SUMDIST)
            s += fixed_term(d2, scale);
    };
    if (SCHED == 1)
        traverse_spatial_wave<D>(nodes, hdr->root, node_count(hdr), pred, wstack, f);
    else if (SCHED == 2)
        traverse_spatial_rope<D>(nodes, hdr->root, node_count(hdr), hdr->start + hdr->n - 1, pred, f);
    else if (SCHED == 3)
        traverse_spatial_q<D>(qnodes, *hdr, node_count(hdr), leaves, kind, pred, st, f);
    else if (SCHED == 4)
        traverse_spatial4<D>(wnodes, hdr->root, node_count(hdr), pred, st, f);
    else
        traverse_spatial<D>(nodes, hdr->root, node_count(hdr), pred, st, f);
    if (!active)
        return;
    counts[qi] = c;
    if (SUMDIST)
        sums[qi] = s;
}

// Packet form of the fused reduction: thread t answers the NQ queries at
// sorted positions NQ*t .. NQ*t + NQ - 1 in one walk over binary nodes
// (float or quantized).
template <int D, bool SUMDIST, int NQ, bool Q = false>
__global__ void k_spatial_reduce_packet(const Node<D> *__restrict__ nodes, const QNode<D> *__restrict__ qnodes,
                                        const float *__restrict__ leaves, int kind,
                                        const TreeHeader *__restrict__ hdr,
                                        const float *__restrict__ queries, int64_t m, float r2, float scale,
                                        const uint32_t *__restrict__ perm, int32_t *__restrict__ counts,
                                        int64_t *__restrict__ sums, int stack_cap)
{
    extern __shared__ int s_stack[];
    const int64_t t = xcd_block() * blockDim.x + threadIdx.x;
    if (t * NQ >= m)
        return;
    Sphere<D> pred[NQ];
    int64_t qi[NQ];
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
        const int64_t p = t * NQ + j;
        qi[j] = p < m ? (perm ? (int64_t)perm[p] : p) : m;
        if (qi[j] < m)
            pred[j].load(queries, qi[j], r2);
        else
            pred[j].dead();
    }
    int spill[kSpill];
    ShortStack<int> st(s_stack + threadIdx.x, blockDim.x, stack_cap, spill);
    int c[NQ];
    long long s[NQ];
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
        c[j] = 0;
        s[j] = 0;
    }
    auto f = [&](int j, int, float d2) {
#pragma unroll
        for (int jj = 0; jj < NQ; ++jj)
            if (jj == j) {
                ++c[jj];
                if (SUMDIST)
                    s[jj] += fixed_term(d2, scale);
            }
    };
    if (Q)
        traverse_spatial_packet_q<D, NQ>(qnodes, *hdr, node_count(hdr), leaves, kind, pred, st, f);
    else
        traverse_spatial_packet<D, NQ>(nodes, hdr->root, node_count(hdr), pred, st, f);
#pragma unroll
    for (int j = 0; j < NQ; ++j)
        if (qi[j] < m) {
            counts[qi[j]] = c[j];
            if (SUMDIST)
                sums[qi[j]] = s[j];
        }
}

// Waves per SIMD the kNN kernel asks the register allocator for.  The 3D
// k = 16 thread walk on float nodes needed 65 registers, one above the
// 8-wave limit: held to 64 (63, no spill) it runs 8 waves per SIMD, and kNN-16
// at 10^7 points took 7.7 ms instead of 8.4 (shell 6.8 instead of 7.4).  The
// 6D k = 8 walk on quantized nodes, held from 88 to 80 registers (6 waves
// instead of 5), spilled and ran slower (7.0 against 6.8 ms), so the other
// shapes are left to the compiler.
template <int D, int K, bool WAVE, int FMT>
constexpr int knn_waves()
{
    return (!WAVE && D <= 3 && K == 16 && FMT == 0) ? 8 : 1;
}

template <int D, int K, bool WAVE, int FMT>
__global__ __attribute__((amdgpu_waves_per_eu(knn_waves<D, K, WAVE, FMT>()))) void k_knn(const Node<D> *__restrict__ nodes, const QNode<D> *__restrict__ qnodes,
                      const Node4<D> *__restrict__ wnodes, const uint64_t *__restrict__ codes, int n_nodes,
                      const float *__restrict__ leaves, int kind,
                      const TreeHeader *__restrict__ hdr, const float *__restrict__ queries, int64_t m, int k_out,
                      const uint32_t *__restrict__ perm, float *__restrict__ out_d2, int32_t *__restrict__ out_idx,
                      int stack_cap, int seed)
{
    extern __shared__ int s_stack[];
    const int64_t t = xcd_block() * blockDim.x + threadIdx.x;
    if (!WAVE && t >= m)
        return;
    const int64_t qi = t < m ? (perm ? (int64_t)perm[t] : t) : m;
    const bool active = qi < m;
    if (!WAVE && !active)
        return;
    float q[D];
#pragma unroll
    for (int d = 0; d < D; ++d)
        q[d] = active ? queries[qi * D + d] : 0.0f;
    TopK<K> best;
    if (WAVE) {
        KnnEntry *wstack = reinterpret_cast<KnnEntry *>(s_stack) + wave_id() * kWaveStack;
        knn_search_wave<D, K>(nodes, n_nodes, leaves, kind, *hdr, q, active, best, wstack, seed);
    } else {
        KnnEntry spill[kSpill];
        ShortStack<KnnEntry> st(reinterpret_cast<KnnEntry *>(s_stack) + threadIdx.x, blockDim.x, stack_cap, spill);
        if (FMT == 1)
            knn_search_q<D, K>(qnodes, n_nodes, leaves, kind, *hdr, q, best, st, seed, SeedKeys{codes, 0, 63 / D});
        else if (FMT == 2)
            knn_search4<D, K>(nodes, wnodes, n_nodes, leaves, kind, *hdr, q, best, st, seed, SeedKeys{codes, 0, 63 / D});
        else
            knn_search<D, K>(nodes, n_nodes, leaves, kind, *hdr, q, best, st, seed, SeedKeys{codes, 0, 63 / D});
    }
    if (active)
        best.store(k_out, out_d2 + qi * k_out, out_idx + qi * k_out, 0);
}

// Callback with output (Section 2.1, query call (2)): the squared distance of
// every match of a radius search's CSR result, evaluated as in the walk (the
// box distance with lo = hi for points) from the build input.  One thread per
// query row, so the row's outputs are contiguous.
template <int D>
__global__ void k_match_distances(const float *__restrict__ values, int64_t n, int kind,
                                  const float *__restrict__ queries, int64_t m, const int64_t *__restrict__ offsets,
                                  const int32_t *__restrict__ indices, float *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        float q[D];
#pragma unroll
        for (int d = 0; d < D; ++d)
            q[d] = queries[i * D + d];
        const int64_t end = offsets[i + 1];
        for (int64_t p = offsets[i]; p < end; ++p) {
            const int64_t j = indices[p];
            if (j < 0 || j >= n) {
                out[p] = NAN;
                continue;
            }
            const float *v = values + j * (kind == ARBORX_BOXES ? 2 * D : D);
            float lo[D], hi[D];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                lo[d] = v[d];
                hi[d] = kind == ARBORX_BOXES ? v[D + d] : v[d];
            }
            out[p] = box_d2<D>(q, lo, hi);
        }
    }
}

// Early-terminating count (Section 2.2): a query's walk over binary nodes
// (float, or with Q the quantized ones) ends once it has counted n_max
// matches; the result is min(count, n_max).
template <int D, bool Q>
__global__ void k_count_up_to(const Node<D> *__restrict__ nodes, const QNode<D> *__restrict__ qnodes,
                              const float *__restrict__ leaves, int kind, const TreeHeader *__restrict__ hdr,
                              const float *__restrict__ queries, int64_t m, float r2, int n_max,
                              const uint32_t *__restrict__ perm, int32_t *__restrict__ counts, int stack_cap)
{
    extern __shared__ int s_stack[];
    const int64_t t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= m)
        return;
    const int64_t qi = perm ? (int64_t)perm[t] : t;
    if (qi < 0 || qi >= m)
        return;
    Sphere<D> pred;
    pred.load(queries, qi, r2);
    int spill[kSpill];
    ShortStack<int> st(s_stack + threadIdx.x, blockDim.x, stack_cap, spill);
    int c = 0;
    auto f = [&](int, float) { ++c; };
    auto stop = [&]() { return c >= n_max; };
    if (n_max > 0) {
        if constexpr (Q)
            traverse_spatial_q<D>(qnodes, *hdr, node_count(hdr), leaves, kind, pred, st, f, stop);
        else
            traverse_spatial<D>(nodes, hdr->root, node_count(hdr), pred, st, f, stop);
    }
    counts[qi] = c < n_max ? c : n_max;
}

// Walk statistics: node fetches per query of the one-query-per-thread radius
// walk (op 0) or kNN walk (op 1, after its seeding), for the touched-bytes
// figure (fetches x node bytes).
template <int D, int K>
__global__ void k_debug_visits(const Node<D> *__restrict__ nodes, const uint64_t *__restrict__ codes, int n_nodes,
                               const float *__restrict__ leaves, int kind, const TreeHeader *__restrict__ hdr,
                               const float *__restrict__ queries, int64_t m, float r2, int op,
                               int32_t *__restrict__ visits, int stack_cap)
{
    extern __shared__ int s_stack[];
    const int64_t qi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (qi >= m)
        return;
    int v = 0;
    if (op == 0) {
        Sphere<D> pred;
        pred.load(queries, qi, r2);
        int spill[kSpill];
        ShortStack<int> st(s_stack + threadIdx.x, blockDim.x, stack_cap, spill);
        auto f = [](int, float) {};
        auto count = [&]() {
            ++v;
            return false;
        };
        traverse_spatial<D>(nodes, hdr->root, n_nodes, pred, st, f, count);
    } else {
        float q[D];
#pragma unroll
        for (int d = 0; d < D; ++d)
            q[d] = queries[qi * D + d];
        TopK<K> best;
        KnnEntry spill[kSpill];
        ShortStack<KnnEntry> st(reinterpret_cast<KnnEntry *>(s_stack) + threadIdx.x, blockDim.x, stack_cap, spill);
        knn_search<D, K>(nodes, n_nodes, leaves, kind, *hdr, q, best, st, 0, SeedKeys{codes, 0, 63 / D}, &v);
    }
    visits[qi] = v;
}

__global__ void k_knn_empty(int64_t total, float *d2, int32_t *idx)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        d2[i] = INFINITY;
        idx[i] = -1;
    }
}

// Morton codes of query centres on a coarse grid (order_bits bits in all:
// 24, or 16 for a two-pass sort), normalised by the tree's bounds.  The order
// only affects speed: queries in one cell of the grid are treated alike.
inline int order_bits(int order) { return order == 2 ? 16 : 24; }

// BOXQ: queries are [m][2][D] rows; the code is of the box centre, or (RAY)
// of the ray's origin row.
template <int D, bool BOXQ, bool RAY = false>
__global__ void k_query_codes(const float *__restrict__ q, int64_t m, const TreeHeader *__restrict__ hdr,
                              uint32_t *__restrict__ codes, uint32_t *__restrict__ ids, int bits)
{
    float lo[D], inv[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = hdr->lo[d];
        const float ext = hdr->hi[d] - hdr->lo[d];
        inv[d] = ext > 0.0f ? 1.0f / ext : 0.0f;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t c[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const float x = RAY ? q[i * 2 * D + d]
                                : (BOXQ ? q[i * 2 * D + d] + 0.5f * (q[i * 2 * D + D + d] - q[i * 2 * D + d])
                                        : q[i * D + d]);
            c[d] = quantise(x, lo[d], inv[d], bits);
        }
        codes[i] = (uint32_t)interleave<D>(c, bits);
        ids[i] = (uint32_t)i;
    }
}

template <typename T>
arborx_status fill_async(T *p, int64_t n, T v, hipStream_t s)
{
    if (n <= 0)
        return ARBORX_OK;
    fill_kernel<T><<<grid_for(n, 256, 65536), 256, 0, s>>>(p, n, v);
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

struct Launch {
    unsigned grid;
    int block;
    int cap;
    size_t lds;
};

Launch traversal_launch(int64_t m, size_t entry_bytes, int op, int dim, bool wave = false)
{
    Launch L;
    launch_shape(op, dim, L.block, L.cap);
    L.grid = (unsigned)((m + L.block - 1) / L.block);
    while (L.cap > 1 && (size_t)L.cap * L.block * entry_bytes > 65536)
        L.cap >>= 1;
    L.lds = wave ? (size_t)(L.block / kWave) * kWaveStack * entry_bytes : (size_t)L.cap * L.block * entry_bytes;
    return L;
}

// Schedule 0 over quantized nodes runs as internal schedule 3, over four-wide
// nodes as internal schedule 4.
int effective_schedule(int op, const TreeDev &t)
{
    const Tuning &tu = tuning(op);
    const int fmt = tree_format(op, t);
    return tu.schedule != 0 ? tu.schedule : (fmt == 1 ? 3 : (fmt == 2 ? 4 : 0));
}

template <int D>
arborx_status count_impl(const TreeDev &t, Pred pred, const float *q, int64_t m, float r2, const uint32_t *perm,
                         int32_t *counts, int32_t *ordered_counts, int32_t *stash, float *stash_d2,
                         const OverflowPool &ovf, hipStream_t s)
{
    const int sched = effective_schedule(OP_SPATIAL, t);
    const int nq = tuning(OP_SPATIAL).packet ? tuning(OP_SPATIAL).packet : (D <= 3 ? 2 : 1);
    const bool out = stash_d2 != nullptr;  // the callback-with-output form (sphere queries only)
    if ((sched == 0 || sched == 3) && nq > 1 && pred == Pred::Sphere) {  // NQ queries per thread, binary nodes
        const Launch L = traversal_launch((m + nq - 1) / nq, sizeof(int), OP_SPATIAL, D);
        const Node<D> *nodes = static_cast<const Node<D> *>(t.nodes);
        const QNode<D> *qnodes = static_cast<const QNode<D> *>(t.qnodes);
        ProfScope ps("spatial_count", s);
#define AX_CP(N, O, QF)                                                                                           \
    k_spatial_count_packet<D, N, O, QF><<<L.grid, L.block, L.lds, s>>>(nodes, qnodes, t.leaves, t.kind, t.hdr, q, m, \
                                                                       r2, perm, counts,                            \
                                                                       perm ? ordered_counts : nullptr, stash,      \
                                                                       stash_d2, ovf, L.cap)
#define AX_CPQ(N, O)         \
    do {                     \
        if (sched == 3)      \
            AX_CP(N, O, true); \
        else                 \
            AX_CP(N, O, false); \
    } while (0)
        if (nq == 2) {
            if (out)
                AX_CPQ(2, true);
            else
                AX_CPQ(2, false);
        } else {
            if (out)
                AX_CPQ(4, true);
            else
                AX_CPQ(4, false);
        }
#undef AX_CPQ
#undef AX_CP
        AX_HIP(hipGetLastError());
        return ARBORX_OK;
    }
    const Launch L = traversal_launch(m, sizeof(int), OP_SPATIAL, D, sched == 1);
    const Node<D> *nodes = static_cast<const Node<D> *>(t.nodes);
    const QNode<D> *qnodes = static_cast<const QNode<D> *>(t.qnodes);
    const Node4<D> *wnodes = static_cast<const Node4<D> *>(t.wnodes);
    ProfScope ps("spatial_count", s);
#define AX_COUNT_O(P, S, O)                                                                                           \
    k_spatial_count<D, P, true, S, O><<<L.grid, L.block, L.lds, s>>>(nodes, qnodes, wnodes, t.leaves, t.kind, t.hdr, q, \
                                                                     m, r2, perm, counts,                             \
                                                                     perm ? ordered_counts : nullptr, stash, stash_d2, \
                                                                     ovf, L.cap)
#define AX_COUNT(P, S) AX_COUNT_O(P, S, false)
    if (pred == Pred::Sphere && out) {
        if (sched == 1)
            AX_COUNT_O(Sphere<D>, 1, true);
        else if (sched == 2)
            AX_COUNT_O(Sphere<D>, 2, true);
        else if (sched == 3)
            AX_COUNT_O(Sphere<D>, 3, true);
        else if (sched == 4)
            AX_COUNT_O(Sphere<D>, 4, true);
        else
            AX_COUNT_O(Sphere<D>, 0, true);
    } else if (pred == Pred::Ray && out) {  // the value slot carries the entry parameter
        if (sched == 1)
            AX_COUNT_O(RayPred<D>, 1, true);
        else if (sched == 2)
            AX_COUNT_O(RayPred<D>, 2, true);
        else if (sched == 3)
            AX_COUNT_O(RayPred<D>, 3, true);
        else if (sched == 4)
            AX_COUNT_O(RayPred<D>, 4, true);
        else
            AX_COUNT_O(RayPred<D>, 0, true);
    } else if (pred == Pred::Ray) {
        if (sched == 1)
            AX_COUNT(RayPred<D>, 1);
        else if (sched == 2)
            AX_COUNT(RayPred<D>, 2);
        else if (sched == 3)
            AX_COUNT(RayPred<D>, 3);
        else if (sched == 4)
            AX_COUNT(RayPred<D>, 4);
        else
            AX_COUNT(RayPred<D>, 0);
    } else if (pred == Pred::Sphere) {
        if (sched == 1)
            AX_COUNT(Sphere<D>, 1);
        else if (sched == 2)
            AX_COUNT(Sphere<D>, 2);
        else if (sched == 3)
            AX_COUNT(Sphere<D>, 3);
        else if (sched == 4)
            AX_COUNT(Sphere<D>, 4);
        else
            AX_COUNT(Sphere<D>, 0);
    } else {
        if (sched == 1)
            AX_COUNT(BoxQuery<D>, 1);
        else if (sched == 2)
            AX_COUNT(BoxQuery<D>, 2);
        else if (sched == 3)
            AX_COUNT(BoxQuery<D>, 3);
        else if (sched == 4)
            AX_COUNT(BoxQuery<D>, 4);
        else
            AX_COUNT(BoxQuery<D>, 0);
    }
#undef AX_COUNT
#undef AX_COUNT_O
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

template <int D>
arborx_status fill_rows_impl(const TreeDev &t, Pred pred, const float *q, int64_t m, float r2, const int32_t *rows,
                             int64_t nrows, const int32_t *head, const int64_t *offsets, int32_t *indices,
                             float *dist, hipStream_t s)
{
    if (nrows <= 0)
        return ARBORX_OK;
    Launch L = traversal_launch(nrows, sizeof(int), OP_SPATIAL, D);
    const Node<D> *nodes = static_cast<const Node<D> *>(t.nodes);
    const QNode<D> *qnodes = static_cast<const QNode<D> *>(t.qnodes);
    const Node4<D> *wnodes = static_cast<const Node4<D> *>(t.wnodes);
    const int fmt = tree_format(OP_SPATIAL, t);
    ProfScope ps("spatial_fill", s);
#define AX_FILL(P, F)                                                                                              \
    k_spatial_fill_rows<D, P, F><<<L.grid, L.block, L.lds, s>>>(nodes, qnodes, wnodes, t.leaves, t.kind, t.hdr, q, m, r2, \
                                                                rows, nrows, head, offsets, indices, dist, L.cap)
    if (pred == Pred::Sphere) {
        if (fmt == 1)
            AX_FILL(Sphere<D>, 1);
        else if (fmt == 2)
            AX_FILL(Sphere<D>, 2);
        else
            AX_FILL(Sphere<D>, 0);
    } else if (pred == Pred::Ray) {
        if (fmt == 1)
            AX_FILL(RayPred<D>, 1);
        else if (fmt == 2)
            AX_FILL(RayPred<D>, 2);
        else
            AX_FILL(RayPred<D>, 0);
    } else {
        if (fmt == 1)
            AX_FILL(BoxQuery<D>, 1);
        else if (fmt == 2)
            AX_FILL(BoxQuery<D>, 2);
        else
            AX_FILL(BoxQuery<D>, 0);
    }
#undef AX_FILL
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

template <int D>
arborx_status reduce_impl(const TreeDev &t, const float *q, int64_t m, float r2, int op, float scale,
                          const uint32_t *perm, int32_t *counts, int64_t *sums, hipStream_t s)
{
    const int sched = effective_schedule(OP_REDUCE, t);
    const int nq = tuning(OP_REDUCE).packet ? tuning(OP_REDUCE).packet : (D <= 3 ? (sched == 3 ? 2 : 4) : 1);
    if ((sched == 0 || sched == 3) && nq > 1) {  // NQ queries per thread over binary nodes
        const Launch L = traversal_launch((m + nq - 1) / nq, sizeof(int), OP_REDUCE, D);
        const Node<D> *nodes = static_cast<const Node<D> *>(t.nodes);
        const QNode<D> *qnodes = static_cast<const QNode<D> *>(t.qnodes);
        ProfScope ps(op == ARBORX_COUNT_SUMDIST ? "reduce_sumdist" : "reduce_count", s);
#define AX_RP(SD, N, QF)                                                                                       \
    k_spatial_reduce_packet<D, SD, N, QF><<<L.grid, L.block, L.lds, s>>>(nodes, qnodes, t.leaves, t.kind, t.hdr, q, \
                                                                         m, r2, scale, perm, counts, sums, L.cap)
#define AX_RPQ(SD, N)          \
    do {                       \
        if (sched == 3)        \
            AX_RP(SD, N, true);  \
        else                   \
            AX_RP(SD, N, false); \
    } while (0)
        if (op == ARBORX_COUNT_SUMDIST) {
            if (nq == 2)
                AX_RPQ(true, 2);
            else
                AX_RPQ(true, 4);
        } else {
            if (nq == 2)
                AX_RPQ(false, 2);
            else
                AX_RPQ(false, 4);
        }
#undef AX_RPQ
#undef AX_RP
        AX_HIP(hipGetLastError());
        return ARBORX_OK;
    }
    const Launch L = traversal_launch(m, sizeof(int), OP_REDUCE, D, sched == 1);
    const Node<D> *nodes = static_cast<const Node<D> *>(t.nodes);
    const QNode<D> *qnodes = static_cast<const QNode<D> *>(t.qnodes);
    const Node4<D> *wnodes = static_cast<const Node4<D> *>(t.wnodes);
    ProfScope ps(op == ARBORX_COUNT_SUMDIST ? "reduce_sumdist" : "reduce_count", s);
#define AX_REDUCE(SD, S)                                                                                      \
    k_spatial_reduce<D, SD, S><<<L.grid, L.block, L.lds, s>>>(nodes, qnodes, wnodes, t.leaves, t.kind, t.hdr, q, m, r2, scale, \
                                                              perm, counts, sums, L.cap)
#define AX_REDUCE_MODE(MD)                 \
    do {                                   \
        if (sched == 1)                    \
            AX_REDUCE(MD, 1);              \
        else if (sched == 2)               \
            AX_REDUCE(MD, 2);              \
        else if (sched == 3)               \
            AX_REDUCE(MD, 3);              \
        else if (sched == 4)               \
            AX_REDUCE(MD, 4);              \
        else                               \
            AX_REDUCE(MD, 0);              \
    } while (0)
    if (op == ARBORX_COUNT_SUMDIST)
        AX_REDUCE_MODE(true);
    else
        AX_REDUCE_MODE(false);
#undef AX_REDUCE_MODE
#undef AX_REDUCE
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

template <int D, int K>
arborx_status knn_launch(const TreeDev &t, const float *q, int64_t m, int k, const uint32_t *perm, float *d2,
                         int32_t *idx, hipStream_t s)
{
    const bool wave = tuning(OP_KNN).schedule == 1;  // kNN has no rope form: schedule 2 walks with the stack
    const int fmt = tree_format(OP_KNN, t);
    const Launch L = traversal_launch(m, sizeof(KnnEntry), OP_KNN, D, wave);
    const Node<D> *nodes = static_cast<const Node<D> *>(t.nodes);
    const QNode<D> *qnodes = static_cast<const QNode<D> *>(t.qnodes);
    const Node4<D> *wnodes = static_cast<const Node4<D> *>(t.wnodes);
    const int seed = tuning(OP_KNN).seed;
    ProfScope ps("knn", s);
#define AX_KNN(W, F)                                                                                              \
    k_knn<D, K, W, F><<<L.grid, L.block, L.lds, s>>>(nodes, qnodes, wnodes, t.codes, tree_nodes(t), t.leaves, t.kind,  \
                                                     t.hdr, q, m, k, perm, d2, idx, L.cap, seed)
    if (wave)
        AX_KNN(true, 0);
    else if (fmt == 1)
        AX_KNN(false, 1);
    else if (fmt == 2)
        AX_KNN(false, 2);
    else
        AX_KNN(false, 0);
#undef AX_KNN
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

template <int D>
arborx_status knn_impl(const TreeDev &t, const float *q, int64_t m, int k, const uint32_t *perm, float *d2,
                       int32_t *idx, hipStream_t s)
{
    if (k <= 1)
        return knn_launch<D, 1>(t, q, m, k, perm, d2, idx, s);
    if (k <= 2)
        return knn_launch<D, 2>(t, q, m, k, perm, d2, idx, s);
    if (k <= 4)
        return knn_launch<D, 4>(t, q, m, k, perm, d2, idx, s);
    if (k <= 8)
        return knn_launch<D, 8>(t, q, m, k, perm, d2, idx, s);
    if (k <= 10)
        return knn_launch<D, 10>(t, q, m, k, perm, d2, idx, s);
    if (k <= 16)
        return knn_launch<D, 16>(t, q, m, k, perm, d2, idx, s);
    if (k <= 32)
        return knn_launch<D, 32>(t, q, m, k, perm, d2, idx, s);
    return knn_launch<D, 64>(t, q, m, k, perm, d2, idx, s);
}

// Query order into caller-given buffers: codes/codes2/ids/ids2 of m entries
// each and a radix workspace of radix_workspace_bytes(m); *perm points into
// ids or ids2.
template <int D>
arborx_status order_into(const TreeDev &t, const float *q, int64_t m, Pred pred, int order, uint32_t *codes,
                         uint32_t *codes2, uint32_t *ids, uint32_t *ids2, void *ws, uint32_t **perm, hipStream_t s)
{
    const int bits = order_bits(order) / D;
    ProfScope ps("order", s);
    if (pred == Pred::Sphere)
        k_query_codes<D, false><<<grid_for(m, 256, 65536), 256, 0, s>>>(q, m, t.hdr, codes, ids, bits);
    else if (pred == Pred::Ray)
        k_query_codes<D, true, true><<<grid_for(m, 256, 65536), 256, 0, s>>>(q, m, t.hdr, codes, ids, bits);
    else
        k_query_codes<D, true><<<grid_for(m, 256, 65536), 256, 0, s>>>(q, m, t.hdr, codes, ids, bits);
    bool alt = false;
    AX_HIP(radix_sort_pairs<uint32_t>(codes, ids, codes2, ids2, m, 0, bits * D, ws, s, &alt));
    *perm = alt ? ids2 : ids;
    return ARBORX_OK;
}

template <int D>
arborx_status order_impl(const TreeDev &t, const float *q, int64_t m, Pred pred, int order, uint32_t **perm,
                         Temps &tmp, hipStream_t s)
{
    uint32_t *codes, *codes2, *ids, *ids2;
    uint8_t *ws;
    arborx_status st;
    if ((st = tmp.get(&codes, m)) != ARBORX_OK || (st = tmp.get(&codes2, m)) != ARBORX_OK ||
        (st = tmp.get(&ids, m)) != ARBORX_OK || (st = tmp.get(&ids2, m)) != ARBORX_OK ||
        (st = tmp.get(&ws, radix_workspace_bytes(m))) != ARBORX_OK)
        return st;
    return order_into<D>(t, q, m, pred, order, codes, codes2, ids, ids2, ws, perm, s);
}

#define AX_DISPATCH_DIM(dim, CALL)                                              \
    switch (dim) {                                                              \
    case 2: { constexpr int D = 2; return CALL; }                               \
    case 3: { constexpr int D = 3; return CALL; }                               \
    case 6: { constexpr int D = 6; return CALL; }                               \
    default: return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in");    \
    }

}  // namespace

arborx_status query_order(const TreeDev &t, const float *queries, int64_t m, Pred pred, int op, uint32_t **perm,
                          Temps &tmp, hipStream_t s)
{
    *perm = nullptr;
    if (!tuning(op).order || t.n == 0 || m <= 1)
        return ARBORX_OK;
    AX_DISPATCH_DIM(t.dim, (order_impl<D>(t, queries, m, pred, tuning(op).order, perm, tmp, s)));
}

arborx_status spatial_count(const TreeDev &t, Pred pred, const float *queries, int64_t m, float radius,
                            const uint32_t *perm, int32_t *counts, int32_t *ordered_counts, int32_t *stash,
                            float *stash_d2, const OverflowPool &ovf, hipStream_t s)
{
    if (m == 0)
        return ARBORX_OK;
    if (t.n == 0)
        return fill_async<int32_t>(counts, m, 0, s);
    arborx_status st = check_nodes(t.qnodes, t.wnodes, t.n, tree_format(OP_SPATIAL, t));
    if (st != ARBORX_OK)
        return st;
    if ((st = fill_async<unsigned long long>(ovf.ctr, (int64_t)kOvfPools * 8, 0ull, s)) != ARBORX_OK)
        return st;
    const float r2 = radius * radius;
    AX_DISPATCH_DIM(t.dim,
                    (count_impl<D>(t, pred, queries, m, r2, perm, counts, ordered_counts, stash, stash_d2, ovf, s)));
}

int64_t overflow_pool_ints(int64_t m, int dim, int factor)
{
    int64_t per = (m * stash_regs(dim) * factor + kOvfPools - 1) / kOvfPools;
    per = (per + kChunk - 1) / kChunk * kChunk;
    const int64_t max_per = (int64_t)INT32_MAX / kOvfPools / kChunk * kChunk;
    per = per < kChunk ? kChunk : (per > max_per ? max_per : per);
    return per * kOvfPools;
}

arborx_status spatial_fill(const TreeDev &t, Pred pred, const float *queries, int64_t m, float radius,
                           const int32_t *counts, const int32_t *stash, const float *stash_d2,
                           const OverflowPool &ovf, const int64_t *offsets, const int32_t *big_list, int64_t nbig,
                           const int32_t *huge_list, int64_t nhuge, int32_t *indices, float *dist, int mode,
                           hipStream_t s, bool sorted)
{
    if (m == 0 || t.n == 0)
        return ARBORX_OK;
    arborx_status st = check_nodes(t.qnodes, t.wnodes, t.n, tree_format(OP_SPATIAL, t));
    if (st != ARBORX_OK)
        return st;
    {
        ProfScope ps("copy_stash", s);
        const unsigned g = grid_for(m, 256, INT32_MAX);
        const int md = dist ? (mode == VALUES_ORDERED ? 2 : 1) : 0;
#define AX_CS(R, M, S) k_copy_stash<R, M, S><<<g, 256, 0, s>>>(stash, stash_d2, m, counts, offsets, indices, dist)
        if (stash_regs(t.dim) == 32) {
            if (md == 2)
                AX_CS(32, 2, true);
            else if (md == 1)
                AX_CS(32, 1, true);
            else if (sorted)
                AX_CS(32, 0, true);
            else
                AX_CS(32, 0, false);
        } else {
            if (md == 2)
                AX_CS(16, 2, true);
            else if (md == 1)
                AX_CS(16, 1, true);
            else if (sorted)
                AX_CS(16, 0, true);
            else
                AX_CS(16, 0, false);
        }
#undef AX_CS
        AX_HIP(hipGetLastError());
    }
    if (nbig > 0) {
        ProfScope ps("copy_overflow", s);
        k_copy_overflow<<<grid_for(nbig, 256 / kWave, 16384), 256, 0, s>>>(stash, stash_d2, stash_regs(t.dim), ovf,
                                                                            counts, offsets, big_list, nbig, indices,
                                                                            dist);
        AX_HIP(hipGetLastError());
    }
    const float r2 = radius * radius;
    switch (t.dim) {
    case 2:
        if ((st = fill_rows_impl<2>(t, pred, queries, m, r2, big_list, nbig, ovf.head, offsets, indices, dist, s)) ==
            ARBORX_OK)
            st = fill_rows_impl<2>(t, pred, queries, m, r2, huge_list, nhuge, nullptr, offsets, indices, dist, s);
        return st;
    case 3:
        if ((st = fill_rows_impl<3>(t, pred, queries, m, r2, big_list, nbig, ovf.head, offsets, indices, dist, s)) ==
            ARBORX_OK)
            st = fill_rows_impl<3>(t, pred, queries, m, r2, huge_list, nhuge, nullptr, offsets, indices, dist, s);
        return st;
    case 6:
        if ((st = fill_rows_impl<6>(t, pred, queries, m, r2, big_list, nbig, ovf.head, offsets, indices, dist, s)) ==
            ARBORX_OK)
            st = fill_rows_impl<6>(t, pred, queries, m, r2, huge_list, nhuge, nullptr, offsets, indices, dist, s);
        return st;
    default:
        return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in");
    }
}

arborx_status sort_big_rows(const int64_t *offsets, int32_t *indices, float *dist, int mode, const int32_t *big_list,
                            int64_t nbig, hipStream_t s)
{
    if (nbig <= 0)
        return ARBORX_OK;
    ProfScope ps("sort_rows", s);
    const unsigned gw = grid_for(nbig, 256 / kWave, 16384), gb = (unsigned)(nbig < 8192 ? nbig : 8192);
    if (dist && mode == VALUES_ORDERED) {
        k_sort_rows_wave<2><<<gw, 256, 0, s>>>(offsets, indices, dist, big_list, nbig);
        k_sort_rows<2><<<gb, 256, 0, s>>>(offsets, indices, dist, big_list, nbig);
    } else if (dist) {
        k_sort_rows_wave<1><<<gw, 256, 0, s>>>(offsets, indices, dist, big_list, nbig);
        k_sort_rows<1><<<gb, 256, 0, s>>>(offsets, indices, dist, big_list, nbig);
    } else {
        k_sort_rows_wave<0><<<gw, 256, 0, s>>>(offsets, indices, dist, big_list, nbig);
        k_sort_rows<0><<<gb, 256, 0, s>>>(offsets, indices, dist, big_list, nbig);
    }
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

arborx_status sort_huge_rows(int64_t n_values, const int64_t *offsets, int32_t *indices, float *dist, int mode,
                             const int32_t *huge_list, int64_t h, Temps &tmp, hipStream_t s)
{
    if (h <= 0)
        return ARBORX_OK;
    int32_t *lens;
    int64_t *starts, *tot_dev;
    uint8_t *sws;
    arborx_status st;
    if ((st = tmp.get(&lens, h)) != ARBORX_OK || (st = tmp.get(&starts, h + 1)) != ARBORX_OK ||
        (st = tmp.get(&tot_dev, 1)) != ARBORX_OK || (st = tmp.get(&sws, scan_workspace_bytes(h))) != ARBORX_OK)
        return st;
    k_huge_lengths<<<grid_for(h, 256, 4096), 256, 0, s>>>(offsets, huge_list, h, lens);
    AX_HIP(csr_offsets(lens, h, starts, tot_dev, sws, s));
    int64_t total = 0;
    AX_HIP(hipMemcpyAsync(&total, tot_dev, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    AX_HIP(hipStreamSynchronize(s));
    int ib = 1, hb = 1;
    while ((1ll << ib) < n_values)
        ++ib;
    while ((1ll << hb) < h)
        ++hb;
    if (ib + hb > 64 || (mode == VALUES_ORDERED && hb > 32))
        return fail(ARBORX_E_UNSUPPORTED, "too many long rows to sort");
    uint64_t *k1, *k2;
    uint32_t *v1, *v2;
    uint8_t *rws;
    if ((st = tmp.get(&k1, total)) != ARBORX_OK || (st = tmp.get(&k2, total)) != ARBORX_OK ||
        (st = tmp.get(&v1, total)) != ARBORX_OK || (st = tmp.get(&v2, total)) != ARBORX_OK ||
        (st = tmp.get(&rws, radix_workspace_bytes(total))) != ARBORX_OK)
        return st;
    k_huge_gather<<<(unsigned)(h < 4096 ? h : 4096), 256, 0, s>>>(offsets, indices, dist, huge_list, h, starts, ib, k1,
                                                                  v1);
    bool alt = false;
    AX_HIP(radix_sort_pairs<uint64_t>(k1, v1, k2, v2, total, 0, ib + hb, rws, s, &alt));
    uint64_t *ks = alt ? k2 : k1, *ko = alt ? k1 : k2;
    uint32_t *vs = alt ? v2 : v1, *vo = alt ? v1 : v2;
    if (mode == VALUES_ORDERED && dist) {
        k_huge_by_value<<<grid_for(total, 256, 65536), 256, 0, s>>>(ks, vs, total, ib, ko, vo);
        AX_HIP(radix_sort_pairs<uint64_t>(ko, vo, ks, vs, total, 0, 32 + hb, rws, s, &alt));
        k_huge_scatter_by_value<<<grid_for(total, 256, 65536), 256, 0, s>>>(alt ? ks : ko, alt ? vs : vo, total, h,
                                                                           offsets, huge_list, starts, indices, dist);
    } else {
        k_huge_scatter<<<grid_for(total, 256, 65536), 256, 0, s>>>(ks, vs, total, ib, h, offsets, huge_list, starts,
                                                                  indices, dist);
    }
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

arborx_status spatial_reduce(const TreeDev &t, const float *queries, int64_t m, float radius, int op,
                             int scale_bits, const uint32_t *perm, int32_t *counts, int64_t *sums, hipStream_t s)
{
    if (m == 0)
        return ARBORX_OK;
    if (t.n == 0) {
        arborx_status st = fill_async<int32_t>(counts, m, 0, s);
        if (st == ARBORX_OK && op == ARBORX_COUNT_SUMDIST)
            st = fill_async<int64_t>(sums, m, 0, s);
        return st;
    }
    arborx_status st = check_nodes(t.qnodes, t.wnodes, t.n, tree_format(OP_REDUCE, t));
    if (st != ARBORX_OK)
        return st;
    const float r2 = radius * radius;
    const float scale = ldexpf(1.0f, scale_bits);
    AX_DISPATCH_DIM(t.dim, (reduce_impl<D>(t, queries, m, r2, op, scale, perm, counts, sums, s)));
}

template <int D>
arborx_status count_up_to_impl(const TreeDev &t, const float *q, int64_t m, float r2, int n_max,
                               const uint32_t *perm, int32_t *counts, hipStream_t s)
{
    // the reductions' node format: quantized nodes where the tree holds them and the tuning walks them
    const bool qf = tree_format(OP_REDUCE, t) == 1 && t.qnodes;
    const Launch L = traversal_launch(m, sizeof(int), OP_REDUCE, D);
    ProfScope ps("count_up_to", s);
    const Node<D> *nodes = static_cast<const Node<D> *>(t.nodes);
    const QNode<D> *qnodes = static_cast<const QNode<D> *>(t.qnodes);
    if (qf)
        k_count_up_to<D, true><<<L.grid, L.block, L.lds, s>>>(nodes, qnodes, t.leaves, t.kind, t.hdr, q, m, r2, n_max,
                                                              perm, counts, L.cap);
    else
        k_count_up_to<D, false><<<L.grid, L.block, L.lds, s>>>(nodes, qnodes, t.leaves, t.kind, t.hdr, q, m, r2,
                                                               n_max, perm, counts, L.cap);
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

arborx_status spatial_count_up_to(const TreeDev &t, const float *queries, int64_t m, float radius, int n_max,
                                  const uint32_t *perm, int32_t *counts, hipStream_t s)
{
    if (m == 0)
        return ARBORX_OK;
    if (t.n == 0 || n_max == 0)
        return fill_async<int32_t>(counts, m, 0, s);
    const float r2 = radius * radius;
    AX_DISPATCH_DIM(t.dim, (count_up_to_impl<D>(t, queries, m, r2, n_max, perm, counts, s)));
}

arborx_status match_distances(const TreeDev &t, const float *values, const float *queries, int64_t m,
                              const int64_t *offsets, const int32_t *indices, float *out, hipStream_t s)
{
    if (m == 0 || t.n == 0)
        return ARBORX_OK;
    ProfScope ps("match_distances", s);
#define AX_MD(DD) k_match_distances<DD><<<grid_for(m, 256, 65536), 256, 0, s>>>(values, t.n, t.kind, queries, m, \
                                                                                offsets, indices, out)
    switch (t.dim) {
    case 2: AX_MD(2); break;
    case 3: AX_MD(3); break;
    case 6: AX_MD(6); break;
    default: return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in");
    }
#undef AX_MD
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

arborx_status knn_query(const TreeDev &t, const float *queries, int64_t m, int k, const uint32_t *perm,
                        float *dist2, int32_t *indices, hipStream_t s)
{
    if (m == 0)
        return ARBORX_OK;
    if (t.n == 0) {
        k_knn_empty<<<grid_for(m * k, 256, 65536), 256, 0, s>>>(m * k, dist2, indices);
        AX_HIP(hipGetLastError());
        return ARBORX_OK;
    }
    arborx_status st = check_nodes(t.qnodes, t.wnodes, t.n, tree_format(OP_KNN, t));
    if (st != ARBORX_OK)
        return st;
    AX_DISPATCH_DIM(t.dim, (knn_impl<D>(t, queries, m, k, perm, dist2, indices, s)));
}


// ---- allocation-free kNN ---------------------------------------------------
// Scratch of arborx_query_knn_noalloc: the query-ordering buffers (two code
// and two id arrays of kNoAllocMaxQueries entries, then the radix sort's tile
// histograms).  One copy per GPU, loaded with the code object and kept until
// the process ends.  In host code `scratch` names a host-side stand-in, so
// only the device address from hipGetSymbolAddress is ever passed to kernels.
constexpr int64_t kNoAllocMaxQueries = ARBORX_NOALLOC_MAX_QUERIES;
constexpr size_t kNoAllocArrayBytes = (size_t)kNoAllocMaxQueries * sizeof(uint32_t);
constexpr size_t kNoAllocWsBytes = size_t(1) << 20;
constexpr size_t kNoAllocScratchBytes = 4 * kNoAllocArrayBytes + kNoAllocWsBytes;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_dev[64] = {};

// Device address of this GPU's scratch, looked up once per device with that
// device current.
static arborx_status scratch_address(void **out)
{
    int dev = -1;
    AX_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64)
        return fail(ARBORX_E_DEVICE, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return ARBORX_OK;
}

arborx_status knn_query_noalloc(const TreeDev &t, const float *queries, int64_t m, int k, float *dist2,
                                int32_t *indices, hipStream_t s)
{
    if (m > kNoAllocMaxQueries)
        return fail(ARBORX_E_CAPACITY, "m = " + std::to_string((long long)m) +
                                           " exceeds the allocation-free limit of " +
                                           std::to_string((long long)kNoAllocMaxQueries) + " queries");
    if (m == 0)
        return ARBORX_OK;
    uint32_t *perm = nullptr;
    const int order = tuning(OP_KNN).order;
    if (order && t.n > 0 && m > 1) {
        if (radix_workspace_bytes(m) > kNoAllocWsBytes)
            return fail(ARBORX_E_CAPACITY, "radix workspace exceeds the allocation-free scratch");
        void *base = nullptr;
        arborx_status st = scratch_address(&base);
        if (st != ARBORX_OK)
            return st;
        unsigned char *b = static_cast<unsigned char *>(base);
        uint32_t *codes = reinterpret_cast<uint32_t *>(b);
        uint32_t *codes2 = reinterpret_cast<uint32_t *>(b + kNoAllocArrayBytes);
        uint32_t *ids = reinterpret_cast<uint32_t *>(b + 2 * kNoAllocArrayBytes);
        uint32_t *ids2 = reinterpret_cast<uint32_t *>(b + 3 * kNoAllocArrayBytes);
        void *ws = b + 4 * kNoAllocArrayBytes;
        switch (t.dim) {
        case 2: st = order_into<2>(t, queries, m, Pred::Sphere, order, codes, codes2, ids, ids2, ws, &perm, s); break;
        case 3: st = order_into<3>(t, queries, m, Pred::Sphere, order, codes, codes2, ids, ids2, ws, &perm, s); break;
        case 6: st = order_into<6>(t, queries, m, Pred::Sphere, order, codes, codes2, ids, ids2, ws, &perm, s); break;
        default: return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in");
        }
        if (st != ARBORX_OK)
            return st;
    }
    return knn_query(t, queries, m, k, perm, dist2, indices, s);
}

arborx_status debug_node_visits(const TreeDev &t, const float *queries, int64_t m, float radius, int op, int k,
                                int32_t *visits, hipStream_t s)
{
    if (m == 0)
        return ARBORX_OK;
    if (t.n == 0)
        return fill_async<int32_t>(visits, m, 0, s);
    const int block = op == 0 ? 256 : 64, cap = 8;
    const size_t lds = (size_t)cap * block * (op == 0 ? sizeof(int) : sizeof(KnnEntry));
    const float r2 = radius * radius;
#define AX_DV(DD, KK)                                                                                                  \
    k_debug_visits<DD, KK><<<grid_for(m, block, INT32_MAX), block, lds, s>>>(                                           \
        static_cast<const Node<DD> *>(t.nodes), t.codes, tree_nodes(t), t.leaves, t.kind, t.hdr, queries, m, r2, op, \
        visits, cap)
#define AX_DV_K(DD)                 \
    do {                            \
        if (op == 0 || k <= 1)      \
            AX_DV(DD, 1);           \
        else if (k <= 8)            \
            AX_DV(DD, 8);           \
        else if (k <= 16)           \
            AX_DV(DD, 16);          \
        else                        \
            AX_DV(DD, 64);          \
    } while (0)
    switch (t.dim) {
    case 2: AX_DV_K(2); break;
    case 3: AX_DV_K(3); break;
    case 6: AX_DV_K(6); break;
    default: return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in");
    }
#undef AX_DV_K
#undef AX_DV
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

}  // namespace ax
