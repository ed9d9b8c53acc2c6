// BVH construction (Section 2.6 of the ArborX 2.0 paper: 64-bit Morton codes,
// a sort, and Apetrei's bottom-up hierarchy construction).
//
//   1. scene bounds      : min/max per dimension over all values;
//   2. Morton-64         : quantise each value's centre to floor(63/D) bits per
//                          dimension and interleave;
//   3. radix sort        : stable sort of (code, value index);
//   4. hierarchy + refit : one thread per leaf climbs the tree.  Internal node
//                          p separates sorted leaves p and p+1.  A subtree over
//                          leaves [l, r] becomes the left child of node r or the
//                          right child of node l-1, whichever boundary is the
//                          smaller split key (the XOR of neighbouring codes,
//                          ties between equal codes broken by position).  Each
//                          thread writes its box into its slot of the parent
//                          and swaps an arrival word into the parent's flag;
//                          the first to arrive stops, the second merges the
//                          sibling's box and continues upwards.  Writing a
//                          leaf's box straight into its parent slot is the
//                          "leaf gather": leaves need no array of their own.
#include <algorithm>
#include <cstddef>
#include <vector>

#include "device_util.hpp"
#include "geometry.hpp"
#include "internal.hpp"
#include "profile.hpp"

namespace ax {
namespace {

constexpr int kBuildBlock = 256;

// Step of the 16-bit frame of [lo, hi]: a hair above (hi - lo) / 65535 so that
// code 65535 decodes at or beyond hi.
// Step of the 16-bit frame [lo, hi]: the smallest float found upward from
// about (hi - lo) / kQMax whose top code decodes to at least hi.  The two
// products are taken before the difference so that an extent beyond the float
// range stays finite; the check makes the guarantee independent of rounding
// and of underflow for tiny extents.
__device__ __forceinline__ float quant_scale(float lo, float hi)
{
    if (!(hi > lo))
        return 0.0f;
    constexpr float k = 1.0f / (float)kQMax;
    float s = (hi * k - lo * k) * (1.0f + 0x1p-18f);
    while (qdecode((uint32_t)kQMax, lo, s) < hi)
        s = nextafterf(s, INFINITY);
    return s;
}

// Largest code whose decoded value is <= x, and smallest whose decoded value
// is >= x.  The estimate from the reciprocal step `inv` is corrected both ways
// against the decode itself, so the result does not depend on its rounding.
__device__ __forceinline__ uint32_t qcode_down(float x, float lo, float scale, float inv)
{
    if (!(scale > 0.0f) || !(x > lo))
        return 0u;
    const float u = floorf((x - lo) * inv);
    uint32_t c = u >= (float)kQMax ? (uint32_t)kQMax : (u > 0.0f ? (uint32_t)u : 0u);
    while (c > 0 && qdecode(c, lo, scale) > x)
        --c;
    while (c < (uint32_t)kQMax && qdecode(c + 1, lo, scale) <= x)
        ++c;
    return c;
}

__device__ __forceinline__ uint32_t qcode_up(float x, float lo, float scale, float inv)
{
    if (!(scale > 0.0f))
        return 0u;
    if (!(x > lo))
        return 0u;
    const float u = ceilf((x - lo) * inv);
    uint32_t c = u >= (float)kQMax ? (uint32_t)kQMax : (u > 0.0f ? (uint32_t)u : 0u);
    while (c < (uint32_t)kQMax && qdecode(c, lo, scale) < x)
        ++c;
    while (c > 0 && qdecode(c - 1, lo, scale) >= x)
        --c;
    return c;
}


template <int D>
__global__ __launch_bounds__(kBuildBlock) void bounds_partial(const float *__restrict__ values, int64_t n, int kind,
                                                              float *__restrict__ partial)
{
    __shared__ float s_lo[kBuildBlock / kWave][D];
    __shared__ float s_hi[kBuildBlock / kWave][D];
    float lo[D], hi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = INFINITY;
        hi[d] = -INFINITY;
    }
    const int stride_v = kind == ARBORX_BOXES ? 2 * D : D;
    const int hoff = kind == ARBORX_BOXES ? D : 0;
    for (int64_t i = (int64_t)blockIdx.x * kBuildBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBuildBlock) {
        const float *v = values + i * stride_v;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lo[d] = fminf(lo[d], v[d]);
            hi[d] = fmaxf(hi[d], v[hoff + d]);
        }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
            lo[d] = fminf(lo[d], __shfl_xor(lo[d], o, kWave));
            hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], o, kWave));
        }
    }
    if (lane_id() == 0) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            s_lo[wave_id()][d] = lo[d];
            s_hi[wave_id()][d] = hi[d];
        }
    }
    __syncthreads();
    if (threadIdx.x < D) {
        const int d = threadIdx.x;
        float a = INFINITY, b = -INFINITY;
        for (int w = 0; w < kBuildBlock / kWave; ++w) {
            a = fminf(a, s_lo[w][d]);
            b = fmaxf(b, s_hi[w][d]);
        }
        partial[(int64_t)blockIdx.x * 2 * D + d] = a;
        partial[(int64_t)blockIdx.x * 2 * D + D + d] = b;
    }
}

template <int D>
__global__ __launch_bounds__(kBuildBlock) void bounds_final(const float *__restrict__ partial, int blocks, int64_t n,
                                                             TreeHeader *hdr)
{
    __shared__ float s_lo[kBuildBlock / kWave][D];
    __shared__ float s_hi[kBuildBlock / kWave][D];
    float a[D], b[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        a[d] = INFINITY;
        b[d] = -INFINITY;
    }
    for (int k = threadIdx.x; k < blocks; k += kBuildBlock)
#pragma unroll
        for (int d = 0; d < D; ++d) {
            a[d] = fminf(a[d], partial[(int64_t)k * 2 * D + d]);
            b[d] = fmaxf(b[d], partial[(int64_t)k * 2 * D + D + d]);
        }
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
            a[d] = fminf(a[d], __shfl_xor(a[d], o, kWave));
            b[d] = fmaxf(b[d], __shfl_xor(b[d], o, kWave));
        }
    if (lane_id() == 0)
#pragma unroll
        for (int d = 0; d < D; ++d) {
            s_lo[wave_id()][d] = a[d];
            s_hi[wave_id()][d] = b[d];
        }
    __syncthreads();
    const int d = threadIdx.x;
    if (d < D) {
        float lo = INFINITY, hi = -INFINITY;
        for (int w = 0; w < kBuildBlock / kWave; ++w) {
            lo = fminf(lo, s_lo[w][d]);
            hi = fmaxf(hi, s_hi[w][d]);
        }
        hdr->lo[d] = lo;
        hdr->hi[d] = hi;
        hdr->qscale[d] = quant_scale(lo, hi);
    }
    if (d == 0) {
        hdr->n = (int32_t)n;
        hdr->root = n > 0 ? 0 : -1;
        hdr->height = 0;
        hdr->start = 0;
    }
}

// Codes of value centres (points: the point; boxes: the box centre).
template <int D>
__global__ __launch_bounds__(kBuildBlock) void morton_kernel(const float *__restrict__ values, int64_t n, int kind,
                                                             const float *__restrict__ blo,
                                                             const float *__restrict__ bhi,
                                                             uint64_t *__restrict__ codes, uint32_t *__restrict__ ids)
{
    constexpr int bits = 63 / D;
    float lo[D], inv[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = blo[d];
        const float ext = bhi[d] - blo[d];
        inv[d] = ext > 0.0f ? 1.0f / ext : 0.0f;
    }
    for (int64_t i = (int64_t)blockIdx.x * kBuildBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBuildBlock) {
        uint32_t c[D];
        if (kind == ARBORX_BOXES) {
            const float *v = values + i * 2 * D;
#pragma unroll
            for (int d = 0; d < D; ++d)
                c[d] = quantise(v[d] + 0.5f * (v[D + d] - v[d]), lo[d], inv[d], bits);
        } else {
            const float *v = values + i * D;
#pragma unroll
            for (int d = 0; d < D; ++d)
                c[d] = quantise(v[d], lo[d], inv[d], bits);
        }
        codes[i] = interleave<D>(c, bits);
        if (ids)
            ids[i] = (uint32_t)i;
    }
}

// Split key between sorted leaves i and i+1: code differences rank above
// position differences (equal codes), so the order is total once ties are
// broken by node index.
__device__ __forceinline__ uint64_t split_key(const uint64_t *__restrict__ codes, int i)
{
    const uint64_t x = codes[i] ^ codes[i + 1];
    return x ? (x | (1ull << 63)) : (uint64_t)(uint32_t)(i ^ (i + 1));
}

template <int D>
__global__ __launch_bounds__(kBuildBlock) void hierarchy_kernel(const uint64_t *__restrict__ codes,
                                                                const uint32_t *__restrict__ ids,
                                                                const float *__restrict__ values, int kind, int n,
                                                                Node<D> *nodes, float *__restrict__ leaves,
                                                                unsigned long long *flags, TreeHeader *hdr)
{
    const int i = blockIdx.x * kBuildBlock + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t id = ids[i];
    if (id >= (uint32_t)n)
        return;
    float lo[D], hi[D];
    if (kind == ARBORX_BOXES) {
        const float *v = values + (int64_t)id * 2 * D;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lo[d] = v[d];
            hi[d] = v[D + d];
        }
    } else {
        const float *v = values + (int64_t)id * D;
#pragma unroll
        for (int d = 0; d < D; ++d)
            lo[d] = hi[d] = v[d];
    }
    int32_t ref = ~(int32_t)id;
    store_leaf<D>(leaves, i, kind, lo, hi, (int32_t)id);
    if (n == 1) {
        Node<D> &nd = nodes[0];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            nd.lo[0][d] = lo[d];
            nd.hi[0][d] = hi[d];
            nd.lo[1][d] = INFINITY;
            nd.hi[1][d] = -INFINITY;
        }
        nd.child[0] = ref;
        nd.child[1] = kEmptyRef;
        nd.range_l = 0;
        nd.range_r = 0;
        hdr->root = 0;
        hdr->height = 1;
        return;
    }
    int l = i, r = i, h = 0;
    while (true) {
        int p, side;
        if (l == 0 || (r != n - 1 && split_key(codes, r) < split_key(codes, l - 1))) {
            p = r;
            side = 0;
        } else {
            p = l - 1;
            side = 1;
        }
        Node<D> *np = nodes + p;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            np->lo[side][d] = lo[d];
            np->hi[side][d] = hi[d];
        }
        np->child[side] = ref;
        // arrival word: (height + 1) << 32 | the outer bound of this subtree's range
        const unsigned long long mine =
            ((unsigned long long)(uint32_t)(h + 1) << 32) | (uint32_t)(side == 0 ? l : r);
        const unsigned long long other =
            __hip_atomic_exchange(flags + p, mine, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (other == 0)
            return;  // first arrival: the sibling's thread finishes this node
        const int oh = (int)(other >> 32) - 1;
        const int ob = (int)(uint32_t)other;
        if (side == 0)
            r = ob;
        else
            l = ob;
        h = (h > oh ? h : oh) + 1;
        const int os = 1 - side;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lo[d] = fminf(lo[d], np->lo[os][d]);
            hi[d] = fmaxf(hi[d], np->hi[os][d]);
        }
        np->range_l = l;
        np->range_r = r;
        ref = p;
        if (l == 0 && r == n - 1) {
            hdr->root = p;
            hdr->height = h;
            return;
        }
    }
}

// ---------------------------------------------------------------------------
// Two-phase form of the same climb.  The tree is identical to the single-pass
// kernel's; only where the arrival handoff happens differs.
//
// Phase 1: one workgroup per chunk of C consecutive sorted leaves.  Arrivals at
// splits p with both neighbours inside the chunk (cs <= p <= ce-2) hand off
// through LDS: flags and the two child slots of each local split live in
// shared memory, so the exchange needs only workgroup scope.  A split whose
// second child reaches outside the chunk gets a single arrival here; its slot
// and arrival word are written to global memory at the end ("pending").  A
// climb that reaches split cs-1 or ce-1 (the chunk's borders) stops and is
// recorded as one of at most two escapes of the chunk.
// Phase 2: one thread per escape continues the climb over the splits whose
// subtrees span chunks, handing off through global memory with device-scope
// acquire/release.  Only these few percent of nodes pay for device-wide
// coherence.
// ---------------------------------------------------------------------------

template <int D>
struct Escape {
    int32_t valid, p, side, l, r, h, ref, pad;
    float lo[D], hi[D];
};

constexpr unsigned long long kDone = ~0ull;

__device__ __forceinline__ unsigned long long arrival_word(int side, int h, int bound)
{
    return ((unsigned long long)side << 48) | ((unsigned long long)(uint32_t)(h + 1) << 32) | (uint32_t)bound;
}

template <int D>
__device__ __forceinline__ void store_node(Node<D> *dst, const Node<D> &nd)
{
    float4 *d4 = reinterpret_cast<float4 *>(dst);
    const float4 *s4 = reinterpret_cast<const float4 *>(&nd);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(Node<D>) / 16); ++k)
        d4[k] = s4[k];
}

template <int D>
__device__ __forceinline__ void load_value_box(const float *values, int kind, uint32_t id, float *lo, float *hi)
{
    if (kind == ARBORX_BOXES) {
        const float *v = values + (int64_t)id * 2 * D;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lo[d] = v[d];
            hi[d] = v[D + d];
        }
    } else {
        const float *v = values + (int64_t)id * D;
#pragma unroll
        for (int d = 0; d < D; ++d)
            lo[d] = hi[d] = v[d];
    }
}

// Quantized form of float node p of a tree with header h.  A point tree's
// leaf child keeps its point and reference unchanged (the point's float words
// fill that child's code bytes); a box tree's leaf child becomes its sorted
// leaf position: the left child of node p is leaf p, the right child leaf
// p + 1.
template <int D>
__device__ __forceinline__ void store_qnode(QNode<D> *__restrict__ dst, const Node<D> &nd, int p, int kind,
                                            const TreeHeader &h)
{
    QNode<D> qn;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(qn.pad) / sizeof(qn.pad[0])); ++k)
        qn.pad[k] = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int32_t ref = nd.child[c];
        if (ref == kEmptyRef) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                qn.q[c][0][d] = (uint16_t)kQMax;
                qn.q[c][1][d] = 0;
            }
            qn.child[c] = kEmptyRef;
            continue;
        }
        if (ref < 0 && kind != ARBORX_BOXES) {
            uint16_t *qc = &qn.q[c][0][0];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const uint32_t bits = __float_as_uint(nd.lo[c][d]);
                qc[2 * d] = (uint16_t)(bits & 0xffffu);
                qc[2 * d + 1] = (uint16_t)(bits >> 16);
            }
            qn.child[c] = ref;
            continue;
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const float inv = h.qscale[d] > 0.0f ? 1.0f / h.qscale[d] : 0.0f;
            qn.q[c][0][d] = (uint16_t)qcode_down(nd.lo[c][d], h.lo[d], h.qscale[d], inv);
            qn.q[c][1][d] = (uint16_t)qcode_up(nd.hi[c][d], h.lo[d], h.qscale[d], inv);
        }
        qn.child[c] = ref >= 0 ? ref : ~(p + c);
    }
    float4 *d4 = reinterpret_cast<float4 *>(dst);
    const float4 *s4 = reinterpret_cast<const float4 *>(&qn);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(QNode<D>) / 16); ++k)
        d4[k] = s4[k];
}

template <int D>
__device__ void write_single_leaf_tree(Node<D> *node, TreeHeader *hdr, const float *lo, const float *hi, int32_t ref,
                                       int index)
{
    Node<D> nd;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        nd.lo[0][d] = lo[d];
        nd.hi[0][d] = hi[d];
        nd.lo[1][d] = INFINITY;
        nd.hi[1][d] = -INFINITY;
    }
    nd.child[0] = ref;
    nd.child[1] = kEmptyRef;
    nd.range_l = index;
    nd.range_r = index;
    store_node(node, nd);
    hdr->root = index;
    hdr->height = 1;
}

template <int D> constexpr int chunk_leaves() { return D <= 3 ? 1024 : 512; }

// Tree (segment) holding sorted leaf i: seg[s] <= i < seg[s+1].  Without
// segments the whole array is one tree.  Climbs never cross a tree's ends, so
// every tree of a forest gets its own root.
__device__ __forceinline__ void segment_of(int i, const int64_t *__restrict__ seg, int nseg, int n, int &s, int &ts,
                                           int &te)
{
    if (!seg) {
        s = 0;
        ts = 0;
        te = n - 1;
        return;
    }
    int lo = 0, hi = nseg;  // find the last s with seg[s] <= i
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg[mid] <= i)
            lo = mid;
        else
            hi = mid;
    }
    s = lo;
    ts = (int)seg[lo];
    te = (int)seg[lo + 1] - 1;
}

// Float nodes -> quantized nodes, a pass over the finished tree (a pass of
// its own measured faster than writing both forms during the climb, whose
// levels run one after another).  Node p belongs to the tree holding sorted
// leaf p (a one-value tree's node sits at its own leaf position).
template <int D>
__global__ void quantize_nodes(const Node<D> *__restrict__ nodes, int n_nodes, const int64_t *__restrict__ seg,
                               int nseg, int n, int kind, const TreeHeader *__restrict__ hdrs,
                               QNode<D> *__restrict__ qnodes)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_nodes)
        return;
    int sg, ts, te;
    segment_of(p < n ? p : n - 1, seg, nseg, n, sg, ts, te);
    Node<D> nd;
    load_node(nodes, p, nd);
    store_qnode<D>(qnodes + p, nd, p, kind, hdrs[sg]);
}


// Four-wide node p from binary node p and its internal children (the tree
// is final).  Slot order: p's left subtree first, so a leaf slot keeps the
// sorted order of the leaves.
template <int D>
__global__ void widen_nodes(const Node<D> *__restrict__ nodes, int n_nodes, Node4<D> *__restrict__ wnodes)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_nodes)
        return;
    Node<D> nd;
    load_node(nodes, p, nd);
    Node4<D> w;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(w.pad) / sizeof(w.pad[0])); ++k)
        w.pad[k] = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        w.child[s] = kEmptyRef;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            w.lo[s][d] = INFINITY;
            w.hi[s][d] = -INFINITY;
        }
    }
    int k = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int32_t ref = nd.child[c];
        if (ref >= 0 && ref < n_nodes) {
            Node<D> ch;
            load_node(nodes, ref, ch);
#pragma unroll
            for (int g = 0; g < 2; ++g) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    w.lo[k][d] = ch.lo[g][d];
                    w.hi[k][d] = ch.hi[g][d];
                }
                w.child[k] = ch.child[g];
                ++k;
            }
        } else if (ref != kEmptyRef) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                w.lo[k][d] = nd.lo[c][d];
                w.hi[k][d] = nd.hi[c][d];
            }
            w.child[k] = ref;
            ++k;
        }
    }
    float4 *dst = reinterpret_cast<float4 *>(wnodes + p);
    const float4 *src = reinterpret_cast<const float4 *>(&w);
#pragma unroll
    for (int q = 0; q < (int)(sizeof(Node4<D>) / 16); ++q)
        dst[q] = src[q];
}

template <int D>
__global__ __launch_bounds__(chunk_leaves<D>()) void hierarchy_chunk_kernel(const uint64_t *__restrict__ codes,
                                                                      const uint32_t *__restrict__ ids,
                                                                      const float *__restrict__ values, int kind,
                                                                      int n, Node<D> *__restrict__ nodes,
                                                                      float *__restrict__ leaves,
                                                                      unsigned long long *__restrict__ gflags,
                                                                      Escape<D> *__restrict__ escapes,
                                                                      const int64_t *__restrict__ seg, int nseg,
                                                                      TreeHeader *hdrs)
{
    constexpr int C = chunk_leaves<D>();
    __shared__ uint64_t s_key[C + 1];             // split keys of splits cs-1 .. ce-1
    __shared__ unsigned long long s_flag[C];      // arrival words of local splits cs .. ce-2
    __shared__ float s_lo[C][2][D], s_hi[C][2][D];  // both child slots of each local split
    __shared__ int32_t s_ref[C][2];

    // one thread per leaf of the chunk, so every climb of the chunk runs at once
    const int cs = blockIdx.x * C;
    const int ce = min(n, cs + C);
    const int tid = threadIdx.x;
    for (int j = tid; j < C; j += C)
        s_flag[j] = 0;
    for (int j = tid; j <= C; j += C) {
        const int g = cs - 1 + j;
        s_key[j] = (g >= 0 && g <= ce - 1 && g <= n - 2) ? split_key(codes, g) : 0ull;
    }
    for (int j = cs + tid; j < ce && j <= n - 2; j += C)
        gflags[j] = 0;
    if (tid < 2)
        escapes[2 * blockIdx.x + tid].valid = 0;
    __syncthreads();

    for (int i = cs + tid; i < ce; i += C) {
        const uint32_t id = ids[i];
        if (id >= (uint32_t)n)
            continue;
        float lo[D], hi[D];
        load_value_box<D>(values, kind, id, lo, hi);
        store_leaf<D>(leaves, i, kind, lo, hi, (int32_t)id);
        int32_t ref = ~(int32_t)id;
        int sg, ts, te;
        segment_of(i, seg, nseg, n, sg, ts, te);
        if (ts == te) {  // a one-value tree: its node slot is the unused split at its end
            write_single_leaf_tree<D>(nodes + ts, hdrs + sg, lo, hi, ref, ts);
            continue;
        }
        int l = i, r = i, h = 0;
        while (true) {
            int p, side;
            if (l == ts || (r != te && s_key[r - cs + 1] < s_key[l - 1 - cs + 1])) {
                p = r;
                side = 0;
            } else {
                p = l - 1;
                side = 1;
            }
            if (p < cs || p > ce - 2) {  // a border split of the chunk: continue in phase 2
                Escape<D> &e = escapes[2 * blockIdx.x + (p >= cs ? 1 : 0)];
                e.p = p;
                e.side = side;
                e.l = l;
                e.r = r;
                e.h = h;
                e.ref = ref;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    e.lo[d] = lo[d];
                    e.hi[d] = hi[d];
                }
                e.valid = 1;
                break;
            }
            const int lp = p - cs;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                s_lo[lp][side][d] = lo[d];
                s_hi[lp][side][d] = hi[d];
            }
            s_ref[lp][side] = ref;
            const unsigned long long other = __hip_atomic_exchange(
                &s_flag[lp], arrival_word(side, h, side == 0 ? l : r), __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (other == 0)
                break;  // first arrival
            const int os = 1 - side;
            const int oh = (int)((other >> 32) & 0xffff) - 1;
            const int ob = (int)(uint32_t)other;
            Node<D> nd;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const float slo = s_lo[lp][os][d], shi = s_hi[lp][os][d];
                nd.lo[0][d] = side == 0 ? lo[d] : slo;
                nd.hi[0][d] = side == 0 ? hi[d] : shi;
                nd.lo[1][d] = side == 0 ? slo : lo[d];
                nd.hi[1][d] = side == 0 ? shi : hi[d];
                lo[d] = fminf(lo[d], slo);
                hi[d] = fmaxf(hi[d], shi);
            }
            const int32_t sref = s_ref[lp][os];
            nd.child[0] = side == 0 ? ref : sref;
            nd.child[1] = side == 0 ? sref : ref;
            if (side == 0)
                r = ob;
            else
                l = ob;
            h = (h > oh ? h : oh) + 1;
            nd.range_l = l;
            nd.range_r = r;
            store_node(nodes + p, nd);
            s_flag[lp] = kDone;
            ref = p;
            if (l == ts && r == te) {
                hdrs[sg].root = p;
                hdrs[sg].height = h;
                break;
            }
        }
    }
    __syncthreads();
    // splits with a single arrival: publish that child's slot for phase 2
    for (int lp = tid; lp <= ce - 2 - cs; lp += C) {
        const unsigned long long w = s_flag[lp];
        if (w != 0 && w != kDone) {
            const int side = (int)(w >> 48);
            Node<D> *np = nodes + cs + lp;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                np->lo[side][d] = s_lo[lp][side][d];
                np->hi[side][d] = s_hi[lp][side][d];
            }
            np->child[side] = s_ref[lp][side];
            gflags[cs + lp] = w;
        }
    }
}

template <int D>
__global__ __launch_bounds__(kBuildBlock) void hierarchy_top_kernel(const uint64_t *__restrict__ codes, int n,
                                                                    Node<D> *nodes, unsigned long long *gflags,
                                                                    const Escape<D> *__restrict__ escapes,
                                                                    int n_escapes, const int64_t *__restrict__ seg,
                                                                    int nseg, TreeHeader *hdrs)
{
    const int e_i = blockIdx.x * kBuildBlock + threadIdx.x;
    if (e_i >= n_escapes)
        return;
    const Escape<D> &e = escapes[e_i];
    if (!e.valid)
        return;
    float lo[D], hi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = e.lo[d];
        hi[d] = e.hi[d];
    }
    int p = e.p, side = e.side, l = e.l, r = e.r, h = e.h;
    int32_t ref = e.ref;
    int sg, ts, te;
    segment_of(l, seg, nseg, n, sg, ts, te);
    // a climb visits at most n-1 splits
    for (int guard = 0; guard < n; ++guard) {
        if (p < 0 || p > n - 2)
            return;
        Node<D> *np = nodes + p;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            np->lo[side][d] = lo[d];
            np->hi[side][d] = hi[d];
        }
        np->child[side] = ref;
        const unsigned long long other = __hip_atomic_exchange(
            gflags + p, arrival_word(side, h, side == 0 ? l : r), __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (other == 0)
            return;
        const int oh = (int)((other >> 32) & 0xffff) - 1;
        const int ob = (int)(uint32_t)other;
        if (side == 0)
            r = ob;
        else
            l = ob;
        h = (h > oh ? h : oh) + 1;
        const int os = 1 - side;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lo[d] = fminf(lo[d], np->lo[os][d]);
            hi[d] = fmaxf(hi[d], np->hi[os][d]);
        }
        np->range_l = l;
        np->range_r = r;
        ref = p;
        if (l == ts && r == te) {
            hdrs[sg].root = p;
            hdrs[sg].height = h;
            return;
        }
        if (l == ts || (r != te && split_key(codes, r) < split_key(codes, l - 1))) {
            p = r;
            side = 0;
        } else {
            p = l - 1;
            side = 1;
        }
    }
}

__global__ void empty_header(TreeHeader *hdr, int dim)
{
    for (int d = 0; d < kMaxDim; ++d)
        hdr->qscale[d] = 0.0f;
    hdr->root = -1;
    hdr->height = 0;
    hdr->n = 0;
    hdr->start = 0;
    for (int d = 0; d < kMaxDim; ++d) {
        hdr->lo[d] = INFINITY;
        hdr->hi[d] = -INFINITY;
    }
    (void)dim;
}

template <int D>
arborx_status build_impl(const float *values, int64_t n, int kind, TreeDev &t, hipStream_t s)
{
    AX_HIP(hipGetLastError());  // clear stale errors from earlier user work
    arborx_status st = dalloc((void **)&t.hdr, sizeof(TreeHeader), s);
    if (st != ARBORX_OK)
        return st;
    t.n = n;
    t.dim = D;
    t.kind = kind;
    if (n == 0) {
        empty_header<<<1, 1, 0, s>>>(t.hdr, D);
        AX_HIP(hipGetLastError());
        return ARBORX_OK;
    }
    const int64_t nn = n > 1 ? n - 1 : 1;
    st = dalloc(&t.nodes, (size_t)nn * sizeof(Node<D>), s);
    if (st != ARBORX_OK)
        return st;
    st = dalloc((void **)&t.leaves, (size_t)n * leaf_floats(D, kind) * sizeof(float), s);
    if (st != ARBORX_OK)
        return st;
    const bool quantized = format_requested(1, D, kind, false), wide = format_requested(2, D, kind, false);
    if (quantized && (st = dalloc(&t.qnodes, (size_t)nn * sizeof(QNode<D>), s)) != ARBORX_OK)
        return st;
    if (wide && (st = dalloc(&t.wnodes, (size_t)nn * sizeof(Node4<D>), s)) != ARBORX_OK)
        return st;

    Temps tmp(s);
    const int pblocks = (int)grid_for(n, kBuildBlock, 1024);
    float *partial;
    uint64_t *codes, *codes2;
    uint32_t *ids, *ids2;
    unsigned long long *flags;
    uint8_t *ws;
    // the sorted codes stay with the tree: kNN finds a query's leaf position by binary search
    if ((st = dalloc((void **)&t.codes, (size_t)n * sizeof(uint64_t), s)) != ARBORX_OK)
        return st;
    codes = t.codes;
    if ((st = tmp.get(&partial, (size_t)pblocks * 2 * D)) != ARBORX_OK ||
        (st = tmp.get(&codes2, n)) != ARBORX_OK || (st = tmp.get(&ids, n)) != ARBORX_OK ||
        (st = tmp.get(&ids2, n)) != ARBORX_OK || (st = tmp.get(&flags, nn)) != ARBORX_OK ||
        (st = tmp.get(&ws, radix_workspace_bytes(n))) != ARBORX_OK)
        return st;

    {
        ProfScope ps("build_bounds", s);
        bounds_partial<D><<<pblocks, kBuildBlock, 0, s>>>(values, n, kind, partial);
        bounds_final<D><<<1, kBuildBlock, 0, s>>>(partial, pblocks, n, t.hdr);
    }
    const float *blo = reinterpret_cast<const float *>(reinterpret_cast<const char *>(t.hdr) + offsetof(TreeHeader, lo));
    const float *bhi = reinterpret_cast<const float *>(reinterpret_cast<const char *>(t.hdr) + offsetof(TreeHeader, hi));
    {
        ProfScope ps("build_morton", s);
        morton_kernel<D><<<grid_for(n, kBuildBlock, 65536), kBuildBlock, 0, s>>>(values, n, kind, blo, bhi, codes,
                                                                                ids);
    }
    bool alt = false;
    {
        ProfScope ps("build_sort", s);
        AX_HIP(radix_sort_pairs<uint64_t>(codes, ids, codes2, ids2, n, 0, (63 / D) * D, ws, s, &alt));
    }
    if (alt) {  // an odd number of passes (none for the dimensions compiled in): keep the result in t.codes
        AX_HIP(hipMemcpyAsync(t.codes, codes2, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        ids = ids2;
    }
    Node<D> *nodes = static_cast<Node<D> *>(t.nodes);
    if (tuning(OP_SPATIAL).build == 1) {
        // single pass: every handoff through device-scope acquire/release
        fill_kernel<unsigned long long><<<grid_for(nn, 256, 65536), 256, 0, s>>>(flags, nn, 0ull);
        ProfScope ps("build_hierarchy", s);
        hierarchy_kernel<D><<<grid_for(n, kBuildBlock), kBuildBlock, 0, s>>>(codes, ids, values, kind, (int)n, nodes,
                                                                             t.leaves, flags, t.hdr);
    } else {
        constexpr int C = chunk_leaves<D>();
        const int chunks = (int)((n + C - 1) / C);
        Escape<D> *esc;
        if ((st = tmp.get(&esc, (size_t)2 * chunks)) != ARBORX_OK)
            return st;
        ProfScope ps("build_hierarchy", s);
        hierarchy_chunk_kernel<D><<<chunks, C, 0, s>>>(codes, ids, values, kind, (int)n, nodes, t.leaves,
                                                                 flags, esc, nullptr, 0, t.hdr);
        if (chunks > 1)
            hierarchy_top_kernel<D><<<grid_for(2 * chunks, kBuildBlock), kBuildBlock, 0, s>>>(
                codes, (int)n, nodes, flags, esc, 2 * chunks, nullptr, 0, t.hdr);
    }
    if (quantized) {
        ProfScope ps("build_quantize", s);
        quantize_nodes<D><<<grid_for(nn, kBuildBlock), kBuildBlock, 0, s>>>(nodes, (int)nn, nullptr, 0, (int)n, t.kind,
                                                                            t.hdr, static_cast<QNode<D> *>(t.qnodes));
    }
    if (wide) {
        ProfScope ps("build_widen", s);
        widen_nodes<D><<<grid_for(nn, kBuildBlock), kBuildBlock, 0, s>>>(nodes, (int)nn,
                                                                         static_cast<Node4<D> *>(t.wnodes));
    }
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

template <int D>
hipError_t morton_impl(const float *pts, int64_t n, const float *bounds, uint64_t *codes, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    morton_kernel<D><<<grid_for(n, kBuildBlock, 65536), kBuildBlock, 0, s>>>(pts, n, ARBORX_POINTS, bounds,
                                                                            bounds + D, codes, nullptr);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Forest build: many trees over one packed value array, tree t holding values
// [seg[t], seg[t+1]).  Work is cut into tiles that never straddle a tree so
// each workgroup knows its tree.  Per-tree bounds are reduced per tile and
// combined with atomics on order-preserving integer images of the floats;
// Morton keys are (tree << mbits) | tree-local code, so one global sort keeps
// every tree contiguous and Morton-ordered inside; the climb then stops at the
// tree ends (segment_of).
// ---------------------------------------------------------------------------

constexpr int kForestTile = 4096;

__device__ __forceinline__ uint32_t float_order(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float order_float(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

template <int D>
__global__ __launch_bounds__(kBuildBlock) void forest_tile_bounds(const float *__restrict__ values, int kind,
                                                                  const int32_t *__restrict__ tile_tree,
                                                                  const int32_t *__restrict__ tile_start,
                                                                  const int32_t *__restrict__ tile_end,
                                                                  uint32_t *__restrict__ tmin,
                                                                  uint32_t *__restrict__ tmax)
{
    __shared__ float s_lo[kBuildBlock / kWave][D];
    __shared__ float s_hi[kBuildBlock / kWave][D];
    const int b = blockIdx.x;
    const int t = tile_tree[b];
    float lo[D], hi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = INFINITY;
        hi[d] = -INFINITY;
    }
    const int stride_v = kind == ARBORX_BOXES ? 2 * D : D;
    const int hoff = kind == ARBORX_BOXES ? D : 0;
    for (int i = tile_start[b] + threadIdx.x; i < tile_end[b]; i += kBuildBlock) {
        const float *v = values + (int64_t)i * stride_v;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lo[d] = fminf(lo[d], v[d]);
            hi[d] = fmaxf(hi[d], v[hoff + d]);
        }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
            lo[d] = fminf(lo[d], __shfl_xor(lo[d], o, kWave));
            hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], o, kWave));
        }
    }
    if (lane_id() == 0) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            s_lo[wave_id()][d] = lo[d];
            s_hi[wave_id()][d] = hi[d];
        }
    }
    __syncthreads();
    if (threadIdx.x < D) {
        const int d = threadIdx.x;
        float a = INFINITY, c = -INFINITY;
        for (int w = 0; w < kBuildBlock / kWave; ++w) {
            a = fminf(a, s_lo[w][d]);
            c = fmaxf(c, s_hi[w][d]);
        }
        atomicMin(&tmin[t * D + d], float_order(a));
        atomicMax(&tmax[t * D + d], float_order(c));
    }
}

template <int D>
__global__ void forest_headers(const int64_t *__restrict__ seg, int T, const uint32_t *__restrict__ tmin,
                               const uint32_t *__restrict__ tmax, TreeHeader *__restrict__ hdrs)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T)
        return;
    const int n = (int)(seg[t + 1] - seg[t]);
    TreeHeader &h = hdrs[t];
    h.n = n;
    h.start = (int)seg[t];
    h.root = -1;
    h.height = 0;
    for (int d = 0; d < kMaxDim; ++d) {
        h.lo[d] = (d < D && n > 0) ? order_float(tmin[t * D + d]) : INFINITY;
        h.hi[d] = (d < D && n > 0) ? order_float(tmax[t * D + d]) : -INFINITY;
        h.qscale[d] = (d < D && n > 0) ? quant_scale(h.lo[d], h.hi[d]) : 0.0f;
    }
}

template <int D>
__global__ __launch_bounds__(kBuildBlock) void forest_tile_morton(const float *__restrict__ values, int kind,
                                                                  const int32_t *__restrict__ tile_tree,
                                                                  const int32_t *__restrict__ tile_start,
                                                                  const int32_t *__restrict__ tile_end,
                                                                  const TreeHeader *__restrict__ hdrs, int mbits,
                                                                  uint64_t *__restrict__ codes,
                                                                  uint32_t *__restrict__ ids)
{
    const int b = blockIdx.x;
    const int t = tile_tree[b];
    const int bits = mbits / D;
    float lo[D], inv[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = hdrs[t].lo[d];
        const float ext = hdrs[t].hi[d] - lo[d];
        inv[d] = ext > 0.0f ? 1.0f / ext : 0.0f;
    }
    for (int i = tile_start[b] + threadIdx.x; i < tile_end[b]; i += kBuildBlock) {
        uint32_t c[D];
        if (kind == ARBORX_BOXES) {
            const float *v = values + (int64_t)i * 2 * D;
#pragma unroll
            for (int d = 0; d < D; ++d)
                c[d] = quantise(v[d] + 0.5f * (v[D + d] - v[d]), lo[d], inv[d], bits);
        } else {
            const float *v = values + (int64_t)i * D;
#pragma unroll
            for (int d = 0; d < D; ++d)
                c[d] = quantise(v[d], lo[d], inv[d], bits);
        }
        codes[i] = ((uint64_t)t << mbits) | interleave<D>(c, bits);
        ids[i] = (uint32_t)i;
    }
}

// The segmentation the build uses, made valid whatever the caller's device
// array holds: seg[0] = 0, seg[T] = n, and in between the running maximum of
// the offsets clamped to [0, n], so segments never overlap or leave the value
// array (a valid array is copied unchanged).  One workgroup: an inclusive
// max-scan over chunks of its width.
constexpr int kSegBlock = 1024;

__global__ __launch_bounds__(kSegBlock) void forest_segments(const int64_t *__restrict__ off, int T, int64_t n,
                                                             int64_t *__restrict__ seg)
{
    __shared__ int64_t s_wmax[kSegBlock / kWave];
    __shared__ int64_t s_carry;
    if (threadIdx.x == 0)
        s_carry = 0;
    __syncthreads();
    for (int base = 0; base <= T; base += kSegBlock) {
        const int i = base + (int)threadIdx.x;
        int64_t v = 0;
        if (i == T)
            v = n;
        else if (i > 0 && i < T)
            v = off[i] < 0 ? 0 : (off[i] > n ? n : off[i]);
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {  // inclusive max-scan across the wavefront
            const int64_t u = __shfl_up(v, o, kWave);
            if (lane_id() >= o)
                v = u > v ? u : v;
        }
        if (lane_id() == kWave - 1)
            s_wmax[wave_id()] = v;
        __syncthreads();
        int64_t before = s_carry;
        for (int w = 0; w < wave_id(); ++w)
            before = s_wmax[w] > before ? s_wmax[w] : before;
        v = v > before ? v : before;
        if (i <= T)
            seg[i] = v;
        __syncthreads();
        if (threadIdx.x == kSegBlock - 1)
            s_carry = v;
        __syncthreads();
    }
}

// Tiles that never straddle a tree, from the device segmentation: tree t
// gets ceil(n_t / kForestTile) tiles, placed by an exclusive scan over the
// trees; entries up to max_tiles past the last are empty tiles (no values).
__global__ __launch_bounds__(kSegBlock) void forest_tiles(const int64_t *__restrict__ seg, int T, int max_tiles,
                                                          int32_t *__restrict__ tile_tree,
                                                          int32_t *__restrict__ tile_start,
                                                          int32_t *__restrict__ tile_end)
{
    __shared__ int32_t s_wsum[kSegBlock / kWave];
    __shared__ int32_t s_carry;
    if (threadIdx.x == 0)
        s_carry = 0;
    __syncthreads();
    for (int base = 0; base < T; base += kSegBlock) {
        const int t = base + (int)threadIdx.x;
        const int64_t a = t < T ? seg[t] : 0, e = t < T ? seg[t + 1] : 0;
        const int cnt = (int)((e - a + kForestTile - 1) / kForestTile);
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int u = __shfl_up(incl, o, kWave);
            if (lane_id() >= o)
                incl += u;
        }
        if (lane_id() == kWave - 1)
            s_wsum[wave_id()] = incl;
        __syncthreads();
        int before = s_carry;
        for (int w = 0; w < wave_id(); ++w)
            before += s_wsum[w];
        const int first = before + incl - cnt;
        for (int j = 0; j < cnt && first + j < max_tiles; ++j) {
            const int64_t ts = a + (int64_t)j * kForestTile;
            tile_tree[first + j] = t;
            tile_start[first + j] = (int32_t)ts;
            tile_end[first + j] = (int32_t)(e < ts + kForestTile ? e : ts + kForestTile);
        }
        __syncthreads();
        if (threadIdx.x == kSegBlock - 1)
            s_carry = before + incl;
        __syncthreads();
    }
    for (int j = s_carry + (int)threadIdx.x; j < max_tiles; j += kSegBlock) {
        tile_tree[j] = 0;
        tile_start[j] = 0;
        tile_end[j] = 0;
    }
}

// The build workspace of a forest of n values in T trees, carved from one
// block: tree bounds, tile tables, keys and ids (two each, for the sort),
// arrival flags, the sort's tile histograms, the climb's escapes, and the
// caller's offsets copied in by the build from host offsets.
struct ForestBuildWs {
    uint32_t *tmin, *tmax;
    int32_t *tiles;
    uint64_t *codes, *codes2;
    uint32_t *ids, *ids2;
    unsigned long long *flags;
    uint8_t *rws;
    void *esc;
    int64_t *offs;
};

template <int D>
size_t forest_build_ws(int64_t n, int T, int max_tiles, uint8_t *base, ForestBuildWs *w)
{
    const int64_t nn = n > 0 ? n : 1;
    const int chunks = (int)((nn + chunk_leaves<D>() - 1) / chunk_leaves<D>());
    size_t at = 0;
    auto take = [&](size_t bytes) {
        uint8_t *p = base ? base + at : nullptr;
        at += (bytes + 255) / 256 * 256;
        return p;
    };
    uint8_t *tmin = take(sizeof(uint32_t) * T * D), *tmax = take(sizeof(uint32_t) * T * D);
    uint8_t *tiles = take(sizeof(int32_t) * 3 * (size_t)max_tiles);
    uint8_t *codes = take(8 * nn), *codes2 = take(8 * nn), *ids = take(4 * nn), *ids2 = take(4 * nn);
    uint8_t *flags = take(8 * nn), *rws = take(radix_workspace_bytes(nn));
    uint8_t *esc = take(sizeof(Escape<D>) * 2 * (size_t)chunks), *offs = take(sizeof(int64_t) * (T + 1));
    if (w) {
        w->tmin = reinterpret_cast<uint32_t *>(tmin);
        w->tmax = reinterpret_cast<uint32_t *>(tmax);
        w->tiles = reinterpret_cast<int32_t *>(tiles);
        w->codes = reinterpret_cast<uint64_t *>(codes);
        w->codes2 = reinterpret_cast<uint64_t *>(codes2);
        w->ids = reinterpret_cast<uint32_t *>(ids);
        w->ids2 = reinterpret_cast<uint32_t *>(ids2);
        w->flags = reinterpret_cast<unsigned long long *>(flags);
        w->rws = rws;
        w->esc = esc;
        w->offs = reinterpret_cast<int64_t *>(offs);
    }
    return at;
}

inline int forest_max_tiles(int64_t n, int T) { return (int)(n / kForestTile) + T + 1; }

// Every device allocation of a forest of n values in T trees: the structure
// and the build workspace.
template <int D>
arborx_status forest_alloc_impl(int64_t n, int T, int kind, ForestDev &f, hipStream_t s)
{
    f.n = n;
    f.dim = D;
    f.kind = kind;
    f.T = T;
    f.max_tiles = forest_max_tiles(n, T);
    arborx_status st;
    if ((st = dalloc((void **)&f.hdrs, sizeof(TreeHeader) * T, s)) != ARBORX_OK ||
        (st = dalloc((void **)&f.seg, sizeof(int64_t) * (T + 1), s)) != ARBORX_OK ||
        (st = dalloc(&f.nodes, (size_t)(n > 0 ? n : 1) * sizeof(Node<D>), s)) != ARBORX_OK ||
        (st = dalloc((void **)&f.leaves, (size_t)(n > 0 ? n : 1) * leaf_floats(D, kind) * sizeof(float), s)) !=
            ARBORX_OK)
        return st;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    if (format_requested(1, D, kind, true) && (st = dalloc(&f.qnodes, nn * sizeof(QNode<D>), s)) != ARBORX_OK)
        return st;
    if (format_requested(2, D, kind, true) && (st = dalloc(&f.wnodes, nn * sizeof(Node4<D>), s)) != ARBORX_OK)
        return st;
    f.bws_bytes = forest_build_ws<D>(n, T, f.max_tiles, nullptr, nullptr);
    return dalloc(&f.bws, f.bws_bytes, s);
}

// Build the forest's trees in place from device-resident values and offsets:
// kernels only (no allocation, no host read, no copy), so the call can be
// captured in a graph and replayed with new contents of the same sizes.
template <int D>
arborx_status forest_rebuild_impl(const float *values, const int64_t *offs, ForestDev &f, hipStream_t s)
{
    AX_HIP(hipGetLastError());
    const int64_t n = f.n;
    const int T = f.T, kind = f.kind, tiles = f.max_tiles;
    ForestBuildWs w;
    forest_build_ws<D>(n, T, tiles, static_cast<uint8_t *>(f.bws), &w);
    int32_t *dtiles = w.tiles;
    forest_segments<<<1, kSegBlock, 0, s>>>(offs, T, n, f.seg);
    forest_tiles<<<1, kSegBlock, 0, s>>>(f.seg, T, tiles, dtiles, dtiles + tiles, dtiles + 2 * tiles);
    fill_kernel<uint32_t><<<grid_for((int64_t)T * D, 256), 256, 0, s>>>(w.tmin, (int64_t)T * D, 0xffffffffu);
    fill_kernel<uint32_t><<<grid_for((int64_t)T * D, 256), 256, 0, s>>>(w.tmax, (int64_t)T * D, 0u);
    {
        ProfScope ps("build_bounds", s);
        forest_tile_bounds<D><<<tiles, kBuildBlock, 0, s>>>(values, kind, dtiles, dtiles + tiles, dtiles + 2 * tiles,
                                                            w.tmin, w.tmax);
        forest_headers<D><<<grid_for(T, 256), 256, 0, s>>>(f.seg, T, w.tmin, w.tmax, f.hdrs);
    }
    AX_HIP(hipGetLastError());
    f.keys = nullptr;
    if (n == 0)
        return ARBORX_OK;
    int tb = 1;
    while ((1 << tb) < T)
        ++tb;
    const int mbits = (63 - tb) / D * D;
    uint64_t *codes = w.codes, *codes2 = w.codes2;
    uint32_t *ids = w.ids, *ids2 = w.ids2;
    {
        ProfScope ps("build_morton", s);
        forest_tile_morton<D><<<tiles, kBuildBlock, 0, s>>>(values, kind, dtiles, dtiles + tiles, dtiles + 2 * tiles,
                                                            f.hdrs, mbits, codes, ids);
    }
    bool alt = false;
    {
        ProfScope ps("build_sort", s);
        AX_HIP(radix_sort_pairs<uint64_t>(codes, ids, codes2, ids2, n, 0, mbits + tb, w.rws, s, &alt));
    }
    if (alt) {
        codes = codes2;
        ids = ids2;
    }
    f.keys = codes;  // kept in the build workspace until the next rebuild: kNN seeds search them
    f.mbits = mbits;
    constexpr int C = chunk_leaves<D>();
    const int chunks = (int)((n + C - 1) / C);
    Escape<D> *esc = static_cast<Escape<D> *>(w.esc);
    Node<D> *nodes = static_cast<Node<D> *>(f.nodes);
    ProfScope ps("build_hierarchy", s);
    hierarchy_chunk_kernel<D><<<chunks, C, 0, s>>>(codes, ids, values, kind, (int)n, nodes, f.leaves, w.flags, esc,
                                                   f.seg, T, f.hdrs);
    if (chunks > 1)
        hierarchy_top_kernel<D><<<grid_for(2 * chunks, kBuildBlock), kBuildBlock, 0, s>>>(
            codes, (int)n, nodes, w.flags, esc, 2 * chunks, f.seg, T, f.hdrs);
    if (f.qnodes)
        quantize_nodes<D><<<grid_for(n, kBuildBlock), kBuildBlock, 0, s>>>(nodes, (int)n, f.seg, T, (int)n, f.kind,
                                                                           f.hdrs, static_cast<QNode<D> *>(f.qnodes));
    if (f.wnodes)
        widen_nodes<D><<<grid_for(n, kBuildBlock), kBuildBlock, 0, s>>>(nodes, (int)n,
                                                                        static_cast<Node4<D> *>(f.wnodes));
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

template <int D>
arborx_status forest_build_impl(const float *values, const int64_t *seg_host, int T, int kind, ForestDev &f,
                                hipStream_t s)
{
    arborx_status st = forest_alloc_impl<D>(seg_host[T], T, kind, f, s);
    if (st != ARBORX_OK)
        return st;
    ForestBuildWs w;
    forest_build_ws<D>(f.n, T, f.max_tiles, static_cast<uint8_t *>(f.bws), &w);
    AX_HIP(hipMemcpyAsync(w.offs, seg_host, sizeof(int64_t) * (T + 1), hipMemcpyHostToDevice, s));
    return forest_rebuild_impl<D>(values, w.offs, f, s);
}

}  // namespace

size_t node_bytes(int dim)
{
    switch (dim) {
    case 2: return sizeof(Node<2>);
    case 3: return sizeof(Node<3>);
    case 6: return sizeof(Node<6>);
    default: return 0;
    }
}

arborx_status build_tree(const float *values, int64_t n, int dim, int kind, TreeDev &t, hipStream_t s)
{
    switch (dim) {
    case 2: return build_impl<2>(values, n, kind, t, s);
    case 3: return build_impl<3>(values, n, kind, t, s);
    case 6: return build_impl<6>(values, n, kind, t, s);
    default: return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in");
    }
}

void forest_release(ForestDev &f, hipStream_t s)
{
    dfree(f.nodes, s);
    dfree(f.qnodes, s);
    f.qnodes = nullptr;
    dfree(f.wnodes, s);
    f.wnodes = nullptr;
    dfree(f.leaves, s);
    dfree(f.hdrs, s);
    dfree(f.seg, s);
    dfree(f.ws, s);
    dfree(f.bws, s);
    f.bws = nullptr;
    f.bws_bytes = 0;
    f.nodes = nullptr;
    f.leaves = nullptr;
    f.hdrs = nullptr;
    f.seg = nullptr;
    f.ws = nullptr;
    f.ws_bytes = 0;
}

arborx_status forest_alloc(int64_t n, int T, int dim, int kind, ForestDev &f, hipStream_t s)
{
    switch (dim) {
    case 2: return forest_alloc_impl<2>(n, T, kind, f, s);
    case 3: return forest_alloc_impl<3>(n, T, kind, f, s);
    case 6: return forest_alloc_impl<6>(n, T, kind, f, s);
    default: return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in");
    }
}

arborx_status forest_rebuild(const float *values, const int64_t *tree_offsets, ForestDev &f, hipStream_t s)
{
    switch (f.dim) {
    case 2: return forest_rebuild_impl<2>(values, tree_offsets, f, s);
    case 3: return forest_rebuild_impl<3>(values, tree_offsets, f, s);
    case 6: return forest_rebuild_impl<6>(values, tree_offsets, f, s);
    default: return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in");
    }
}

arborx_status build_forest(const float *values, const int64_t *seg_host, int T, int dim, int kind, ForestDev &f,
                           hipStream_t s)
{
    switch (dim) {
    case 2: return forest_build_impl<2>(values, seg_host, T, kind, f, s);
    case 3: return forest_build_impl<3>(values, seg_host, T, kind, f, s);
    case 6: return forest_build_impl<6>(values, seg_host, T, kind, f, s);
    default: return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in");
    }
}

hipError_t morton64_points(const float *pts, int64_t n, int dim, const float *bounds, uint64_t *codes, hipStream_t s)
{
    switch (dim) {
    case 2: return morton_impl<2>(pts, n, bounds, codes, s);
    case 3: return morton_impl<3>(pts, n, bounds, codes, s);
    case 6: return morton_impl<6>(pts, n, bounds, codes, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ax
