// Device-side geometry: node layout, squared distances, overlap, Morton codes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ax {

// Child reference stored in a node: >= 0 is an internal node index, < 0 is a
// leaf holding value ~ref.  kEmptyRef marks the unused slot of a one-value tree.
constexpr int32_t kEmptyRef = INT32_MIN;

// Internal node of the binary hierarchy.  It stores the bounding boxes of its
// two children, so one 16*D+16 byte fetch decides both children (64 B in 3D).
// A leaf needs no storage of its own: its box is the value's box (a point is
// the degenerate box [p, p]) held in the parent slot, and its reference is the
// value's input index.
template <int D>
struct alignas(16) Node {
    float lo[2][D];
    float hi[2][D];
    int32_t child[2];
    int32_t range_l;  // leaf range [range_l, range_r] in sorted order
    int32_t range_r;
};
static_assert(sizeof(Node<3>) == 64, "3D node is 64 bytes");
static_assert(sizeof(Node<6>) == 112, "6D node is 112 bytes");

// Leaves in sorted (Morton) order, one record per value: the point (or the
// box lo and hi rows) followed by the value's input index, padded to 16 bytes.
// A 3D point leaf is {x, y, z, index}: 16 bytes.
__host__ __device__ constexpr int leaf_floats(int dim, int kind)
{
    return ((kind == 1 ? 2 * dim : dim) + 1 + 3) / 4 * 4;
}

template <int D>
__device__ __forceinline__ void store_leaf(float *leaves, int64_t pos, int kind, const float *lo, const float *hi,
                                           int32_t id)
{
    float4 *dst = reinterpret_cast<float4 *>(leaves + pos * leaf_floats(D, kind));
    if (kind == 1) {
        constexpr int F = leaf_floats(D, 1);
        float v[F];
#pragma unroll
        for (int k = 0; k < F; ++k)
            v[k] = 0.0f;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            v[d] = lo[d];
            v[D + d] = hi[d];
        }
        v[2 * D] = __int_as_float(id);
#pragma unroll
        for (int k = 0; k < F / 4; ++k)
            dst[k] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
    } else {
        constexpr int F = leaf_floats(D, 0);
        float v[F];
#pragma unroll
        for (int k = 0; k < F; ++k)
            v[k] = 0.0f;
#pragma unroll
        for (int d = 0; d < D; ++d)
            v[d] = lo[d];
        v[D] = __int_as_float(id);
#pragma unroll
        for (int k = 0; k < F / 4; ++k)
            dst[k] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
    }
}

// The same node with each child box stored as 16-bit codes in the tree's
// frame (lo + code * qscale per dimension), rounded outward so that the
// decoded box always contains the true one: tests on it are conservative.
// In a tree of points a leaf child is stored exactly instead: the point's D
// float32 words take the 4*D bytes of that child's codes, and the reference
// is ~value index as in the float node, so leaf tests need no second fetch
// and give the float node's results bit for bit.  In a tree of boxes a leaf
// child refers to its sorted leaf record (~position), whose exact box decides
// the match.  32 bytes in 3D, half the float node; 64 bytes in 6D.
template <int D>
struct alignas(16) QNode {
    uint16_t q[2][2][D];  // [child][lo, hi][dim]
    int32_t child[2];     // >= 0 node, < 0 leaf record ~ref, kEmptyRef empty
    int32_t pad[(16 - (8 * D + 8) % 16) % 16 / 4];
};
static_assert(sizeof(QNode<3>) == 32, "3D quantized node is 32 bytes");

constexpr int kQMax = 65535;

// Four-wide node: binary node p with its two levels collapsed.  The slots are
// p's children, each internal child replaced by its own two children, so one
// fetch decides up to four subtrees.  A slot reference >= 0 names a binary
// node whose four-wide node is visited next, < 0 is a leaf holding value ~ref,
// kEmptyRef an unused slot (box lo = +inf, hi = -inf).  128 bytes in 3D.
template <int D>
struct alignas(16) Node4 {
    float lo[4][D];
    float hi[4][D];
    int32_t child[4];
    int32_t pad[(16 - (32 * D + 16) % 16) % 16 / 4 + (D == 3 ? 4 : 0)];
};
static_assert(sizeof(Node4<3>) == 128, "3D four-wide node is 128 bytes");

template <int D>
__device__ __forceinline__ void load_node4(const Node4<D> *__restrict__ nodes, int32_t i, Node4<D> &out)
{
    const float4 *src = reinterpret_cast<const float4 *>(nodes + i);
    float4 *dst = reinterpret_cast<float4 *>(&out);
#pragma unroll
    for (int k = 0; k < (int)((sizeof(Node4<D>) - (D == 3 ? 16 : 0)) / 16); ++k)
        dst[k] = src[k];
}

__device__ __forceinline__ float qdecode(uint32_t code, float lo, float scale) { return fmaf((float)code, scale, lo); }

template <int D>
__device__ __forceinline__ void load_qnode(const QNode<D> *__restrict__ nodes, int32_t i, QNode<D> &out)
{
    const float4 *src = reinterpret_cast<const float4 *>(nodes + i);
    float4 *dst = reinterpret_cast<float4 *>(&out);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(QNode<D>) / 16); ++k)
        dst[k] = src[k];
}

// Child c of a quantized node as a box.  `exact` (a point tree's leaf child)
// reads the stored point; otherwise the codes decode outward-rounded.  Both
// forms are evaluated and selected, so the choice costs no branch.
template <int D>
__device__ __forceinline__ void qchild(const QNode<D> &nd, int c, bool exact, const float *flo, const float *fsc,
                                       float (&lo)[D], float (&hi)[D])
{
    const uint16_t *qc = &nd.q[c][0][0];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const float p = __uint_as_float((uint32_t)qc[2 * d] | ((uint32_t)qc[2 * d + 1] << 16));
        const float l = qdecode(qc[d], flo[d], fsc[d]);
        const float h = qdecode(qc[D + d], flo[d], fsc[d]);
        lo[d] = exact ? p : l;
        hi[d] = exact ? p : h;
    }
}

template <int D>
__device__ __forceinline__ void load_node(const Node<D> *__restrict__ nodes, int32_t i, Node<D> &out)
{
    const float4 *src = reinterpret_cast<const float4 *>(nodes + i);
    float4 *dst = reinterpret_cast<float4 *>(&out);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(Node<D>) / 16); ++k)
        dst[k] = src[k];
}

// Squared distance from point q to the closed box [lo, hi]: per dimension the
// gap to the nearer face (0 inside), each square and each sum rounded once,
// dimensions summed from 0 upwards.  For a degenerate box [p, p] it equals the
// point-to-point squared distance bit for bit, because |fl(p - q)| = |fl(q - p)|.
// The signed gap is q - med3(q, lo, hi): for lo <= hi the median is q
// clamped to the box, so the difference is fl(q - lo) below the box (whose
// square equals that of fl(lo - q)), fl(q - hi) above it and 0 inside, with
// no branch.  The one box with lo > hi, the empty slot of a one-value tree,
// is never tested for a match: its reference is checked first.
template <int D>
__device__ __forceinline__ float box_d2(const float *q, const float *lo, const float *hi)
{
#pragma clang fp contract(off)
    float acc = 0.0f;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const float t = q[d] - __builtin_amdgcn_fmed3f(q[d], lo[d], hi[d]);
        float s = t * t;
        acc = acc + s;
    }
    return acc;
}

// Closed overlap of [alo, ahi] and [blo, bhi] in every dimension.
template <int D>
__device__ __forceinline__ bool boxes_overlap(const float *alo, const float *ahi, const float *blo, const float *bhi)
{
    bool ok = true;
#pragma unroll
    for (int d = 0; d < D; ++d)
        ok = ok & (alo[d] <= bhi[d]) & (blo[d] <= ahi[d]);
    return ok;
}

// Spread the low 21 bits of x so that bit i moves to bit 3i.
__device__ __forceinline__ uint64_t spread3_21(uint64_t x)
{
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// Quantise coordinate x of [lo, lo + 1/inv] into 2^bits cells (bits <= 31).
// The upper clamp is done on the integer side: 2^bits - 1 is not a float for
// bits > 24.
__device__ __forceinline__ uint32_t quantise(float x, float lo, float inv, int bits)
{
    const float cells = (float)(1u << bits);
    const float u = fmaxf((x - lo) * inv * cells, 0.0f);
    return u >= cells ? (1u << bits) - 1u : (uint32_t)u;
}

// Morton code of cell coordinates c[0..D) with `bits` bits each, dimension 0
// most significant within each group of D bits.
template <int D>
__device__ __forceinline__ uint64_t interleave(const uint32_t *c, int bits)
{
    if constexpr (D == 3) {
        if (bits == 21)
            return (spread3_21(c[0]) << 2) | (spread3_21(c[1]) << 1) | spread3_21(c[2]);
    }
    uint64_t code = 0;
    for (int b = bits - 1; b >= 0; --b)
#pragma unroll
        for (int d = 0; d < D; ++d)
            code = (code << 1) | ((c[d] >> b) & 1u);
    return code;
}

}  // namespace ax
