// Device-side traversal pieces shared by the single-tree and forest queries:
// the short stack, query predicates, the depth-first spatial walk, the sorted
// register buffers, and the seeded nearest-first kNN walk.
#pragma once

#include "device_util.hpp"
#include "geometry.hpp"
#include "internal.hpp"

namespace ax {
namespace {

// Deepest tree the build can make.  Along a root-to-leaf path the split keys
// (code XOR of neighbouring leaves, or position XOR for equal codes) strictly
// decrease, and two splits with the same highest bit always have a larger
// split between them in sorted order, so no path repeats a highest bit: at
// most 63 code bits + 31 position bits + the leaf edge.
constexpr int kMaxTreeHeight = 95;
// Spill entries behind the LDS ring.  A binary walk pushes at most one entry
// per level, a four-wide walk at most three per four-wide level (two binary
// levels), so no walk ever holds more than 3 * ceil(95 / 2) = 144 deferred
// entries, even with a one-entry ring: the spill area never overflows.
constexpr int kSpill = 160;
static_assert(kSpill >= 3 * ((kMaxTreeHeight + 1) / 2), "spill area below the four-wide walk's bound");

// The ring indices live in registers; only the rarely used spill area (a
// separate private array owned by the caller) sits in scratch memory.  Keeping
// the array out of this struct lets the compiler hold the counters in
// registers instead of reloading them from scratch on every push and pop.
template <typename E>
struct ShortStack {
    E *lds;  // this thread's column: entry j at lds[j << shift] (the stride is the block size, a power of two)
    E *spill;
    int shift, mask;
    int base = 0, cnt = 0, ns = 0;
    __device__ ShortStack(E *col, int stride, int cap, E *spill_) : lds(col), spill(spill_), shift(__ffs(stride) - 1),
                                                                     mask(cap - 1) {}
    __device__ __forceinline__ bool empty() const { return cnt == 0 && ns == 0; }
    __device__ __forceinline__ void clear() { base = cnt = ns = 0; }
    __device__ __forceinline__ void push(E x)
    {
        if (cnt == mask + 1) {  // ring full: move the oldest LDS entry to the spill area
            if (ns < kSpill)    // always true (see kSpill); the check only keeps the store in bounds
                spill[ns++] = lds[(base & mask) << shift];
            ++base;
            --cnt;
        }
        lds[((base + cnt) & mask) << shift] = x;
        ++cnt;
    }
    // The newest spilled entry sits just below the ring's oldest one: when the
    // ring is empty it moves back first, so every pop reads LDS.
    __device__ __forceinline__ E pop()
    {
        if (cnt == 0) {
            --base;
            lds[(base & mask) << shift] = spill[--ns];
            cnt = 1;
        }
        --cnt;
        return lds[((base + cnt) & mask) << shift];
    }
};

// Blocks are dealt round-robin over the 8 XCDs; renumber them so that each
// XCD (and its L2) works on one contiguous run of Morton-ordered queries.
__device__ __forceinline__ int64_t xcd_block()
{
    constexpr int64_t X = 8;
    const int64_t b = blockIdx.x, G = gridDim.x;
    const int64_t q = G / X, r = G % X, x = b % X;
    return x * q + (x < r ? x : r) + b / X;
}

template <int D>
struct Sphere {
    float c[D];
    float r2;
    __device__ __forceinline__ bool hit(const float *lo, const float *hi, float &d2) const
    {
        d2 = box_d2<D>(c, lo, hi);
        return d2 <= r2;
    }
    __device__ __forceinline__ void load(const float *q, int64_t i, float rr)
    {
#pragma unroll
        for (int d = 0; d < D; ++d)
            c[d] = q[i * D + d];
        r2 = rr;
    }
    __device__ __forceinline__ void dead()  // matches nothing: d2 >= 0 > r2
    {
#pragma unroll
        for (int d = 0; d < D; ++d)
            c[d] = 0.0f;
        r2 = -1.0f;
    }
};

template <int D>
struct BoxQuery {
    float lo[D], hi[D];
    __device__ __forceinline__ bool hit(const float *blo, const float *bhi, float &d2) const
    {
        d2 = 0.0f;
        return boxes_overlap<D>(lo, hi, blo, bhi);
    }
    __device__ __forceinline__ void load(const float *q, int64_t i, float)
    {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lo[d] = q[i * 2 * D + d];
            hi[d] = q[i * 2 * D + D + d];
        }
    }
    __device__ __forceinline__ void dead()  // an empty box overlaps nothing
    {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lo[d] = INFINITY;
            hi[d] = -INFINITY;
        }
    }
};

// A ray o + t*dir, t >= 0 (Section 2.5).  It meets a closed box when its slab
// intervals overlap: slabs taken in dimension order from tmin = 0, tmax =
// +inf, t1 = (lo - o)/dir and t2 = (hi - o)/dir with correctly rounded
// division, a zero direction component requiring lo <= o <= hi.  The entry
// parameter tmin is reported in the distance slot.  Subtraction and division
// are monotone, so a box inside another is met no earlier: pruning by a
// parent's box is exact.
template <int D>
struct RayPred {
    float o[D], dir[D];
    __device__ __forceinline__ void load(const float *rays, int64_t i, float)
    {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            o[d] = rays[i * 2 * D + d];
            dir[d] = rays[i * 2 * D + D + d];
        }
    }
    __device__ __forceinline__ void dead()  // origin at +inf, no direction: outside every finite box
    {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            o[d] = INFINITY;
            dir[d] = 0.0f;
        }
    }
    __device__ __forceinline__ bool hit(const float *lo, const float *hi, float &t) const
    {
        float tmin = 0.0f, tmax = INFINITY;
        bool inside = true;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if (dir[k] == 0.0f) {
                inside = inside && !(o[k] < lo[k] || o[k] > hi[k]);
                continue;
            }
            const float t1 = (lo[k] - o[k]) / dir[k];
            const float t2 = (hi[k] - o[k]) / dir[k];
            const float tn = t1 < t2 ? t1 : t2, tf = t1 < t2 ? t2 : t1;
            tmin = tn > tmin ? tn : tmin;
            tmax = tf < tmax ? tf : tmax;
        }
        t = tmin;
        return inside && !(tmin > tmax);
    }
};

// Exact test of the sorted leaf record `pos` (the value's own box) against
// the predicate, calling f(index, d2) on a match.
template <int D, class P, class F>
__device__ __forceinline__ void leaf_exact(const float *__restrict__ leaves, int kind, int pos, const P &pred, F &f)
{
    const float *lf = leaves + (int64_t)pos * leaf_floats(D, kind);
    float lo[D], hi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = lf[d];
        hi[d] = kind == ARBORX_BOXES ? lf[D + d] : lf[d];
    }
    float d2;
    if (pred.hit(lo, hi, d2))
        f(__float_as_int(lf[kind == ARBORX_BOXES ? 2 * D : D]), d2);
}

struct NeverStop {
    __device__ __forceinline__ constexpr bool operator()() const { return false; }
};

// Depth-first walk calling f(index, d2) on every matching value; with a stop
// functor, the walk ends as soon as stop() holds after a node's matches were
// reported (the early termination of Section 2.2).
// A depth-first walk enters each internal node at most once, so `limit`
// iterations (more than the node count) bound every walk even on a corrupt
// tree, and node indices are range-checked before use.
template <int D, class P, class F, class S = NeverStop>
__device__ __forceinline__ void traverse_spatial(const Node<D> *__restrict__ nodes, int root, int n_nodes,
                                                 const P &pred, ShortStack<int> &st, F &f, const S &stop = S())
{
    int cur = root;
    for (int iter = 0; iter <= n_nodes; ++iter) {
        if ((unsigned)cur >= (unsigned)n_nodes)
            break;
        Node<D> nd;
        load_node(nodes, cur, nd);
        float d0, d1;
        bool h0 = pred.hit(nd.lo[0], nd.hi[0], d0);
        bool h1 = pred.hit(nd.lo[1], nd.hi[1], d1);
        const int c0 = nd.child[0], c1 = nd.child[1];
        if (h0 && c0 < 0) {
            if (c0 != kEmptyRef)
                f(~c0, d0);
            h0 = false;
        }
        if (h1 && c1 < 0) {
            if (c1 != kEmptyRef)
                f(~c1, d1);
            h1 = false;
        }
        if (stop())
            break;
        if (h0) {
            if (h1)
                st.push(c1);
            cur = c0;
        } else if (h1) {
            cur = c1;
        } else {
            if (st.empty())
                break;
            cur = st.pop();
        }
    }
}

// The depth-first walk over four-wide nodes: one fetch tests up to four
// subtrees; matching leaf slots are reported, the first matching internal slot
// is entered and the others are deferred on the stack.
template <int D, class P, class F>
__device__ __forceinline__ void traverse_spatial4(const Node4<D> *__restrict__ nodes, int root, int n_nodes,
                                                  const P &pred, ShortStack<int> &st, F &f)
{
    int cur = root;
    for (int iter = 0; iter <= n_nodes; ++iter) {
        if ((unsigned)cur >= (unsigned)n_nodes)
            break;
        Node4<D> nd;
        load_node4(nodes, cur, nd);
        int next = -1;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            float d;
            const bool h = pred.hit(nd.lo[s], nd.hi[s], d);
            const int c = nd.child[s];
            if (h && c < 0 && c != kEmptyRef)
                f(~c, d);
            if (h && c >= 0) {
                if (next >= 0)
                    st.push(next);
                next = c;
            }
        }
        cur = next >= 0 ? next : (st.empty() ? -1 : st.pop());
    }
}

// Packet walk: one thread answers NQ queries (Morton neighbours) in a single
// depth-first walk over the union of their paths.  A child is entered when
// any query's predicate admits it; leaves are tested per query, calling
// f(j, index, d2) for query j.  Neighbouring queries share most of their
// paths, so a thread makes fewer dependent node fetches per query.
template <int D, int NQ, class P, class F>
__device__ __forceinline__ void traverse_spatial_packet(const Node<D> *__restrict__ nodes, int root, int n_nodes,
                                                        const P (&pred)[NQ], ShortStack<int> &st, F &f)
{
    int cur = root;
    for (int iter = 0; iter <= n_nodes; ++iter) {
        if ((unsigned)cur >= (unsigned)n_nodes)
            break;
        Node<D> nd;
        load_node(nodes, cur, nd);
        const int c0 = nd.child[0], c1 = nd.child[1];
        bool g0 = false, g1 = false;
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            float d0, d1;
            const bool h0 = pred[j].hit(nd.lo[0], nd.hi[0], d0);
            const bool h1 = pred[j].hit(nd.lo[1], nd.hi[1], d1);
            if (h0 && c0 < 0 && c0 != kEmptyRef)
                f(j, ~c0, d0);
            if (h1 && c1 < 0 && c1 != kEmptyRef)
                f(j, ~c1, d1);
            g0 = g0 | h0;
            g1 = g1 | h1;
        }
        g0 = g0 && c0 >= 0;
        g1 = g1 && c1 >= 0;
        if (g0) {
            if (g1)
                st.push(c1);
            cur = c0;
        } else if (g1) {
            cur = c1;
        } else {
            if (st.empty())
                break;
            cur = st.pop();
        }
    }
}

// Wavefront-packet form of the walk: the 64 lanes (64 Morton-neighbouring
// queries) visit the union of their paths together.  The node index is the
// same in every lane, so each node is fetched once per wavefront through the
// scalar cache, and the stack of deferred nodes is one per wavefront in LDS.
// A stack entry is pushed only at a level where some lane needs both
// children, so its depth never exceeds the tree height (kMaxTreeHeight),
// below kWaveStack.  Lanes without a query
// (`active` false) carry a predicate that matches nothing.
constexpr int kWaveStack = 128;
static_assert(kWaveStack > kMaxTreeHeight, "wavefront stack below the tree height bound");

template <int D, class P, class F>
__device__ __forceinline__ void traverse_spatial_wave(const Node<D> *__restrict__ nodes, int root, int n_nodes,
                                                      const P &pred, int *wstack, F &f)
{
    int sp = 0;
    int cur = root;
    for (int iter = 0; iter <= n_nodes; ++iter) {
        cur = __builtin_amdgcn_readfirstlane(cur);
        if ((unsigned)cur >= (unsigned)n_nodes)
            break;
        Node<D> nd;
        load_node(nodes, cur, nd);
        float d0, d1;
        bool h0 = pred.hit(nd.lo[0], nd.hi[0], d0);
        bool h1 = pred.hit(nd.lo[1], nd.hi[1], d1);
        const int c0 = nd.child[0], c1 = nd.child[1];
        if (c0 < 0) {
            if (h0 && c0 != kEmptyRef)
                f(~c0, d0);
            h0 = false;
        }
        if (c1 < 0) {
            if (h1 && c1 != kEmptyRef)
                f(~c1, d1);
            h1 = false;
        }
        const bool any0 = __ballot(h0) != 0, any1 = __ballot(h1) != 0;
        if (any0) {
            if (any1) {
                if (sp < kWaveStack)
                    wstack[sp] = c1;
                ++sp;
            }
            cur = c0;
        } else if (any1) {
            cur = c1;
        } else {
            if (sp == 0)
                break;
            --sp;
            cur = sp < kWaveStack ? wstack[sp] : -1;
        }
    }
}

// Stackless walk with ropes (the paper's spatial traversal, Section 2.6).  The
// walk position is a child slot (node p, side).  Its rope, the slot the
// depth-first order visits after the whole subtree in it, needs no storage:
// after (p, left) comes (p, right); the right child of p covers leaves
// [p + 1, range_r(p)], and the next subtree in leaf order is the right child
// of the node splitting leaves range_r(p) and range_r(p) + 1, i.e. (range_r(p),
// right), unless range_r(p) is the last leaf of the tree.  Every slot is tested
// at most once, so 2 * n_nodes steps bound the walk.
template <int D, class P, class F>
__device__ __forceinline__ void traverse_spatial_rope(const Node<D> *__restrict__ nodes, int root, int n_nodes,
                                                      int last_leaf, const P &pred, F &f)
{
    int p = root, side = 0;
    Node<D> nd;
    int loaded = -1;
    for (int iter = 0; iter <= 2 * n_nodes; ++iter) {
        if ((unsigned)p >= (unsigned)n_nodes)
            break;
        if (p != loaded) {
            load_node(nodes, p, nd);
            loaded = p;
        }
        float lo[D], hi[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lo[d] = side ? nd.lo[1][d] : nd.lo[0][d];
            hi[d] = side ? nd.hi[1][d] : nd.hi[0][d];
        }
        const int c = side ? nd.child[1] : nd.child[0];
        float d2;
        if (c != kEmptyRef && pred.hit(lo, hi, d2)) {
            if (c >= 0) {
                p = c;
                side = 0;
                continue;
            }
            f(~c, d2);
        }
        if (side == 0) {
            side = 1;
        } else {
            if (nd.range_r >= last_leaf)
                break;
            p = nd.range_r;
        }
    }
}

// Pair-search walk (Section 2.6 names a dedicated traversal for searching
// pairs of objects) for the value at sorted position p of a single tree: the
// rope walk started at p's own rope.  In depth-first order the slot after leaf
// p is (node p, right side) -- node p separates leaves p and p + 1, whichever
// of nodes p - 1 and p holds the leaf -- and the ropes from there reach
// exactly the subtrees of positions p + 1 .. last_leaf.  So each unordered
// pair of values is met once, from its earlier position, and no walk touches
// the part of the tree before its own leaf.  f(q, index, d2) gets the
// partner's sorted position (a leaf in slot (node, side) sits at position
// node + side), its value index and its distance.
template <int D, class P, class F>
__device__ __forceinline__ void traverse_pairs_after(const Node<D> *__restrict__ nodes, int n_nodes, int p,
                                                     int last_leaf, const P &pred, F &f)
{
    if (p >= last_leaf)
        return;
    int cur = p, side = 1;
    Node<D> nd;
    int loaded = -1;
    for (int iter = 0; iter <= 2 * n_nodes; ++iter) {
        if ((unsigned)cur >= (unsigned)n_nodes)
            break;
        if (cur != loaded) {
            load_node(nodes, cur, nd);
            loaded = cur;
        }
        float lo[D], hi[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lo[d] = side ? nd.lo[1][d] : nd.lo[0][d];
            hi[d] = side ? nd.hi[1][d] : nd.hi[0][d];
        }
        const int c = side ? nd.child[1] : nd.child[0];
        float d2;
        if (c != kEmptyRef && pred.hit(lo, hi, d2)) {
            if (c >= 0) {
                cur = c;
                side = 0;
                continue;
            }
            f(cur + side, ~c, d2);
        }
        if (side == 0) {
            side = 1;
        } else {
            if (nd.range_r >= last_leaf)
                break;
            cur = nd.range_r;
        }
    }
}

// Top-down packet form of the pair-search walk: one thread takes the NQ
// consecutive sorted positions p0 .. p0 + NQ - 1 of a single tree and walks
// from the root over the union of their paths.  Node c separates leaves c and
// c + 1, so its left child holds positions [range_l, c] and its right child
// [c + 1, range_r]; query j enters a child only if the child's box admits it
// and the child holds a position after p0 + j.  Each unordered pair is thus
// reported once, to the query at its earlier position, as
// f(j, partner position, partner index, d2); the walk over the shared upper
// levels is paid once per NQ queries.  Queries past the tree carry a
// predicate that matches nothing.
template <int D, int NQ, class P, class F>
__device__ __forceinline__ void traverse_pairs_packet(const Node<D> *__restrict__ nodes, int root, int n_nodes, int p0,
                                                      const P (&pred)[NQ], ShortStack<int> &st, F &f)
{
    int cur = root;
    for (int iter = 0; iter <= n_nodes; ++iter) {
        if ((unsigned)cur >= (unsigned)n_nodes)
            break;
        Node<D> nd;
        load_node(nodes, cur, nd);
        const int c0 = nd.child[0], c1 = nd.child[1];
        bool g0 = false, g1 = false;
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            float d0, d1;
            const bool h0 = cur > p0 + j && pred[j].hit(nd.lo[0], nd.hi[0], d0);
            const bool h1 = nd.range_r > p0 + j && pred[j].hit(nd.lo[1], nd.hi[1], d1);
            if (h0 && c0 < 0 && c0 != kEmptyRef)
                f(j, cur, ~c0, d0);
            if (h1 && c1 < 0 && c1 != kEmptyRef)
                f(j, cur + 1, ~c1, d1);
            g0 = g0 | h0;
            g1 = g1 | h1;
        }
        g0 = g0 && c0 >= 0;
        g1 = g1 && c1 >= 0;
        if (g0) {
            if (g1)
                st.push(c1);
            cur = c0;
        } else if (g1) {
            cur = c1;
        } else {
            if (st.empty())
                break;
            cur = st.pop();
        }
    }
}

// Both child boxes of a quantized node in the tree's frame; `points` says the
// tree holds points, whose leaf children are stored exactly.
template <int D>
__device__ __forceinline__ void qboxes(const QNode<D> &nd, bool points, const float *flo, const float *fsc,
                                       float (&lo)[2][D], float (&hi)[2][D])
{
    qchild<D>(nd, 0, points && nd.child[0] < 0, flo, fsc, lo[0], hi[0]);
    qchild<D>(nd, 1, points && nd.child[1] < 0, flo, fsc, lo[1], hi[1]);
}

// The short-stack walk over quantized nodes.  Internal child boxes decode to
// supersets of the true boxes, so no matching subtree is skipped.  A point
// tree's leaf child is exact in the node and reported from it; a box tree's
// leaf whose decoded box passes is tested exactly on its leaf record.  (An
// empty slot's bytes are never reported: its reference is checked first.)
// An optional stop functor ends the walk as in traverse_spatial.
template <int D, class P, class F, class S = NeverStop>
__device__ __forceinline__ void traverse_spatial_q(const QNode<D> *__restrict__ nodes, const TreeHeader &h,
                                                   int n_nodes, const float *__restrict__ leaves, int kind,
                                                   const P &pred, ShortStack<int> &st, F &f, const S &stop = S())
{
    const bool points = kind != ARBORX_BOXES;
    float flo[D], fsc[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        flo[d] = h.lo[d];
        fsc[d] = h.qscale[d];
    }
    int cur = h.root;
    for (int iter = 0; iter <= n_nodes; ++iter) {
        if ((unsigned)cur >= (unsigned)n_nodes)
            break;
        QNode<D> nd;
        load_qnode(nodes, cur, nd);
        float lo[2][D], hi[2][D];
        qboxes<D>(nd, points, flo, fsc, lo, hi);
        float d0, d1;
        bool h0 = pred.hit(lo[0], hi[0], d0);
        bool h1 = pred.hit(lo[1], hi[1], d1);
        const int c0 = nd.child[0], c1 = nd.child[1];
        if (h0 && c0 < 0) {
            if (c0 != kEmptyRef) {
                if (points)
                    f(~c0, d0);
                else
                    leaf_exact<D>(leaves, kind, ~c0, pred, f);
            }
            h0 = false;
        }
        if (h1 && c1 < 0) {
            if (c1 != kEmptyRef) {
                if (points)
                    f(~c1, d1);
                else
                    leaf_exact<D>(leaves, kind, ~c1, pred, f);
            }
            h1 = false;
        }
        if (stop())
            break;
        if (h0) {
            if (h1)
                st.push(c1);
            cur = c0;
        } else if (h1) {
            cur = c1;
        } else {
            if (st.empty())
                break;
            cur = st.pop();
        }
    }
}

// Packet walk over quantized nodes: as traverse_spatial_packet, one decode
// of the node's child boxes serving all NQ queries; leaves as in
// traverse_spatial_q.
template <int D, int NQ, class P, class F>
__device__ __forceinline__ void traverse_spatial_packet_q(const QNode<D> *__restrict__ nodes, const TreeHeader &h,
                                                          int n_nodes, const float *__restrict__ leaves, int kind,
                                                          const P (&pred)[NQ], ShortStack<int> &st, F &f)
{
    const bool points = kind != ARBORX_BOXES;
    float flo[D], fsc[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        flo[d] = h.lo[d];
        fsc[d] = h.qscale[d];
    }
    int cur = h.root;
    for (int iter = 0; iter <= n_nodes; ++iter) {
        if ((unsigned)cur >= (unsigned)n_nodes)
            break;
        QNode<D> nd;
        load_qnode(nodes, cur, nd);
        float lo[2][D], hi[2][D];
        qboxes<D>(nd, points, flo, fsc, lo, hi);
        const int c0 = nd.child[0], c1 = nd.child[1];
        bool g0 = false, g1 = false;
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            float d0, d1;
            const bool h0 = pred[j].hit(lo[0], hi[0], d0);
            const bool h1 = pred[j].hit(lo[1], hi[1], d1);
            auto fj = [&](int idx, float d) { f(j, idx, d); };
            if (h0 && c0 < 0 && c0 != kEmptyRef) {
                if (points)
                    f(j, ~c0, d0);
                else
                    leaf_exact<D>(leaves, kind, ~c0, pred[j], fj);
            }
            if (h1 && c1 < 0 && c1 != kEmptyRef) {
                if (points)
                    f(j, ~c1, d1);
                else
                    leaf_exact<D>(leaves, kind, ~c1, pred[j], fj);
            }
            g0 = g0 | h0;
            g1 = g1 | h1;
        }
        g0 = g0 && c0 >= 0;
        g1 = g1 && c1 >= 0;
        if (g0) {
            if (g1)
                st.push(c1);
            cur = c0;
        } else if (g1) {
            cur = c1;
        } else {
            if (st.empty())
                break;
            cur = st.pop();
        }
    }
}

// Pair walk over the quantized nodes of a tree of points, one leaf (sorted
// position p) per thread: f(q, index, d2) for every later position q whose
// point is in range.  A node is entered only when its leaf range holds a
// position after p: the root unless p is the last leaf; a left child [l, c]
// when c > p; a right child always, as its range ends where its parent's does.
// So only the leaf children need a position test (the left leaf sits at c,
// the right one at c + 1) and the node needs no stored range.
template <int D, class P, class F>
__device__ __forceinline__ void traverse_pairs_q(const QNode<D> *__restrict__ nodes, const TreeHeader &h,
                                                 int n_nodes, int p, const P &pred, ShortStack<int> &st, F &f)
{
    if (p >= h.start + h.n - 1)
        return;
    float flo[D], fsc[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        flo[d] = h.lo[d];
        fsc[d] = h.qscale[d];
    }
    int cur = h.root;
    for (int iter = 0; iter <= n_nodes; ++iter) {
        if ((unsigned)cur >= (unsigned)n_nodes)
            break;
        QNode<D> nd;
        load_qnode(nodes, cur, nd);
        float lo[2][D], hi[2][D];
        qboxes<D>(nd, true, flo, fsc, lo, hi);
        const int c0 = nd.child[0], c1 = nd.child[1];
        float d0, d1;
        const bool h0 = cur > p && pred.hit(lo[0], hi[0], d0);
        const bool h1 = (c1 >= 0 || cur + 1 > p) && pred.hit(lo[1], hi[1], d1);
        if (h0 && c0 < 0 && c0 != kEmptyRef)
            f(cur, ~c0, d0);
        if (h1 && c1 < 0 && c1 != kEmptyRef)
            f(cur + 1, ~c1, d1);
        const bool g0 = h0 && c0 >= 0;
        const bool g1 = h1 && c1 >= 0;
        if (g0) {
            if (g1)
                st.push(c1);
            cur = c0;
        } else if (g1) {
            cur = c1;
        } else {
            if (st.empty())
                break;
            cur = st.pop();
        }
    }
}

// One term of the fixed-point distance sum: trunc(sqrtf(d2) * scale), scale
// a power of two.
__device__ __forceinline__ long long fixed_term(float d2, float scale)
{
    const float dist = sqrtf(d2);       // correctly rounded
    const float scaled = dist * scale;  // exact: scale is a power of two
    return (long long)(unsigned long long)scaled;  // scaled >= 0: the unsigned conversion is shorter
}

// Store x in slot k of buf (k < C), with static indices only.
template <int C, typename T>
__device__ __forceinline__ void append_at(T (&buf)[C], int k, T x)
{
#pragma unroll
    for (int s = 0; s < C; ++s)
        buf[s] = s == k ? x : buf[s];
}

// Ascending bitonic sorting network over C (a power of two) registers.
template <int C, typename T>
__device__ __forceinline__ void sort_network(T (&v)[C])
{
#pragma unroll
    for (int k = 2; k <= C; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
            for (int i = 0; i < C; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const T a = v[i], b = v[l];
                    const bool up = (i & k) == 0;
                    const T lo = a < b ? a : b, hi = a < b ? b : a;
                    v[i] = up ? lo : hi;
                    v[l] = up ? hi : lo;
                }
            }
}

struct KnnEntry {
    int32_t ref;
    float d2;
};

// The K best (distance, index) pairs of one query in ascending order, each
// packed as one 64-bit key: the float32 bits of a distance >= 0 order like the
// distance itself, so comparing keys compares distances first and breaks ties
// by the smaller index, with no mask arithmetic.  An empty slot holds index
// INT32_MAX.
template <int K>
struct TopK {
    uint64_t key[K];

    __device__ static __forceinline__ uint64_t pack(float d, int id)
    {
        return ((uint64_t)__float_as_uint(d) << 32) | (uint32_t)id;
    }
    __device__ __forceinline__ void reset(float bound)
    {
#pragma unroll
        for (int s = 0; s < K; ++s)
            key[s] = pack(bound, INT32_MAX);
    }
    // distance of the K-th best: a box farther than this cannot contribute
    __device__ __forceinline__ float bound() const { return __uint_as_float((uint32_t)(key[K - 1] >> 32)); }
    // Insertion from the back: the new key displaces the last slot and moves
    // left past larger keys.  A candidate that gets in usually ranks near the
    // end, so the walk stops as soon as no lane of the wavefront still moves.
    __device__ __forceinline__ void offer(float d, int id)
    {
        const uint64_t v = pack(d, id);
        bool moving = v < key[K - 1];
        if (!moving)
            return;
#pragma unroll
        for (int s = K - 1; s > 0; --s) {
            const uint64_t prev = key[s - 1];
            const bool shift = moving && v < prev;
            key[s] = shift ? prev : (moving ? v : key[s]);
            moving = shift;
            if (__ballot(moving) == 0)
                return;
        }
        if (moving)
            key[0] = v;
    }
    // Write the first k_out, indices relative to `base`; empty slots become (+inf, -1).
    __device__ __forceinline__ void store(int k_out, float *d2, int32_t *idx, int base) const
    {
#pragma unroll
        for (int s = 0; s < K; ++s) {
            if (s < k_out) {
                const int id = (int)(uint32_t)key[s];
                const bool empty = id == INT32_MAX;
                d2[s] = empty ? INFINITY : __uint_as_float((uint32_t)(key[s] >> 32));
                idx[s] = empty ? -1 : id - base;
            }
        }
    }
};

// Squared distance from q to the value stored in leaf record `pos`.
template <int D>
__device__ __forceinline__ float leaf_d2(const float *__restrict__ leaves, int kind, int64_t pos, const float *q)
{
    const float *lf = leaves + pos * leaf_floats(D, kind);
    float lo[D], hi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = lf[d];
        hi[d] = kind == ARBORX_BOXES ? lf[D + d] : lf[d];
    }
    return box_d2<D>(q, lo, hi);
}

// Sorted leaf keys a kNN seed searches for the query's position: a tree's
// Morton codes (no prefix, 63/D bits per dimension), or a forest's keys, whose
// segment for tree t holds (t << mbits) | the tree-local code (mbits/D bits per
// dimension, on that tree's bounds).  Without codes a greedy descent finds the
// position.
struct SeedKeys {
    const uint64_t *codes = nullptr;
    uint64_t prefix = 0;
    int bits = 0;
};

// Position of q among the sorted leaves of the tree of hdr: the first leaf
// whose key (the build's, on the tree's bounds) is not below q's, found by
// binary search over the tree's segment of the keys, clamped to the tree.
template <int D>
__device__ __forceinline__ int leaf_position(const SeedKeys &keys, const TreeHeader &hdr, const float *q)
{
    uint32_t c[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const float ext = hdr.hi[d] - hdr.lo[d];
        c[d] = quantise(q[d], hdr.lo[d], ext > 0.0f ? 1.0f / ext : 0.0f, keys.bits);
    }
    const uint64_t key = keys.prefix | interleave<D>(c, keys.bits);
    const uint64_t *__restrict__ codes = keys.codes;
    int lo = hdr.start, hi = hdr.start + hdr.n;  // first code >= key in [lo, hi)
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (codes[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < hdr.start + hdr.n ? lo : hdr.start + hdr.n - 1;
}

// Width of the register window that selects the mode-0 seed bound: the
// smallest power of two holding 2K distances.
template <int K>
constexpr int seed_width()
{
    int w = 1;
    while (w < 2 * K)
        w <<= 1;
    return w;
}

// Bitonic compare-exchange network on register words, fully unrolled so
// that every index is a compile-time constant: sorts v[LO .. LO + N) (N a
// power of two) ascending if UP, else descending.  The words are the bit
// patterns of distances >= 0 (or NaN), which order as unsigned integers like
// the distances, NaN after +inf.
template <int W, int LO, int N, bool UP>
__device__ __forceinline__ void bitonic_sort_range(uint32_t (&v)[W])
{
#pragma unroll
    for (int k = 2; k <= N; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const bool asc = ((i & k) == 0) == UP;
                    const uint32_t a = v[LO + i], b = v[LO + l];
                    const uint32_t mn = a < b ? a : b, mx = a < b ? b : a;
                    v[LO + i] = asc ? mn : mx;
                    v[LO + l] = asc ? mx : mn;
                }
            }
}

// Starting bound for the kNN walk from the sorted leaves around position pos
// (where a greedy descent towards q ends).  mode 0: the k-th smallest distance
// among the 2k leaves around pos; mode 2: the largest distance among the k
// leaves around pos (a looser bound).  Either is at least the true k-th
// neighbour distance, so the slots start as k copies of (bound, INT32_MAX),
// which admit every true result.  Needs n >= k.
//
// For k <= 16 the k-th smallest of the window is selected in registers with a
// sorting network (the distances' bit patterns sorted as unsigned words);
// when the window is exactly 2k wide only its two halves are sorted, one up
// and one down: the elementwise minima of the halves are then the k smallest
// of the window, so their maximum is the k-th smallest.
template <int D, int K>
__device__ __forceinline__ void seed_window(const float *__restrict__ leaves, int kind, const TreeHeader &hdr, int pos,
                                            const float *q, TopK<K> &best, int mode)
{
    const int lo_lim = hdr.start, hi_lim = hdr.start + hdr.n;
    if (mode == 2) {
        int w0 = pos - K / 2;
        w0 = w0 > hi_lim - K ? hi_lim - K : w0;
        w0 = w0 < lo_lim ? lo_lim : w0;
        float b = 0.0f;
#pragma unroll 4
        for (int p = w0; p < w0 + K; ++p)
            b = fmaxf(b, leaf_d2<D>(leaves, kind, p, q));
        best.reset(b);
        return;
    }
    int w0 = pos - K;
    w0 = w0 > hi_lim - 2 * K ? hi_lim - 2 * K : w0;
    w0 = w0 < lo_lim ? lo_lim : w0;
    const int w1 = (w0 + 2 * K < hi_lim) ? w0 + 2 * K : hi_lim;
    if constexpr (K <= 16) {
        constexpr int W = seed_width<K>();
        constexpr uint32_t kInfBits = 0x7f800000u;
        uint32_t v[W];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const int p = w0 + i;
            v[i] = (i < 2 * K && p < w1) ? __float_as_uint(leaf_d2<D>(leaves, kind, p, q)) : kInfBits;
        }
        uint32_t kth;
        if constexpr (W == 2 * K && K > 1) {
            bitonic_sort_range<W, 0, K, true>(v);
            bitonic_sort_range<W, K, K, false>(v);
            kth = 0;
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const uint32_t mn = v[i] < v[K + i] ? v[i] : v[K + i];
                kth = mn > kth ? mn : kth;
            }
        } else {
            bitonic_sort_range<W, 0, W, true>(v);
            kth = v[K - 1];
        }
        best.reset(__uint_as_float(kth < kInfBits ? kth : kInfBits));
        return;
    }
    for (int p = w0; p < w1; ++p)
        best.offer(leaf_d2<D>(leaves, kind, p, q), p);  // distinct keys; only distances matter
    best.reset(best.bound());
}

// Seeding of a kNN walk: the query's position in the tree's sorted leaves
// (binary search over the kept leaf keys, a tree's codes or its segment of a
// forest's keys, or a greedy nearer-child descent when there are none); the K-th smallest distance among the 2K leaves around
// it bounds the K-th nearest distance from above, so the walk starts with that
// bound instead of +inf.  The heap then starts as K copies of
// (bound, INT32_MAX): every value at distance < bound, or == bound, orders
// before them, so all true results are still admitted, and none of the
// placeholders survive when the tree has at least K values.
template <int D, int K>
__device__ __forceinline__ void knn_seed(const Node<D> *__restrict__ nodes, int n_nodes,
                                         const float *__restrict__ leaves, int kind, const TreeHeader &hdr,
                                         const float *q, TopK<K> &best, int seed, const SeedKeys &keys)
{
    const int n = hdr.n;
    best.reset(INFINITY);
    if (seed != 1 && n >= K) {
        int cur = keys.codes ? -1 : hdr.root, pos = keys.codes ? leaf_position<D>(keys, hdr, q) : hdr.start;
        for (int iter = 0; iter <= n_nodes; ++iter) {
            if ((unsigned)cur >= (unsigned)n_nodes)
                break;
            Node<D> nd;
            load_node(nodes, cur, nd);
            const float d0 = box_d2<D>(q, nd.lo[0], nd.hi[0]);
            const float d1 = box_d2<D>(q, nd.lo[1], nd.hi[1]);
            const int go = d1 < d0 ? 1 : 0;
            const int c = go ? nd.child[1] : nd.child[0];
            if (c < 0) {
                pos = cur + go;  // node cur separates sorted leaves cur and cur + 1
                break;
            }
            cur = c;
        }
        // window of 2K leaves around pos inside [start, start + n)
        seed_window<D, K>(leaves, kind, hdr, pos, q, best, seed);
    }
}

// Nearest-first walk keeping the K best (d2, index) pairs sorted in
// registers; a subtree is skipped only if its box is strictly farther than the
// current K-th pair, so equal-distance values with smaller indices are found.
// Software-pipelined: the next node is chosen from the current node's box
// distances and the bound before this node's leaves are offered (a bound that
// can only be looser, so nothing is lost), its fetch is issued, and the leaf
// insertions and the stack push run while it is in flight.
template <int D, int K>
__device__ __forceinline__ void knn_search(const Node<D> *__restrict__ nodes, int n_nodes,
                                           const float *__restrict__ leaves, int kind, const TreeHeader &hdr,
                                           const float *q, TopK<K> &best, ShortStack<KnnEntry> &st, int seed,
                                           const SeedKeys &keys, int *visits = nullptr)
{
    knn_seed<D, K>(nodes, n_nodes, leaves, kind, hdr, q, best, seed, keys);
    if (hdr.n <= 0)
        return;
    int cur = hdr.root;
    Node<D> nd;
    if ((unsigned)cur < (unsigned)n_nodes)
        load_node(nodes, cur, nd);
    for (int iter = 0; iter <= n_nodes; ++iter) {
        if ((unsigned)cur >= (unsigned)n_nodes)
            break;
        if (visits)  // node fetches, for the walk statistics of the debug entry point
            ++*visits;
        const float d0 = box_d2<D>(q, nd.lo[0], nd.hi[0]);
        const float d1 = box_d2<D>(q, nd.lo[1], nd.hi[1]);
        const int c0 = nd.child[0], c1 = nd.child[1];
        const float bound = best.bound();
        const bool k0 = c0 >= 0 && !(d0 > bound);
        const bool k1 = c1 >= 0 && !(d1 > bound);
        int next = -1;
        if (k0 && k1) {
            const bool near1 = d1 < d0;
            st.push(near1 ? KnnEntry{c0, d0} : KnnEntry{c1, d1});
            next = near1 ? c1 : c0;
        } else if (k0) {
            next = c0;
        } else if (k1) {
            next = c1;
        } else {
            while (!st.empty()) {
                const KnnEntry e = st.pop();
                if (!(e.d2 > bound)) {
                    next = e.ref;
                    break;
                }
            }
        }
        if ((unsigned)next < (unsigned)n_nodes)
            load_node(nodes, next, nd);  // in flight during the insertions below
        if (c0 < 0 && c0 != kEmptyRef)
            best.offer(d0, ~c0);
        if (c1 < 0 && c1 != kEmptyRef)
            best.offer(d1, ~c1);
        cur = next;
    }
}

// Order two (distance, reference, admitted) candidates so that the first is
// the farther admitted one; candidates not admitted go last.
__device__ __forceinline__ void far_first(float &da, int &ra, bool &ka, float &db, int &rb, bool &kb)
{
    const bool swap = (kb && !ka) || (ka && kb && db > da);
    const float td = da;
    const int tr = ra;
    const bool tk = ka;
    da = swap ? db : da;
    ra = swap ? rb : ra;
    ka = swap ? kb : ka;
    db = swap ? td : db;
    rb = swap ? tr : rb;
    kb = swap ? tk : kb;
}

// kNN over four-wide nodes: leaf slots are offered; admitted internal slots
// are sorted farthest first, the nearest is entered and the others are pushed
// with their distances (the nearest of them on top).  Seeding as knn_search,
// on the binary nodes.
template <int D, int K>
__device__ __forceinline__ void knn_search4(const Node<D> *__restrict__ nodes, const Node4<D> *__restrict__ wnodes,
                                            int n_nodes, const float *__restrict__ leaves, int kind,
                                            const TreeHeader &hdr, const float *q, TopK<K> &best,
                                            ShortStack<KnnEntry> &st, int seed, const SeedKeys &keys)
{
    const int n = hdr.n;
    best.reset(INFINITY);
    if (n <= 0)
        return;
    if (seed != 1 && n >= K) {
        int cur = keys.codes ? -1 : hdr.root, pos = keys.codes ? leaf_position<D>(keys, hdr, q) : hdr.start;
        for (int iter = 0; iter <= n_nodes; ++iter) {
            if ((unsigned)cur >= (unsigned)n_nodes)
                break;
            Node<D> nd;
            load_node(nodes, cur, nd);
            const float d0 = box_d2<D>(q, nd.lo[0], nd.hi[0]);
            const float d1 = box_d2<D>(q, nd.lo[1], nd.hi[1]);
            const int go = d1 < d0 ? 1 : 0;
            const int c = go ? nd.child[1] : nd.child[0];
            if (c < 0) {
                pos = cur + go;
                break;
            }
            cur = c;
        }
        seed_window<D, K>(leaves, kind, hdr, pos, q, best, seed);
    }
    int cur = hdr.root;
    for (int iter = 0; iter <= n_nodes; ++iter) {
        if ((unsigned)cur >= (unsigned)n_nodes)
            break;
        Node4<D> nd;
        load_node4(wnodes, cur, nd);
        float d[4];
        int r[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            d[s] = box_d2<D>(q, nd.lo[s], nd.hi[s]);
            r[s] = nd.child[s];
            if (r[s] < 0 && r[s] != kEmptyRef)
                best.offer(d[s], ~r[s]);
        }
        const float bound = best.bound();
        bool k[4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
            k[s] = r[s] >= 0 && !(d[s] > bound);
        // sorting network on four: farthest admitted first, not admitted last
        far_first(d[0], r[0], k[0], d[1], r[1], k[1]);
        far_first(d[2], r[2], k[2], d[3], r[3], k[3]);
        far_first(d[0], r[0], k[0], d[2], r[2], k[2]);
        far_first(d[1], r[1], k[1], d[3], r[3], k[3]);
        far_first(d[1], r[1], k[1], d[2], r[2], k[2]);
        int next = -1;
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if (k[s]) {
                if (next >= 0)
                    st.push(KnnEntry{next, d[s - 1 >= 0 ? s - 1 : 0]});
                next = r[s];
            }
        if (next < 0) {
            while (!st.empty()) {
                const KnnEntry e = st.pop();
                if (!(e.d2 > best.bound())) {
                    next = e.ref;
                    break;
                }
            }
        }
        cur = next;
    }
}

__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1)
        v = fminf(v, __shfl_xor(v, o, kWave));
    return v;
}

// Wavefront-packet kNN walk (single tree: every lane shares the root).  Each
// lane keeps its own top-K and bound; a child is entered when some lane's
// bound admits it.  The nearer child for most lanes goes first; the deferred
// child is stored with the smallest distance any lane has to it, and is
// skipped at pop time only when that distance exceeds every lane's bound.
// Seeding (per lane) is as in knn_search.
template <int D, int K>
__device__ __forceinline__ void knn_search_wave(const Node<D> *__restrict__ nodes, int n_nodes,
                                                const float *__restrict__ leaves, int kind, const TreeHeader &hdr,
                                                const float *q, bool active, TopK<K> &best,
                                                KnnEntry *wstack, int seed)
{
    const int n = hdr.n;
    best.reset(INFINITY);
    if (n <= 0)
        return;
    if (active && seed != 1 && n >= K) {
        int cur = hdr.root, pos = hdr.start;
        for (int iter = 0; iter <= n_nodes; ++iter) {
            if ((unsigned)cur >= (unsigned)n_nodes)
                break;
            Node<D> nd;
            load_node(nodes, cur, nd);
            const float d0 = box_d2<D>(q, nd.lo[0], nd.hi[0]);
            const float d1 = box_d2<D>(q, nd.lo[1], nd.hi[1]);
            const int go = d1 < d0 ? 1 : 0;
            const int c = go ? nd.child[1] : nd.child[0];
            if (c < 0) {
                pos = cur + go;
                break;
            }
            cur = c;
        }
        seed_window<D, K>(leaves, kind, hdr, pos, q, best, seed);
    }
    int sp = 0;
    int cur = hdr.root;
    for (int iter = 0; iter <= n_nodes; ++iter) {
        cur = __builtin_amdgcn_readfirstlane(cur);
        if ((unsigned)cur >= (unsigned)n_nodes)
            break;
        Node<D> nd;
        load_node(nodes, cur, nd);
        const float d0 = box_d2<D>(q, nd.lo[0], nd.hi[0]);
        const float d1 = box_d2<D>(q, nd.lo[1], nd.hi[1]);
        const int c0 = nd.child[0], c1 = nd.child[1];
        if (active && c0 < 0 && c0 != kEmptyRef)
            best.offer(d0, ~c0);
        if (active && c1 < 0 && c1 != kEmptyRef)
            best.offer(d1, ~c1);
        const bool k0 = active && c0 >= 0 && !(d0 > best.bound());
        const bool k1 = active && c1 >= 0 && !(d1 > best.bound());
        const bool any0 = __ballot(k0) != 0, any1 = __ballot(k1) != 0;
        if (any0 && any1) {
            const bool want1 = (k0 || k1) && d1 < d0;
            const bool want0 = (k0 || k1) && !(d1 < d0);
            const bool first1 = __popcll(__ballot(want1)) > __popcll(__ballot(want0));
            const int far = first1 ? c0 : c1;
            const float dfar = wave_min(first1 ? (k0 ? d0 : INFINITY) : (k1 ? d1 : INFINITY));
            if (sp < kWaveStack)
                wstack[sp] = KnnEntry{far, dfar};
            ++sp;
            cur = first1 ? c1 : c0;
        } else if (any0) {
            cur = c0;
        } else if (any1) {
            cur = c1;
        } else {
            cur = -1;
            while (sp > 0) {
                --sp;
                const KnnEntry e = sp < kWaveStack ? wstack[sp] : KnnEntry{-1, INFINITY};
                if (__ballot(active && !(e.d2 > best.bound())) != 0) {
                    cur = e.ref;
                    break;
                }
            }
            if (cur < 0)
                break;
        }
    }
}

// kNN over quantized nodes: as knn_search (seeded, software-pipelined),
// pruning with the decoded (larger) internal boxes.  A point tree's leaves are
// offered with their exact distances from the node; a box tree's leaves that
// pass the bound are offered from their records.
template <int D, int K>
__device__ __forceinline__ void knn_search_q(const QNode<D> *__restrict__ nodes, int n_nodes,
                                             const float *__restrict__ leaves, int kind, const TreeHeader &hdr,
                                             const float *q, TopK<K> &best, ShortStack<KnnEntry> &st,
                                             int seed, const SeedKeys &keys)
{
    const int n = hdr.n;
    best.reset(INFINITY);
    if (n <= 0)
        return;
    const bool points = kind != ARBORX_BOXES;
    float flo[D], fsc[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        flo[d] = hdr.lo[d];
        fsc[d] = hdr.qscale[d];
    }
    if (seed != 1 && n >= K) {
        int cur = keys.codes ? -1 : hdr.root, pos = keys.codes ? leaf_position<D>(keys, hdr, q) : hdr.start;
        for (int iter = 0; iter <= n_nodes; ++iter) {
            if ((unsigned)cur >= (unsigned)n_nodes)
                break;
            QNode<D> nd;
            load_qnode(nodes, cur, nd);
            float lo[2][D], hi[2][D];
            qboxes<D>(nd, points, flo, fsc, lo, hi);
            const float d0 = box_d2<D>(q, lo[0], hi[0]);
            const float d1 = box_d2<D>(q, lo[1], hi[1]);
            const int go = (d1 < d0 && nd.child[1] != kEmptyRef) ? 1 : 0;
            const int c = go ? nd.child[1] : nd.child[0];
            if (c < 0) {
                pos = cur + go;  // node cur separates sorted leaves cur and cur + 1
                break;
            }
            cur = c;
        }
        seed_window<D, K>(leaves, kind, hdr, pos, q, best, seed);
    }
    int cur = hdr.root;
    QNode<D> nd;
    if ((unsigned)cur < (unsigned)n_nodes)
        load_qnode(nodes, cur, nd);
    for (int iter = 0; iter <= n_nodes; ++iter) {
        if ((unsigned)cur >= (unsigned)n_nodes)
            break;
        float lo[2][D], hi[2][D];
        qboxes<D>(nd, points, flo, fsc, lo, hi);
        const float d0 = box_d2<D>(q, lo[0], hi[0]);
        const float d1 = box_d2<D>(q, lo[1], hi[1]);
        const int c0 = nd.child[0], c1 = nd.child[1];
        const float bound = best.bound();
        const bool k0 = c0 >= 0 && !(d0 > bound);
        const bool k1 = c1 >= 0 && !(d1 > bound);
        int next = -1;
        if (k0 && k1) {
            const bool near1 = d1 < d0;
            st.push(near1 ? KnnEntry{c0, d0} : KnnEntry{c1, d1});
            next = near1 ? c1 : c0;
        } else if (k0) {
            next = c0;
        } else if (k1) {
            next = c1;
        } else {
            while (!st.empty()) {
                const KnnEntry e = st.pop();
                if (!(e.d2 > bound)) {
                    next = e.ref;
                    break;
                }
            }
        }
        if ((unsigned)next < (unsigned)n_nodes)
            load_qnode(nodes, next, nd);  // in flight during the insertions below
        if (points) {
            if (c0 < 0 && c0 != kEmptyRef)
                best.offer(d0, ~c0);
            if (c1 < 0 && c1 != kEmptyRef)
                best.offer(d1, ~c1);
        } else {
            const int lf = leaf_floats(D, kind);
            if (c0 < 0 && c0 != kEmptyRef && !(d0 > best.bound()))
                best.offer(leaf_d2<D>(leaves, kind, ~c0, q), __float_as_int(leaves[(int64_t)(~c0) * lf + 2 * D]));
            if (c1 < 0 && c1 != kEmptyRef && !(d1 > best.bound()))
                best.offer(leaf_d2<D>(leaves, kind, ~c1, q), __float_as_int(leaves[(int64_t)(~c1) * lf + 2 * D]));
        }
        cur = next;
    }
}

}  // namespace
}  // namespace ax
