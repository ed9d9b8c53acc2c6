// Ray predicates over the hierarchy (Section 2.5: rays traced against the
// index's boxes).  A ray is o + t*dir, t >= 0; it meets a closed box when its
// slab intervals overlap (the same float32 slab arithmetic as the oracle, with
// correctly rounded division), and t at entry orders the hits.  The hit count
// is a depth-first walk; the first k hits are a nearest-first walk keeping a
// register top-k ordered by (entry t, index), pruning subtrees entered after
// the k-th hit.  A box inside another is met no earlier, so both prunings are
// exact.
#include "device_util.hpp"
#include "geometry.hpp"
#include "internal.hpp"
#include "profile.hpp"
#include "traverse.hpp"

namespace ax {
namespace {

__device__ __forceinline__ int ray_nodes(const TreeHeader *hdr) { return hdr->n > 1 ? hdr->n - 1 : 1; }

// Thread t answers ray perm[t] (origins in Morton order: neighbouring rays
// start in the same part of the tree), or ray t without an order.
template <int D>
__global__ void k_ray_count(const Node<D> *__restrict__ nodes, const TreeHeader *__restrict__ hdr,
                            const float *__restrict__ rays, int64_t m, const uint32_t *__restrict__ perm,
                            int32_t *__restrict__ counts, int stack_cap)
{
    extern __shared__ int s_stack[];
    const int64_t t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= m)
        return;
    const int64_t i = perm ? (int64_t)perm[t] : t;
    if (i >= m)
        return;
    RayPred<D> p;
    p.load(rays, i, 0.0f);
    int spill[kSpill];
    ShortStack<int> st(s_stack + threadIdx.x, blockDim.x, stack_cap, spill);
    int c = 0;
    auto f = [&](int, float) { ++c; };
    if (hdr->n > 0)
        traverse_spatial<D>(nodes, hdr->root, ray_nodes(hdr), p, st, f);
    counts[i] = c;
}

template <int D, int K>
__global__ void k_ray_nearest(const Node<D> *__restrict__ nodes, const TreeHeader *__restrict__ hdr,
                              const float *__restrict__ rays, int64_t m, const uint32_t *__restrict__ perm, int k_out,
                              float *__restrict__ t_out, int32_t *__restrict__ idx_out, int stack_cap)
{
    extern __shared__ int s_stack[];
    const int64_t t0 = xcd_block() * blockDim.x + threadIdx.x;
    if (t0 >= m)
        return;
    const int64_t i = perm ? (int64_t)perm[t0] : t0;
    if (i >= m)
        return;
    RayPred<D> p;
    p.load(rays, i, 0.0f);
    KnnEntry spill[kSpill];
    ShortStack<KnnEntry> st(reinterpret_cast<KnnEntry *>(s_stack) + threadIdx.x, blockDim.x, stack_cap, spill);
    TopK<K> best;
    best.reset(INFINITY);
    const int n_nodes = ray_nodes(hdr);
    int cur = hdr->n > 0 ? hdr->root : -1;
    for (int iter = 0; iter <= n_nodes; ++iter) {
        if ((unsigned)cur >= (unsigned)n_nodes)
            break;
        Node<D> nd;
        load_node(nodes, cur, nd);
        float t0, t1;
        const bool h0 = p.hit(nd.lo[0], nd.hi[0], t0);
        const bool h1 = p.hit(nd.lo[1], nd.hi[1], t1);
        const int c0 = nd.child[0], c1 = nd.child[1];
        if (h0 && c0 < 0 && c0 != kEmptyRef)
            best.offer(t0, ~c0);
        if (h1 && c1 < 0 && c1 != kEmptyRef)
            best.offer(t1, ~c1);
        const bool k0 = h0 && c0 >= 0 && !(t0 > best.bound());
        const bool k1 = h1 && c1 >= 0 && !(t1 > best.bound());
        if (k0 && k1) {
            if (t1 < t0) {
                st.push(KnnEntry{c0, t0});
                cur = c1;
            } else {
                st.push(KnnEntry{c1, t1});
                cur = c0;
            }
        } else if (k0) {
            cur = c0;
        } else if (k1) {
            cur = c1;
        } else {
            bool found = false;
            while (!st.empty()) {
                const KnnEntry e = st.pop();
                if (!(e.d2 > best.bound())) {
                    cur = e.ref;
                    found = true;
                    break;
                }
            }
            if (!found)
                break;
        }
    }
    best.store(k_out, t_out + i * k_out, idx_out + i * k_out, 0);
}

constexpr int kRayBlock = 64;

template <int D>
arborx_status ray_count_impl(const TreeDev &t, const float *rays, int64_t m, const uint32_t *perm, int32_t *counts,
                             hipStream_t s)
{
    const int cap = 8;
    ProfScope ps("ray_count", s);
    k_ray_count<D><<<(unsigned)((m + kRayBlock - 1) / kRayBlock), kRayBlock, (size_t)cap * kRayBlock * sizeof(int),
                     s>>>(static_cast<const Node<D> *>(t.nodes), t.hdr, rays, m, perm, counts, cap);
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

template <int D, int K>
arborx_status ray_nearest_launch(const TreeDev &t, const float *rays, int64_t m, const uint32_t *perm, int k,
                                 float *t_out, int32_t *idx_out, hipStream_t s)
{
    const int cap = 8;
    ProfScope ps("ray_nearest", s);
    k_ray_nearest<D, K><<<(unsigned)((m + kRayBlock - 1) / kRayBlock), kRayBlock,
                          (size_t)cap * kRayBlock * sizeof(KnnEntry), s>>>(static_cast<const Node<D> *>(t.nodes),
                                                                           t.hdr, rays, m, perm, k, t_out, idx_out,
                                                                           cap);
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

template <int D>
arborx_status ray_nearest_impl(const TreeDev &t, const float *rays, int64_t m, const uint32_t *perm, int k,
                               float *t_out, int32_t *idx_out, hipStream_t s)
{
    if (k <= 1)
        return ray_nearest_launch<D, 1>(t, rays, m, perm, k, t_out, idx_out, s);
    if (k <= 4)
        return ray_nearest_launch<D, 4>(t, rays, m, perm, k, t_out, idx_out, s);
    if (k <= 16)
        return ray_nearest_launch<D, 16>(t, rays, m, perm, k, t_out, idx_out, s);
    return ray_nearest_launch<D, 64>(t, rays, m, perm, k, t_out, idx_out, s);
}

}  // namespace

arborx_status ray_count(const TreeDev &t, const float *rays, int64_t m, const uint32_t *perm, int32_t *counts,
                        hipStream_t s)
{
    if (m == 0)
        return ARBORX_OK;
    switch (t.dim) {
    case 2: return ray_count_impl<2>(t, rays, m, perm, counts, s);
    case 3: return ray_count_impl<3>(t, rays, m, perm, counts, s);
    case 6: return ray_count_impl<6>(t, rays, m, perm, counts, s);
    default: return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in");
    }
}

arborx_status ray_nearest(const TreeDev &t, const float *rays, int64_t m, const uint32_t *perm, int k, float *t_out,
                          int32_t *idx_out, hipStream_t s)
{
    if (m == 0)
        return ARBORX_OK;
    switch (t.dim) {
    case 2: return ray_nearest_impl<2>(t, rays, m, perm, k, t_out, idx_out, s);
    case 3: return ray_nearest_impl<3>(t, rays, m, perm, k, t_out, idx_out, s);
    case 6: return ray_nearest_impl<6>(t, rays, m, perm, k, t_out, idx_out, s);
    default: return fail(ARBORX_E_UNSUPPORTED, "dimension not compiled in");
    }
}

}  // namespace ax
