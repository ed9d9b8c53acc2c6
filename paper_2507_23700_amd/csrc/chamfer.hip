// Chamfer loss of nearest-neighbour pairs between point clouds, and its gradient.
//
// Pair p holds clouds A_p and B_p (3D).  The forward pass puts all 2P clouds in
// one forest (trees 0..P-1 are A_0..A_{P-1}, trees P..2P-1 are B_0..B_{P-1}) and
// answers one k = 1 nearest query per point against the other cloud of its pair
// (the nearest predicate of Section 2.1 with ties to the smaller index):
//   L_p = sum_i |a_i - b_nn(i)|^2 + sum_j |b_j - a_nn(j)|^2,
// float32 squared distances summed in float64.  With the assignment held fixed
// the gradient is
//   dL/da_i = 2 (a_i - b_nn(i)) + sum_{j : nn(j) = i} 2 (a_i - b_j),
// and symmetrically for b; the backward pass evaluates it in float64 from the
// float32 coordinates, one thread per point: a first pass stores each point's
// own term, a second scatters the reverse terms with float64 atomics, and the
// result is rounded once to float32.
#include <vector>

#include "device_util.hpp"
#include "internal.hpp"
#include "profile.hpp"

namespace ax {
namespace {

__device__ __forceinline__ int pair_of(const int64_t *__restrict__ off, int P, int64_t i)
{
    int lo = 0, hi = P;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= i)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// One workgroup per pair: loss[p] = sum of the pair's nearest squared distances (float64).
__global__ __launch_bounds__(256) void k_pair_loss(const float *__restrict__ d2, const int32_t *__restrict__ idx,
                                                   const int64_t *__restrict__ seg, int P, float *__restrict__ loss)
{
    __shared__ double wsum[256 / kWave];
    const int p = blockIdx.x;
    double s = 0.0;
    for (int part = 0; part < 2; ++part) {
        const int t = part == 0 ? p : P + p;
        for (int64_t i = seg[t] + threadIdx.x; i < seg[t + 1]; i += blockDim.x)
            if (idx[i] >= 0)
                s += (double)d2[i];
    }
    s = wave_sum(s);
    if (lane_id() == 0)
        wsum[wave_id()] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < 256 / kWave; ++w)
            tot += wsum[w];
        loss[p] = (float)tot;
    }
}

// The term of point i of one side (src, offsets soff) with its nearest
// neighbour in the other side (dst, doff): 2 g (x_i - y_nn(i)), or 0.
__device__ __forceinline__ bool own_term(const float *__restrict__ src, const int64_t *__restrict__ soff,
                                         const float *__restrict__ dst, const int64_t *__restrict__ doff,
                                         const int32_t *__restrict__ nn, const float *__restrict__ grad_loss, int P,
                                         int64_t i, double (&t)[3], int64_t &jj)
{
    t[0] = t[1] = t[2] = 0.0;
    const int32_t j = nn[i];
    if (j < 0)
        return false;
    const int p = pair_of(soff, P, i);
    jj = doff[p] + j;
    if (jj >= doff[p + 1])
        return false;
    const double g2 = 2.0 * (double)grad_loss[p];
#pragma unroll
    for (int d = 0; d < 3; ++d)
        t[d] = g2 * ((double)src[i * 3 + d] - (double)dst[jj * 3 + d]);
    return true;
}

// First pass: g_src[i] = 2 g (x_i - y_nn(i)), a plain store per point.
__global__ void k_chamfer_own(const float *__restrict__ src, const int64_t *__restrict__ soff, int64_t ns,
                              const float *__restrict__ dst, const int64_t *__restrict__ doff,
                              const int32_t *__restrict__ nn, const float *__restrict__ grad_loss, int P,
                              double *__restrict__ gsrc)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
        double t[3];
        int64_t jj = 0;
        own_term(src, soff, dst, doff, nn, grad_loss, P, i, t, jj);
#pragma unroll
        for (int d = 0; d < 3; ++d)
            gsrc[i * 3 + d] = t[d];
    }
}

// Second pass, after both first passes: g_dst[nn(i)] -= 2 g (x_i - y_nn(i)).
__global__ void k_chamfer_reverse(const float *__restrict__ src, const int64_t *__restrict__ soff, int64_t ns,
                                  const float *__restrict__ dst, const int64_t *__restrict__ doff,
                                  const int32_t *__restrict__ nn, const float *__restrict__ grad_loss, int P,
                                  double *__restrict__ gdst)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
        double t[3];
        int64_t jj = 0;
        if (own_term(src, soff, dst, doff, nn, grad_loss, P, i, t, jj))
#pragma unroll
            for (int d = 0; d < 3; ++d)
                atomicAdd(&gdst[jj * 3 + d], -t[d]);
    }
}

__global__ void k_to_float(const double *__restrict__ x, int64_t n, float *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (float)x[i];
}

__global__ void k_copy_i32(const int32_t *__restrict__ x, int64_t n, int32_t *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = x[i];
}

}  // namespace

arborx_status chamfer_forward(const float *a, const int64_t *a_off, const float *b, const int64_t *b_off, int P,
                              float *loss, int32_t *nn_ab, int32_t *nn_ba, hipStream_t s)
{
    const int64_t na = a_off[P], nb = b_off[P], n = na + nb;
    std::vector<int64_t> seg(2 * P + 1);
    std::vector<int32_t> btree(2 * P);
    for (int p = 0; p <= P; ++p) {
        seg[p] = a_off[p];
        seg[P + p] = na + b_off[p];
    }
    for (int p = 0; p < P; ++p) {
        btree[p] = P + p;  // A_p queries search B_p
        btree[P + p] = p;  // B_p queries search A_p
    }
    Temps tmp(s);
    float *pts, *d2;
    int32_t *idx, *dbt;
    arborx_status st;
    if ((st = tmp.get(&pts, (size_t)3 * (n > 0 ? n : 1))) != ARBORX_OK || (st = tmp.get(&d2, n > 0 ? n : 1)) != ARBORX_OK ||
        (st = tmp.get(&idx, n > 0 ? n : 1)) != ARBORX_OK || (st = tmp.get(&dbt, 2 * P)) != ARBORX_OK)
        return st;
    if (na > 0)
        AX_HIP(hipMemcpyAsync(pts, a, 12 * na, hipMemcpyDeviceToDevice, s));
    if (nb > 0)
        AX_HIP(hipMemcpyAsync(pts + 3 * na, b, 12 * nb, hipMemcpyDeviceToDevice, s));
    AX_HIP(hipMemcpyAsync(dbt, btree.data(), 4 * 2 * P, hipMemcpyHostToDevice, s));
    ForestDev f;
    st = build_forest(pts, seg.data(), 2 * P, 3, ARBORX_POINTS, f, s);
    if (st == ARBORX_OK)
        st = forest_query_knn(f, pts, n, f.seg, dbt, 2 * P, 1, d2, idx, s);
    if (st == ARBORX_OK) {
        ProfScope ps("chamfer_loss", s);
        k_pair_loss<<<P, 256, 0, s>>>(d2, idx, f.seg, P, loss);
        if (na > 0)
            k_copy_i32<<<grid_for(na, 256, 65536), 256, 0, s>>>(idx, na, nn_ab);
        if (nb > 0)
            k_copy_i32<<<grid_for(nb, 256, 65536), 256, 0, s>>>(idx + na, nb, nn_ba);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            st = hip_fail(e, "chamfer loss");
    }
    forest_release(f, s);
    return st;
}

arborx_status chamfer_backward(const float *a, const int64_t *a_off, const float *b, const int64_t *b_off, int P,
                               const int32_t *nn_ab, const int32_t *nn_ba, const float *grad_loss, float *grad_a,
                               float *grad_b, hipStream_t s)
{
    const int64_t na = a_off[P], nb = b_off[P];
    Temps tmp(s);
    double *ga, *gb;
    int64_t *aoff, *boff;
    arborx_status st;
    if ((st = tmp.get(&ga, (size_t)3 * (na > 0 ? na : 1))) != ARBORX_OK ||
        (st = tmp.get(&gb, (size_t)3 * (nb > 0 ? nb : 1))) != ARBORX_OK ||
        (st = tmp.get(&aoff, P + 1)) != ARBORX_OK || (st = tmp.get(&boff, P + 1)) != ARBORX_OK)
        return st;
    AX_HIP(hipMemcpyAsync(aoff, a_off, 8 * (P + 1), hipMemcpyHostToDevice, s));
    AX_HIP(hipMemcpyAsync(boff, b_off, 8 * (P + 1), hipMemcpyHostToDevice, s));
    ProfScope ps("chamfer_backward", s);
    if (na > 0)
        k_chamfer_own<<<grid_for(na, 256, 65536), 256, 0, s>>>(a, aoff, na, b, boff, nn_ab, grad_loss, P, ga);
    if (nb > 0)
        k_chamfer_own<<<grid_for(nb, 256, 65536), 256, 0, s>>>(b, boff, nb, a, aoff, nn_ba, grad_loss, P, gb);
    if (na > 0)
        k_chamfer_reverse<<<grid_for(na, 256, 65536), 256, 0, s>>>(a, aoff, na, b, boff, nn_ab, grad_loss, P, gb);
    if (nb > 0)
        k_chamfer_reverse<<<grid_for(nb, 256, 65536), 256, 0, s>>>(b, boff, nb, a, aoff, nn_ba, grad_loss, P, ga);
    if (na > 0)
        k_to_float<<<grid_for(3 * na, 256, 65536), 256, 0, s>>>(ga, 3 * na, grad_a);
    if (nb > 0)
        k_to_float<<<grid_for(3 * nb, 256, 65536), 256, 0, s>>>(gb, 3 * nb, grad_b);
    AX_HIP(hipGetLastError());
    return ARBORX_OK;
}

}  // namespace ax
