// Wavefront (64 lanes) and workgroup helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ax {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x / kWave); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v)
{
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T t = __shfl_up(v, o, kWave);
        if (lane >= o)
            v += t;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1)
        v += __shfl_xor(v, o, kWave);
    return v;
}

// Exclusive scan across a workgroup of BLOCK threads.  `wsum` is LDS scratch of
// BLOCK/64 entries.  Returns the exclusive prefix; *total gets the block sum.
// Contains two workgroup barriers; every thread of the block must call it.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *wsum, T *total)
{
    constexpr int W = BLOCK / kWave;
    T inc = wave_inclusive_scan(v);
    if (lane_id() == kWave - 1)
        wsum[wave_id()] = inc;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        T s = wsum[w];
        off += (w < wave_id()) ? s : T(0);
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

template <typename T>
__global__ void fill_kernel(T *p, int64_t n, T v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

template <typename T>
__global__ void iota_kernel(T *p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = (T)i;
}

}  // namespace ax
