// Stable LSD radix sort of (key, uint32 value) pairs, 8-bit digits.
//
// One pass = four launches:
//   hist    : per 4096-key tile, a 256-bin digit histogram (LDS atomics),
//             stored digit-major so that one scan over [digit][tile] yields
//             every tile's global output offset per digit;
//   totals  : one workgroup per digit sums its row of tile counts;
//   scan    : one workgroup per digit scans its row of tile counts and adds
//             the number of keys with smaller digits;
//   scatter : per tile, keys are ranked stably inside each wavefront with
//             ballots (8 ballots identify the lanes sharing a digit, the
//             popcount of those below a lane is its rank), the tile is
//             reordered by digit in LDS and written out in digit runs, so
//             consecutive lanes write consecutive addresses.
// Sorting is what the paper names as the decisive construction cost (Section
// 2.6: switching to a vendor sort took construction from 17 s to 0.02 s).
#include "device_util.hpp"
#include "internal.hpp"

namespace ax {
namespace {

constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;
constexpr int kTile = kSortBlock * kSortItems;  // keys per tile
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
static_assert(kSortBlock == kRadix, "one thread per digit in the per-tile steps");

template <typename K>
__global__ __launch_bounds__(kSortBlock) void radix_hist(const K *__restrict__ keys, int64_t n, int shift,
                                                         uint32_t mask, uint32_t *__restrict__ tile_hist,
                                                         int num_tiles)
{
    __shared__ uint32_t h[kRadix];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll 4
    for (int j = 0; j < kSortItems; ++j) {
        int64_t i = base + (int64_t)j * kSortBlock + threadIdx.x;
        if (i < n)
            atomicAdd(&h[(uint32_t)(keys[i] >> shift) & mask], 1u);
    }
    __syncthreads();
    tile_hist[(int64_t)threadIdx.x * num_tiles + blockIdx.x] = h[threadIdx.x];
}

// digit_total[d] = sum over tiles of tile_hist[d][t]: one workgroup per digit.
__global__ __launch_bounds__(kSortBlock) void radix_totals(const uint32_t *__restrict__ tile_hist, int num_tiles,
                                                           uint32_t *__restrict__ digit_total)
{
    __shared__ uint32_t wsum[kSortBlock / kWave];
    const uint32_t *row = tile_hist + (int64_t)blockIdx.x * num_tiles;
    uint32_t s = 0;
    for (int i = threadIdx.x; i < num_tiles; i += kSortBlock)
        s += row[i];
    s = wave_sum(s);
    if (lane_id() == 0)
        wsum[wave_id()] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kSortBlock / kWave; ++w)
            t += wsum[w];
        digit_total[blockIdx.x] = t;
    }
}

// In place: tile_hist[d][t] <- (keys with digit < d) + sum_{t' < t} tile_hist[d][t'].
__global__ __launch_bounds__(kSortBlock) void radix_scan(uint32_t *__restrict__ tile_hist,
                                                         const uint32_t *__restrict__ digit_total, int num_tiles)
{
    __shared__ uint32_t wsum[kSortBlock / kWave];
    const int d = blockIdx.x;
    uint32_t base = 0;
    uint32_t v = ((int)threadIdx.x < d) ? digit_total[threadIdx.x] : 0u;
    block_exclusive_scan<kSortBlock>(v, wsum, &base);
    uint32_t carry = base;
    uint32_t *row = tile_hist + (int64_t)d * num_tiles;
    constexpr int PER = 4;
    for (int start = 0; start < num_tiles; start += kSortBlock * PER) {
        const int i0 = start + (int)threadIdx.x * PER;
        uint32_t x[PER];
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            x[k] = (i0 + k < num_tiles) ? row[i0 + k] : 0u;
            s += x[k];
        }
        uint32_t chunk = 0;
        uint32_t run = carry + block_exclusive_scan<kSortBlock>(s, wsum, &chunk);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if (i0 + k < num_tiles)
                row[i0 + k] = run;
            run += x[k];
        }
        carry += chunk;
    }
}

template <typename K>
__global__ __launch_bounds__(kSortBlock) void radix_scatter(const K *__restrict__ keys_in,
                                                            const uint32_t *__restrict__ vals_in,
                                                            K *__restrict__ keys_out, uint32_t *__restrict__ vals_out,
                                                            int64_t n, int shift, uint32_t mask,
                                                            const uint32_t *__restrict__ tile_off, int num_tiles)
{
    constexpr int W = kSortBlock / kWave;  // wavefronts per tile
    constexpr int PER_WAVE = kTile / W;    // contiguous keys per wavefront
    constexpr int ROUNDS = PER_WAVE / kWave;
    __shared__ K s_keys[kTile];
    __shared__ uint32_t s_vals[kTile];
    __shared__ uint32_t s_wcnt[W][kRadix];
    __shared__ uint32_t s_dstart[kRadix];
    __shared__ uint32_t s_goff[kRadix];
    __shared__ uint32_t s_wsum[W];

    const int lane = lane_id(), w = wave_id();
    for (int i = threadIdx.x; i < W * kRadix; i += kSortBlock)
        (&s_wcnt[0][0])[i] = 0;
    s_goff[threadIdx.x] = tile_off[(int64_t)threadIdx.x * num_tiles + blockIdx.x];
    __syncthreads();

    const int64_t tile_base = (int64_t)blockIdx.x * kTile;
    const int64_t wbase = tile_base + (int64_t)w * PER_WAVE;
    const uint64_t lt = lanemask_lt();
    K k[ROUNDS];
    uint32_t v[ROUNDS];
    uint32_t rank[ROUNDS];
#pragma unroll
    for (int j = 0; j < ROUNDS; ++j) {
        const int64_t i = wbase + (int64_t)j * kWave + lane;
        const bool valid = i < n;
        const K key = valid ? keys_in[i] : K(0);
        k[j] = key;
        v[j] = valid ? vals_in[i] : 0u;
        const uint32_t d = (uint32_t)(key >> shift) & mask;
        // lanes of this round holding the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t r = (uint32_t)__popcll(peers & lt);
        uint32_t prior = 0;
        if (valid && r == 0)
            prior = atomicAdd(&s_wcnt[w][d], (uint32_t)__popcll(peers));
        const int leader = valid ? (__ffsll((unsigned long long)peers) - 1) : lane;
        prior = __shfl(prior, leader, kWave);
        rank[j] = prior + r;
    }
    __syncthreads();
    {
        // per digit: exclusive prefix over wavefronts, then over digits
        const int d = threadIdx.x;
        uint32_t run = 0;
#pragma unroll
        for (int ww = 0; ww < W; ++ww) {
            const uint32_t c = s_wcnt[ww][d];
            s_wcnt[ww][d] = run;
            run += c;
        }
        uint32_t tot = 0;
        s_dstart[d] = block_exclusive_scan<kSortBlock>(run, s_wsum, &tot);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ROUNDS; ++j) {
        const int64_t i = wbase + (int64_t)j * kWave + lane;
        if (i < n) {
            const uint32_t d = (uint32_t)(k[j] >> shift) & mask;
            const uint32_t pos = s_dstart[d] + s_wcnt[w][d] + rank[j];
            if (pos < (uint32_t)kTile) {
                s_keys[pos] = k[j];
                s_vals[pos] = v[j];
            }
        }
    }
    __syncthreads();
    const int64_t left = n - tile_base;
    const int tile_n = left < kTile ? (int)left : kTile;
    for (int p = threadIdx.x; p < tile_n; p += kSortBlock) {
        const K key = s_keys[p];
        const uint32_t d = (uint32_t)(key >> shift) & mask;
        const uint32_t g = s_goff[d] + (uint32_t)(p - (int)s_dstart[d]);
        if ((int64_t)g < n) {
            keys_out[g] = key;
            vals_out[g] = s_vals[p];
        }
    }
}

}  // namespace

size_t radix_workspace_bytes(int64_t n)
{
    const int64_t tiles = (n + kTile - 1) / kTile;
    return (size_t)(tiles * kRadix + 8 * kRadix) * sizeof(uint32_t) + 256;
}

template <typename K>
hipError_t radix_sort_pairs(K *keys, uint32_t *vals, K *keys_alt, uint32_t *vals_alt, int64_t n, int begin, int end,
                            void *workspace, hipStream_t s, bool *in_alt)
{
    *in_alt = false;
    if (n <= 1 || end <= begin)
        return hipSuccess;
    if (n > (int64_t)UINT32_MAX)
        return hipErrorInvalidValue;
    const int tiles = (int)((n + kTile - 1) / kTile);
    uint32_t *tile_hist = static_cast<uint32_t *>(workspace);
    uint32_t *totals = tile_hist + (size_t)tiles * kRadix;
    const int passes = (end - begin + kRadixBits - 1) / kRadixBits;
    if (passes > 8)
        return hipErrorInvalidValue;
    K *kin = keys, *kout = keys_alt;
    uint32_t *vin = vals, *vout = vals_alt;
    for (int p = 0; p < passes; ++p) {
        const int shift = begin + p * kRadixBits;
        const int bits = (end - shift) < kRadixBits ? (end - shift) : kRadixBits;
        const uint32_t mask = (1u << bits) - 1u;
        radix_hist<K><<<tiles, kSortBlock, 0, s>>>(kin, n, shift, mask, tile_hist, tiles);
        radix_totals<<<kRadix, kSortBlock, 0, s>>>(tile_hist, tiles, totals + p * kRadix);
        radix_scan<<<kRadix, kSortBlock, 0, s>>>(tile_hist, totals + p * kRadix, tiles);
        radix_scatter<K><<<tiles, kSortBlock, 0, s>>>(kin, vin, kout, vout, n, shift, mask, tile_hist, tiles);
        K *tk = kin;
        kin = kout;
        kout = tk;
        uint32_t *tv = vin;
        vin = vout;
        vout = tv;
    }
    *in_alt = (passes & 1) != 0;
    return hipGetLastError();
}

template hipError_t radix_sort_pairs<uint64_t>(uint64_t *, uint32_t *, uint64_t *, uint32_t *, int64_t, int, int,
                                               void *, hipStream_t, bool *);
template hipError_t radix_sort_pairs<uint32_t>(uint32_t *, uint32_t *, uint32_t *, uint32_t *, int64_t, int, int,
                                               void *, hipStream_t, bool *);

}  // namespace ax
