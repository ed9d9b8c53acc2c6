// CSR offsets from per-query counts: offsets[0] = 0, offsets[i+1] = offsets[i] + counts[i]
// (the offsets array of the compressed-sparse-row result, Section 2.1).
// Reduce-then-scan over 4096-count tiles: tile sums, one-workgroup scan of the
// tile sums, then each tile scans itself from its prefix.
#include "device_util.hpp"
#include "internal.hpp"

namespace ax {
namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanBlock * kScanItems;

__global__ __launch_bounds__(kScanBlock) void scan_tile_sums(const int32_t *__restrict__ counts, int64_t m,
                                                             int64_t *__restrict__ tile_sums)
{
    __shared__ int64_t wsum[kScanBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
#pragma unroll 4
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + (int64_t)j * kScanBlock + threadIdx.x;
        if (i < m)
            s += counts[i];
    }
    int64_t tot = 0;
    block_exclusive_scan<kScanBlock>(s, wsum, &tot);
    if (threadIdx.x == 0)
        tile_sums[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of the tile sums in place; the grand total goes to *total.
__global__ __launch_bounds__(kScanBlock) void scan_tile_prefix(int64_t *__restrict__ tile_sums, int64_t tiles,
                                                               int64_t *__restrict__ total)
{
    __shared__ int64_t wsum[kScanBlock / kWave];
    int64_t carry = 0;
    for (int64_t start = 0; start < tiles; start += kScanBlock) {
        const int64_t i = start + threadIdx.x;
        const int64_t x = i < tiles ? tile_sums[i] : 0;
        int64_t chunk = 0;
        const int64_t ex = block_exclusive_scan<kScanBlock>(x, wsum, &chunk);
        if (i < tiles)
            tile_sums[i] = carry + ex;
        carry += chunk;
    }
    if (threadIdx.x == 0)
        *total = carry;
}

// Each thread owns kScanItems consecutive counts.
__global__ __launch_bounds__(kScanBlock) void scan_apply(const int32_t *__restrict__ counts, int64_t m,
                                                         const int64_t *__restrict__ tile_prefix,
                                                         int64_t *__restrict__ offsets)
{
    __shared__ int64_t wsum[kScanBlock / kWave];
    const int64_t i0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t c[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        c[j] = (i0 + j < m) ? counts[i0 + j] : 0;
        s += c[j];
    }
    int64_t tot = 0;
    int64_t run = tile_prefix[blockIdx.x] + block_exclusive_scan<kScanBlock>(s, wsum, &tot);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (i0 + j < m)
            offsets[i0 + j] = run;
        run += c[j];
        if (i0 + j == m - 1)
            offsets[m] = run;
    }
}

// CSR offsets plus ordered lists of long rows.  Per tile the scan carries the
// count sum and a packed pair of flag counts (low 32 bits: rows longer than
// `regs` but at most kRowSortBlock; high 32 bits: longer rows), so the
// row ids of both kinds are compacted in row order without atomics.
__device__ __forceinline__ int64_t row_flags(int32_t c, int regs)
{
    return (c > regs && c <= kRowSortBlock) ? 1ll : (c > kRowSortBlock ? (1ll << 32) : 0ll);
}

// counts[i] is row i's length; lcounts[i] is the length of the row listed at
// position i (the same array, or the lengths in traversal order).
__global__ __launch_bounds__(kScanBlock) void csr_tile_sums(const int32_t *__restrict__ counts,
                                                            const int32_t *__restrict__ lcounts, int64_t m, int regs,
                                                            int64_t *__restrict__ tile_sums,
                                                            int64_t *__restrict__ tile_flags)
{
    __shared__ int64_t wsum[kScanBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0, f = 0;
#pragma unroll 4
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + (int64_t)j * kScanBlock + threadIdx.x;
        if (i < m) {
            s += counts[i];
            f += row_flags(lcounts[i], regs);
        }
    }
    int64_t tot = 0, ftot = 0;
    block_exclusive_scan<kScanBlock>(s, wsum, &tot);
    block_exclusive_scan<kScanBlock>(f, wsum, &ftot);
    if (threadIdx.x == 0) {
        tile_sums[blockIdx.x] = tot;
        tile_flags[blockIdx.x] = ftot;
    }
}

__global__ __launch_bounds__(kScanBlock) void csr_tile_prefix(int64_t *__restrict__ tile_sums,
                                                              int64_t *__restrict__ tile_flags, int64_t tiles,
                                                              QueryHeader *__restrict__ qh)
{
    __shared__ int64_t wsum[kScanBlock / kWave];
    int64_t carry = 0, fcarry = 0;
    for (int64_t start = 0; start < tiles; start += kScanBlock) {
        const int64_t i = start + threadIdx.x;
        const int64_t x = i < tiles ? tile_sums[i] : 0;
        const int64_t f = i < tiles ? tile_flags[i] : 0;
        int64_t chunk = 0, fchunk = 0;
        const int64_t ex = block_exclusive_scan<kScanBlock>(x, wsum, &chunk);
        const int64_t fex = block_exclusive_scan<kScanBlock>(f, wsum, &fchunk);
        if (i < tiles) {
            tile_sums[i] = carry + ex;
            tile_flags[i] = fcarry + fex;
        }
        carry += chunk;
        fcarry += fchunk;
    }
    if (threadIdx.x == 0) {
        qh->total = (unsigned long long)carry;
        qh->big_rows = (unsigned long long)(fcarry & 0xffffffffll);
        qh->huge_rows = (unsigned long long)(fcarry >> 32);
    }
}

// Offsets in row order; long rows listed in the order of lcounts, as order[i]
// (the row at position i) or i when order is NULL.
__global__ __launch_bounds__(kScanBlock) void csr_apply(const int32_t *__restrict__ counts,
                                                        const int32_t *__restrict__ lcounts,
                                                        const uint32_t *__restrict__ order, int64_t m, int regs,
                                                        const int64_t *__restrict__ tile_prefix,
                                                        const int64_t *__restrict__ tile_flags,
                                                        int64_t *__restrict__ offsets, int32_t *__restrict__ big_list,
                                                        int32_t *__restrict__ huge_list)
{
    __shared__ int64_t wsum[kScanBlock / kWave];
    const int64_t i0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t c[kScanItems], lc[kScanItems];
    if (i0 + kScanItems <= m) {  // whole chunk: 16-byte loads (i0 is a multiple of kScanItems)
#pragma unroll
        for (int j = 0; j < kScanItems; j += 4) {
            const int4 a = *reinterpret_cast<const int4 *>(counts + i0 + j);
            const int4 b = *reinterpret_cast<const int4 *>(lcounts + i0 + j);
            c[j] = a.x, c[j + 1] = a.y, c[j + 2] = a.z, c[j + 3] = a.w;
            lc[j] = b.x, lc[j + 1] = b.y, lc[j + 2] = b.z, lc[j + 3] = b.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            c[j] = (i0 + j < m) ? counts[i0 + j] : 0;
            lc[j] = (i0 + j < m) ? lcounts[i0 + j] : 0;
        }
    }
    int64_t s = 0, f = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        s += c[j];
        f += row_flags(lc[j], regs);
    }
    int64_t tot = 0, ftot = 0;
    int64_t run = tile_prefix[blockIdx.x] + block_exclusive_scan<kScanBlock>(s, wsum, &tot);
    int64_t frun = tile_flags[blockIdx.x] + block_exclusive_scan<kScanBlock>(f, wsum, &ftot);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = i0 + j;
        if (i < m) {
            offsets[i] = run;
            const int64_t fl = row_flags(lc[j], regs);
            if (fl != 0) {
                const int32_t row = order ? (int32_t)order[i] : (int32_t)i;
                if (fl == 1)
                    big_list[frun & 0xffffffffll] = row;
                else
                    huge_list[frun >> 32] = row;
            }
            frun += fl;
        }
        run += c[j];
        if (i == m - 1)
            offsets[m] = run;
    }
}

__global__ void csr_empty(int64_t *offsets, QueryHeader *qh)
{
    offsets[0] = 0;
    qh->total = 0;
    qh->big_rows = 0;
    qh->huge_rows = 0;
}

__global__ void scan_empty(int64_t *offsets, int64_t *total)
{
    offsets[0] = 0;
    *total = 0;
}

}  // namespace

size_t scan_workspace_bytes(int64_t m) { return (size_t)2 * ((m + kScanTile - 1) / kScanTile + 1) * sizeof(int64_t); }

hipError_t csr_offsets_lists(const int32_t *counts, const int32_t *ordered_counts, const uint32_t *order, int64_t m,
                             int regs, int64_t *offsets, int32_t *big_list, int32_t *huge_list, QueryHeader *qh,
                             void *workspace, hipStream_t s)
{
    if (m == 0) {
        csr_empty<<<1, 1, 0, s>>>(offsets, qh);
        return hipGetLastError();
    }
    const int64_t tiles = (m + kScanTile - 1) / kScanTile;
    int64_t *tile_sums = static_cast<int64_t *>(workspace);
    int64_t *tile_flags = tile_sums + tiles + 1;
    const int32_t *lc = order ? ordered_counts : counts;
    csr_tile_sums<<<(unsigned)tiles, kScanBlock, 0, s>>>(counts, lc, m, regs, tile_sums, tile_flags);
    csr_tile_prefix<<<1, kScanBlock, 0, s>>>(tile_sums, tile_flags, tiles, qh);
    csr_apply<<<(unsigned)tiles, kScanBlock, 0, s>>>(counts, lc, order, m, regs, tile_sums, tile_flags, offsets, big_list,
                                                     huge_list);
    return hipGetLastError();
}

hipError_t csr_offsets(const int32_t *counts, int64_t m, int64_t *offsets, int64_t *total_dev, void *workspace,
                       hipStream_t s)
{
    if (m == 0) {
        scan_empty<<<1, 1, 0, s>>>(offsets, total_dev);
        return hipGetLastError();
    }
    const int64_t tiles = (m + kScanTile - 1) / kScanTile;
    int64_t *tile_sums = static_cast<int64_t *>(workspace);
    scan_tile_sums<<<(unsigned)tiles, kScanBlock, 0, s>>>(counts, m, tile_sums);
    scan_tile_prefix<<<1, kScanBlock, 0, s>>>(tile_sums, tiles, total_dev);
    scan_apply<<<(unsigned)tiles, kScanBlock, 0, s>>>(counts, m, tile_sums, offsets);
    return hipGetLastError();
}

}  // namespace ax
