// Device-wide exclusive scan of uint32 values.  Tiles of 4096 values; each
// downsweep block scans its tile with 16 consecutive values per thread and
// adds the sum of all earlier tiles.  That sum comes from a per-tile
// reduction launched first: up to 2048 tiles each downsweep block adds up
// the earlier tiles' sums itself (two launches), beyond that a single-block
// scan of the tile sums runs in between (three launches).  Up to 16384
// values one 1024-thread block does everything in one launch.  Sums are
// carried in 64 bits; the 64-bit grand total is written for the host, which
// rejects totals that do not fit the 32-bit offsets.
#include "lfr_internal.h"

namespace lfr {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanBlock * kScanItems;
constexpr int kScanBigBlock = 1024;
constexpr int kScanSingle = kScanBigBlock * kScanItems;     // values of a one-launch scan
constexpr int kScanFoldLoads = 8;
constexpr int kScanFoldTiles = kScanBlock * kScanFoldLoads;  // tiles a downsweep block sums itself

// Inclusive scan of one value per thread across a block of B threads; the
// block's total goes to *block_total.
template <int B>
__device__ inline uint64_t block_inclusive_scan(uint64_t v, uint64_t *wave_sums, uint64_t *block_total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    if (lane == 63) wave_sums[wave] = v;
    __syncthreads();
    uint64_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < B / 64; ++w) {
        const uint64_t s = wave_sums[w];
        if (w < wave) before += s;
        total += s;
    }
    __syncthreads();
    *block_total = total;
    return v + before;
}

__global__ void __launch_bounds__(kScanBlock) scan_reduce_kernel(const uint32_t *in, int64_t n, uint64_t *partial)
{
    __shared__ uint64_t ws[kScanBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    // all loads first (index 0 stands in past the end and counts nothing):
    // a load guarded by its own bounds test would wait for each in turn
    uint32_t v[kScanItems];
#pragma unroll
    for (int it = 0; it < kScanItems; ++it) {
        const int64_t idx = base + it * kScanBlock + threadIdx.x;
        v[it] = in[idx < n ? idx : 0];
    }
    uint64_t s = 0;
#pragma unroll
    for (int it = 0; it < kScanItems; ++it) {
        const int64_t idx = base + it * kScanBlock + threadIdx.x;
        s += idx < n ? v[it] : 0u;
    }
    uint64_t total;
    block_inclusive_scan<kScanBlock>(s, ws, &total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Exclusive scan of the tile sums in place (one block), for more tiles than
// a downsweep block adds up itself.
__global__ void __launch_bounds__(kScanBlock) scan_partials_kernel(uint64_t *partial, int64_t nb, uint64_t *total_out)
{
    __shared__ uint64_t ws[kScanBlock / 64];
    uint64_t carry = 0;
    for (int64_t base = 0; base < nb; base += kScanBlock) {
        const int64_t idx = base + threadIdx.x;
        const uint64_t v = idx < nb ? partial[idx] : 0;
        uint64_t tot;
        const uint64_t inc = block_inclusive_scan<kScanBlock>(v, ws, &tot);
        if (idx < nb) partial[idx] = carry + inc - v;
        carry += tot;
    }
    if (threadIdx.x == 0 && total_out) *total_out = carry;
}

// Downsweep of tile blockIdx.x (B x 16 values, thread t on values 16t ..
// 16t + 15 of the tile, read and written as 16-byte vectors when in and out
// are 16-byte aligned).  The tile's offset is partial[blockIdx.x] when the
// tile sums were scanned (kFold false); otherwise (kFold, at most
// kScanFoldTiles tiles) this block adds up the sums partial[0 .. blockIdx.x)
// of the earlier tiles, and the last tile writes the grand total.
template <int B, bool kFold>
__global__ void __launch_bounds__(B) scan_down_kernel(const uint32_t *in, uint32_t *out, int64_t n,
                                                       const uint64_t *partial, uint64_t *total_out)
{
    __shared__ uint64_t ws[B / 64];
    uint64_t carry;
    if (kFold) {
        // every load issued before any is summed (index 0 stands in past the end)
        uint64_t p[kScanFoldLoads];
#pragma unroll
        for (int q = 0; q < kScanFoldLoads; ++q) {
            const int j = q * B + (int)threadIdx.x;
            p[q] = partial[j < (int)blockIdx.x ? j : 0];
        }
        uint64_t c = 0;
#pragma unroll
        for (int q = 0; q < kScanFoldLoads; ++q) c += q * B + (int)threadIdx.x < (int)blockIdx.x ? p[q] : 0ull;
        block_inclusive_scan<B>(c, ws, &carry);
    } else {
        carry = partial[blockIdx.x];
    }
    const int64_t t0 = (int64_t)blockIdx.x * (B * kScanItems) + (int64_t)threadIdx.x * kScanItems;
    const bool vec = t0 + kScanItems <= n && ((((uintptr_t)in | (uintptr_t)out) & 15u) == 0);
    uint32_t v[kScanItems];
    if (vec) {
        const uint4 *pv = reinterpret_cast<const uint4 *>(in + t0);
#pragma unroll
        for (int j = 0; j < kScanItems / 4; ++j) {
            const uint4 q = pv[j];
            v[4 * j] = q.x;
            v[4 * j + 1] = q.y;
            v[4 * j + 2] = q.z;
            v[4 * j + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = in[t0 + k < n ? t0 + k : 0];
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = t0 + k < n ? v[k] : 0u;
    }
    uint64_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) sum += v[k];
    uint64_t tot;
    const uint64_t inc = block_inclusive_scan<B>(sum, ws, &tot);
    uint64_t run = carry + inc - sum;
    uint32_t o[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        o[k] = (uint32_t)run;
        run += v[k];
    }
    if (vec) {
        uint4 *q = reinterpret_cast<uint4 *>(out + t0);
#pragma unroll
        for (int j = 0; j < kScanItems / 4; ++j) q[j] = make_uint4(o[4 * j], o[4 * j + 1], o[4 * j + 2], o[4 * j + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (t0 + k < n) out[t0 + k] = o[k];
    }
    if (kFold && total_out && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *total_out = carry + tot;
}

size_t scan_temp_bytes(int64_t n)
{
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    return (size_t)(nb > 0 ? nb : 1) * sizeof(uint64_t);
}

hipError_t launch_exclusive_scan(const uint32_t *in, uint32_t *out, int64_t n, void *temp, uint64_t *total,
                                 hipStream_t s)
{
    uint64_t *partial = (uint64_t *)temp;
    if (n == 0) {
        // nothing to read: only the total (zero)
        if (total) hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(kScanBlock), 0, s, partial, (int64_t)0, total);
        return hipGetLastError();
    }
    if (n <= kScanSingle) {
        // one block; with no earlier tile it reads no tile sum
        hipLaunchKernelGGL((scan_down_kernel<kScanBigBlock, true>), dim3(1), dim3(kScanBigBlock), 0, s, in, out, n,
                           (const uint64_t *)partial, total);
        return hipGetLastError();
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, n, partial);
    if (nb <= kScanFoldTiles) {
        hipLaunchKernelGGL((scan_down_kernel<kScanBlock, true>), dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, out,
                           n, (const uint64_t *)partial, total);
    } else {
        hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(kScanBlock), 0, s, partial, nb, total);
        hipLaunchKernelGGL((scan_down_kernel<kScanBlock, false>), dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, out,
                           n, (const uint64_t *)partial, (uint64_t *)nullptr);
    }
    return hipGetLastError();
}

}  // namespace lfr
