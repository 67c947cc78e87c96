// Device-wide exclusive scan of uint32 values (three phases: per-tile sums,
// a single-block scan of the tile sums, per-tile downsweep).  Sums are
// carried in 64 bits; the 64-bit grand total is written for the host, which
// rejects totals that do not fit the 32-bit offsets.
#include "lfr_internal.h"

namespace lfr {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanBlock * kScanItems;

// Inclusive scan of one value per thread across a 256-thread block.
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
    for (int w = 0; w < kScanBlock / 64; ++w) {
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
    block_inclusive_scan(s, ws, &total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanBlock) scan_partials_kernel(uint64_t *partial, int64_t nb, uint64_t *total_out)
{
    __shared__ uint64_t ws[kScanBlock / 64];
    uint64_t carry = 0;
    for (int64_t base = 0; base < nb; base += kScanBlock) {
        const int64_t idx = base + threadIdx.x;
        const uint64_t v = idx < nb ? partial[idx] : 0;
        uint64_t tot;
        const uint64_t inc = block_inclusive_scan(v, ws, &tot);
        if (idx < nb) partial[idx] = carry + inc - v;
        carry += tot;
    }
    if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ void __launch_bounds__(kScanBlock) scan_down_kernel(const uint32_t *in, uint32_t *out, int64_t n,
                                                                const uint64_t *partial)
{
    __shared__ uint64_t ws[kScanBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint64_t carry = partial[blockIdx.x];
    // items in striped order (it-major, then thread): the scan order is the
    // index order because idx = base + it*256 + tid
    for (int it = 0; it < kScanItems; ++it) {
        const int64_t idx = base + it * kScanBlock + threadIdx.x;
        const uint64_t v = idx < n ? in[idx] : 0;
        uint64_t tot;
        const uint64_t inc = block_inclusive_scan(v, ws, &tot);
        if (idx < n) out[idx] = (uint32_t)(carry + inc - v);
        carry += tot;
    }
}

// The same downsweep with each thread on 16 consecutive items (read and
// written as four 16-byte vectors): one block scan per tile instead of
// sixteen.  For 16-byte aligned in / out.
__global__ void __launch_bounds__(kScanBlock) scan_down_blocked_kernel(const uint32_t *in, uint32_t *out, int64_t n,
                                                                        const uint64_t *partial)
{
    __shared__ uint64_t ws[kScanBlock / 64];
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    const bool full = t0 + kScanItems <= n;
    uint32_t v[kScanItems];
    if (full) {
        const uint4 *p = reinterpret_cast<const uint4 *>(in + t0);
#pragma unroll
        for (int j = 0; j < kScanItems / 4; ++j) {
            const uint4 q = p[j];
            v[4 * j] = q.x;
            v[4 * j + 1] = q.y;
            v[4 * j + 2] = q.z;
            v[4 * j + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = t0 + k < n ? in[t0 + k] : 0u;
    }
    uint64_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) sum += v[k];
    uint64_t tot;
    const uint64_t inc = block_inclusive_scan(sum, ws, &tot);
    uint64_t run = partial[blockIdx.x] + inc - sum;
    uint32_t o[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        o[k] = (uint32_t)run;
        run += v[k];
    }
    if (full) {
        uint4 *q = reinterpret_cast<uint4 *>(out + t0);
#pragma unroll
        for (int j = 0; j < kScanItems / 4; ++j) q[j] = make_uint4(o[4 * j], o[4 * j + 1], o[4 * j + 2], o[4 * j + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (t0 + k < n) out[t0 + k] = o[k];
    }
}

size_t scan_temp_bytes(int64_t n)
{
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    return (size_t)(nb > 0 ? nb : 1) * sizeof(uint64_t);
}

hipError_t launch_exclusive_scan(const uint32_t *in, uint32_t *out, int64_t n, void *temp, uint64_t *total,
                                 hipStream_t s)
{
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    uint64_t *partial = (uint64_t *)temp;
    if (n == 0) {
        if (total) hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(kScanBlock), 0, s, partial, (int64_t)0, total);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, n, partial);
    hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(kScanBlock), 0, s, partial, nb, total);
    if ((((uintptr_t)in | (uintptr_t)out) & 15u) == 0)
        hipLaunchKernelGGL(scan_down_blocked_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, out, n,
                           (const uint64_t *)partial);
    else
        hipLaunchKernelGGL(scan_down_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, out, n,
                           (const uint64_t *)partial);
    return hipGetLastError();
}

}  // namespace lfr
