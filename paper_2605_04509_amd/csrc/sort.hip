// Stable LSD radix sort of (key, value) pairs, 8-bit digits.
//
// Per pass: (1) every 4096-key tile builds a 256-bin digit histogram in LDS;
// (2) the [digit][tile] histogram matrix is exclusive-scanned, giving every
// (digit, tile) its first output slot; (3) every tile re-reads its keys and
// scatters them.  Stability inside a tile comes from processing its keys in
// index order, 256 at a time: each wavefront matches equal digits with eight
// 64-bit ballots (one per digit bit), ranks a key by the popcount of equal
// lanes below it, and the four wavefronts' per-digit counts are prefixed in
// wavefront order through LDS.
#include "lfr_internal.h"

namespace lfr {

constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortBlock * kSortItems;
constexpr int kSortWaves = kSortBlock / 64;

template <typename K>
__global__ void __launch_bounds__(kSortBlock) sort_hist_kernel(const K *__restrict__ keys, int64_t n, int shift,
                                                                uint32_t mask, uint32_t *hist, int64_t nb)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t idx = base + it * kSortBlock + threadIdx.x;
        if (idx < n) atomicAdd(&h[(uint32_t)(keys[idx] >> shift) & mask], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

template <typename K>
__global__ void __launch_bounds__(kSortBlock) sort_scatter_kernel(const K *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                                   K *__restrict__ kout, uint32_t *__restrict__ vout,
                                                                   int64_t n, int shift, uint32_t mask,
                                                                   const uint32_t *__restrict__ offs, int64_t nb)
{
    __shared__ uint32_t base_of[256];               // next free slot per digit
    __shared__ uint32_t wave_cnt[kSortWaves][256];  // per-wavefront counts, then offsets
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    base_of[threadIdx.x] = offs[(int64_t)threadIdx.x * nb + blockIdx.x];
    const int64_t tile = (int64_t)blockIdx.x * kSortTile;
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t idx = tile + it * kSortBlock + threadIdx.x;
        const bool valid = idx < n;
        K key = 0;
        uint32_t val = 0, digit = 0;
        if (valid) {
            key = kin[idx];
            val = vin[idx];
            digit = (uint32_t)(key >> shift) & mask;
        }
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (digit >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
        const bool leader = valid && (peers & lt_mask) == 0;
        // clear this wavefront's counters (4 per lane), then publish counts
#pragma unroll
        for (int k = 0; k < 4; ++k) wave_cnt[wave][lane * 4 + k] = 0;
        __syncthreads();
        if (leader) wave_cnt[wave][digit] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            const int d = threadIdx.x;
            uint32_t run = base_of[d];
#pragma unroll
            for (int w = 0; w < kSortWaves; ++w) {
                const uint32_t c = wave_cnt[w][d];
                wave_cnt[w][d] = run;
                run += c;
            }
            base_of[d] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = wave_cnt[wave][digit] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
    }
}

static int64_t sort_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

size_t sort_temp_bytes(int64_t n)
{
    const int64_t nb = sort_tiles(n) > 0 ? sort_tiles(n) : 1;
    const int64_t nh = 256 * nb;
    // hist + offsets + scan temp
    return (size_t)(2 * nh * sizeof(uint32_t)) + scan_temp_bytes(nh) + 64;
}

template <typename K>
static hipError_t radix_sort_impl(K *k0, uint32_t *v0, K *k1, uint32_t *v1, int64_t n, int b0, int b1,
                                  void *temp, bool *in_alt, hipStream_t s, hipEvent_t *ev = nullptr,
                                  int *n_timed = nullptr)
{
    *in_alt = false;
    if (n_timed) *n_timed = 0;
    if (n <= 1 || b1 <= b0) return hipSuccess;
    const int64_t nb = sort_tiles(n);
    const int64_t nh = 256 * nb;
    uint32_t *hist = (uint32_t *)temp;
    uint32_t *offs = hist + nh;
    void *stemp = (void *)(((uintptr_t)(offs + nh) + 63) & ~(uintptr_t)63);
    K *ki = k0, *ko = k1;
    uint32_t *vi = v0, *vo = v1;
    for (int shift = b0; shift < b1; shift += 8) {
        const int bits = (b1 - shift) < 8 ? (b1 - shift) : 8;
        const uint32_t mask = (1u << bits) - 1u;
        hipLaunchKernelGGL(sort_hist_kernel<K>, dim3((unsigned)nb), dim3(kSortBlock), 0, s, ki, n, shift, mask,
                           hist, nb);
        hipError_t e = launch_exclusive_scan(hist, offs, nh, stemp, nullptr, s);
        if (e != hipSuccess) return e;
        const int pass = (shift - b0) / 8;
        const bool timed = ev && pass < kSortTimedPasses;
        if (timed) (void)hipEventRecord(ev[2 * pass], s);
        hipLaunchKernelGGL(sort_scatter_kernel<K>, dim3((unsigned)nb), dim3(kSortBlock), 0, s, ki, vi, ko, vo, n,
                           shift, mask, offs, nb);
        if (timed) {
            (void)hipEventRecord(ev[2 * pass + 1], s);
            *n_timed = pass + 1;
        }
        K *tk = ki;
        ki = ko;
        ko = tk;
        uint32_t *tv = vi;
        vi = vo;
        vo = tv;
        *in_alt = !*in_alt;
    }
    return hipGetLastError();
}

hipError_t radix_sort_u32(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n, int b0, int b1,
                          void *temp, bool *in_alt, hipStream_t s, hipEvent_t *ev, int *n_timed)
{
    return radix_sort_impl<uint32_t>(k0, v0, k1, v1, n, b0, b1, temp, in_alt, s, ev, n_timed);
}

hipError_t radix_sort_u64(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n, int b0, int b1,
                          void *temp, bool *in_alt, hipStream_t s)
{
    return radix_sort_impl<uint64_t>(k0, v0, k1, v1, n, b0, b1, temp, in_alt, s);
}

}  // namespace lfr
