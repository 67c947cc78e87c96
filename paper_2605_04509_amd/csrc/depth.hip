// Depth order of the (Gaussian, cluster) items for chunked key generation.
//
// Pairs are generated chunk by chunk in depth order (section 4.2 "Sorting"
// and "Key Generation", appendix B.2): every chunk but the last is a range of
// depth ranks of each cluster, the last one holds everything deeper.  Only
// the ranks of the ranked chunks need a full depth order.  So instead of
// sorting all K' x M items, each cluster k gets a threshold thr[k] on the
// depth key with at most R valid items below it (R = the ranks the ranked
// chunks cover).  Those items (the near set) are copied in index order into
// a segment of ncap >= R entries per cluster (the rest of the segment holds
// invalid keys) and sorted there by the segmented radix sort.  Items with a
// valid key >= thr[k] (the far set) are binned as the last chunk in index
// order, the depth key travelling in the pair key so that a 64-bit sort puts
// each (tile, cluster) list in depth order.
//
// Near and far are split by key value, so every near key is below every far
// key of the cluster; the copy and both sorts are stable, so equal depths
// stay in index order.  The result is the (depth, i) order of one full sort.
//
// The threshold lies on a grid of 2^20 key values (sign, exponent and three
// mantissa bits of the float32 depth): from a 2048-bin histogram of each
// cluster's valid keys (positive float32 bits, below 2^31) it is the largest
// bin boundary with at most R keys below it.
#include "lfr_internal.h"

namespace lfr {

constexpr int kSplitBins = 2048;
constexpr int kSplitShift = 20;
constexpr int kSplitTile = 4096;  // keys per tile: the sort's segment granule
constexpr int kSplitBlock = 256;
constexpr int kSplitItems = kSplitTile / kSplitBlock;
constexpr int kSplitTilesPerBlock = 4;  // histogram tiles per block (one cluster)

// Histogram of bin = key >> 20 over the valid keys of each cluster's segment.
// Block (x, k) covers tiles [x t, (x + 1) t) of cluster k's segment.  A
// cluster's keys fall in few bins, so the lanes of one atomic instruction
// often share a bin: lane l counts into copy l & 3 of the histogram (copies
// kSplitBins + 1 words apart, so a bin's copies lie in different banks),
// which cuts those collisions fourfold.
constexpr int kSplitCopies = 4;
__global__ void __launch_bounds__(kSplitBlock) split_hist_kernel(const uint32_t *__restrict__ dkey, int64_t Mp,
                                                                  uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[kSplitCopies * (kSplitBins + 1)];
    const int k = blockIdx.y;
    uint32_t *hc = h + (threadIdx.x & (kSplitCopies - 1)) * (kSplitBins + 1);
    for (int b = threadIdx.x; b < kSplitCopies * (kSplitBins + 1); b += kSplitBlock) h[b] = 0u;
    __syncthreads();
    const int64_t tps = Mp / kSplitTile;
    const int64_t t0 = (int64_t)blockIdx.x * kSplitTilesPerBlock;
    const int64_t t1 = min(t0 + kSplitTilesPerBlock, tps);
    const uint32_t *seg = dkey + (int64_t)k * Mp;
    for (int64_t t = t0; t < t1; ++t) {
        uint32_t v[kSplitItems];
#pragma unroll
        for (int it = 0; it < kSplitItems; ++it) v[it] = seg[t * kSplitTile + it * kSplitBlock + threadIdx.x];
#pragma unroll
        for (int it = 0; it < kSplitItems; ++it)
            if (v[it] < 0x80000000u) atomicAdd(&hc[v[it] >> kSplitShift], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kSplitBins; b += kSplitBlock) {
        uint32_t c = 0;
#pragma unroll
        for (int q = 0; q < kSplitCopies; ++q) c += h[q * (kSplitBins + 1) + b];
        if (c) atomicAdd(&hist[(int64_t)k * kSplitBins + b], c);
    }
}

// thr[k] = (largest bin boundary b with at most R keys in bins below b) << 20;
// one wavefront per cluster, 32 bins per lane.
__global__ void __launch_bounds__(64) split_select_kernel(const uint32_t *__restrict__ hist, int64_t R,
                                                           uint32_t *__restrict__ thr)
{
    const int k = blockIdx.x, lane = threadIdx.x;
    constexpr int kPer = kSplitBins / 64;
    const uint32_t *h = hist + (int64_t)k * kSplitBins + lane * kPer;
    uint32_t v[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) v[j] = h[j];
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) s += v[j];
    uint64_t incl = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    uint64_t below = incl - s;  // keys in the bins before this lane's first
    int best = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        if (below <= (uint64_t)R) best = lane * kPer + j;
        below += v[j];
    }
    if (lane == 63 && below <= (uint64_t)R) best = kSplitBins;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) best = max(best, __shfl_xor(best, d, 64));
    if (lane == 0) thr[k] = (uint32_t)best << kSplitShift;
}

// Keys below the threshold in each 4096-key tile (tile t of the [K'][Mp]
// array; tps tiles per cluster).
__global__ void __launch_bounds__(kSplitBlock) split_count_kernel(const uint32_t *__restrict__ dkey, int64_t tps,
                                                                   const uint32_t *__restrict__ thr,
                                                                   uint32_t *__restrict__ tile_cnt)
{
    __shared__ uint32_t ws[kSplitBlock / 64];
    const int64_t t = blockIdx.x;
    const uint32_t th = thr[t / tps];
    const uint32_t *tk = dkey + t * kSplitTile;
    uint32_t v[kSplitItems];
#pragma unroll
    for (int it = 0; it < kSplitItems; ++it) v[it] = tk[it * kSplitBlock + threadIdx.x];
    uint32_t c = 0;
#pragma unroll
    for (int it = 0; it < kSplitItems; ++it) c += (uint32_t)__popcll(__ballot(v[it] < th));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) ws[wave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t sum = 0;
#pragma unroll
        for (int w = 0; w < kSplitBlock / 64; ++w) sum += ws[w];
        tile_cnt[t] = sum;
    }
}

// Stable copy of the near keys: tile t's keys below the threshold go, in
// index order, to cluster k's segment of near_key / near_val (value = the
// Gaussian index) from slot tile_off[t] - tile_off[k tps].  Wavefront w
// covers the 1024 consecutive keys [1024 w, 1024 (w + 1)) of the tile.
__global__ void __launch_bounds__(kSplitBlock) split_write_kernel(const uint32_t *__restrict__ dkey, int64_t tps,
                                                                   const uint32_t *__restrict__ thr,
                                                                   const uint32_t *__restrict__ tile_off,
                                                                   int64_t ncap, uint32_t *__restrict__ near_key,
                                                                   uint32_t *__restrict__ near_val)
{
    constexpr int kPerWave = kSplitTile / (kSplitBlock / 64);  // 1024
    constexpr int kIt = kPerWave / 64;                         // 16
    __shared__ uint32_t ws[kSplitBlock / 64];
    const int64_t t = blockIdx.x;
    const int64_t k = t / tps;
    const uint32_t th = thr[k];
    const uint32_t off = tile_off[t] - tile_off[k * tps];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    const int64_t l0 = (t - k * tps) * kSplitTile + (int64_t)wave * kPerWave;  // index within the cluster
    const uint32_t *wk = dkey + t * kSplitTile + (int64_t)wave * kPerWave;
    uint32_t v[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) v[it] = wk[it * 64 + lane];
    uint32_t c = 0;
#pragma unroll
    for (int it = 0; it < kIt; ++it) c += (uint32_t)__popcll(__ballot(v[it] < th));
    if (lane == 0) ws[wave] = c;
    __syncthreads();
    uint32_t pos = off;
    for (int w = 0; w < wave; ++w) pos += ws[w];
    uint32_t *ok = near_key + k * ncap;
    uint32_t *ov = near_val + k * ncap;
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const bool nr = v[it] < th;
        const uint64_t b = __ballot(nr);
        const uint32_t p = pos + (uint32_t)__popcll(b & lt_mask);
        if (nr && p < (uint32_t)ncap) {
            ok[p] = v[it];
            ov[p] = (uint32_t)(l0 + it * 64 + lane);
        }
        pos += (uint32_t)__popcll(b);
    }
}

size_t split_temp_bytes(int n_clusters, int64_t Mp)
{
    const int64_t nt = (int64_t)n_clusters * (Mp / kSplitTile);
    return (size_t)n_clusters * kSplitBins * 4 + (size_t)n_clusters * 4 + 2 * (size_t)nt * 4 + 256 +
           scan_temp_bytes(nt);
}

hipError_t launch_depth_split(const uint32_t *dkey, int n_clusters, int64_t Mp, int64_t R, int64_t ncap,
                              void *temp, uint32_t **thr_out, uint32_t *near_key, uint32_t *near_val, hipStream_t s)
{
    if (Mp % kSplitTile != 0 || ncap % kSplitTile != 0 || R > ncap || n_clusters <= 0) return hipErrorInvalidValue;
    const int64_t tps = Mp / kSplitTile, nt = (int64_t)n_clusters * tps;
    uint32_t *hist = (uint32_t *)temp;
    uint32_t *thr = hist + (int64_t)n_clusters * kSplitBins;
    uint32_t *tile_cnt = thr + n_clusters;
    uint32_t *tile_off = tile_cnt + nt;
    void *stemp = (void *)(((uintptr_t)(tile_off + nt) + 255) & ~(uintptr_t)255);
    *thr_out = thr;
    hipError_t e = launch_fill_u32(hist, 0u, (int64_t)n_clusters * kSplitBins, s);
    if (e != hipSuccess) return e;
    e = launch_fill_u32(near_key, 0xFFFFFFFFu, (int64_t)n_clusters * ncap, s);
    if (e != hipSuccess) return e;
    const unsigned hb = (unsigned)((tps + kSplitTilesPerBlock - 1) / kSplitTilesPerBlock);
    hipLaunchKernelGGL(split_hist_kernel, dim3(hb, (unsigned)n_clusters), dim3(kSplitBlock), 0, s, dkey, Mp, hist);
    hipLaunchKernelGGL(split_select_kernel, dim3((unsigned)n_clusters), dim3(64), 0, s, hist, R, thr);
    hipLaunchKernelGGL(split_count_kernel, dim3((unsigned)nt), dim3(kSplitBlock), 0, s, dkey, tps, thr, tile_cnt);
    e = launch_exclusive_scan(tile_cnt, tile_off, nt, stemp, nullptr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(split_write_kernel, dim3((unsigned)nt), dim3(kSplitBlock), 0, s, dkey, tps, thr, tile_off,
                       ncap, near_key, near_val);
    return hipGetLastError();
}

}  // namespace lfr
