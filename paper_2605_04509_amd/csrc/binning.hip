// Key generation with reuse (section 4.2 "Key Generation", appendix B.2
// GenerateKeys): for each (Gaussian i, cluster k) the tiles touched by the
// union over the cluster's views j of the box around mean2d(i, j) with the
// cluster's half extents; one (key, i) pair per tile of that union, key =
// (tile << cluster_bits) | k.
//
// The pairs of one cluster are emitted in the cluster's depth order (the
// per-cluster depth sort runs before emission), so a stable sort on the
// tile bits alone leaves every (tile, cluster) list sorted by (depth, i):
// the order of the 64-bit key (t, k, depth) of Eq. 7 / appendix B.2.
//
// Tile coverage is conservative (the box bounds the alpha >= 1/255 region
// with margins), so the rendered result does not depend on the tiling.
#include "lfr_internal.h"

namespace lfr {

struct TileRect {
    int x0, x1, y0, y1;  // inclusive tile ranges
};

// Box of one view in tile coordinates; false if it misses the panel.
__device__ inline bool view_rect(float2 m, float2 e, const BinParams &bp, TileRect &r)
{
    // pixel x is covered when |x + 0.5 - mx| <= ex
    const float fx0 = fmaxf(ceilf(m.x - e.x - 0.5f), 0.0f);
    const float fx1 = fminf(floorf(m.x + e.x - 0.5f), (float)(bp.W - 1));
    const float fy0 = fmaxf(ceilf(m.y - e.y - 0.5f), 0.0f);
    const float fy1 = fminf(floorf(m.y + e.y - 0.5f), (float)(bp.H - 1));
    if (!(fx0 <= fx1) || !(fy0 <= fy1)) return false;
    r.x0 = (int)fx0 / bp.tw;
    r.x1 = (int)fx1 / bp.tw;
    r.y0 = (int)fy0 / bp.th;
    r.y1 = (int)fy1 / bp.th;
    return true;
}

// Collect the rectangles of the cluster's views, sorted by x0.
__device__ inline int cluster_rects(const BinParams &bp, const float2 *mean2d, float2 e, int k, int64_t i,
                                    TileRect *rects)
{
    int n = 0;
    const int v0 = bp.cv_off[k], v1 = bp.cv_off[k + 1];
    for (int v = v0; v < v1; ++v) {
        const float2 m = mean2d[(int64_t)bp.cv_list[v] * bp.M + i];
        if (isnan(m.x)) continue;
        TileRect r;
        if (!view_rect(m, e, bp, r)) continue;
        int p = n++;
        while (p > 0 && rects[p - 1].x0 > r.x0) {
            rects[p] = rects[p - 1];
            --p;
        }
        rects[p] = r;
    }
    return n;
}

// Walk the union row by row; with kEmit write the keys, else count.
template <bool kEmit>
__device__ inline uint32_t union_tiles(const TileRect *rects, int n, const BinParams &bp, uint32_t k,
                                       uint32_t i, uint32_t *keys, uint32_t *vals, uint32_t limit = 0)
{
    if (n == 0) return 0;
    int ylo = rects[0].y0, yhi = rects[0].y1;
    for (int a = 1; a < n; ++a) {
        ylo = min(ylo, rects[a].y0);
        yhi = max(yhi, rects[a].y1);
    }
    uint32_t cnt = 0;
    for (int ty = ylo; ty <= yhi; ++ty) {
        int end = -1;
        for (int a = 0; a < n; ++a) {
            const TileRect &r = rects[a];
            if (ty < r.y0 || ty > r.y1 || r.x1 <= end) continue;
            const int from = max(r.x0, end + 1);
            if (kEmit) {
                const uint32_t rowbase = (uint32_t)ty * (uint32_t)bp.TX;
                for (int tx = from; tx <= r.x1 && cnt < limit; ++tx) {
                    keys[cnt] = ((rowbase + (uint32_t)tx) << bp.cluster_bits) | k;
                    vals[cnt] = i;
                    ++cnt;
                }
            } else {
                cnt += (uint32_t)(r.x1 - from + 1);
            }
            end = r.x1;
        }
    }
    return cnt;
}

__global__ void __launch_bounds__(256) tile_count_kernel(BinParams bp, const float2 *__restrict__ mean2d,
                                                          const float2 *__restrict__ ext,
                                                          const uint64_t *__restrict__ dkey,
                                                          uint32_t *__restrict__ counts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (i >= bp.M) return;
    const int64_t idx = (int64_t)k * bp.M + i;
    uint32_t cnt = 0;
    if ((uint32_t)dkey[idx] != 0xFFFFFFFFu) {
        TileRect rects[kMaxClusterViews];
        const int n = cluster_rects(bp, mean2d, ext[idx], k, i, rects);
        cnt = union_tiles<false>(rects, n, bp, 0, 0, nullptr, nullptr);
    }
    counts[idx] = cnt;
}

// counts_sorted[e] = counts[cluster(e) * M + i(e)] for the depth-sorted order.
__global__ void __launch_bounds__(256) gather_counts_kernel(const uint64_t *__restrict__ dkey_sorted,
                                                             const uint32_t *__restrict__ dval_sorted, int64_t M,
                                                             int64_t n, const uint32_t *__restrict__ counts,
                                                             uint32_t *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const uint64_t key = dkey_sorted[e];
    out[e] = (uint32_t)key == 0xFFFFFFFFu ? 0u : counts[(int64_t)(key >> 32) * M + dval_sorted[e]];
}

__global__ void __launch_bounds__(256) tile_emit_kernel(BinParams bp, const float2 *__restrict__ mean2d,
                                                         const float2 *__restrict__ ext,
                                                         const uint64_t *__restrict__ dkey_sorted,
                                                         const uint32_t *__restrict__ dval_sorted,
                                                         const uint32_t *__restrict__ offsets,
                                                         const uint32_t *__restrict__ counts_sorted,
                                                         uint32_t *__restrict__ pair_keys,
                                                         uint32_t *__restrict__ pair_vals, int64_t n)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const uint64_t key = dkey_sorted[e];
    if ((uint32_t)key == 0xFFFFFFFFu) return;
    const int k = (int)(key >> 32);
    const uint32_t i = dval_sorted[e];
    TileRect rects[kMaxClusterViews];
    const int nr = cluster_rects(bp, mean2d, ext[(int64_t)k * bp.M + i], k, i, rects);
    const uint32_t off = offsets[e];
    // bounded by the count pass, so the pair buffer can never be overrun
    union_tiles<true>(rects, nr, bp, (uint32_t)k, i, pair_keys + off, pair_vals + off, counts_sorted[e]);
}

__global__ void __launch_bounds__(256) fill_kernel(uint32_t *p, uint32_t v, int64_t n)
{
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x)
        p[s] = v;
}

// [start, end) of every (tile, cluster) list, indexed by the list's key.
__global__ void __launch_bounds__(256) ranges_kernel(const uint32_t *__restrict__ keys, int64_t P, uint2 *ranges)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const uint32_t k = keys[p];
    if (p == 0 || keys[p - 1] != k) ranges[k].x = (uint32_t)p;
    if (p == P - 1 || keys[p + 1] != k) ranges[k].y = (uint32_t)(p + 1);
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_tile_count(const BinParams &bp, const float2 *mean2d, const float2 *ext, const uint64_t *dkey,
                             uint32_t *counts, hipStream_t s)
{
    if (bp.M == 0 || bp.n_clusters == 0) return hipSuccess;
    hipLaunchKernelGGL(tile_count_kernel, dim3(blocks_for(bp.M), bp.n_clusters), dim3(256), 0, s, bp, mean2d, ext,
                       dkey, counts);
    return hipGetLastError();
}

hipError_t launch_gather_counts(const uint64_t *dkey_sorted, const uint32_t *dval_sorted, int64_t M, int64_t n,
                                const uint32_t *counts, uint32_t *counts_sorted, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(gather_counts_kernel, dim3(blocks_for(n)), dim3(256), 0, s, dkey_sorted, dval_sorted, M, n,
                       counts, counts_sorted);
    return hipGetLastError();
}

hipError_t launch_tile_emit(const BinParams &bp, const float2 *mean2d, const float2 *ext,
                            const uint64_t *dkey_sorted, const uint32_t *dval_sorted, const uint32_t *offsets,
                            const uint32_t *counts_sorted, uint32_t *pair_keys, uint32_t *pair_vals, hipStream_t s)
{
    const int64_t n = bp.M * bp.n_clusters;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(tile_emit_kernel, dim3(blocks_for(n)), dim3(256), 0, s, bp, mean2d, ext, dkey_sorted,
                       dval_sorted, offsets, counts_sorted, pair_keys, pair_vals, n);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)g), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_ranges(const uint32_t *keys, int64_t P, uint2 *ranges, hipStream_t s)
{
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(ranges_kernel, dim3(blocks_for(P)), dim3(256), 0, s, keys, P, ranges);
    return hipGetLastError();
}

}  // namespace lfr
