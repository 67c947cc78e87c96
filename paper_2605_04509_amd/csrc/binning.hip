// Key generation with reuse (section 4.2 "Key Generation", appendix B.2
// GenerateKeys): for each (Gaussian i, cluster k) the tiles touched by the
// union over the cluster's views j of the box around mean2d(i, j) with the
// cluster's half extents; one (key, i) pair per tile of that union, key =
// (tile << cluster_bits) | k.
//
// The Gaussians of every cluster are first sorted by depth; pairs are then
// generated chunk by chunk in that order (a chunk is a range of depth ranks,
// the same for every cluster), so a stable sort on the tile bits alone
// leaves every (tile, cluster) list sorted by (depth, i): the order of the
// 64-bit key (t, k, depth) of Eq. 7 / appendix B.2.  A tile is skipped when
// its (tile, cluster) list has no unsaturated subpixel left (`alive` bits,
// maintained by the blend between chunks): those lists would never be read.
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

// The boxes of one (Gaussian, cluster) item: up to kRegViews kept in
// registers; items with more views recompute their boxes from the means.
constexpr int kRegViews = 4;
struct Item {
    int k = 0;
    uint32_t i = 0;
    float2 e = make_float2(0.f, 0.f);
    int nv = 0;          // views of the cluster (boxes possibly empty)
    int ylo = 1, yhi = 0, wlo = 1, whi = 0;  // tile-row and 32-tile-word bounds of the union
    TileRect r[kRegViews];
    bool ok[kRegViews];
};

__device__ inline bool item_rect(const BinParams &bp, const float2 *mean2d, const Item &it, int v, TileRect &r)
{
    if (v < kRegViews) {
        r = it.r[v];
        return it.ok[v];
    }
    const float2 m = mean2d[(int64_t)bp.cv_list[bp.cv_off[it.k] + v] * bp.M + it.i];
    return !isnan(m.x) && view_rect(m, it.e, bp, r);
}

__device__ inline void item_init(const BinParams &bp, const float2 *mean2d, const float2 *ext, int k, uint32_t i,
                                 Item &it)
{
    it.k = k;
    it.i = i;
    it.e = ext[(int64_t)k * bp.M + i];
    it.nv = bp.cv_off[k + 1] - bp.cv_off[k];
    int ylo = 1 << 30, yhi = -1, xlo = 1 << 30, xhi = -1;
    for (int v = 0; v < it.nv; ++v) {
        const float2 m = mean2d[(int64_t)bp.cv_list[bp.cv_off[k] + v] * bp.M + i];
        TileRect r;
        const bool ok = !isnan(m.x) && view_rect(m, it.e, bp, r);
        if (v < kRegViews) {
            it.r[v] = r;
            it.ok[v] = ok;
        }
        if (ok) {
            ylo = min(ylo, r.y0);
            yhi = max(yhi, r.y1);
            xlo = min(xlo, r.x0);
            xhi = max(xhi, r.x1);
        }
    }
    it.ylo = ylo;
    it.yhi = yhi;
    it.wlo = xlo >> 5;
    it.whi = xhi >= 0 ? (xhi >> 5) : -1;
}

__device__ inline int item_units(const Item &it)
{
    return it.yhi < it.ylo ? 0 : (it.yhi - it.ylo + 1) * (it.whi - it.wlo + 1);
}

// Alive tiles of the union in one (tile row, 32-tile word) unit: OR of the
// views' interval masks, AND the list-alive bits.
__device__ inline uint32_t unit_mask(const BinParams &bp, const float2 *mean2d, const Item &it, int u)
{
    const int nw = it.whi - it.wlo + 1;
    const int ty = it.ylo + u / nw;
    const int w = it.wlo + u % nw;
    uint32_t m = 0;
    for (int v = 0; v < it.nv; ++v) {
        TileRect r;
        if (!item_rect(bp, mean2d, it, v, r) || ty < r.y0 || ty > r.y1) continue;
        const int lo = r.x0 - (w << 5), hi = r.x1 - (w << 5);
        if (hi < 0 || lo > 31) continue;
        const uint32_t mh = hi >= 31 ? 0xFFFFFFFFu : ((2u << hi) - 1u);
        const uint32_t ml = lo <= 0 ? 0xFFFFFFFFu : (0xFFFFFFFFu << lo);
        m |= mh & ml;
    }
    const uint32_t *alive_k = bp.alive + (int64_t)it.k * bp.TY * bp.alive_words;
    return m & alive_k[(int64_t)ty * bp.alive_words + w];
}

__device__ inline void unit_emit(const BinParams &bp, const Item &it, int u, uint32_t m, uint32_t *keys,
                                 uint32_t *vals)
{
    const int nw = it.whi - it.wlo + 1;
    const int ty = it.ylo + u / nw;
    const int w = it.wlo + u % nw;
    const uint32_t base = (uint32_t)ty * (uint32_t)bp.TX + ((uint32_t)w << 5);
    int n = 0;
    while (m) {
        const int b = __ffs(m) - 1;
        m &= m - 1u;
        keys[n] = ((base + (uint32_t)b) << bp.cluster_bits) | (uint32_t)it.k;
        vals[n] = it.i;
        ++n;
    }
}

// Items with at most this many (row, word) units are handled by their own
// lane; larger ones by the whole wavefront, one at a time.
constexpr int kLaneUnits = 6;

// Items of one chunk: depth ranks [r0, r0 + len) of every cluster; item
// (k, r) sits at k * M + r of the depth-sorted arrays and at k * len + (r - r0)
// of the chunk's count / offset arrays.  The order of pairs inside one item
// is irrelevant (each tile appears at most once per item), so cooperative
// emission may place them in any order within the item's slot range.
template <bool kEmit>
__global__ void __launch_bounds__(256) chunk_tiles_kernel(BinParams bp, const float2 *__restrict__ mean2d,
                                                           const float2 *__restrict__ ext,
                                                           const uint64_t *__restrict__ dkey_sorted,
                                                           const uint32_t *__restrict__ dval_sorted, int64_t r0,
                                                           int64_t len, uint32_t *__restrict__ counts,
                                                           const uint32_t *__restrict__ offsets,
                                                           uint32_t *__restrict__ pair_keys,
                                                           uint32_t *__restrict__ pair_vals)
{
    const int64_t rl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const bool in = rl < len;
    const int64_t o = (int64_t)k * len + rl;
    Item it;
    bool valid = false;
    if (in) {
        const int64_t e = (int64_t)k * bp.M + r0 + rl;
        valid = (uint32_t)dkey_sorted[e] != 0xFFFFFFFFu;
        if (valid) item_init(bp, mean2d, ext, k, dval_sorted[e], it);
    }
    const int units = valid ? item_units(it) : 0;
    const bool big = units > kLaneUnits;
    uint32_t cnt = 0;
    uint32_t off = 0, limit = 0;
    if (kEmit && valid) {
        off = offsets[o];
        limit = counts[o];
    }
    if (valid && !big) {
        for (int u = 0; u < units; ++u) {
            const uint32_t m = unit_mask(bp, mean2d, it, u);
            if (kEmit && m) {
                // bounded by the count pass, so the pair buffer is never overrun
                if (cnt + (uint32_t)__popc(m) <= limit) unit_emit(bp, it, u, m, pair_keys + off + cnt, pair_vals + off + cnt);
            }
            cnt += (uint32_t)__popc(m);
        }
    }
    // large items: the whole wavefront walks one item's units at a time
    uint64_t todo = __ballot(big);
    while (todo) {
        const int src = __ffsll((long long)todo) - 1;
        todo &= todo - 1ull;
        Item w;
        w.k = k;
        w.i = (uint32_t)__shfl((int)it.i, src, 64);
        item_init(bp, mean2d, ext, k, w.i, w);
        const int wu = item_units(w);
        const uint32_t woff = (uint32_t)__shfl((int)off, src, 64);
        const uint32_t wlimit = (uint32_t)__shfl((int)limit, src, 64);
        uint32_t total = 0;  // running count of the units before this round
        for (int ub = 0; ub < wu; ub += 64) {
            const int u = ub + lane;
            const uint32_t m = u < wu ? unit_mask(bp, mean2d, w, u) : 0u;
            const uint32_t c = (uint32_t)__popc(m);
            if (kEmit) {
                uint32_t incl = c;  // inclusive scan of c over the wavefront
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const uint32_t t = (uint32_t)__shfl_up((int)incl, d, 64);
                    if (lane >= d) incl += t;
                }
                const uint32_t at = total + incl - c;
                if (c && at + c <= wlimit) unit_emit(bp, w, u, m, pair_keys + woff + at, pair_vals + woff + at);
                total += (uint32_t)__shfl((int)incl, 63, 64);
            } else {
                uint32_t sum = c;
#pragma unroll
                for (int d = 32; d > 0; d >>= 1) sum += (uint32_t)__shfl_xor((int)sum, d, 64);
                total += sum;
            }
        }
        if (lane == src) cnt = total;
    }
    if (!kEmit && in) counts[o] = valid ? cnt : 0u;
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

// alive bit of (cluster k, tile t) = (number of unsaturated subpixels of the
// (t, k) list) > 0; one thread per 32-bit word of a tile row.
__global__ void __launch_bounds__(256) alive_bits_kernel(const uint32_t *__restrict__ tc_alive, int n_clusters,
                                                          int TX, int TY, int words, int cluster_bits,
                                                          uint32_t *__restrict__ bits)
{
    const int64_t wid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)n_clusters * TY * words;
    if (wid >= n) return;
    const int w = (int)(wid % words);
    const int64_t rowid = wid / words;
    const int ty = (int)(rowid % TY);
    const int k = (int)(rowid / TY);
    uint32_t m = 0;
    for (int b = 0; b < 32; ++b) {
        const int tx = (w << 5) + b;
        if (tx >= TX) break;
        const uint32_t t = (uint32_t)(ty * TX + tx);
        if (tc_alive[(t << cluster_bits) | (uint32_t)k] > 0) m |= 1u << b;
    }
    bits[wid] = m;
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_chunk_count(const BinParams &bp, const float2 *mean2d, const float2 *ext,
                              const uint64_t *dkey_sorted, const uint32_t *dval_sorted, int64_t r0, int64_t len,
                              uint32_t *counts, hipStream_t s)
{
    if (len == 0 || bp.n_clusters == 0) return hipSuccess;
    hipLaunchKernelGGL(chunk_tiles_kernel<false>, dim3(blocks_for(len), bp.n_clusters), dim3(256), 0, s, bp, mean2d,
                       ext, dkey_sorted, dval_sorted, r0, len, counts, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                       (uint32_t *)nullptr);
    return hipGetLastError();
}

hipError_t launch_chunk_emit(const BinParams &bp, const float2 *mean2d, const float2 *ext,
                             const uint64_t *dkey_sorted, const uint32_t *dval_sorted, int64_t r0, int64_t len,
                             uint32_t *counts, const uint32_t *offsets, uint32_t *pair_keys, uint32_t *pair_vals,
                             hipStream_t s)
{
    if (len == 0 || bp.n_clusters == 0) return hipSuccess;
    hipLaunchKernelGGL(chunk_tiles_kernel<true>, dim3(blocks_for(len), bp.n_clusters), dim3(256), 0, s, bp, mean2d,
                       ext, dkey_sorted, dval_sorted, r0, len, counts, offsets, pair_keys, pair_vals);
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

hipError_t launch_alive_bits(const uint32_t *tc_alive, int n_clusters, int TX, int TY, int words, int cluster_bits,
                             uint32_t *bits, hipStream_t s)
{
    const int64_t n = (int64_t)n_clusters * TY * words;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(alive_bits_kernel, dim3(blocks_for(n)), dim3(256), 0, s, tc_alive, n_clusters, TX, TY, words,
                       cluster_bits, bits);
    return hipGetLastError();
}

}  // namespace lfr
