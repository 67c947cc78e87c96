// Display precompute: the lenticular view-index map V (section 3.1, Eq. 1-3),
// the per-tile view-sorted subpixel LUT Psi (section 4.3, Eq. 8) and the
// blend work items derived from Psi.  Run once per display (and once per
// cluster size for the work items); none of it is part of the frame time.
#include "lfr_internal.h"

namespace lfr {

// Eq. 1-3 in exact integer arithmetic: with every length scaled by Q (the
// lcm of the lens parameters' denominators), d_offset*Q = D is an integer,
// x_offset*Q = D mod P (P = L_x*Q, mathematical mod) and
// j = floor(N * x_offset / L_x) = floor(N * (D mod P) / P).
// The host checks that every intermediate fits in int64.
__global__ void __launch_bounds__(256) view_map_kernel(ViewMapParams p, uint16_t *V)
{
    const int64_t n = 3ll * p.W * p.H;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pix = s / 3;
        const int64_t u = s - 3 * pix;
        const int64_t y = pix / p.W;
        const int64_t x = pix - y * p.W;
        const int64_t D = (3 * x + u) * p.qa + y * p.qb - p.qc;
        int64_t X = D % p.P;
        if (X < 0) X += p.P;
        V[s] = (uint16_t)(((int64_t)p.N * X) / p.P);
    }
}

__global__ void __launch_bounds__(256) referenced_kernel(const uint16_t *V, int64_t n, uint32_t *mask)
{
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x)
        mask[V[s]] = 1u;  // every writer stores the same value
}

static int grid_for(int64_t n, int block, int cap = 65536)
{
    int64_t g = (n + block - 1) / block;
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

hipError_t launch_view_map(const ViewMapParams &p, uint16_t *V, hipStream_t s)
{
    const int64_t n = 3ll * p.W * p.H;
    hipLaunchKernelGGL(view_map_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, V);
    return hipGetLastError();
}

hipError_t launch_referenced_views(const uint16_t *V, int64_t n, uint32_t *mask, hipStream_t s)
{
    hipLaunchKernelGGL(referenced_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, V, n, mask);
    return hipGetLastError();
}

// Geometry of tile t: origin, in-panel size, and the position of its first
// subpixel in Psi (tiles are concatenated in row-major tile order).
struct TileGeom {
    int x0, y0, w, h;
    int64_t off;
};

__device__ inline TileGeom tile_geom(int t, int W, int H, int tw, int th)
{
    const int TX = (W + tw - 1) / tw;
    const int ty = t / TX, tx = t - ty * TX;
    TileGeom g;
    g.x0 = tx * tw;
    g.y0 = ty * th;
    g.w = min(tw, W - g.x0);
    g.h = min(th, H - g.y0);
    // all tile rows above cover th full pixel rows; tiles to the left in this
    // tile row cover tx*tw columns of g.h rows
    g.off = 3ll * ((int64_t)ty * th * W + (int64_t)tx * tw * g.h);
    return g;
}

__device__ inline uint32_t tile_subpixel(const TileGeom &g, int W, int r)
{
    const int row = 3 * g.w;
    const int ly = r / row;
    const int rem = r - ly * row;
    const int lx = rem / 3;
    const int u = rem - 3 * lx;
    return (uint32_t)((((int64_t)(g.y0 + ly)) * W + (g.x0 + lx)) * 3 + u);
}

// Psi for one tile: the tile's subpixels in row-major order (local rank r)
// stably sorted by V.  Keys (V << 15) | r are unique (r < 3 * 8192 < 32768;
// V < 2^16, so keys stay below the all-ones padding), so a bitonic sort in
// LDS yields exactly the stable order.  One 256-thread block per tile; LDS
// holds next_pow2(3 * tw * th) keys (at most 32768, 128 KB of the CU's
// 160 KB).
__global__ void __launch_bounds__(256) remap_kernel(const uint16_t *V, int W, int H, int tw, int th,
                                                    uint32_t *psi)
{
    extern __shared__ uint32_t keys[];
    const TileGeom g = tile_geom(blockIdx.x, W, H, tw, th);
    const int n = 3 * g.w * g.h;
    int n2 = 1;
    while (n2 < n) n2 <<= 1;
    for (int r = threadIdx.x; r < n2; r += blockDim.x)
        keys[r] = r < n ? (((uint32_t)V[tile_subpixel(g, W, r)] << 15) | (uint32_t)r) : 0xFFFFFFFFu;
    __syncthreads();
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n2; i += blockDim.x) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const uint32_t a = keys[i], b = keys[ixj];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        keys[i] = b;
                        keys[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int r = threadIdx.x; r < n; r += blockDim.x)
        psi[g.off + r] = tile_subpixel(g, W, (int)(keys[r] & 0x7FFFu));
}

hipError_t launch_remap(const uint16_t *V, int W, int H, int tw, int th, uint32_t *psi, hipStream_t s)
{
    const int T = ((W + tw - 1) / tw) * ((H + th - 1) / th);
    int n2 = 1;
    while (n2 < 3 * tw * th) n2 <<= 1;
    const size_t lds = (size_t)n2 * sizeof(uint32_t);
    if (lds > 65536) {
        // more than the default 64 KB of dynamic LDS per workgroup
        const hipError_t e =
            hipFuncSetAttribute((const void *)remap_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(remap_kernel, dim3(T), dim3(256), lds, s, V, W, H, tw, th, psi);
    return hipGetLastError();
}

// Work items for the remapped blend: walk each tile's subpixels in Psi order
// and cut a new item whenever the cluster changes, 64 subpixels are reached,
// or a new view would exceed kMaxWaveViews distinct views.  One thread per
// tile; `emit` selects counting or writing.
template <bool kEmit>
__global__ void __launch_bounds__(64) task_kernel(const uint16_t *V, const uint32_t *psi,
                                                  const int32_t *view_cluster, const int32_t *view_slot, int W,
                                                  int H, int tw, int th, int T, uint32_t *counts,
                                                  const uint32_t *offsets, Task *tasks)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const TileGeom g = tile_geom(t, W, H, tw, th);
    const int n = 3 * g.w * g.h;
    uint32_t nt = 0;
    int cur = -2, cnt = 0, nviews = 0, last_v = -1;
    Task tk{};
    Task *out = kEmit ? tasks + offsets[t] : nullptr;
    // 16 subpixels at a time: their Psi entries, views and clusters are each
    // loaded together, then walked one by one in order
    constexpr int kStep = 16;
    for (int r0 = 0; r0 < n; r0 += kStep) {
        int vs[kStep], cs[kStep];
#pragma unroll
        for (int q = 0; q < kStep; ++q) vs[q] = (int)psi[g.off + min(r0 + q, n - 1)];
#pragma unroll
        for (int q = 0; q < kStep; ++q) vs[q] = V[vs[q]];
#pragma unroll
        for (int q = 0; q < kStep; ++q) cs[q] = view_cluster[vs[q]];
#pragma unroll
        for (int q = 0; q < kStep; ++q) {
            const int r = r0 + q;
            if (r >= n) break;
            const int v = vs[q], c = cs[q];
            if (c < 0) continue;
            const bool new_view = v != last_v;
            if (c != cur || cnt == kWave || (new_view && nviews == kMaxWaveViews)) {
                if (kEmit && cur >= 0) out[nt - 1] = tk;
                ++nt;
                cur = c;
                cnt = 0;
                nviews = 0;
                last_v = -1;
                tk = Task{};
                tk.tile = (uint32_t)t;
                tk.cluster = (uint32_t)c;
                tk.start = (uint32_t)(g.off + r);
                for (int e = 0; e < 4; ++e) tk.run_start[e] = (uint8_t)kWave;
            }
            if (v != last_v) {
                if (kEmit) {
                    tk.run_start[nviews] = (uint8_t)cnt;
                    tk.slot[nviews] = (uint16_t)view_slot[v];
                }
                ++nviews;
                last_v = v;
            }
            ++cnt;
            tk.count = (uint16_t)cnt;
            tk.n_runs = (uint16_t)nviews;
        }
    }
    if (kEmit) {
        if (cur >= 0) out[nt - 1] = tk;
    } else {
        counts[t] = nt;
    }
}

hipError_t launch_task_count(const uint16_t *V, const uint32_t *psi, const int32_t *view_cluster,
                             int W, int H, int tw, int th, uint32_t *counts, hipStream_t s)
{
    const int T = ((W + tw - 1) / tw) * ((H + th - 1) / th);
    hipLaunchKernelGGL(task_kernel<false>, dim3((T + 63) / 64), dim3(64), 0, s, V, psi, view_cluster,
                       (const int32_t *)nullptr, W, H, tw, th, T, counts, (const uint32_t *)nullptr,
                       (Task *)nullptr);
    return hipGetLastError();
}

hipError_t launch_task_emit(const uint16_t *V, const uint32_t *psi, const int32_t *view_cluster,
                            const int32_t *view_slot, int W, int H, int tw, int th, const uint32_t *offsets,
                            Task *tasks, hipStream_t s)
{
    const int T = ((W + tw - 1) / tw) * ((H + th - 1) / th);
    hipLaunchKernelGGL(task_kernel<true>, dim3((T + 63) / 64), dim3(64), 0, s, V, psi, view_cluster, view_slot,
                       W, H, tw, th, T, (uint32_t *)nullptr, offsets, tasks);
    return hipGetLastError();
}

// Subpixels of every (tile, cluster) list: one thread per subpixel.
__global__ void __launch_bounds__(256) tc_count_kernel(const uint16_t *V, const int32_t *view_cluster, int W, int H,
                                                        int tw, int th, int cluster_bits, uint32_t *counts)
{
    const int64_t n = 3ll * W * H;
    const int TX = (W + tw - 1) / tw;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
        const int c = view_cluster[V[s]];
        if (c < 0) continue;
        const int64_t pix = s / 3;
        const int y = (int)(pix / W), x = (int)(pix - (int64_t)y * W);
        const uint32_t t = (uint32_t)((y / th) * TX + x / tw);
        atomicAdd(&counts[(t << cluster_bits) | (uint32_t)c], 1u);
    }
}

hipError_t launch_tc_count(const uint16_t *V, const int32_t *view_cluster, int W, int H, int tw, int th,
                           int cluster_bits, uint32_t *counts, hipStream_t s)
{
    hipLaunchKernelGGL(tc_count_kernel, dim3(grid_for(3ll * W * H, 256)), dim3(256), 0, s, V, view_cluster, W, H, tw,
                       th, cluster_bits, counts);
    return hipGetLastError();
}

}  // namespace lfr
