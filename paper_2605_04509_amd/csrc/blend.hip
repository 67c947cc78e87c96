// Alpha blending (section 4.3, Eq. 9-10; appendix B.2 Alpha-Blend).
//
// The subpixel blends are resumable: lists arrive in depth chunks (see
// binning.hip) and each launch continues every unsaturated subpixel from its
// saved (T, C), in the same front-to-back order as one uninterrupted pass.
// A subpixel's output is written when it saturates or after the last chunk.
//
// Every kernel here evaluates one (subpixel, Gaussian) step with the same
// inline function, so the remapped path, the row-major path and the
// full-frame baseline produce bit-identical values for the same inputs:
//   w = dx + beta*dy (one rounding), E = A' w^2 + G' dy^2,
//   alpha = min(0.99, o * 2^-E); skip if alpha < 1/255;
//   T' = T (1 - alpha); stop (without blending) if T' < 1e-4;
//   C += c * alpha * T; T = T'.
#include "lfr_internal.h"

namespace lfr {

// Large finite stand-in for a mean that is invalid in a view: E becomes
// +inf and alpha 0, so the Gaussian is skipped without a branch.
constexpr float kFarMean = 1e30f;

__device__ __forceinline__ float step_alpha(const float4 a, const float2 m, float px, float py)
{
    const float dx = px - m.x;
    const float dy = py - m.y;
    const float w = fmaf(a.y, dy, dx);
    const float E = fmaf(a.x * w, w, (a.z * dy) * dy);
    return fminf(kAlphaMax, a.w * __builtin_amdgcn_exp2f(-E));
}

__device__ __forceinline__ float2 sanitize_mean(float2 m)
{
    return isnan(m.x) ? make_float2(kFarMean, kFarMean) : m;
}

// Block index -> task index such that each of the 8 XCDs (which receive
// blocks round-robin) works on one contiguous range of tasks; neighbouring
// tiles then share their XCD's L2.  The grid has 8 * per blocks.
__device__ __forceinline__ int xcd_task(int b, int per) { return (b & 7) * per + (b >> 3); }

// Sum of a per-lane count over the wavefront, added once to a counter.
__device__ __forceinline__ void add_work(unsigned long long *dst, unsigned long long v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(dst, v);
}

// Saved per-subpixel state: (T, C), T negated once the subpixel saturated.
__device__ __forceinline__ void load_state(const BlendParams &bp, uint32_t at, float &T, float &C, bool &done)
{
    const float2 st = bp.state[at];
    done = st.x < 0.0f;
    T = fabsf(st.x);
    C = st.y;
}

// One 64-lane wavefront per task: up to 64 subpixels of one tile and one
// cluster, in Psi order.  Gaussians of the (tile, cluster) list are staged
// 64 at a time into LDS (record + the mean for each distinct view of the
// wavefront; the next batch is fetched into registers while the current one
// is evaluated), then every lane walks the batch.  The walk is branch-free:
// a lane that has stopped keeps executing with its updates masked by selects,
// and the wavefront leaves as soon as all of its lanes have stopped (checked
// every 16 Gaussians).  Batches are padded to a multiple of 4 with
// zero-opacity entries, whose alpha is 0 and never passes the cutoff.
template <bool kCount>
__global__ void __launch_bounds__(64) blend_remap_kernel(BlendParams bp, const Task *__restrict__ tasks,
                                                          int n_tasks, int per)
{
    __shared__ float4 s_a[kWave];
    __shared__ float s_c[kWave * 4];
    __shared__ float2 s_mu[kMaxWaveViews][kWave];
    __shared__ int s_slot[kMaxWaveViews];

    const int ti = xcd_task(blockIdx.x, per);
    if (ti >= n_tasks) return;
    if (!bp.first && !bp.task_alive[ti]) return;
    const Task tk = tasks[ti];
    const int lane = threadIdx.x;
    const bool active = lane < (int)tk.count;
    const uint32_t at = tk.start + (active ? lane : (int)tk.count - 1);
    const uint32_t p = bp.psi[at];
    const int j = bp.V[p];
    const uint32_t pix = p / 3;
    const int u = (int)(p - 3 * pix);
    const uint32_t y = pix / (uint32_t)bp.W;
    const uint32_t x = pix - y * (uint32_t)bp.W;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;

    // distinct views of this wavefront (Psi is sorted by view inside a tile)
    const int jprev = __shfl_up(j, 1, 64);
    const bool first = lane == 0 || j != jprev;
    const uint64_t runs = __ballot(first);
    const int my_run = __popcll(runs & ((2ull << lane) - 1ull)) - 1;
    const int n_runs = __popcll(runs);
    if (first) s_slot[my_run] = bp.view_slot[j];

    const uint32_t list = (tk.tile << bp.cluster_bits) | tk.cluster;
    const uint2 range = bp.ranges[list];
    const GaussRec *rec = bp.rec + (int64_t)tk.cluster * bp.M;
    float T = 1.0f, C = 0.0f;
    bool done = !active;
    if (!bp.first && active) load_state(bp, at, T, C, done);
    const bool was_done = done;
    unsigned long long n_eval = 0, n_blend = 0;
    __syncthreads();
    int slots[kMaxWaveViews];
#pragma unroll
    for (int q = 0; q < kMaxWaveViews; ++q) slots[q] = q < n_runs ? s_slot[q] : 0;

    // registers holding the batch being fetched
    float4 ga = make_float4(0.f, 0.f, 0.f, 0.f), gc = ga;
    float2 gm[kMaxWaveViews];
    auto fetch = [&](uint32_t base) {
        const uint32_t e = base + (uint32_t)lane;
        ga = make_float4(0.f, 0.f, 0.f, 0.f);
        gc = ga;
#pragma unroll
        for (int q = 0; q < kMaxWaveViews; ++q) gm[q] = make_float2(0.f, 0.f);
        if (e < range.y) {
            const uint32_t i = bp.vals[e];
            const GaussRec g = rec[i];
            ga = g.a;
            gc = g.c;
#pragma unroll
            for (int q = 0; q < kMaxWaveViews; ++q)
                if (q < n_runs) gm[q] = sanitize_mean(bp.mean2d[(int64_t)slots[q] * bp.M + i]);
        }
    };
    if (__ballot(!done) != 0 && range.x < range.y) {
        fetch(range.x);
        for (uint32_t base = range.x; base < range.y; base += kWave) {
            s_a[lane] = ga;
            *reinterpret_cast<float4 *>(&s_c[lane * 4]) = gc;
#pragma unroll
            for (int q = 0; q < kMaxWaveViews; ++q)
                if (q < n_runs) s_mu[q][lane] = gm[q];
            __syncthreads();
            if (base + kWave < range.y) fetch(base + kWave);
            const int nb = (int)min((uint32_t)kWave, range.y - base);
            const int nb4 = (nb + 3) & ~3;
            for (int g0 = 0; g0 < nb4; g0 += 16) {
                const int g1 = min(g0 + 16, nb4);
#pragma unroll 4
                for (int g = g0; g < g1; ++g) {
                    const float alpha = step_alpha(s_a[g], s_mu[my_run][g], px, py);
                    const float Tn = T * (1.0f - alpha);
                    const bool pass = !done && alpha >= kAlphaMin;
                    const bool take = pass && Tn >= kTStop;
                    if (kCount) {
                        n_eval += (!done && g < nb) ? 1u : 0u;
                        n_blend += take ? 1u : 0u;
                    }
                    C = take ? fmaf(s_c[g * 4 + u] * alpha, T, C) : C;
                    T = take ? Tn : T;
                    done = done || (pass && !take);
                }
                if (__ballot(!done) == 0) break;
            }
            if (__ballot(!done) == 0) break;
            __syncthreads();
        }
    }
    const uint64_t newly = __ballot(active && done && !was_done);
    const bool all_done = __ballot(!done) == 0;
    if (all_done || bp.last) {
        if (active) bp.out[p] = C + T * bp.bg[u];
    } else if (active) {
        bp.state[at] = make_float2(done ? -T : T, C);
    }
    if (lane == 0) {
        if (all_done) bp.task_alive[ti] = 0;
        const uint32_t nn = (uint32_t)__popcll(newly);
        if (nn) {
            atomicSub(&bp.tc_alive[list], nn);
            atomicSub(bp.alive_total, nn);
        }
    }
    if (kCount) {
        add_work(bp.work, n_eval);
        add_work(bp.work + 1, n_blend);
    }
}

// Row-major thread order (no remap): a 256-thread block per tile, each
// thread takes subpixels r = tid, tid+256, ... of the tile's row-major list
// and walks its own (tile, cluster) list from global memory.  State is kept
// per panel subpixel.
template <bool kCount>
__global__ void __launch_bounds__(256) blend_rowmajor_kernel(BlendParams bp)
{
    unsigned long long n_eval = 0, n_blend = 0;
    const int t = blockIdx.x;
    const int ty = t / bp.TX, tx = t - ty * bp.TX;
    const int x0 = tx * bp.tw, y0 = ty * bp.th;
    const int w = min(bp.tw, bp.W - x0), h = min(bp.th, bp.H - y0);
    const int n = 3 * w * h;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        const int ly = r / (3 * w);
        const int rem = r - ly * 3 * w;
        const int lx = rem / 3;
        const int u = rem - 3 * lx;
        const int x = x0 + lx, y = y0 + ly;
        const uint32_t p = (uint32_t)(((int64_t)y * bp.W + x) * 3 + u);
        float T = 1.0f, C = 0.0f;
        bool done = false;
        if (!bp.first) {
            load_state(bp, p, T, C, done);
            if (done) continue;
        }
        const int j = bp.V[p];
        const int c = bp.view_cluster[j];
        const int slot = bp.view_slot[j];
        const uint32_t list = ((uint32_t)t << bp.cluster_bits) | (uint32_t)c;
        const uint2 range = bp.ranges[list];
        const GaussRec *rec = bp.rec + (int64_t)c * bp.M;
        const float2 *mu = bp.mean2d + (int64_t)slot * bp.M;
        const float px = (float)x + 0.5f, py = (float)y + 0.5f;
        for (uint32_t e = range.x; e < range.y; ++e) {
            const uint32_t i = bp.vals[e];
            const GaussRec g = rec[i];
            const float alpha = step_alpha(g.a, sanitize_mean(mu[i]), px, py);
            if (kCount) ++n_eval;
            if (alpha < kAlphaMin) continue;
            const float Tn = T * (1.0f - alpha);
            if (Tn < kTStop) {
                done = true;
                break;
            }
            const float col = u == 0 ? g.c.x : (u == 1 ? g.c.y : g.c.z);
            C = fmaf(col * alpha, T, C);
            T = Tn;
            if (kCount) ++n_blend;
        }
        if (done || bp.last) bp.out[p] = C + T * bp.bg[u];
        if (done) {
            if (!bp.last) bp.state[p] = make_float2(-T, C);
            atomicSub(&bp.tc_alive[list], 1u);
            atomicSub(bp.alive_total, 1u);
        } else if (!bp.last) {
            bp.state[p] = make_float2(T, C);
        }
    }
    if (kCount) {
        add_work(bp.work, n_eval);
        add_work(bp.work + 1, n_blend);
    }
}

// Standard single-view 3DGS tile blend for the full-frame baseline: one
// block per (tile, view), one thread per pixel, batches of Gaussians staged
// through LDS, RGB sharing one alpha and one transmittance.
__global__ void __launch_bounds__(1024) blend_fullframe_kernel(FullFrameParams fp)
{
    extern __shared__ float4 smem[];
    const int nthr = blockDim.x;
    float4 *s_a = smem;                                        // [nthr]
    float4 *s_c = smem + nthr;                                 // [nthr]
    float2 *s_mu = reinterpret_cast<float2 *>(smem + 2 * nthr);  // [nthr]
    const int t = blockIdx.x, b = blockIdx.y;
    const int ty = t / fp.TX, tx = t - ty * fp.TX;
    const int lx = threadIdx.x % fp.tw, ly = threadIdx.x / fp.tw;
    const int x = tx * fp.tw + lx, y = ty * fp.th + ly;
    const bool inside = x < fp.W && y < fp.H;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const uint2 range = fp.ranges[((uint32_t)t << fp.cluster_bits) | (uint32_t)b];
    const GaussRec *rec = fp.rec + (int64_t)b * fp.M;
    const float2 *mu = fp.mean2d + (int64_t)b * fp.M;
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    bool done = !inside;
    for (uint32_t base = range.x; base < range.y; base += (uint32_t)nthr) {
        const int nb = (int)min((uint32_t)nthr, range.y - base);
        __syncthreads();
        if ((int)threadIdx.x < nb) {
            const uint32_t i = fp.vals[base + threadIdx.x];
            const GaussRec g = rec[i];
            s_a[threadIdx.x] = g.a;
            s_c[threadIdx.x] = g.c;
            s_mu[threadIdx.x] = sanitize_mean(mu[i]);
        }
        __syncthreads();
        if (!done) {
            for (int g = 0; g < nb; ++g) {
                const float alpha = step_alpha(s_a[g], s_mu[g], px, py);
                if (alpha < kAlphaMin) continue;
                const float Tn = T * (1.0f - alpha);
                if (Tn < kTStop) {
                    done = true;
                    break;
                }
                const float4 c = s_c[g];
                C0 = fmaf(c.x * alpha, T, C0);
                C1 = fmaf(c.y * alpha, T, C1);
                C2 = fmaf(c.z * alpha, T, C2);
                T = Tn;
            }
        }
        if (__syncthreads_count(!done) == 0) break;
    }
    if (inside) {
        float *o = fp.images + ((int64_t)b * fp.H * fp.W + (int64_t)y * fp.W + x) * 3;
        o[0] = C0 + T * fp.bg[0];
        o[1] = C1 + T * fp.bg[1];
        o[2] = C2 + T * fp.bg[2];
    }
}

__global__ void __launch_bounds__(256) interlace_kernel(const uint16_t *__restrict__ V, int64_t n,
                                                         const int32_t *__restrict__ batch_slot,
                                                         const float *__restrict__ images, int64_t stride,
                                                         float *__restrict__ out)
{
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
        const int b = batch_slot[V[s]];
        if (b >= 0) out[s] = images[(int64_t)b * stride + s];
    }
}

hipError_t launch_blend_remap(const BlendParams &bp, const Task *tasks, int n_tasks, hipStream_t s)
{
    if (n_tasks == 0) return hipSuccess;
    const int per = (n_tasks + 7) / 8;
    if (bp.work)
        hipLaunchKernelGGL(blend_remap_kernel<true>, dim3((unsigned)(8 * per)), dim3(kWave), 0, s, bp, tasks, n_tasks, per);
    else
        hipLaunchKernelGGL(blend_remap_kernel<false>, dim3((unsigned)(8 * per)), dim3(kWave), 0, s, bp, tasks, n_tasks, per);
    return hipGetLastError();
}

hipError_t launch_blend_rowmajor(const BlendParams &bp, hipStream_t s)
{
    const int T = bp.TX * ((bp.H + bp.th - 1) / bp.th);
    if (bp.work)
        hipLaunchKernelGGL(blend_rowmajor_kernel<true>, dim3((unsigned)T), dim3(256), 0, s, bp);
    else
        hipLaunchKernelGGL(blend_rowmajor_kernel<false>, dim3((unsigned)T), dim3(256), 0, s, bp);
    return hipGetLastError();
}

hipError_t launch_blend_fullframe(const FullFrameParams &fp, hipStream_t s)
{
    const int T = fp.TX * fp.TY;
    const int nthr = fp.tw * fp.th;
    const size_t shm = (size_t)nthr * (2 * sizeof(float4) + sizeof(float2));
    hipLaunchKernelGGL(blend_fullframe_kernel, dim3((unsigned)T, (unsigned)fp.n_views), dim3(nthr), shm, s, fp);
    return hipGetLastError();
}

hipError_t launch_interlace(const uint16_t *V, int64_t n_sub, const int32_t *batch_slot, const float *images,
                            int64_t stride, float *out, hipStream_t s)
{
    int64_t g = (n_sub + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(interlace_kernel, dim3((unsigned)g), dim3(256), 0, s, V, n_sub, batch_slot, images, stride,
                       out);
    return hipGetLastError();
}

}  // namespace lfr
