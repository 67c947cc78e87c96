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


// Intermediates of one step, shared by the forward and the reverse blend so
// that both evaluate alpha with the same float32 operations.
struct StepEval {
    float dy, w, ex, raw;  // raw = o 2^-E before the clamp
};

// E of the sample (px, py) for record a = (A', beta, G', o) and mean m.
__device__ __forceinline__ float step_exponent(const float4 a, const float2 m, float px, float py, StepEval &s)
{
    const float dx = px - m.x;
    s.dy = py - m.y;
    s.w = fmaf(a.y, s.dy, dx);
    return fmaf(a.x * s.w, s.w, (a.z * s.dy) * s.dy);
}

// alpha = min(0.99, o 2^-E).
__device__ __forceinline__ float step_alpha_of(float o, float E, StepEval &s)
{
    s.ex = __builtin_amdgcn_exp2f(-E);
    s.raw = o * s.ex;
    return fminf(kAlphaMax, s.raw);
}

__device__ __forceinline__ float step_eval(const float4 a, const float2 m, float px, float py, StepEval &s)
{
    return step_alpha_of(a.w, step_exponent(a, m, px, py, s), s);
}

__device__ __forceinline__ float step_alpha(const float4 a, const float2 m, float px, float py)
{
    StepEval s;
    return step_eval(a, m, px, py, s);
}

__device__ __forceinline__ float2 sanitize_mean(float2 m)
{
    return isnan(m.x) ? make_float2(kFarMean, kFarMean) : m;
}

// Block index -> task index.  Blocks are dealt to the 8 XCDs round-robin;
// XCD x runs task groups x, x + 8, x + 16, ... (groups of 2^sh consecutive
// tasks) in order.  Tasks are ordered cluster by cluster over blocks of
// neighbouring tiles, so a group sized to about one such block keeps the
// tasks that read the same Gaussians' records on one XCD and its L2, while
// every XCD sweeps the whole panel: the work per tile varies strongly
// across the panel, and contiguous eighths of it would leave some XCDs idle
// early.  The grid is rounded up to whole rounds of 8 groups.
__device__ __forceinline__ int xcd_task(int b, int sh)
{
    const int x = b & 7, l = b >> 3;
    return ((((l >> sh) << 3) + x) << sh) + (l & ((1 << sh) - 1));
}
static unsigned xcd_grid(int n_tasks, int sh)
{
    const int r = 8 << sh;
    return (unsigned)((n_tasks + r - 1) / r * r);
}

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
// 64 at a time into LDS (record, colour, cutoff exponent and the mean for
// each distinct view of the wavefront; the next batch is fetched into
// registers while the current one is evaluated), then every lane walks the
// batch.  The walk is branch-free per lane: a lane that has stopped keeps
// executing with its updates masked by selects, and the wavefront leaves as
// soon as all of its lanes have stopped (checked every 16 Gaussians).  A step
// in which no unfinished lane is within the cutoff exponent of the Gaussian
// is skipped as a whole (nothing would change).  Batches are padded to a
// multiple of 4 with zero-opacity entries, which never pass the cutoff.
//
// A lane that stops folds the background into its colour, C + T bg (the same
// operations as the final write), and sets T = 0: afterwards T (1 - alpha)
// can never pass the stop test, so T = 0 is its "finished" state, here and in
// the saved per-subpixel state between depth chunks.  The output C + T bg is
// then C + 0 = C, the same value as writing C + T bg at the stop.
// kSave (single-chunk renders) also writes each subpixel's final T (before
// the fold) and the end of its blended list for the backward.
template <bool kCount, bool kSave>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(6))) blend_remap_kernel(BlendParams bp, const Task *__restrict__ tasks,
                                                          int n_tasks, int xcd_shift)
{
    __shared__ float4 s_a[kWave];
    __shared__ float s_c[kWave * 4];
    __shared__ float2 s_mu[kMaxWaveViews][kWave];
    __shared__ float4 s_box[kMaxWaveViews];         // per view run: unfinished lanes' x0, x1, y0, y1
    __shared__ uint32_t s_pos[kSave || kCount ? kWave : 1];  // list position of each staged entry

    const int ti = xcd_task(blockIdx.x, xcd_shift);
    if (ti >= n_tasks) return;
    // the item and its alive flag are loaded together (the test reads both;
    // an item always has at least one lane)
    const Task tk = tasks[ti];
    if ((!bp.first && !bp.task_alive[ti]) || tk.count == 0) return;
    const int lane = threadIdx.x;
    const bool active = lane < (int)tk.count;
    const uint32_t at = tk.start + (active ? lane : (int)tk.count - 1);
    const uint32_t p = bp.psi[at];
    const uint32_t pix = p / 3;
    const int u = (int)(p - 3 * pix);
    const uint32_t y = pix / (uint32_t)bp.W;
    const uint32_t x = pix - y * (uint32_t)bp.W;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const float bgu = bp.bg[u];
    // this lane's view run (the task's lanes are runs of one view each)
    const int n_runs = tk.n_runs;
    const int my_run = (lane >= (int)tk.run_start[1]) + (lane >= (int)tk.run_start[2]) + (lane >= (int)tk.run_start[3]);

    const uint32_t list = (tk.tile << bp.cluster_bits) | tk.cluster;
    const uint2 range = bp.ranges[list];
    const GaussRec *rec = bp.rec + (int64_t)tk.cluster * bp.M;
    // a merged batch group: the frame's output and its slice of the state
    float *const out = bp.out_frames ? bp.out_frames[tk.frame] : bp.out;
    float2 *const state = bp.state + (int64_t)tk.frame * bp.n_sub;
    float T = 1.0f, C = 0.0f;
    if (!bp.first && active) {
        const float2 st = state[at];
        T = st.x;
        C = st.y;
    }
    if (!active) T = 0.0f;
    const bool was_done = T == 0.0f;
    float Tsave = T;
    unsigned long long n_blend = 0, n_steps = 0, n_live = 0;
    uint32_t endp = 0;
    uint32_t stopl = range.y;  // (counting) list position after this lane's stop
    // sample-centre bounding box of each view run's unfinished lanes
    {
#pragma unroll
        for (int q = 0; q < kMaxWaveViews; ++q) {
            if (q >= n_runs) break;
            const bool in = (T > 0.0f) & (my_run == q);
            float x0 = in ? px : 3e38f, x1 = in ? px : -3e38f, y0 = in ? py : 3e38f, y1 = in ? py : -3e38f;
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) {
                x0 = fminf(x0, __shfl_xor(x0, d, 64));
                x1 = fmaxf(x1, __shfl_xor(x1, d, 64));
                y0 = fminf(y0, __shfl_xor(y0, d, 64));
                y1 = fmaxf(y1, __shfl_xor(y1, d, 64));
            }
            if (lane == 0) s_box[q] = make_float4(x0, x1, y0, y1);
        }
    }
    __syncthreads();
    int slots[kMaxWaveViews];
#pragma unroll
    for (int q = 0; q < kMaxWaveViews; ++q) slots[q] = tk.slot[q];
    // a cluster of at most kItemViews views keeps its means in the record, so
    // an entry's conic, colour and means come from one cache line; the runs'
    // views are then record slots (view slots are numbered in view order)
    const int cv0 = bp.cv_off[tk.cluster];
    const bool inline_means = bp.cv_off[tk.cluster + 1] - cv0 <= kItemViews;

    // Registers holding the batch being fetched, and the Gaussian indices of
    // the batch after it.  fetch() only issues loads (the record and means of
    // batch `base`, whose indices arrived during the previous batch, and the
    // indices of the next one); their values are first used when the batch
    // is staged, after the walk of the batch before it.
    float4 ga = make_float4(0.f, 0.f, 0.f, 0.f), gc = ga;
    float2 gm[kMaxWaveViews];
    uint32_t nidx = 0;
    auto load_index = [&](uint32_t base) {
        const uint32_t e = base + (uint32_t)lane;
        nidx = e < range.y ? bp.vals[e] : 0u;
    };
    auto fetch = [&](uint32_t base) {
        const uint32_t e = base + (uint32_t)lane;
        ga = make_float4(0.f, 0.f, 0.f, 0.f);
        gc = ga;
#pragma unroll
        for (int q = 0; q < kMaxWaveViews; ++q) gm[q] = make_float2(0.f, 0.f);
        if (e < range.y) {
            const uint32_t i = nidx;
            ga = rec[i].a;
            gc = rec[i].c;  // .w: the cutoff exponent
#pragma unroll
            for (int q = 0; q < kMaxWaveViews; ++q)
                if (q < n_runs)
                    gm[q] = inline_means ? rec[i].m[slots[q] - cv0] : bp.mean2d[(int64_t)slots[q] * bp.M + i];
        }
        load_index(base + kWave);
    };
    // Whether this lane's fetched Gaussian can reach any unfinished lane: the
    // region E <= E_cut lies in |dy| <= sqrt(E_cut / G'), |dx| <= sqrt(E_cut /
    // A') + |beta| |dy| (E = A'(dx + beta dy)^2 + G' dy^2), widened by 0.1%
    // and 1e-3 px for rounding (far above the one-ulp error of the hardware
    // reciprocal and square root used here); outside it alpha < 0.9986 / 255
    // for every lane, so dropping the Gaussian changes nothing.  (A cutoff of
    // exactly 0 with a vanishing conic term gives NaN and drops the Gaussian:
    // a cutoff below 0.01 never passes.)
    auto relevant = [&](uint32_t base) -> bool {
#pragma unroll
        for (int q = 0; q < kMaxWaveViews; ++q) gm[q] = sanitize_mean(gm[q]);
        if (base + (uint32_t)lane >= range.y) return false;
        const float thr = gc.w;
        if (!(thr >= 0.0f)) return false;
        const float hy = __builtin_amdgcn_sqrtf(thr * __builtin_amdgcn_rcpf(ga.z)) * 1.001f + 1e-3f;
        const float hx = __builtin_amdgcn_sqrtf(thr * __builtin_amdgcn_rcpf(ga.x)) * 1.001f + fabsf(ga.y) * hy + 1e-3f;
        bool r = false;
#pragma unroll
        for (int q = 0; q < kMaxWaveViews; ++q) {
            if (q >= n_runs) break;
            const float4 b = s_box[q];
            r = r | ((gm[q].x + hx >= b.x) & (gm[q].x - hx <= b.y) & (gm[q].y + hy >= b.z) & (gm[q].y - hy <= b.w));
        }
        return r;
    };
    if (__ballot(T > 0.0f) != 0 && range.x < range.y) {
        load_index(range.x);
        fetch(range.x);
        for (uint32_t base = range.x; base < range.y; base += kWave) {
            // stage the relevant entries of this batch, compacted in list order
            const bool rel = relevant(base);
            const uint64_t rmask = __ballot(rel);
            const int nb = __popcll(rmask);
            if (rel) {
                const int pos = __popcll(rmask & ((1ull << lane) - 1ull));
                s_a[pos] = ga;
                *reinterpret_cast<float4 *>(&s_c[pos * 4]) = gc;
#pragma unroll
                for (int q = 0; q < kMaxWaveViews; ++q)
                    if (q < n_runs) s_mu[q][pos] = gm[q];
                if (kSave || kCount) s_pos[pos] = base + (uint32_t)lane;
            }
            if (lane >= nb && lane < ((nb + 3) & ~3)) {
                // padding up to a multiple of 4 (slots no relevant entry uses,
                // whatever this lane's own entry was): zero opacity, never passes
                s_a[lane] = make_float4(0.f, 0.f, 0.f, 0.f);
                s_c[lane * 4 + 3] = -__builtin_inff();
#pragma unroll
                for (int q = 0; q < kMaxWaveViews; ++q)
                    if (q < n_runs) s_mu[q][lane] = make_float2(0.f, 0.f);
            }
            __syncthreads();
            if (base + kWave < range.y) fetch(base + kWave);
            const int nb4 = (nb + 3) & ~3;
            for (int g0 = 0; g0 < nb4; g0 += 16) {
                const int g1 = min(g0 + 16, nb4);
                // groups of 4 steps with a constant-trip inner loop, so the
                // steps unroll despite the wavefront votes inside them
                for (int g4 = g0; g4 < g1; g4 += 4) {
                    // the group's LDS reads are all issued before its first step
                    float4 A[4];
                    float2 MU[4];
                    float CU[4], TH[4];
#pragma unroll
                    for (int gk = 0; gk < 4; ++gk) {
                        A[gk] = s_a[g4 + gk];
                        CU[gk] = s_c[(g4 + gk) * 4 + u];
                        TH[gk] = s_c[(g4 + gk) * 4 + 3];
                        MU[gk] = s_mu[my_run][g4 + gk];
                    }
                    // the four exponents are independent: compute them together,
                    // and skip the whole group when no unfinished lane is within
                    // any of the four cutoffs
                    StepEval st[4];
                    float E[4];
#pragma unroll
                    for (int gk = 0; gk < 4; ++gk) E[gk] = step_exponent(A[gk], MU[gk], px, py, st[gk]);
                    // lane masks of "within the cutoff", combined on the scalar unit
                    uint64_t within[4];
#pragma unroll
                    for (int gk = 0; gk < 4; ++gk) within[gk] = __ballot(E[gk] <= TH[gk]);
                    const bool skip_group =
                        ((within[0] | within[1] | within[2] | within[3]) & __ballot(T > 0.0f)) == 0;
                    if (kCount) n_steps += lane == 0 ? (unsigned)min(4, nb - g4) : 0u;
                    if (skip_group) continue;
#pragma unroll
                    for (int gk = 0; gk < 4; ++gk) {
                        const int g = g4 + gk;
                        // no unfinished lane within this cutoff: nothing changes
                        if ((within[gk] & __ballot(T > 0.0f)) == 0) continue;
                        const float alpha = step_alpha_of(A[gk].w, E[gk], st[gk]);
                        const float Tn = T * (1.0f - alpha);
                        const bool pass = alpha >= kAlphaMin;
                        const bool take = pass & (Tn >= kTStop);
                        const bool stop = pass & !take & (T > 0.0f);
                        if (kCount) {
                            n_blend += take ? 1u : 0u;
                            const bool live = __ballot(pass & (T > 0.0f)) != 0;
                            n_live += (lane == 0 && live) ? 1u : 0u;
                            stopl = stop ? s_pos[g] + 1u : stopl;
                        }
                        // branch-free update: fma(0, T, C) = C for a lane that does not take
                        const float wgt = take ? CU[gk] * alpha : 0.0f;
                        const float Ct = fmaf(wgt, T, C);
                        C = stop ? C + T * bgu : Ct;
                        if (kSave) {
                            endp = take ? s_pos[g] + 1u : endp;
                            Tsave = stop ? T : (take ? Tn : Tsave);
                        }
                        T = take ? Tn : (stop ? 0.0f : T);
                    }
                }
                if (__ballot(T > 0.0f) == 0) break;
            }
            if (__ballot(T > 0.0f) == 0) break;
            __syncthreads();
        }
    }
    const bool done = T == 0.0f;
    const uint64_t newly = __ballot(active && done && !was_done);
    const bool all_done = __ballot(!done) == 0;
    if (all_done || bp.last) {
        if (active) {
            out[p] = C + T * bgu;
            if (kSave) {
                bp.save_T[p] = Tsave;
                bp.save_end[p] = endp;
            }
        }
    } else if (active) {
        state[at] = make_float2(T, C);
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
        // the method evaluates every list entry up to and including the one
        // at which the lane stops (culled entries included)
        add_work(bp.work, was_done ? 0ull : (unsigned long long)(stopl - range.x));
        add_work(bp.work + 1, n_blend);
        add_work(bp.work + 2, n_steps);
        add_work(bp.work + 3, n_live);
    }
}

// Row-major thread order (no remap): a 256-thread block per tile, each
// thread takes subpixels r = tid, tid+256, ... of the tile's row-major list
// and walks its own (tile, cluster) list from global memory.  State is kept
// per panel subpixel.
template <bool kCount, bool kSave>
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
        uint32_t endp = 0;
        for (uint32_t e = range.x; e < range.y; ++e) {
            const uint32_t i = bp.vals[e];
            const float4 ga = rec[i].a;
            const float alpha = step_alpha(ga, sanitize_mean(mu[i]), px, py);
            if (kCount) ++n_eval;
            if (alpha < kAlphaMin) continue;
            const float Tn = T * (1.0f - alpha);
            if (Tn < kTStop) {
                done = true;
                break;
            }
            const float4 gc = rec[i].c;
            const float col = u == 0 ? gc.x : (u == 1 ? gc.y : gc.z);
            C = fmaf(col * alpha, T, C);
            T = Tn;
            endp = e + 1;
            if (kCount) ++n_blend;
        }
        if (done || bp.last) bp.out[p] = C + T * bp.bg[u];
        if (kSave) {
            bp.save_T[p] = T;
            bp.save_end[p] = endp;
        }
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
            s_a[threadIdx.x] = rec[i].a;
            s_c[threadIdx.x] = rec[i].c;
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

// ---------------------------------------------------------------------------
// Reverse blend (derivative of Eq. 9-10 with the forward's decisions held).
//
// For one subpixel with blended list e = 0..n-1 (alpha_e, colour c_e, T_e the
// transmittance in front of e) and output I = sum_e c_e alpha_e T_e + T_n bg:
//   dI/dc_e     = alpha_e T_e
//   dI/dalpha_e = c_e T_e - (sum_{h>e} c_h alpha_h T_h + T_n bg) / (1 - alpha_e)
// Walking the list back to front from its saved end, T_e = T_{e+1}/(1-alpha_e)
// recovers the transmittance from the saved T_n, and the bracket is a running
// sum.  Through alpha = o 2^-E (no clamp active): dalpha/do = 2^-E,
// dalpha/dE = -alpha ln 2, and E = A'(dx + beta dy)^2 + G' dy^2 with
// (dx, dy) = sample - mean gives the record and mean derivatives.
//
// One wavefront per work item, as in the forward: the (tile, cluster) list is
// staged 64 entries at a time from the top of the wavefront's highest list
// end downwards.  Each entry's seven record derivatives (and the two mean
// derivatives per view of the wavefront) are summed over the 64 lanes and
// added to the per-(cluster, Gaussian) and per-(view, Gaussian) gradient
// buffers with one float atomic per value.
// ---------------------------------------------------------------------------
constexpr float kLn2 = 0.69314718055994530942f;

template <int kCtrl>
__device__ __forceinline__ float dpp_get(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, 0xF, 0xF, false));
}

// Value of lane (lane ^ m) for m = 1, 2, 4, 8 with DPP inside 16-lane rows
// (quad permutations for 1 and 2, a row shift in the lane's direction for 4
// and 8), and through a lane permute for 16 and 32.
// (Both row shifts are computed by every lane before the select: a DPP read
// in a divergent branch would read lanes the branch has switched off.)
template <int m>
__device__ __forceinline__ float lane_xor(float v, int lane)
{
    if constexpr (m == 1) {
        return dpp_get<0xB1>(v);
    } else if constexpr (m == 2) {
        return dpp_get<0x4E>(v);
    } else if constexpr (m == 4) {
        const float from_below = dpp_get<0x114>(v), from_above = dpp_get<0x104>(v);
        return (lane & 4) ? from_below : from_above;
    } else if constexpr (m == 8) {
        const float from_below = dpp_get<0x118>(v), from_above = dpp_get<0x108>(v);
        return (lane & 8) ? from_below : from_above;
    } else {
        return __shfl_xor(v, m, 64);
    }
}

// One halving step of a transposed reduction: lanes with bit m set keep the
// upper half of their n values, the others the lower half, each adding the
// half its partner (lane ^ m) gives away.
template <int m, int n>
__device__ __forceinline__ void halve(float (&v)[16], int lane)
{
    const bool up = (lane & m) != 0;
#pragma unroll
    for (int j = 0; j < n / 2; ++j) {
        const float keep = up ? v[j + n / 2] : v[j];
        const float give = up ? v[j] : v[j + n / 2];
        v[j] = keep + lane_xor<m>(give, lane);
    }
}

// Sums of 16 per-lane values over the wavefront: after halving steps on
// lane bits 0..3 each lane holds one value index's sum over its 16-lane
// row, and two more exchanges add the four rows.  Lane l ends with the sum
// of value (bit-reversed l & 15).
__device__ __forceinline__ float wave_sum16(float (&v)[16], int lane)
{
    halve<1, 16>(v, lane);
    halve<2, 8>(v, lane);
    halve<4, 4>(v, lane);
    halve<8, 2>(v, lane);
    float r = v[0];
    r += lane_xor<16>(r, lane);
    r += lane_xor<32>(r, lane);
    return r;
}

__device__ __forceinline__ int rev4(int l)
{
    return ((l & 1) << 3) | ((l & 2) << 1) | ((l & 4) >> 1) | ((l & 8) >> 3);
}

__global__ void __launch_bounds__(64) blend_backward_kernel(BwdParams bp, const Task *__restrict__ tasks,
                                                             int n_tasks, int xcd_shift)
{
    __shared__ float4 s_a[kWave];
    __shared__ float s_c[kWave * 4];
    __shared__ float2 s_mu[kMaxWaveViews][kWave];
    __shared__ uint32_t s_i[kWave];

    const int ti = xcd_task(blockIdx.x, xcd_shift);
    if (ti >= n_tasks) return;
    const Task tk = tasks[ti];
    const int lane = threadIdx.x;
    const bool active = lane < (int)tk.count;
    const uint32_t at = tk.start + (active ? lane : (int)tk.count - 1);
    const uint32_t p = bp.psi[at];
    const uint32_t pix = p / 3;
    const int u = (int)(p - 3 * pix);
    const uint32_t y = pix / (uint32_t)bp.W;
    const uint32_t x = pix - y * (uint32_t)bp.W;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const int n_runs = tk.n_runs;
    const int my_run = (lane >= (int)tk.run_start[1]) + (lane >= (int)tk.run_start[2]) + (lane >= (int)tk.run_start[3]);

    const float gout = active ? bp.grad_out[p] : 0.0f;
    const uint32_t end = (active && gout != 0.0f) ? bp.save_end[p] : 0u;
    float T = active ? bp.save_T[p] : 0.0f;
    float rest = T * bp.bg[u];
    const uint32_t list = (tk.tile << bp.cluster_bits) | tk.cluster;
    const uint2 range = bp.ranges[list];
    uint32_t hi = end;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) hi = max(hi, (uint32_t)__shfl_xor((int)hi, d, 64));
    if (hi <= range.x) return;
    int slots[kMaxWaveViews];
#pragma unroll
    for (int q = 0; q < kMaxWaveViews; ++q) slots[q] = tk.slot[q];
    const GaussRec *rec = bp.rec + (int64_t)tk.cluster * bp.M;
    const int cv0 = bp.cv_off[tk.cluster];
    const bool inline_means = bp.cv_off[tk.cluster + 1] - cv0 <= kItemViews;
    float *drec = reinterpret_cast<float *>(bp.d_rec + (int64_t)tk.cluster * bp.M);
    float *dmean = reinterpret_cast<float *>(bp.d_mean2d);

    for (uint32_t top = hi; top > range.x;) {
        const uint32_t b0 = top - range.x > (uint32_t)kWave ? top - (uint32_t)kWave : range.x;
        const int nb = (int)(top - b0);
        if (lane < nb) {
            const uint32_t i = bp.vals[b0 + lane];
            s_a[lane] = rec[i].a;
            *reinterpret_cast<float4 *>(&s_c[lane * 4]) = rec[i].c;  // .w: the cutoff exponent
            s_i[lane] = i;
#pragma unroll
            for (int q = 0; q < kMaxWaveViews; ++q)
                if (q < n_runs)
                    s_mu[q][lane] = sanitize_mean(inline_means ? rec[i].m[slots[q] - cv0]
                                                               : bp.mean2d[(int64_t)slots[q] * bp.M + i]);
        }
        __syncthreads();
        for (int g = nb - 1; g >= 0; --g) {
            const float4 a = s_a[g];
            StepEval st;
            const float E = step_exponent(a, s_mu[my_run][g], px, py, st);
            const bool in_list = b0 + (uint32_t)g < end;
            if (__ballot(in_list && E <= s_c[g * 4 + 3]) == 0) continue;
            const float alpha = step_alpha_of(a.w, E, st);
            const bool on = in_list && alpha >= kAlphaMin;
            if (__ballot(on) == 0) continue;
            const float c = s_c[g * 4 + u];
            const float inv = __builtin_amdgcn_rcpf(1.0f - alpha);
            const float Tg = T * inv;
            const float dc = on ? gout * alpha * Tg : 0.0f;
            const float da = gout * (c * Tg - rest * inv);
            rest = on ? fmaf(c * alpha, Tg, rest) : rest;
            T = on ? Tg : T;
            // lanes that do not take this entry contribute exact zeros (their
            // w may be huge for a view where the mean is invalid, so the
            // products are selected, not multiplied by zero)
            const bool smooth = on && st.raw <= kAlphaMax;
            const float dE = -da * st.raw * kLn2;
            const float t2 = 2.0f * a.x * st.w;
            // the mean of the lane's view: d/dmean = -d/d(dx, dy)
            const float dmx = smooth ? -dE * t2 : 0.0f;
            const float dmy = smooth ? -dE * fmaf(t2, a.y, 2.0f * a.z * st.dy) : 0.0f;
            // values 0..6: record derivatives dA', dbeta, dG', do, dr, dg, db;
            // 8 + 2q, 9 + 2q: mean derivatives of the task's view q
            float v[16];
            v[0] = smooth ? dE * st.w * st.w : 0.0f;
            v[1] = smooth ? dE * t2 * st.dy : 0.0f;
            v[2] = smooth ? dE * st.dy * st.dy : 0.0f;
            v[3] = smooth ? da * st.ex : 0.0f;
            v[4] = u == 0 ? dc : 0.0f;
            v[5] = u == 1 ? dc : 0.0f;
            v[6] = u == 2 ? dc : 0.0f;
            v[7] = 0.0f;
#pragma unroll
            for (int q = 0; q < kMaxWaveViews; ++q) {
                v[8 + 2 * q] = my_run == q ? dmx : 0.0f;
                v[9 + 2 * q] = my_run == q ? dmy : 0.0f;
            }
            const float sum = wave_sum16(v, lane);
            const uint32_t i = s_i[g];
            const int idx = rev4(lane & 15);
            if (lane < 16 && idx < 7) {
                unsafeAtomicAdd(drec + (int64_t)i * 8 + idx, sum);
            } else if (lane < 16 && idx >= 8) {
                const int q = (idx - 8) >> 1;
                // (selects, not slots[q]: a per-lane index could put the array in scratch)
                const int sq = q == 0 ? slots[0] : q == 1 ? slots[1] : q == 2 ? slots[2] : slots[3];
                if (q < n_runs && sum != 0.0f)
                    unsafeAtomicAdd(dmean + ((int64_t)sq * bp.M + i) * 2 + (idx & 1), sum);
            }
        }
        __syncthreads();
        top = b0;
    }
}

hipError_t launch_blend_remap(const BlendParams &bp, const Task *tasks, int n_tasks, int xcd_shift, hipStream_t s)
{
    if (n_tasks == 0) return hipSuccess;
    if (xcd_shift < 0 || xcd_shift > 12) return hipErrorInvalidValue;
    const dim3 grid(xcd_grid(n_tasks, xcd_shift)), block(kWave);
    if (bp.work && bp.save_T)
        hipLaunchKernelGGL((blend_remap_kernel<true, true>), grid, block, 0, s, bp, tasks, n_tasks, xcd_shift);
    else if (bp.work)
        hipLaunchKernelGGL((blend_remap_kernel<true, false>), grid, block, 0, s, bp, tasks, n_tasks, xcd_shift);
    else if (bp.save_T)
        hipLaunchKernelGGL((blend_remap_kernel<false, true>), grid, block, 0, s, bp, tasks, n_tasks, xcd_shift);
    else
        hipLaunchKernelGGL((blend_remap_kernel<false, false>), grid, block, 0, s, bp, tasks, n_tasks, xcd_shift);
    return hipGetLastError();
}

hipError_t launch_blend_rowmajor(const BlendParams &bp, hipStream_t s)
{
    const dim3 grid((unsigned)(bp.TX * ((bp.H + bp.th - 1) / bp.th))), block(256);
    if (bp.work && bp.save_T)
        hipLaunchKernelGGL((blend_rowmajor_kernel<true, true>), grid, block, 0, s, bp);
    else if (bp.work)
        hipLaunchKernelGGL((blend_rowmajor_kernel<true, false>), grid, block, 0, s, bp);
    else if (bp.save_T)
        hipLaunchKernelGGL((blend_rowmajor_kernel<false, true>), grid, block, 0, s, bp);
    else
        hipLaunchKernelGGL((blend_rowmajor_kernel<false, false>), grid, block, 0, s, bp);
    return hipGetLastError();
}

hipError_t launch_blend_backward(const BwdParams &bp, const Task *tasks, int n_tasks, int xcd_shift, hipStream_t s)
{
    if (n_tasks == 0) return hipSuccess;
    if (xcd_shift < 0 || xcd_shift > 12) return hipErrorInvalidValue;
    hipLaunchKernelGGL(blend_backward_kernel, dim3(xcd_grid(n_tasks, xcd_shift)), dim3(kWave), 0, s, bp, tasks,
                       n_tasks, xcd_shift);
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
