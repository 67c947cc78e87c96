// Projection with cross-view attribute reuse (section 4.2 Eq. 5-6, appendix
// B.2 "Projection"): per Gaussian, the 2D mean for every projected view and
// the 2D covariance, depth and SH colour once per cluster, at the cluster's
// representative view.
//
// Layout: one thread per Gaussian.  A block first copies its Gaussians' SH
// coefficients into LDS with coalesced loads (rows of odd pitch, so the
// per-thread reads that follow are free of bank conflicts); each thread
// then builds the 3D covariance once and loops over the clusters: the full
// record at the representative view, then the mean in each projected view
// of the cluster (every projected view belongs to exactly one cluster), whose
// tile boxes are unioned while the mean is still in registers.  Each output
// plane [slot][M] is written coalesced across the wavefront.  A (cluster,
// Gaussian) whose boxes miss the panel in every view of the cluster gets the
// "invalid" depth key and no record: it sorts last and is never binned.
//
// Arithmetic is double precision with FMA contraction disabled (the library
// is built with -ffp-contract=off); results are rounded to float32 once, when
// stored.  The evaluation order of every expression is fixed, and quotients
// by the depth, the determinant, the conic's last pivot and the direction's
// norm are taken as products with a reciprocal accurate to about one double
// ulp (recip below), so the stored float32 values equal those of the plain
// double formulas except where the exact value lies within a few double ulps
// of a float32 rounding boundary (about one value in 10^8).  The tile-box
// extents, which only need to be conservative, are computed in float32.
#include "lfr_internal.h"

namespace lfr {

// 1/x for the finite, positive, normal x it is used on (depths beyond the
// near plane, determinants and pivots of the dilated covariance, direction
// norms): the hardware reciprocal estimate refined by two Newton steps.
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

struct Cov3 {
    double xx, xy, xz, yy, yz, zz;
};

// Sigma = M M^T with M = R(q) diag(exp(log_scale)), q normalized.
__device__ inline Cov3 cov3d(const float ls[3], const float q[4])
{
    double qw = q[0], qx = q[1], qy = q[2], qz = q[3];
    const double qn = sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz);
    qw = qw / qn;
    qx = qx / qn;
    qy = qy / qn;
    qz = qz / qn;
    const double r00 = 1.0 - 2.0 * (qy * qy + qz * qz), r01 = 2.0 * (qx * qy - qw * qz),
                 r02 = 2.0 * (qx * qz + qw * qy);
    const double r10 = 2.0 * (qx * qy + qw * qz), r11 = 1.0 - 2.0 * (qx * qx + qz * qz),
                 r12 = 2.0 * (qy * qz - qw * qx);
    const double r20 = 2.0 * (qx * qz - qw * qy), r21 = 2.0 * (qy * qz + qw * qx),
                 r22 = 1.0 - 2.0 * (qx * qx + qy * qy);
    const double s0 = exp((double)ls[0]), s1 = exp((double)ls[1]), s2 = exp((double)ls[2]);
    const double m00 = r00 * s0, m01 = r01 * s1, m02 = r02 * s2;
    const double m10 = r10 * s0, m11 = r11 * s1, m12 = r12 * s2;
    const double m20 = r20 * s0, m21 = r21 * s1, m22 = r22 * s2;
    Cov3 c;
    c.xx = (m00 * m00 + m01 * m01) + m02 * m02;
    c.xy = (m00 * m10 + m01 * m11) + m02 * m12;
    c.xz = (m00 * m20 + m01 * m21) + m02 * m22;
    c.yy = (m10 * m10 + m11 * m11) + m12 * m12;
    c.yz = (m10 * m20 + m11 * m21) + m12 * m22;
    c.zz = (m20 * m20 + m21 * m21) + m22 * m22;
    return c;
}

// Real SH basis (Condon-Shortley phase, m = -l..l) at unit direction (x,y,z),
// dotted with the coefficients of one channel: acc = sum_b Y_b * sh_b.
template <int DEG>
__device__ inline void sh_colour(const float *shc, double x, double y, double z, float col[3])
{
    constexpr double pi = 3.14159265358979323846;
    double Y[16];
    Y[0] = 0.5 * __builtin_sqrt(1.0 / pi);
    if (DEG >= 1) {
        const double c1 = __builtin_sqrt(3.0 / (4.0 * pi));
        Y[1] = -c1 * y;
        Y[2] = c1 * z;
        Y[3] = -c1 * x;
    }
    if (DEG >= 2) {
        const double xx = x * x, yy = y * y, zz = z * z;
        const double c2a = 0.5 * __builtin_sqrt(15.0 / pi);
        const double c2b = 0.25 * __builtin_sqrt(5.0 / pi);
        const double c2c = 0.25 * __builtin_sqrt(15.0 / pi);
        Y[4] = c2a * (x * y);
        Y[5] = -c2a * (y * z);
        Y[6] = c2b * (2.0 * zz - xx - yy);
        Y[7] = -c2a * (x * z);
        Y[8] = c2c * (xx - yy);
        if (DEG >= 3) {
            const double c3a = 0.25 * __builtin_sqrt(35.0 / (2.0 * pi));
            const double c3b = 0.5 * __builtin_sqrt(105.0 / pi);
            const double c3c = 0.25 * __builtin_sqrt(21.0 / (2.0 * pi));
            const double c3d = 0.25 * __builtin_sqrt(7.0 / pi);
            const double c3e = 0.25 * __builtin_sqrt(105.0 / pi);
            Y[9] = -c3a * (y * (3.0 * xx - yy));
            Y[10] = c3b * (x * y * z);
            Y[11] = -c3c * (y * (4.0 * zz - xx - yy));
            Y[12] = c3d * (z * (2.0 * zz - 3.0 * xx - 3.0 * yy));
            Y[13] = -c3c * (x * (4.0 * zz - xx - yy));
            Y[14] = c3e * (z * (xx - yy));
            Y[15] = -c3a * (x * (xx - 3.0 * yy));
        }
    }
    constexpr int NB = (DEG + 1) * (DEG + 1);
    // the dot product with fused multiply-adds (one rounding per term)
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b) acc = fma(Y[b], (double)shc[b * 3 + u], acc);
        acc = acc + 0.5;
        col[u] = (float)(acc > 0.0 ? acc : 0.0);
    }
}

struct MeanProj {
    double tx, ty, tz, iz, ux, uy;   // iz = 1 / tz
    float depth;
    float2 m2d;
    bool valid;  // finite and in front of the near plane
};

// Eq. 5: camera-space point, depth and pixel position of the mean.
__device__ inline MeanProj project_mean(const DevCamera &c, double mx, double my, double mz, bool finite)
{
    MeanProj p;
    p.tx = ((c.R[0] * mx + c.R[1] * my) + c.R[2] * mz) + c.t[0];
    p.ty = ((c.R[3] * mx + c.R[4] * my) + c.R[5] * mz) + c.t[1];
    p.tz = ((c.R[6] * mx + c.R[7] * my) + c.R[8] * mz) + c.t[2];
    p.depth = (float)p.tz;
    p.valid = finite && p.depth > kNearZ;
    p.iz = recip(p.tz);
    p.ux = p.tx * p.iz;
    p.uy = p.ty * p.iz;
    p.m2d = make_float2((float)(c.fx * p.ux + c.cx), (float)(c.fy * p.uy + c.cy));
    p.valid = p.valid && isfinite(p.m2d.x) && isfinite(p.m2d.y);
    return p;
}

struct FullProj {
    float conic[3];
    float colour[3];
    float2 ext;
    bool valid;
};

// Eq. 4/6 at one camera: EWA 2D covariance (Jacobian at the clamped mean
// direction, +0.3 dilation), its inverse in LDL^T form pre-scaled by
// log2(e)/2, SH colour along camera->mean, and conservative half extents of
// the region where alpha can reach 1/255.
// tau_o: the squared-Mahalanobis cutoff 2 ln(255 o) + 0.01 of the Gaussian
// (cutoff_tau).
template <int DEG>
__device__ inline FullProj project_full(const DevCamera &c, const MeanProj &m, const Cov3 &S,
                                        double mx, double my, double mz, float tau_o, const float *shc)
{
    FullProj f = {};
    const double *R = c.R;
    // J (2 x 3, zero in (0,1) and (1,0)) at the clamped mean direction; with
    // N = J R (2 x 3), Sigma2D = N Sigma N^T + 0.3 I: the quadratic forms of
    // the symmetric Sigma in the rows n0, n1 of N
    const double cxl = m.ux < -c.limx ? -c.limx : (m.ux > c.limx ? c.limx : m.ux);
    const double cyl = m.uy < -c.limy ? -c.limy : (m.uy > c.limy ? c.limy : m.uy);
    const double j00 = c.fx * m.iz, j02 = -(c.fx * cxl) * m.iz;
    const double j11 = c.fy * m.iz, j12 = -(c.fy * cyl) * m.iz;
    const double n00 = j00 * R[0] + j02 * R[6], n01 = j00 * R[1] + j02 * R[7], n02 = j00 * R[2] + j02 * R[8];
    const double n10 = j11 * R[3] + j12 * R[6], n11 = j11 * R[4] + j12 * R[7], n12 = j11 * R[5] + j12 * R[8];
    // Sigma n0 and Sigma n1
    const double u0 = (S.xx * n00 + S.xy * n01) + S.xz * n02;
    const double u1 = (S.xy * n00 + S.yy * n01) + S.yz * n02;
    const double u2 = (S.xz * n00 + S.yz * n01) + S.zz * n02;
    const double w0 = (S.xx * n10 + S.xy * n11) + S.xz * n12;
    const double w1 = (S.xy * n10 + S.yy * n11) + S.yz * n12;
    const double w2 = (S.xz * n10 + S.yz * n11) + S.zz * n12;
    const double sa = ((n00 * u0 + n01 * u1) + n02 * u2) + kDilation;
    const double sb = (n00 * w0 + n01 * w1) + n02 * w2;
    const double sc = ((n10 * w0 + n11 * w1) + n12 * w2) + kDilation;
    const double det = sa * sc - sb * sb;
    if (!(det > 0.0)) return f;
    const double rsc = recip(sc);
    const double A = sc * recip(det), beta = -sb * rsc, G = rsc;
    f.conic[0] = (float)(A * kHalfLog2e);
    f.conic[1] = (float)beta;
    f.conic[2] = (float)(G * kHalfLog2e);
    // colour
    double dx = mx - c.campos[0], dy = my - c.campos[1], dz = mz - c.campos[2];
    const double rdn = recip(sqrt((dx * dx + dy * dy) + dz * dz));
    dx = dx * rdn;
    dy = dy * rdn;
    dz = dz * rdn;
    sh_colour<DEG>(shc, dx, dy, dz, f.colour);
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) ok = ok && isfinite(f.conic[k]) && isfinite(f.colour[k]);
    ok = ok && f.conic[0] > 0.0f && f.conic[2] > 0.0f;
    if (!ok) return f;
    // Extents of {d : o 2^-E(d) >= 1/255}, i.e. d^T Sigma^-1 d <= tau with
    // tau = 2 ln(255 o) (tau_o: per Gaussian, + 0.01), for the float32 conic
    // actually stored, with margins (x 1.0001 + 0.02 px) that dominate both
    // the float32 evaluation error here and that of the blend.
    constexpr float kInvHalfLog2e = (float)(1.0 / kHalfLog2e);
    const float Ar = f.conic[0] * kInvHalfLog2e, br = f.conic[1], Gr = f.conic[2] * kInvHalfLog2e;
    // (hardware reciprocals and square roots: their error of about one ulp is
    // far inside the margins)
    const float iG = __builtin_amdgcn_rcpf(Gr);
    const float S00 = __builtin_amdgcn_rcpf(Ar) + (br * br) * iG, S11 = iG;
    f.ext = make_float2(__builtin_amdgcn_sqrtf(tau_o * S00) * 1.0001f + 0.02f,
                        __builtin_amdgcn_sqrtf(tau_o * S11) * 1.0001f + 0.02f);
    f.valid = isfinite(f.ext.x) && isfinite(f.ext.y);
    return f;
}

// 2 ln(255 o) + 0.01 (0.01 for o <= 1/255): the extents' cutoff.
__device__ inline float cutoff_tau(float o)
{
    const double tau = 2.0 * log(255.0 * (double)o);
    return (float)((tau > 0.0 ? tau : 0.0) + 0.01);
}

struct GaussIn {
    float mu[3], ls[3], q[4], o;
    bool finite;
};

// Parameters of Gaussian i; the SH coefficients are copied to shc from the
// scene, or (from_scene false) are already there and only checked.
template <int DEG>
__device__ inline void load_gaussian(const SceneDev &sc, int64_t i, GaussIn &g, float *shc,
                                     bool from_scene = true)
{
    constexpr int NB = (DEG + 1) * (DEG + 1);
    bool fin = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        g.mu[k] = sc.means[3 * i + k];
        g.ls[k] = sc.log_scales[3 * i + k];
        fin &= isfinite(g.mu[k]);
        fin &= isfinite(g.ls[k]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        g.q[k] = sc.quats[4 * i + k];
        fin &= isfinite(g.q[k]);
    }
    g.o = sc.opac[i];
    fin &= isfinite(g.o);
    const float *s = sc.sh + (int64_t)NB * 3 * i;
#pragma unroll
    for (int k = 0; k < NB * 3; ++k) {
        if (from_scene) shc[k] = s[k];
        fin &= isfinite(shc[k]);
    }
    g.finite = fin;
}

// Tile box (inclusive tile ranges) of the pixels whose centres lie within
// the half extents e of mean m; false if it misses the panel.
__device__ inline bool tile_box(float2 m, float2 e, const TileGrid &tg, ushort4 &b)
{
    // pixel x is covered when |x + 0.5 - mx| <= ex
    const float fx0 = fmaxf(ceilf(m.x - e.x - 0.5f), 0.0f);
    const float fx1 = fminf(floorf(m.x + e.x - 0.5f), (float)(tg.W - 1));
    const float fy0 = fmaxf(ceilf(m.y - e.y - 0.5f), 0.0f);
    const float fy1 = fminf(floorf(m.y + e.y - 0.5f), (float)(tg.H - 1));
    if (!(fx0 <= fx1) || !(fy0 <= fy1)) return false;
    b = make_ushort4((unsigned short)((int)fx0 >> tg.tw_shift), (unsigned short)((int)fx1 >> tg.tw_shift),
                     (unsigned short)((int)fy0 >> tg.th_shift), (unsigned short)((int)fy1 >> tg.th_shift));
    return true;
}

constexpr int kProjBlock = 64;

// Store of the 64 lanes' records (Q pieces of 16 bytes each), consecutive in
// memory from dst, as Q stores of 1 KB each, through the wavefront's 1 KB
// LDS buffer: in round j the 64 / Q lanes whose records the round covers
// put them into the buffer, then every lane stores the buffer's 16-byte
// piece `lane`.  Each store fills whole cache lines, where a per-lane
// record store would write 16 bytes into each of 64 lines.  The buffer is
// private to the wavefront; the wavefront-scope fences keep the compiler
// from moving a round's buffer writes across the previous round's reads (a
// wavefront's LDS accesses are performed in program order).
template <int Q>
__device__ __forceinline__ void wave_store(uint4 *dst, const uint4 (&pc)[Q], int lane, uint4 *buf)
{
    constexpr int R = 64 / Q;  // records per round
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        const int rl = lane - j * R;
        if (rl >= 0 && rl < R) {
#pragma unroll
            for (int p = 0; p < Q; ++p) buf[rl * Q + p] = pc[p];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        dst[j * 64 + lane] = buf[lane];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

template <int DEG>
__global__ void __launch_bounds__(kProjBlock) project_kernel(SceneDev sc, const DevCamera *__restrict__ cams, TileGrid tg,
                                                      int n_clusters, const int32_t *__restrict__ cluster_cam,
                                                      ProjectOut out)
{
    constexpr int NS = (DEG + 1) * (DEG + 1) * 3;  // SH floats per Gaussian
    constexpr int PITCH = NS | 1;
    __shared__ float s_sh[kProjBlock * PITCH];
    __shared__ uint4 s_stage[kProjBlock / 64][64];  // each wavefront's record-store buffer
    const int64_t i0 = (int64_t)blockIdx.x * kProjBlock;
    const int64_t i = i0 + threadIdx.x;
    const int64_t M = sc.M, Mp = out.Mp;
    {
        const int64_t nb = M - i0 < kProjBlock ? (M - i0 > 0 ? M - i0 : 0) : kProjBlock;
        const float *src = sc.sh + i0 * NS;
        if (nb == kProjBlock) {
            // a full block: 16 loads in flight before their LDS stores (a
            // loop of load-then-store would wait for every load in turn)
#pragma unroll
            for (int c = 0; c < NS; c += 16) {
                float v[16];
#pragma unroll
                for (int q = 0; q < 16; ++q)
                    if (c + q < NS) v[q] = src[(c + q) * kProjBlock + threadIdx.x];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    if (c + q >= NS) break;
                    const int e = (c + q) * kProjBlock + threadIdx.x;
                    const int r = e / NS;
                    s_sh[r * PITCH + (e - r * NS)] = v[q];
                }
            }
        } else {
            for (int e = threadIdx.x; e < (int)nb * NS; e += kProjBlock) {
                const int r = e / NS;
                s_sh[r * PITCH + (e - r * NS)] = src[e];
            }
        }
    }
    __syncthreads();
    if (i >= M) {
        // padding of each cluster's depth-key segment: sorts last, never read
        if (i < Mp)
            for (int k = 0; k < n_clusters; ++k) {
                out.dkey[(int64_t)k * Mp + i] = 0xFFFFFFFFu;
                if (out.dval) out.dval[(int64_t)k * Mp + i] = 0u;
            }
        return;
    }
    GaussIn g;
    float *shc = s_sh + threadIdx.x * PITCH;
    load_gaussian<DEG>(sc, i, g, shc, false);
    const double mx = g.mu[0], my = g.mu[1], mz = g.mu[2];
    // all 64 Gaussians of this wavefront exist: its records are written with
    // whole-wavefront stores (also those of pairs that are not binned, which
    // nothing reads)
    const int lane = threadIdx.x & 63;
    const bool full_wave = i - lane + 64 <= M;
    const bool want_cov = g.finite && g.o >= kAlphaMin;
    Cov3 S = {};
    if (want_cov) S = cov3d(g.ls, g.q);
    // per-Gaussian cutoffs: of the extents and of the blend (log2(255 o) + 0.01)
    const float tau_o = cutoff_tau(g.o);
    const float ecut = (float)(log2(255.0 * (double)g.o) + 0.01);
    for (int k = 0; k < n_clusters; ++k) {
        const DevCamera &c = cams[cluster_cam[k]];
        const MeanProj m = project_mean(c, mx, my, mz, g.finite);
        FullProj f = {};
        if (want_cov && m.valid) f = project_full<DEG>(c, m, S, mx, my, mz, tau_o, shc);
        const int64_t idx = (int64_t)k * M + i, kidx = (int64_t)k * Mp + i;
        if (out.dval) out.dval[kidx] = (uint32_t)i;
        // the cluster's views: mean planes, the record's means (the first
        // kItemViews views, placed by selects rather than a dynamic index so
        // that the record stays in registers), and the union of the tile
        // boxes of this Gaussian's mean in each view with the cluster's extents
        float2 mv[kItemViews];
#pragma unroll
        for (int q = 0; q < kItemViews; ++q) mv[q] = make_float2(kFarMean, kFarMean);
        int nv = 0;
        unsigned short x0 = 0xFFFF, x1 = 0, y0 = 0xFFFF, y1 = 0;
        // a cluster of more views keeps the box of its binned views' means
        float2 hlo = make_float2(kFarMean, kFarMean), hhi = make_float2(-kFarMean, -kFarMean);
        for (int v = tg.cv_off[k]; v < tg.cv_off[k + 1]; ++v) {
            const MeanProj mj = project_mean(cams[tg.cv_cam[v]], mx, my, mz, g.finite);
            const float2 m2 = mj.valid ? mj.m2d : make_float2(kFarMean, kFarMean);
            if (out.mean2d) out.mean2d[(int64_t)tg.cv_list[v] * M + i] = m2;
            const int l = v - tg.cv_off[k];
#pragma unroll
            for (int q = 0; q < kItemViews; ++q)
                if (q == l) mv[q] = m2;
            ushort4 b;
            if (!f.valid || !mj.valid || !tile_box(m2, f.ext, tg, b)) continue;
            ++nv;
            hlo = make_float2(fminf(hlo.x, m2.x), fminf(hlo.y, m2.y));
            hhi = make_float2(fmaxf(hhi.x, m2.x), fmaxf(hhi.y, m2.y));
            x0 = min(x0, b.x);
            x1 = max(x1, b.y);
            y0 = min(y0, b.z);
            y1 = max(y1, b.w);
        }
        const bool binned = nv != 0;
        GaussRec r;
        r.a = make_float4(f.conic[0], f.conic[1], f.conic[2], g.o);
        r.c = make_float4(f.colour[0], f.colour[1], f.colour[2], ecut);
#pragma unroll
        for (int q = 0; q < kItemViews; ++q) r.m[q] = mv[q];
        if (tg.cv_off[k + 1] - tg.cv_off[k] > kItemViews) {
            r.m[0] = hlo;
            r.m[1] = hhi;
        }
        const ushort4 box = make_ushort4(x0, x1, y0, y1);
        if (full_wave) {
            uint4 rp[4];
            __builtin_memcpy(rp, &r, sizeof(GaussRec));
            wave_store<4>(reinterpret_cast<uint4 *>(out.rec + (idx - lane)), rp, lane, s_stage[threadIdx.x >> 6]);
            out.ibox[idx] = box;
        } else if (binned) {
            out.rec[idx] = r;
            out.ibox[idx] = box;
        }
        out.dkey[kidx] = binned ? __float_as_uint(m.depth) : 0xFFFFFFFFu;
    }
}

template <int DEG>
__global__ void __launch_bounds__(256) project_records_kernel(SceneDev sc, const DevCamera *__restrict__ cam,
                                                              lfr_proj_record *out)
{
    constexpr int NB = (DEG + 1) * (DEG + 1);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sc.M) return;
    GaussIn g;
    float shc[NB * 3];
    load_gaussian<DEG>(sc, i, g, shc);
    const double mx = g.mu[0], my = g.mu[1], mz = g.mu[2];
    const MeanProj m = project_mean(*cam, mx, my, mz, g.finite);
    lfr_proj_record r;
    const float nanf_ = __builtin_nanf("");
    r.mean2d[0] = m.valid ? m.m2d.x : nanf_;
    r.mean2d[1] = m.valid ? m.m2d.y : nanf_;
    r.depth = m.depth;
    r.opacity = g.o;
    r.valid_mean = m.valid ? 1 : 0;
    r.valid = 0;
    for (int k = 0; k < 3; ++k) r.conic[k] = r.color[k] = 0.0f;
    if (m.valid && g.o >= kAlphaMin) {
        const Cov3 S = cov3d(g.ls, g.q);
        const FullProj f = project_full<DEG>(*cam, m, S, mx, my, mz, cutoff_tau(g.o), shc);
        if (f.valid) {
            for (int k = 0; k < 3; ++k) {
                r.conic[k] = f.conic[k];
                r.color[k] = f.colour[k];
            }
            r.valid = 1;
        }
    }
    out[i] = r;
}

hipError_t launch_project(const SceneDev &sc, const DevCamera *cams, const TileGrid &tg, int n_clusters,
                          const int32_t *cluster_cam, const ProjectOut &out, hipStream_t s)
{
    const int64_t n = sc.M > out.Mp ? sc.M : out.Mp;
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)((n + kProjBlock - 1) / kProjBlock)), block(kProjBlock);
    switch (sc.deg) {
    case 0: hipLaunchKernelGGL(project_kernel<0>, grid, block, 0, s, sc, cams, tg, n_clusters, cluster_cam, out); break;
    case 1: hipLaunchKernelGGL(project_kernel<1>, grid, block, 0, s, sc, cams, tg, n_clusters, cluster_cam, out); break;
    case 2: hipLaunchKernelGGL(project_kernel<2>, grid, block, 0, s, sc, cams, tg, n_clusters, cluster_cam, out); break;
    default: hipLaunchKernelGGL(project_kernel<3>, grid, block, 0, s, sc, cams, tg, n_clusters, cluster_cam, out); break;
    }
    return hipGetLastError();
}

hipError_t launch_project_records(const SceneDev &sc, const DevCamera *cam, int W, int H,
                                  lfr_proj_record *out, hipStream_t s)
{
    (void)W;
    (void)H;
    if (sc.M == 0) return hipSuccess;
    const dim3 grid((unsigned)((sc.M + 255) / 256)), block(256);
    switch (sc.deg) {
    case 0: hipLaunchKernelGGL(project_records_kernel<0>, grid, block, 0, s, sc, cam, out); break;
    case 1: hipLaunchKernelGGL(project_records_kernel<1>, grid, block, 0, s, sc, cam, out); break;
    case 2: hipLaunchKernelGGL(project_records_kernel<2>, grid, block, 0, s, sc, cam, out); break;
    default: hipLaunchKernelGGL(project_records_kernel<3>, grid, block, 0, s, sc, cam, out); break;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Projection backward: the reverse of project_mean, project_full, cov3d and
// sh_colour for the gradients the reverse blend left in the per-(cluster,
// Gaussian) records and per-(view, Gaussian) means.  Double precision, one
// thread per Gaussian, so every parameter gradient is written once without
// atomics.  Clamped quantities (Jacobian direction, colour at 0) pass no
// derivative.
// ---------------------------------------------------------------------------

// Real SH basis at (x, y, z) and its gradient, treating each basis function
// as the polynomial it is written as (the direction's normalization is
// chained separately).
template <int DEG>
__device__ inline void sh_basis_grad(double x, double y, double z, double Y[16], double Gx[16], double Gy[16],
                                     double Gz[16])
{
    constexpr double pi = 3.14159265358979323846;
#pragma unroll
    for (int b = 0; b < 16; ++b) Y[b] = Gx[b] = Gy[b] = Gz[b] = 0.0;
    Y[0] = 0.5 * __builtin_sqrt(1.0 / pi);
    if (DEG >= 1) {
        const double c1 = __builtin_sqrt(3.0 / (4.0 * pi));
        Y[1] = -c1 * y;  Gy[1] = -c1;
        Y[2] = c1 * z;   Gz[2] = c1;
        Y[3] = -c1 * x;  Gx[3] = -c1;
    }
    if (DEG >= 2) {
        const double xx = x * x, yy = y * y, zz = z * z;
        const double c2a = 0.5 * __builtin_sqrt(15.0 / pi);
        const double c2b = 0.25 * __builtin_sqrt(5.0 / pi);
        const double c2c = 0.25 * __builtin_sqrt(15.0 / pi);
        Y[4] = c2a * (x * y);                  Gx[4] = c2a * y;          Gy[4] = c2a * x;
        Y[5] = -c2a * (y * z);                 Gy[5] = -c2a * z;         Gz[5] = -c2a * y;
        Y[6] = c2b * (2.0 * zz - xx - yy);     Gx[6] = -2.0 * c2b * x;   Gy[6] = -2.0 * c2b * y;  Gz[6] = 4.0 * c2b * z;
        Y[7] = -c2a * (x * z);                 Gx[7] = -c2a * z;         Gz[7] = -c2a * x;
        Y[8] = c2c * (xx - yy);                Gx[8] = 2.0 * c2c * x;    Gy[8] = -2.0 * c2c * y;
        if (DEG >= 3) {
            const double c3a = 0.25 * __builtin_sqrt(35.0 / (2.0 * pi));
            const double c3b = 0.5 * __builtin_sqrt(105.0 / pi);
            const double c3c = 0.25 * __builtin_sqrt(21.0 / (2.0 * pi));
            const double c3d = 0.25 * __builtin_sqrt(7.0 / pi);
            const double c3e = 0.25 * __builtin_sqrt(105.0 / pi);
            Y[9] = -c3a * (y * (3.0 * xx - yy));
            Gx[9] = -6.0 * c3a * x * y;            Gy[9] = -3.0 * c3a * (xx - yy);
            Y[10] = c3b * (x * y * z);
            Gx[10] = c3b * y * z;                  Gy[10] = c3b * x * z;        Gz[10] = c3b * x * y;
            Y[11] = -c3c * (y * (4.0 * zz - xx - yy));
            Gx[11] = 2.0 * c3c * x * y;            Gy[11] = -c3c * (4.0 * zz - xx - 3.0 * yy);
            Gz[11] = -8.0 * c3c * y * z;
            Y[12] = c3d * (z * (2.0 * zz - 3.0 * xx - 3.0 * yy));
            Gx[12] = -6.0 * c3d * x * z;           Gy[12] = -6.0 * c3d * y * z;
            Gz[12] = c3d * (6.0 * zz - 3.0 * xx - 3.0 * yy);
            Y[13] = -c3c * (x * (4.0 * zz - xx - yy));
            Gx[13] = -c3c * (4.0 * zz - 3.0 * xx - yy);
            Gy[13] = 2.0 * c3c * x * y;            Gz[13] = -8.0 * c3c * x * z;
            Y[14] = c3e * (z * (xx - yy));
            Gx[14] = 2.0 * c3e * x * z;            Gy[14] = -2.0 * c3e * y * z;  Gz[14] = c3e * (xx - yy);
            Y[15] = -c3a * (x * (xx - 3.0 * yy));
            Gx[15] = -3.0 * c3a * (xx - yy);       Gy[15] = 6.0 * c3a * x * y;
        }
    }
}

// d(loss)/d(pixel mean) in one camera -> d(loss)/d(world mean).
__device__ inline void mean_grad(const DevCamera &c, const MeanProj &m, float2 dm, double dmu[3])
{
    const double dux = c.fx * (double)dm.x, duy = c.fy * (double)dm.y;
    const double dtx = dux / m.tz, dty = duy / m.tz, dtz = -(dux * m.tx + duy * m.ty) / (m.tz * m.tz);
#pragma unroll
    for (int k = 0; k < 3; ++k) dmu[k] += (c.R[k] * dtx + c.R[3 + k] * dty) + c.R[6 + k] * dtz;
}

// Record gradients at one cluster's representative camera -> world mean,
// world covariance (symmetric, entries xx xy xz yy yz zz) and SH.
template <int DEG>
__device__ inline void record_grad(const DevCamera &c, const MeanProj &m, const Cov3 &S, double mx, double my,
                                   double mz, const float *shc, const GradRec &g, double dmu[3], double dS[6],
                                   float *dsh)
{
    const double *R = c.R;
    // forward: V = R S R^T, J, Sigma2D (the same expressions as project_full)
    const double s00 = S.xx, s01 = S.xy, s02 = S.xz, s11 = S.yy, s12 = S.yz, s22 = S.zz;
    const double a00 = (R[0] * s00 + R[1] * s01) + R[2] * s02;
    const double a01 = (R[0] * s01 + R[1] * s11) + R[2] * s12;
    const double a02 = (R[0] * s02 + R[1] * s12) + R[2] * s22;
    const double a10 = (R[3] * s00 + R[4] * s01) + R[5] * s02;
    const double a11 = (R[3] * s01 + R[4] * s11) + R[5] * s12;
    const double a12 = (R[3] * s02 + R[4] * s12) + R[5] * s22;
    const double a20 = (R[6] * s00 + R[7] * s01) + R[8] * s02;
    const double a21 = (R[6] * s01 + R[7] * s11) + R[8] * s12;
    const double a22 = (R[6] * s02 + R[7] * s12) + R[8] * s22;
    const double v00 = (a00 * R[0] + a01 * R[1]) + a02 * R[2];
    const double v01 = (a00 * R[3] + a01 * R[4]) + a02 * R[5];
    const double v02 = (a00 * R[6] + a01 * R[7]) + a02 * R[8];
    const double v11 = (a10 * R[3] + a11 * R[4]) + a12 * R[5];
    const double v12 = (a10 * R[6] + a11 * R[7]) + a12 * R[8];
    const double v20 = (a20 * R[0] + a21 * R[1]) + a22 * R[2];
    const double v21 = (a20 * R[3] + a21 * R[4]) + a22 * R[5];
    const double v22 = (a20 * R[6] + a21 * R[7]) + a22 * R[8];
    const double cxl = m.ux < -c.limx ? -c.limx : (m.ux > c.limx ? c.limx : m.ux);
    const double cyl = m.uy < -c.limy ? -c.limy : (m.uy > c.limy ? c.limy : m.uy);
    const double tz = m.tz, tz2 = tz * tz;
    const double j00 = c.fx / tz, j02 = -(c.fx * cxl) / tz;
    const double j11 = c.fy / tz, j12 = -(c.fy * cyl) / tz;
    const double k00 = j00 * v00 + j02 * v20, k01 = j00 * v01 + j02 * v21, k02 = j00 * v02 + j02 * v22;
    const double k10 = j11 * v01 + j12 * v20, k11 = j11 * v11 + j12 * v21, k12 = j11 * v12 + j12 * v22;
    const double sa = (k00 * j00 + k02 * j02) + kDilation;
    const double sb = k01 * j11 + k02 * j12;
    const double sc = (k11 * j11 + k12 * j12) + kDilation;
    const double det = sa * sc - sb * sb;

    // A' = h sc/det, beta = -sb/sc, G' = h/sc  ->  d(sa, sb, sc)
    const double gA = (double)g.a.x * kHalfLog2e, gB = (double)g.a.y, gG = (double)g.a.z * kHalfLog2e;
    const double id2 = 1.0 / (det * det), isc = 1.0 / sc;
    const double dsa = -gA * sc * sc * id2;
    const double dsb = 2.0 * gA * sb * sc * id2 - gB * isc;
    const double dsc = -gA * sb * sb * id2 + gB * sb * isc * isc - gG * isc * isc;
    // Sigma2D = J V J^T with the symmetric upstream P = [[dsa, dsb/2], [dsb/2, dsc]]:
    // dV = J^T P J, dJ = 2 P (J V)
    const double p00 = dsa, p01 = 0.5 * dsb, p11 = dsc;
    const double q0 = p00 * j02 + p01 * j12, q1 = p01 * j02 + p11 * j12;
    const double D00 = j00 * j00 * p00, D01 = j00 * j11 * p01, D02 = j00 * q0;
    const double D11 = j11 * j11 * p11, D12 = j11 * q1, D22 = j02 * q0 + j12 * q1;
    const double dj00 = 2.0 * (p00 * k00 + p01 * k10), dj02 = 2.0 * (p00 * k02 + p01 * k12);
    const double dj11 = 2.0 * (p01 * k01 + p11 * k11), dj12 = 2.0 * (p01 * k02 + p11 * k12);
    // J -> camera-space mean (the clamped direction passes nothing)
    double dtz = (-dj00 * c.fx + dj02 * c.fx * cxl - dj11 * c.fy + dj12 * c.fy * cyl) / tz2;
    double dtx = 0.0, dty = 0.0;
    if (cxl == m.ux) {
        const double d = -dj02 * c.fx / tz;
        dtx += d / tz;
        dtz -= d * m.tx / tz2;
    }
    if (cyl == m.uy) {
        const double d = -dj12 * c.fy / tz;
        dty += d / tz;
        dtz -= d * m.ty / tz2;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) dmu[k] += (R[k] * dtx + R[3 + k] * dty) + R[6 + k] * dtz;
    // V = R S R^T -> dS = R^T D R
    const double D[9] = {D00, D01, D02, D01, D11, D12, D02, D12, D22};
    double B[9];  // D R
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) B[r * 3 + k] = (D[r * 3] * R[k] + D[r * 3 + 1] * R[3 + k]) + D[r * 3 + 2] * R[6 + k];
    auto rtb = [&](int a, int b) { return (R[a] * B[b] + R[3 + a] * B[3 + b]) + R[6 + a] * B[6 + b]; };
    dS[0] += rtb(0, 0);
    dS[1] += rtb(0, 1);
    dS[2] += rtb(0, 2);
    dS[3] += rtb(1, 1);
    dS[4] += rtb(1, 2);
    dS[5] += rtb(2, 2);

    // colour along the direction camera -> mean
    const float dcol[3] = {g.c.x, g.c.y, g.c.z};
    if (dcol[0] == 0.0f && dcol[1] == 0.0f && dcol[2] == 0.0f) return;
    double vx = mx - c.campos[0], vy = my - c.campos[1], vz = mz - c.campos[2];
    const double dn = sqrt((vx * vx + vy * vy) + vz * vz);
    vx = vx / dn;
    vy = vy / dn;
    vz = vz / dn;
    double Y[16], Gx[16], Gy[16], Gz[16];
    sh_basis_grad<DEG>(vx, vy, vz, Y, Gx, Gy, Gz);
    constexpr int NB = (DEG + 1) * (DEG + 1);
    double ex = 0.0, ey = 0.0, ez = 0.0;
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        if (dcol[u] == 0.0f) continue;
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b) acc = acc + Y[b] * (double)shc[b * 3 + u];
        acc = acc + 0.5;
        if (!(acc > 0.0)) continue;
        const double dc = dcol[u];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const double h = shc[b * 3 + u];
            dsh[b * 3 + u] += (float)(Y[b] * dc);
            ex += dc * h * Gx[b];
            ey += dc * h * Gy[b];
            ez += dc * h * Gz[b];
        }
    }
    const double dot = (ex * vx + ey * vy) + ez * vz;
    dmu[0] += (ex - vx * dot) / dn;
    dmu[1] += (ey - vy * dot) / dn;
    dmu[2] += (ez - vz * dot) / dn;
}

template <int DEG>
__global__ void __launch_bounds__(256) project_backward_kernel(SceneDev sc, const DevCamera *__restrict__ cams,
                                                               int n_clusters, const int32_t *__restrict__ cluster_cam,
                                                               int n_views, const int32_t *__restrict__ view_cam,
                                                               const GradRec *__restrict__ d_rec,
                                                               const float2 *__restrict__ d_mean2d, SceneGrads out)
{
    constexpr int NB = (DEG + 1) * (DEG + 1);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sc.M) return;
    const int64_t M = sc.M;
    GaussIn g;
    float shc[NB * 3];
    load_gaussian<DEG>(sc, i, g, shc);
    const double mx = g.mu[0], my = g.mu[1], mz = g.mu[2];
    double dmu[3] = {0.0, 0.0, 0.0}, dS[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, dop = 0.0;
    float dsh[NB * 3];
#pragma unroll
    for (int k = 0; k < NB * 3; ++k) dsh[k] = 0.0f;
    const bool want_cov = g.finite && g.o >= kAlphaMin;
    Cov3 S = {};
    if (want_cov) S = cov3d(g.ls, g.q);
    if (want_cov) {
        for (int k = 0; k < n_clusters; ++k) {
            const GradRec gr = d_rec[(int64_t)k * M + i];
            if (gr.a.x == 0.0f && gr.a.y == 0.0f && gr.a.z == 0.0f && gr.a.w == 0.0f && gr.c.x == 0.0f &&
                gr.c.y == 0.0f && gr.c.z == 0.0f)
                continue;
            dop += (double)gr.a.w;
            const DevCamera &c = cams[cluster_cam[k]];
            const MeanProj m = project_mean(c, mx, my, mz, g.finite);
            if (m.valid) record_grad<DEG>(c, m, S, mx, my, mz, shc, gr, dmu, dS, dsh);
        }
    }
    for (int v = 0; v < n_views; ++v) {
        const float2 dm = d_mean2d[(int64_t)v * M + i];
        if (dm.x == 0.0f && dm.y == 0.0f) continue;
        const DevCamera &c = cams[view_cam[v]];
        const MeanProj m = project_mean(c, mx, my, mz, g.finite);
        if (m.valid) mean_grad(c, m, dm, dmu);
    }
    // Sigma = Mq Mq^T with Mq = Rq(q/|q|) diag(exp(log_scale)): dMq = 2 dS Mq
    double dls[3] = {0.0, 0.0, 0.0}, dq[4] = {0.0, 0.0, 0.0, 0.0};
    if (want_cov) {
        const double qn = sqrt((((double)g.q[0] * g.q[0] + (double)g.q[1] * g.q[1]) + (double)g.q[2] * g.q[2]) +
                               (double)g.q[3] * g.q[3]);
        const double w = g.q[0] / qn, x = g.q[1] / qn, y = g.q[2] / qn, z = g.q[3] / qn;
        const double Rq[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z),       2.0 * (x * z + w * y),
                              2.0 * (x * y + w * z),       1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
                              2.0 * (x * z - w * y),       2.0 * (y * z + w * x),       1.0 - 2.0 * (x * x + y * y)};
        const double sv[3] = {exp((double)g.ls[0]), exp((double)g.ls[1]), exp((double)g.ls[2])};
        const double Gm[9] = {dS[0], dS[1], dS[2], dS[1], dS[3], dS[4], dS[2], dS[4], dS[5]};
        double gR[9];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double ds = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                // dMq[a][b] = 2 sum_k G[a][k] Rq[k][b] s_b
                const double dM = 2.0 * ((Gm[a * 3] * Rq[b] + Gm[a * 3 + 1] * Rq[3 + b]) + Gm[a * 3 + 2] * Rq[6 + b]) * sv[b];
                gR[a * 3 + b] = dM * sv[b];
                ds += dM * Rq[a * 3 + b];
            }
            dls[b] = ds * sv[b];
        }
        // Rq of the unit quaternion (w, x, y, z), grouped by entry pairs
        const double dw = 2.0 * (x * (gR[7] - gR[5]) + y * (gR[2] - gR[6]) + z * (gR[3] - gR[1]));
        const double dx = 2.0 * (y * (gR[1] + gR[3]) + z * (gR[2] + gR[6]) + w * (gR[7] - gR[5]) - 2.0 * x * (gR[4] + gR[8]));
        const double dy = 2.0 * (x * (gR[1] + gR[3]) + z * (gR[5] + gR[7]) + w * (gR[2] - gR[6]) - 2.0 * y * (gR[0] + gR[8]));
        const double dz = 2.0 * (x * (gR[2] + gR[6]) + y * (gR[5] + gR[7]) + w * (gR[3] - gR[1]) - 2.0 * z * (gR[0] + gR[4]));
        // through the normalization q / |q|
        const double proj = ((dw * w + dx * x) + dy * y) + dz * z;
        dq[0] = (dw - w * proj) / qn;
        dq[1] = (dx - x * proj) / qn;
        dq[2] = (dy - y * proj) / qn;
        dq[3] = (dz - z * proj) / qn;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        out.means[3 * i + k] = (float)dmu[k];
        out.log_scales[3 * i + k] = (float)dls[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) out.quats[4 * i + k] = (float)dq[k];
    out.opac[i] = (float)dop;
    float *o = out.sh + (int64_t)NB * 3 * i;
#pragma unroll
    for (int k = 0; k < NB * 3; ++k) o[k] = dsh[k];
}

hipError_t launch_project_backward(const SceneDev &sc, const DevCamera *cams, int n_clusters,
                                   const int32_t *cluster_cam, int n_views, const int32_t *view_cam,
                                   const GradRec *d_rec, const float2 *d_mean2d, const SceneGrads &out,
                                   hipStream_t s)
{
    if (sc.M == 0) return hipSuccess;
    const dim3 grid((unsigned)((sc.M + 255) / 256)), block(256);
    switch (sc.deg) {
    case 0: hipLaunchKernelGGL(project_backward_kernel<0>, grid, block, 0, s, sc, cams, n_clusters, cluster_cam, n_views, view_cam, d_rec, d_mean2d, out); break;
    case 1: hipLaunchKernelGGL(project_backward_kernel<1>, grid, block, 0, s, sc, cams, n_clusters, cluster_cam, n_views, view_cam, d_rec, d_mean2d, out); break;
    case 2: hipLaunchKernelGGL(project_backward_kernel<2>, grid, block, 0, s, sc, cams, n_clusters, cluster_cam, n_views, view_cam, d_rec, d_mean2d, out); break;
    default: hipLaunchKernelGGL(project_backward_kernel<3>, grid, block, 0, s, sc, cams, n_clusters, cluster_cam, n_views, view_cam, d_rec, d_mean2d, out); break;
    }
    return hipGetLastError();
}

}  // namespace lfr
