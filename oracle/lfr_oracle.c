/*
 * lfr_oracle.c -- CPU oracle for subpixel-level 3D Gaussian rasterization of
 * one interlaced light-field image (CoherentRaster, arXiv 2605.04509).
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow reference written from the paper
 * (single-threaded unless orc_set_threads asks for more; the results are
 * bit-identical for any thread count).  It shares no code with the HIP library; only the tests,
 * the smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared lfr_oracle.c -lm -lpthread
 *
 * What each function follows:
 *   orc_view_map         section 3.1, Eq. 1-3 (lenticular view-index map)
 *   orc_cluster_table    appendix B.1 (contiguous view clusters, padding,
 *                        median representative)
 *   orc_remap            section 4.3, Eq. 8 (per-tile view-sorted LUT Psi)
 *   orc_project          section 4.1 Eq. 4, section 4.2 Eq. 5-6 (projection
 *                        of mean, covariance, depth and SH colour)
 *   orc_render_subpixels section 4.3 Eq. 9-10 with the reuse rule of
 *                        section 4.2 (mean per view, the rest per cluster)
 *   orc_render_view      section 3.3 (standard full-frame 3DGS blend)
 *
 * Parity pins live in tests/test_oracle_*.py.
 */
#include "lfr_oracle.h"
#include "lfr_oracle_impl.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define FLAG_SAFETY 4.0

/* ------------------------------------------------------------------------ */
/* Eq. 1-3                                                                  */
/* ------------------------------------------------------------------------ */

typedef __int128 i128;

static i128 gcd128(i128 a, i128 b)
{
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    while (b != 0) {
        i128 t = a % b;
        a = b;
        b = t;
    }
    return a;
}

static i128 lcm128(i128 a, i128 b) { return a / gcd128(a, b) * b; }

int orc_view_map(int32_t W, int32_t H, int32_t N,
                 int64_t tan_num, int64_t tan_den,
                 int64_t pitch_num, int64_t pitch_den,
                 int64_t off_num, int64_t off_den, int32_t *V)
{
    if (W <= 0 || H <= 0 || N <= 0 || tan_den <= 0 || pitch_den <= 0 ||
        off_den <= 0 || pitch_num <= 0)
        return -1;
    /* Scale every length by Q so that d_offset and L_x become integers:
     * D = Q * d_offset = Q*(3x+u) + Q*3y*tan(alpha) - Q*K_offset, P = Q*L_x.
     * Then x_offset*Q = D mod P (mathematical mod, in [0, P)) and
     * j = floor(N * x_offset / L_x) = floor(N * (D mod P) / P).            */
    i128 Q = lcm128(lcm128(tan_den, pitch_den), off_den);
    i128 P = (i128)pitch_num * (Q / pitch_den);
    for (int32_t y = 0; y < H; ++y)
        for (int32_t x = 0; x < W; ++x)
            for (int32_t u = 0; u < 3; ++u) {
                i128 D = (i128)(3 * (int64_t)x + u) * Q
                       + (i128)3 * y * tan_num * (Q / tan_den)
                       - (i128)off_num * (Q / off_den);
                i128 X = D % P;
                if (X < 0) X += P;
                V[((int64_t)y * W + x) * 3 + u] = (int32_t)(((i128)N * X) / P);
            }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Appendix B.1                                                             */
/* ------------------------------------------------------------------------ */

int32_t orc_cluster_table(int32_t N, int32_t S, int32_t *slots, int32_t *rep)
{
    if (N <= 0 || S <= 0) return -1;
    int32_t K = (N + S - 1) / S;
    for (int32_t k = 0; k < K; ++k) {
        for (int32_t l = 0; l < S; ++l) {
            int32_t j = k * S + l;
            slots[k * S + l] = j < N ? j : N - 1;      /* pad with v_{N-1} */
        }
        rep[k] = slots[k * S + S / 2];                  /* median index     */
    }
    return K;
}

/* ------------------------------------------------------------------------ */
/* Section 4.3                                                              */
/* ------------------------------------------------------------------------ */

typedef struct { int32_t v; uint32_t p; } vp_pair;

static int cmp_vp(const void *a, const void *b)
{
    const vp_pair *x = (const vp_pair *)a, *y = (const vp_pair *)b;
    if (x->v != y->v) return x->v < y->v ? -1 : 1;
    return x->p < y->p ? -1 : (x->p > y->p);
}

int orc_remap(int32_t W, int32_t H, int32_t tw, int32_t th,
              const int32_t *V, uint32_t *psi)
{
    if (W <= 0 || H <= 0 || tw <= 0 || th <= 0) return -1;
    int32_t TX = (W + tw - 1) / tw, TY = (H + th - 1) / th;
    vp_pair *buf = (vp_pair *)malloc(sizeof(vp_pair) * 3 * (size_t)tw * th);
    if (!buf) return -1;
    int64_t pos = 0;
    for (int32_t ty = 0; ty < TY; ++ty)
        for (int32_t tx = 0; tx < TX; ++tx) {
            int32_t n = 0;
            for (int32_t y = ty * th; y < (ty + 1) * th && y < H; ++y)
                for (int32_t x = tx * tw; x < (tx + 1) * tw && x < W; ++x)
                    for (int32_t u = 0; u < 3; ++u) {
                        uint32_t p = (uint32_t)(((int64_t)y * W + x) * 3 + u);
                        buf[n].v = V[p];
                        buf[n].p = p;
                        ++n;
                    }
            /* (V, p) pairs are unique, so sorting by them is the stable sort
             * of the row-major list by V. */
            qsort(buf, (size_t)n, sizeof(vp_pair), cmp_vp);
            for (int32_t e = 0; e < n; ++e) psi[pos++] = buf[e].p;
        }
    free(buf);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Spherical harmonics: real basis with the Condon-Shortley phase, bands     */
/* ordered m = -l..l, evaluated at a unit direction (x, y, z).               */
/* ------------------------------------------------------------------------ */

void orc_sh_basis(int32_t degree, const double d[3], double *Y)
{
    const double pi = 3.14159265358979323846;
    double x = d[0], y = d[1], z = d[2];
    Y[0] = 0.5 * sqrt(1.0 / pi);
    if (degree < 1) return;
    double c1 = sqrt(3.0 / (4.0 * pi));
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    if (degree < 2) return;
    double xx = x * x, yy = y * y, zz = z * z;
    double c2a = 0.5 * sqrt(15.0 / pi);
    double c2b = 0.25 * sqrt(5.0 / pi);
    double c2c = 0.25 * sqrt(15.0 / pi);
    Y[4] = c2a * (x * y);
    Y[5] = -c2a * (y * z);
    Y[6] = c2b * (2.0 * zz - xx - yy);
    Y[7] = -c2a * (x * z);
    Y[8] = c2c * (xx - yy);
    if (degree < 3) return;
    double c3a = 0.25 * sqrt(35.0 / (2.0 * pi));
    double c3b = 0.5 * sqrt(105.0 / pi);
    double c3c = 0.25 * sqrt(21.0 / (2.0 * pi));
    double c3d = 0.25 * sqrt(7.0 / pi);
    double c3e = 0.25 * sqrt(105.0 / pi);
    Y[9] = -c3a * (y * (3.0 * xx - yy));
    Y[10] = c3b * (x * y * z);
    Y[11] = -c3c * (y * (4.0 * zz - xx - yy));
    Y[12] = c3d * (z * (2.0 * zz - 3.0 * xx - 3.0 * yy));
    Y[13] = -c3c * (x * (4.0 * zz - xx - yy));
    Y[14] = c3e * (z * (xx - yy));
    Y[15] = -c3a * (x * (xx - 3.0 * yy));
}

/* ------------------------------------------------------------------------ */
/* Eq. 4-6: projection                                                      */
/* ------------------------------------------------------------------------ */

void orc_load_cam(const float *c, int32_t W, int32_t H, orc_cam *o)
{
    for (int k = 0; k < 9; ++k) o->R[k] = c[k];
    for (int k = 0; k < 3; ++k) o->t[k] = c[9 + k];
    o->fx = c[12];
    o->fy = c[13];
    o->cx = c[14];
    o->cy = c[15];
    o->limx = CLAMP_FOV * ((0.5 * (double)W) / o->fx);
    o->limy = CLAMP_FOV * ((0.5 * (double)H) / o->fy);
    for (int a = 0; a < 3; ++a)
        o->campos[a] = -((o->R[0 + a] * o->t[0] + o->R[3 + a] * o->t[1]) + o->R[6 + a] * o->t[2]);
}

double orc_clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

static void project_one(const float *mu, const float *ls, const float *q, float o,
                        const float *sh, int32_t nb, int32_t deg, const orc_cam *c,
                        orc_proj *out)
{
    memset(out, 0, sizeof *out);
    out->opacity = o;
    int finite = isfinite(o);
    for (int k = 0; k < 3; ++k) finite = finite && isfinite(mu[k]) && isfinite(ls[k]);
    for (int k = 0; k < 4; ++k) finite = finite && isfinite(q[k]);
    for (int k = 0; k < nb * 3; ++k) finite = finite && isfinite(sh[k]);

    /* Eq. 5: the mean, through the world->camera transform and the pinhole */
    double mx = mu[0], my = mu[1], mz = mu[2];
    const double *R = c->R;
    double tx = ((R[0] * mx + R[1] * my) + R[2] * mz) + c->t[0];
    double ty = ((R[3] * mx + R[4] * my) + R[5] * mz) + c->t[1];
    double tz = ((R[6] * mx + R[7] * my) + R[8] * mz) + c->t[2];
    float depth = (float)tz;
    out->depth = depth;
    if (!(finite && depth > NEAR_Z)) return;
    double ux = tx / tz, uy = ty / tz;
    out->mean2d[0] = (float)(c->fx * ux + c->cx);
    out->mean2d[1] = (float)(c->fy * uy + c->cy);
    out->valid_mean = isfinite(out->mean2d[0]) && isfinite(out->mean2d[1]);
    if (!out->valid_mean) return;
    if (!(o >= ALPHA_MIN)) return;

    /* 3D covariance Sigma = R_q S S^T R_q^T from the unit quaternion and the
     * per-axis scales exp(log_scale). */
    double qw = q[0], qx = q[1], qy = q[2], qz = q[3];
    double qn = sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz);
    qw = qw / qn; qx = qx / qn; qy = qy / qn; qz = qz / qn;
    double Rq[9] = {
        1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz), 2.0 * (qx * qz + qw * qy),
        2.0 * (qx * qy + qw * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx),
        2.0 * (qx * qz - qw * qy), 2.0 * (qy * qz + qw * qx), 1.0 - 2.0 * (qx * qx + qy * qy)};
    double s[3] = {exp((double)ls[0]), exp((double)ls[1]), exp((double)ls[2])};
    double Mq[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Mq[a * 3 + b] = Rq[a * 3 + b] * s[b];
    double Sig[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            Sig[a * 3 + b] = (Mq[a * 3 + 0] * Mq[b * 3 + 0] + Mq[a * 3 + 1] * Mq[b * 3 + 1])
                           + Mq[a * 3 + 2] * Mq[b * 3 + 2];
    /* camera-space covariance  Vc = R Sigma R^T */
    double T1[9], Vc[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            T1[a * 3 + b] = (R[a * 3 + 0] * Sig[0 * 3 + b] + R[a * 3 + 1] * Sig[1 * 3 + b])
                          + R[a * 3 + 2] * Sig[2 * 3 + b];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            Vc[a * 3 + b] = (T1[a * 3 + 0] * R[b * 3 + 0] + T1[a * 3 + 1] * R[b * 3 + 1])
                          + T1[a * 3 + 2] * R[b * 3 + 2];
    /* EWA: Jacobian of the pinhole at the (clamped) mean direction */
    double cxl = orc_clampd(ux, -c->limx, c->limx);
    double cyl = orc_clampd(uy, -c->limy, c->limy);
    double j00 = c->fx / tz, j02 = -(c->fx * cxl) / tz;
    double j11 = c->fy / tz, j12 = -(c->fy * cyl) / tz;
    /* K = J Vc (rows 0 and 1), Sigma2D = K J^T */
    double K00 = j00 * Vc[0] + j02 * Vc[6];
    double K01 = j00 * Vc[1] + j02 * Vc[7];
    double K02 = j00 * Vc[2] + j02 * Vc[8];
    double K11 = j11 * Vc[4] + j12 * Vc[7];
    double K12 = j11 * Vc[5] + j12 * Vc[8];
    double sa = (K00 * j00 + K02 * j02) + DILATION;
    double sb = K01 * j11 + K02 * j12;
    double sc = (K11 * j11 + K12 * j12) + DILATION;
    double det = sa * sc - sb * sb;
    if (!(det > 0.0)) return;
    /* Inverse covariance Q = [[sc, -sb], [-sb, sa]] / det, in LDL^T form:
     * d^T Q d = A (dx + beta dy)^2 + G dy^2 with A = sc/det, beta = -sb/sc,
     * G = 1/sc; stored pre-scaled by log2(e)/2 so that alpha = o 2^-E. */
    const double half_log2e = 0.5 * 1.44269504088896340736;
    double A = sc / det, beta = -sb / sc, G = 1.0 / sc;
    out->conic[0] = (float)(A * half_log2e);
    out->conic[1] = (float)beta;
    out->conic[2] = (float)(G * half_log2e);

    /* Eq. 6 colour: SH evaluated along the unit direction camera -> mean */
    double dv[3] = {mx - c->campos[0], my - c->campos[1], mz - c->campos[2]};
    double dn = sqrt((dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2]);
    dv[0] = dv[0] / dn; dv[1] = dv[1] / dn; dv[2] = dv[2] / dn;
    double Y[16];
    orc_sh_basis(deg, dv, Y);
    for (int u = 0; u < 3; ++u) {
        double acc = 0.0;
        for (int b = 0; b < nb; ++b) acc = acc + Y[b] * (double)sh[b * 3 + u];
        acc = acc + 0.5;
        out->color[u] = (float)(acc > 0.0 ? acc : 0.0);
    }
    int ok = 1;
    for (int k = 0; k < 3; ++k) ok = ok && isfinite(out->conic[k]) && isfinite(out->color[k]);
    ok = ok && out->conic[0] > 0.0f && out->conic[2] > 0.0f;
    out->valid = ok;
}

/* ------------------------------------------------------------------------ */
/* Host threads.  Every parallel loop below splits independent items (one   */
/* Gaussian, one subpixel, one image row) over threads; each item is         */
/* computed by exactly the same operations as in a single-threaded run, so   */
/* the results are bit-identical for any thread count.                      */
/* ------------------------------------------------------------------------ */

static int orc_threads = 1;

void orc_set_threads(int32_t n) { orc_threads = n < 1 ? 1 : (n > 256 ? 256 : n); }
int32_t orc_get_threads(void) { return orc_threads; }

typedef void (*range_fn)(void *arg, int64_t begin, int64_t end);
typedef struct { range_fn fn; void *arg; int64_t begin, end; } range_job;

static void *run_range(void *p)
{
    range_job *j = (range_job *)p;
    j->fn(j->arg, j->begin, j->end);
    return NULL;
}

/* fn(arg, b, e) over contiguous pieces of [0, n). */
static void parallel_for(int64_t n, int64_t min_per_thread, range_fn fn, void *arg)
{
    int64_t nt = orc_threads;
    if (min_per_thread < 1) min_per_thread = 1;
    if (nt > n / min_per_thread) nt = n / min_per_thread;
    if (nt <= 1) {
        if (n > 0) fn(arg, 0, n);
        return;
    }
    pthread_t tid[256];
    range_job job[256];
    int started[256];
    for (int64_t t = 0; t < nt; ++t) {
        job[t].fn = fn;
        job[t].arg = arg;
        job[t].begin = n * t / nt;
        job[t].end = n * (t + 1) / nt;
        started[t] = t > 0 && pthread_create(&tid[t], NULL, run_range, &job[t]) == 0;
    }
    run_range(&job[0]);
    for (int64_t t = 1; t < nt; ++t) {
        if (started[t]) pthread_join(tid[t], NULL);
        else run_range(&job[t]);      /* could not start a thread: do it here */
    }
}

typedef struct {
    int32_t deg, nb;
    const float *means, *log_scales, *quats, *opac, *sh;
    const orc_cam *c;
    orc_proj *out;
} project_job;

static void project_range(void *p, int64_t b, int64_t e)
{
    const project_job *j = (const project_job *)p;
    for (int64_t i = b; i < e; ++i)
        project_one(j->means + 3 * i, j->log_scales + 3 * i, j->quats + 4 * i, j->opac[i],
                    j->sh + (int64_t)j->nb * 3 * i, j->nb, j->deg, j->c, j->out + i);
}

void orc_project(int64_t M, int32_t deg, const float *means, const float *log_scales,
                 const float *quats, const float *opac, const float *sh, const float *cam,
                 int32_t W, int32_t H, orc_proj *out)
{
    orc_cam c;
    orc_load_cam(cam, W, H, &c);
    project_job j = {deg, (deg + 1) * (deg + 1), means, log_scales, quats, opac, sh, &c, out};
    parallel_for(M, 4096, project_range, &j);
}

/* ------------------------------------------------------------------------ */
/* Eq. 9-10: front-to-back blend                                            */
/* ------------------------------------------------------------------------ */

typedef struct { float d; int64_t i; } depth_key;

static int cmp_depth(const void *a, const void *b)
{
    const depth_key *x = (const depth_key *)a, *y = (const depth_key *)b;
    if (x->d != y->d) return x->d < y->d ? -1 : 1;
    return x->i < y->i ? -1 : (x->i > y->i);
}

/* Indices of the Gaussians valid at `rep`, ordered by (float32 depth, i). */
static int64_t depth_order(int64_t M, const orc_proj *rep, int64_t *order)
{
    depth_key *keys = (depth_key *)malloc(sizeof(depth_key) * (size_t)(M > 0 ? M : 1));
    int64_t n = 0;
    for (int64_t i = 0; i < M; ++i)
        if (rep[i].valid) {
            keys[n].d = rep[i].depth;
            keys[n].i = i;
            ++n;
        }
    qsort(keys, (size_t)n, sizeof(depth_key), cmp_depth);
    for (int64_t e = 0; e < n; ++e) order[e] = keys[e].i;
    free(keys);
    return n;
}

/* The walk over one ordered list at sample position (px, py) for the
 * channels [u0, u1).  Mean and validity come from `view`, the conic, colour
 * and opacity from `rep` (the same array on the exact path).
 *
 * Near-threshold decisions.  A float32 evaluation of the same formulas (dx,
 * dy, w = dx + beta dy, A' w^2 + G' dy^2, exp2 within one ulp, the opacity
 * product) has, to first order in the unit roundoff u, an error in E of at
 * most u * SE and a relative error in alpha of at most ea = ln2 * u * SE + 3u;
 * T carries the accumulated bound relT.  An alpha or T' within FLAG_SAFETY
 * times its bound of its threshold may fall on the other side in float32.
 * The main walk takes every decision on the float32-rounded value and
 * records the first such event (flags bit 0: alpha near 1/255, bit 1: T' near
 * 1e-4; tflag = T before it).  With `branch` set, the walk also follows the
 * other outcome of every flagged decision (a depth-first tree of at most
 * MAX_PATHS leaves) and keeps the range [lo, hi] of the values its leaves
 * reach: every value a float32 renderer can legitimately produce, up to its
 * own rounding of the sums. */
#define MAX_PATHS 64

typedef struct {
    const int64_t *order;
    int64_t n;
    const orc_proj *rep, *view;
    double px, py;
    int u0, u1;
    const float *bg;
    int branch;
    int paths, overflow;
    double lo[3], hi[3];
    float out[3];
    int32_t flag;
    double tflag;
} walk_t;

/* Continue the walk at list position e with state (T, C, relT).  At position
 * fe the alpha-cutoff and stop decisions are forced to fcut / fstop when
 * those are >= 0 (a branch taking the other outcome). */
static void walk(walk_t *w, int64_t e, double T, const double *Cin, double relT,
                 int64_t fe, int fcut, int fstop, int main_path)
{
    double C[3] = {Cin[0], Cin[1], Cin[2]};
    for (; e < w->n; ++e) {
        int64_t i = w->order[e];
        const orc_proj *g = w->rep + i, *m = w->view + i;
        if (!m->valid_mean) continue;
        double dx = w->px - (double)m->mean2d[0];
        double dy = w->py - (double)m->mean2d[1];
        double beta = (double)g->conic[1];
        double ww = dx + beta * dy;
        double E = (double)g->conic[0] * ww * ww + (double)g->conic[2] * dy * dy;
        double alpha = (double)g->opacity * exp2(-E);
        int clamped = alpha > ALPHA_MAX;
        if (clamped) alpha = ALPHA_MAX;
        double SE = 2.0 * (double)g->conic[0] * fabs(ww) * (fabs(dx) + fabs(beta * dy) + fabs(ww))
                  + (double)g->conic[0] * ww * ww + 4.0 * (double)g->conic[2] * dy * dy + E;
        double ea = clamped ? 1e-6 : 0.6931471805599453 * U32 * SE + 3.0 * U32;
        int forced = e == fe;
        int near_cut = fabs(alpha - 1.0 / 255.0) <= FLAG_SAFETY * ea * alpha;
        if (near_cut && main_path && !w->flag) {
            w->tflag = T;
            w->flag |= 1;
        } else if (near_cut && main_path) {
            w->flag |= 1;
        }
        int pass = (float)alpha >= ALPHA_MIN;
        if (forced && fcut >= 0) {
            pass = fcut;
        } else if (near_cut && w->branch) {
            if (w->paths + 1 < MAX_PATHS) {
                ++w->paths;
                walk(w, e, T, C, relT, e, !pass, -1, 0);
            } else {
                w->overflow = 1;
            }
        }
        if (!pass) continue;
        double Tn = T * (1.0 - alpha);
        double step = (clamped ? 1e-6 : alpha / (1.0 - alpha) * ea) + 2.0 * U32;
        int near_stop = fabs(Tn - 1e-4) <= FLAG_SAFETY * (relT + step) * Tn;
        if (near_stop && main_path && !w->flag) {
            w->tflag = T;
            w->flag |= 2;
        } else if (near_stop && main_path) {
            w->flag |= 2;
        }
        int stop = (float)Tn < T_STOP;
        if (forced && fstop >= 0) {
            stop = fstop;
        } else if (near_stop && w->branch) {
            if (w->paths + 1 < MAX_PATHS) {
                ++w->paths;
                walk(w, e, T, C, relT, e, pass, !stop, 0);
            } else {
                w->overflow = 1;
            }
        }
        if (stop) break;
        for (int u = w->u0; u < w->u1; ++u) C[u] = C[u] + (double)g->color[u] * alpha * T;
        T = Tn;
        relT += step;
    }
    for (int u = w->u0; u < w->u1; ++u) {
        double v = (double)(float)(C[u] + T * (double)w->bg[u]);
        if (v < w->lo[u]) w->lo[u] = v;
        if (v > w->hi[u]) w->hi[u] = v;
        if (main_path) w->out[u] = (float)(C[u] + T * (double)w->bg[u]);
    }
}

static void blend_walk(walk_t *w, double px, double py, int u0, int u1)
{
    const double zero[3] = {0.0, 0.0, 0.0};
    w->px = px;
    w->py = py;
    w->u0 = u0;
    w->u1 = u1;
    w->paths = 1;
    w->overflow = 0;
    w->flag = 0;
    w->tflag = 0.0;
    for (int u = 0; u < 3; ++u) {
        w->lo[u] = INFINITY;
        w->hi[u] = -INFINITY;
        w->out[u] = 0.0f;
    }
    walk(w, 0, 1.0, zero, 0.0, -1, -1, -1, 1);
}

/* One view's samples of orc_render_subpixels_ex. */
typedef struct {
    const int64_t *order;
    int64_t n;
    const orc_proj *rep, *view;
    const float *bg;
    int32_t W;
    const int64_t *samples;   /* all samples */
    const int64_t *which;     /* indices into samples of this view's */
    float *out;
    int32_t *flags;
    double *tflag;
    float *lo, *hi;
    int32_t *paths;
} view_job;

static void view_range(void *p, int64_t b, int64_t e)
{
    const view_job *j = (const view_job *)p;
    walk_t w;
    w.order = j->order;
    w.n = j->n;
    w.rep = j->rep;
    w.view = j->view;
    w.bg = j->bg;
    w.branch = j->lo != NULL;
    for (int64_t q = b; q < e; ++q) {
        int64_t s = j->which[q];
        int64_t p = j->samples[s];
        int32_t u = (int32_t)(p % 3);
        int64_t pix = p / 3;
        blend_walk(&w, (double)(pix % j->W) + 0.5, (double)(pix / j->W) + 0.5, u, u + 1);
        j->out[s] = w.out[u];
        if (j->flags) j->flags[s] = w.flag;
        if (j->tflag) j->tflag[s] = w.tflag;
        if (j->lo) {
            j->lo[s] = (float)w.lo[u];
            j->hi[s] = (float)w.hi[u];
            j->paths[s] = w.overflow ? -w.paths : w.paths;
        }
    }
}

int orc_render_subpixels_ex(int64_t M, int32_t deg, const float *means, const float *log_scales,
                            const float *quats, const float *opac, const float *sh,
                            const float *cams, int32_t N, const int32_t *V, int32_t W, int32_t H,
                            int32_t S, const float *bg, int64_t n_samples, const int64_t *samples,
                            float *out, int32_t *flags, double *tflag,
                            float *lo, float *hi, int32_t *paths)
{
    if (M < 0 || N <= 0 || S <= 0 || W <= 0 || H <= 0) return -1;
    if ((lo != NULL) != (hi != NULL) || (lo != NULL) != (paths != NULL)) return -1;
    int64_t total = 3 * (int64_t)W * H;
    for (int64_t s = 0; s < n_samples; ++s)
        if (samples[s] < 0 || samples[s] >= total) return -1;
    int32_t K = (N + S - 1) / S;
    int32_t *slots = (int32_t *)malloc(sizeof(int32_t) * (size_t)K * S);
    int32_t *rep = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    orc_cluster_table(N, S, slots, rep);
    size_t mm = (size_t)(M > 0 ? M : 1);
    orc_proj *prep = (orc_proj *)malloc(sizeof(orc_proj) * mm);
    orc_proj *pview = (orc_proj *)malloc(sizeof(orc_proj) * mm);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * mm);
    int64_t *which = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_samples > 0 ? n_samples : 1));
    char *need = (char *)malloc((size_t)N);
    for (int32_t k = 0; k < K; ++k) {
        /* any sample in this cluster? */
        int any = 0;
        memset(need, 0, (size_t)N);
        for (int64_t s = 0; s < n_samples; ++s) {
            int32_t j = V[samples[s]];
            if (j / S == k) { need[j] = 1; any = 1; }
        }
        if (!any) continue;
        int32_t r = rep[k];
        orc_project(M, deg, means, log_scales, quats, opac, sh, cams + 16 * (int64_t)r, W, H, prep);
        int64_t n = depth_order(M, prep, order);
        for (int32_t j = 0; j < N; ++j) {
            if (!need[j]) continue;
            const orc_proj *pv = prep;
            if (j != r) {
                orc_project(M, deg, means, log_scales, quats, opac, sh, cams + 16 * (int64_t)j, W, H, pview);
                pv = pview;
            }
            int64_t nw = 0;
            for (int64_t s = 0; s < n_samples; ++s)
                if (V[samples[s]] == j) which[nw++] = s;
            view_job job = {order, n, prep, pv, bg, W, samples, which, out, flags, tflag, lo, hi, paths};
            parallel_for(nw, 1, view_range, &job);
        }
    }
    free(slots); free(rep); free(prep); free(pview); free(order); free(which); free(need);
    return 0;
}

int orc_render_subpixels(int64_t M, int32_t deg, const float *means, const float *log_scales,
                         const float *quats, const float *opac, const float *sh,
                         const float *cams, int32_t N, const int32_t *V, int32_t W, int32_t H,
                         int32_t S, const float *bg, int64_t n_samples, const int64_t *samples,
                         float *out, int32_t *flags, double *tflag)
{
    return orc_render_subpixels_ex(M, deg, means, log_scales, quats, opac, sh, cams, N, V, W, H, S, bg,
                                   n_samples, samples, out, flags, tflag, NULL, NULL, NULL);
}

typedef struct {
    const int64_t *order;
    int64_t n;
    const orc_proj *pr;
    const float *bg;
    int32_t W;
    float *img;
    int32_t *flags;
    double *tflag;
} rows_job;

static void rows_range(void *p, int64_t b, int64_t e)
{
    const rows_job *j = (const rows_job *)p;
    walk_t w;
    w.order = j->order;
    w.n = j->n;
    w.rep = j->pr;
    w.view = j->pr;
    w.bg = j->bg;
    w.branch = 0;
    for (int64_t y = b; y < e; ++y)
        for (int32_t x = 0; x < j->W; ++x) {
            int64_t pix = y * j->W + x;
            blend_walk(&w, x + 0.5, (double)y + 0.5, 0, 3);
            for (int u = 0; u < 3; ++u) j->img[3 * pix + u] = w.out[u];
            if (j->flags) j->flags[pix] = w.flag;
            if (j->tflag) j->tflag[pix] = w.tflag;
        }
}

void orc_render_view(int64_t M, int32_t deg, const float *means, const float *log_scales,
                     const float *quats, const float *opac, const float *sh, const float *cam,
                     int32_t W, int32_t H, const float *bg, float *img, int32_t *flags,
                     double *tflag)
{
    size_t mm = (size_t)(M > 0 ? M : 1);
    orc_proj *pr = (orc_proj *)malloc(sizeof(orc_proj) * mm);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * mm);
    orc_project(M, deg, means, log_scales, quats, opac, sh, cam, W, H, pr);
    int64_t n = depth_order(M, pr, order);
    rows_job job = {order, n, pr, bg, W, img, flags, tflag};
    parallel_for(H, 1, rows_range, &job);
    free(pr);
    free(order);
}
