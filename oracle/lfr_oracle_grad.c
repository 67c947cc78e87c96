/*
 * lfr_oracle_grad.c -- gradient oracle: the subpixel renderer of section 4.3
 * (Eq. 9-10, with the reuse rule of section 4.2, Eq. 5-6) evaluated in IEEE
 * double precision with nothing rounded to float32, and its analytic
 * reverse-mode derivative with respect to every scene parameter.
 *
 * TEST INFRASTRUCTURE ONLY.  It shares no code with the HIP library; only
 * the tests may load it.
 *
 * The paper defines the forward renderer only; the derivative is the chain
 * rule applied to that definition, step by step:
 *
 *   blend      out = sum_e c_e a_e T_e + T_end bg,  T_{e+1} = T_e (1 - a_e)
 *              a = min(0.99, o 2^-E),  E = A'(dx + beta dy)^2 + G' dy^2,
 *              (dx, dy) = sample centre - projected mean of the blended view
 *   conic      A' = h sc/det, beta = -sb/sc, G' = h/sc,  h = log2(e)/2,
 *              det = sa sc - sb^2, [[sa, sb], [sb, sc]] = J Vc J^T + 0.3 I
 *   camera     Vc = R Sigma R^T, J = pinhole Jacobian at the clamped mean
 *              direction, t = R mu + t_cam
 *   3D shape   Sigma = M M^T, M = R(q / |q|) diag(exp(log_scale))
 *   colour     c_u = max(0, sum_b Y_b(d) h_bu + 1/2), d = (mu - campos)/|.|
 *   mean       m2d = (fx tx/tz + cx, fy ty/tz + cy) in the blended view
 *
 * The discrete decisions (which Gaussians are valid, their depth order,
 * which pass the 1/255 cutoff, where the 1e-4 transmittance stop falls,
 * the 0.99 alpha clamp, the colour clamp at 0 and the Jacobian clamp) are
 * taken once per evaluation and held fixed; derivatives through an active
 * clamp are zero.  The decisions are taken either on the double values
 * (mode 0: the function whose finite differences the analytic gradient must
 * match) or exactly as the float32-attribute oracle takes them (mode 1: the
 * decisions of a float32 rasterizer).
 */
#include "lfr_oracle.h"
#include "lfr_oracle_impl.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define LN2 0.69314718055994530942

/* Everything the reverse pass needs about one Gaussian seen from one camera. */
typedef struct {
    double t[3], ux, uy, m2d[2];
    int valid_mean;
    double qn, qh[4], Rq[9], s[3], M[9], Vc[9];
    double cxl, cyl;
    int clx, cly;                /* Jacobian clamp active on x / y */
    double j00, j02, j11, j12;
    double sa, sb, sc, det;
    double A, beta, G;           /* A', beta, G' */
    double dn, dir[3], Y[16], raw[3], color[3];
    double depth;
    int valid;
} p64;

static void mat3_mul(const double *a, const double *b, double *c)
{
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k)
            c[r * 3 + k] = (a[r * 3 + 0] * b[0 * 3 + k] + a[r * 3 + 1] * b[1 * 3 + k]) + a[r * 3 + 2] * b[2 * 3 + k];
}

static void mat3_transpose(const double *a, double *t)
{
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) t[k * 3 + r] = a[r * 3 + k];
}

/* The forward projection in double precision (section 4.1 Eq. 4, section
 * 4.2 Eq. 5-6), with the same validity rules as the float32 oracle applied
 * to the double values. */
static void project64(const float *mu, const float *ls, const float *q, float o, const float *sh,
                      int nb, int deg, const orc_cam *c, p64 *P)
{
    memset(P, 0, sizeof *P);
    int finite = isfinite(o);
    for (int k = 0; k < 3; ++k) finite = finite && isfinite(mu[k]) && isfinite(ls[k]);
    for (int k = 0; k < 4; ++k) finite = finite && isfinite(q[k]);
    for (int k = 0; k < nb * 3; ++k) finite = finite && isfinite(sh[k]);
    const double *R = c->R;
    const double m[3] = {mu[0], mu[1], mu[2]};
    for (int a = 0; a < 3; ++a) P->t[a] = ((R[a * 3] * m[0] + R[a * 3 + 1] * m[1]) + R[a * 3 + 2] * m[2]) + c->t[a];
    P->depth = P->t[2];
    if (!(finite && P->t[2] > (double)NEAR_Z)) return;
    P->ux = P->t[0] / P->t[2];
    P->uy = P->t[1] / P->t[2];
    P->m2d[0] = c->fx * P->ux + c->cx;
    P->m2d[1] = c->fy * P->uy + c->cy;
    P->valid_mean = isfinite(P->m2d[0]) && isfinite(P->m2d[1]);
    if (!P->valid_mean || !(o >= ALPHA_MIN)) return;

    /* Sigma = M M^T, M = R(q^) diag(s) */
    P->qn = sqrt((((double)q[0] * q[0] + (double)q[1] * q[1]) + (double)q[2] * q[2]) + (double)q[3] * q[3]);
    for (int k = 0; k < 4; ++k) P->qh[k] = q[k] / P->qn;
    const double w = P->qh[0], x = P->qh[1], y = P->qh[2], z = P->qh[3];
    double *Rq = P->Rq;
    Rq[0] = 1.0 - 2.0 * (y * y + z * z); Rq[1] = 2.0 * (x * y - w * z);       Rq[2] = 2.0 * (x * z + w * y);
    Rq[3] = 2.0 * (x * y + w * z);       Rq[4] = 1.0 - 2.0 * (x * x + z * z); Rq[5] = 2.0 * (y * z - w * x);
    Rq[6] = 2.0 * (x * z - w * y);       Rq[7] = 2.0 * (y * z + w * x);       Rq[8] = 1.0 - 2.0 * (x * x + y * y);
    for (int b = 0; b < 3; ++b) P->s[b] = exp((double)ls[b]);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) P->M[a * 3 + b] = Rq[a * 3 + b] * P->s[b];
    double Mt[9], Sig[9], RS[9], Rt[9];
    mat3_transpose(P->M, Mt);
    mat3_mul(P->M, Mt, Sig);
    mat3_mul(R, Sig, RS);
    mat3_transpose(R, Rt);
    mat3_mul(RS, Rt, P->Vc);

    /* EWA: J at the clamped direction, Sigma2D = J Vc J^T + 0.3 I */
    P->cxl = orc_clampd(P->ux, -c->limx, c->limx);
    P->cyl = orc_clampd(P->uy, -c->limy, c->limy);
    P->clx = P->cxl != P->ux;
    P->cly = P->cyl != P->uy;
    const double tz = P->t[2];
    P->j00 = c->fx / tz;
    P->j02 = -(c->fx * P->cxl) / tz;
    P->j11 = c->fy / tz;
    P->j12 = -(c->fy * P->cyl) / tz;
    const double J[6] = {P->j00, 0.0, P->j02, 0.0, P->j11, P->j12};
    double S2[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) acc += J[a * 3 + k] * P->Vc[k * 3 + l] * J[b * 3 + l];
            S2[a * 2 + b] = acc;
        }
    P->sa = S2[0] + DILATION;
    P->sb = 0.5 * (S2[1] + S2[2]);
    P->sc = S2[3] + DILATION;
    P->det = P->sa * P->sc - P->sb * P->sb;
    if (!(P->det > 0.0)) return;
    P->A = HALF_LOG2E * P->sc / P->det;
    P->beta = -P->sb / P->sc;
    P->G = HALF_LOG2E / P->sc;

    /* colour along the unit direction camera -> mean */
    double v[3] = {m[0] - c->campos[0], m[1] - c->campos[1], m[2] - c->campos[2]};
    P->dn = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    for (int k = 0; k < 3; ++k) P->dir[k] = v[k] / P->dn;
    orc_sh_basis(deg, P->dir, P->Y);
    for (int u = 0; u < 3; ++u) {
        double acc = 0.0;
        for (int b = 0; b < nb; ++b) acc = acc + P->Y[b] * (double)sh[b * 3 + u];
        P->raw[u] = acc + 0.5;
        P->color[u] = P->raw[u] > 0.0 ? P->raw[u] : 0.0;
    }
    int ok = P->A > 0.0 && P->G > 0.0 && isfinite(P->A) && isfinite(P->beta) && isfinite(P->G);
    for (int u = 0; u < 3; ++u) ok = ok && isfinite(P->color[u]);
    P->valid = ok;
}

/* Gradient of the real SH basis polynomials (as functions on R^3, in the
 * form the basis is written) at d: dY[b][k] = dY_b / d d_k. */
static void sh_basis_grad(int deg, const double d[3], double dY[16][3])
{
    const double pi = 3.14159265358979323846;
    const double x = d[0], y = d[1], z = d[2];
    memset(dY, 0, sizeof(double) * 48);
    if (deg < 1) return;
    const double c1 = sqrt(3.0 / (4.0 * pi));
    dY[1][1] = -c1;
    dY[2][2] = c1;
    dY[3][0] = -c1;
    if (deg < 2) return;
    const double c2a = 0.5 * sqrt(15.0 / pi), c2b = 0.25 * sqrt(5.0 / pi), c2c = 0.25 * sqrt(15.0 / pi);
    dY[4][0] = c2a * y;          dY[4][1] = c2a * x;
    dY[5][1] = -c2a * z;         dY[5][2] = -c2a * y;
    dY[6][0] = -2.0 * c2b * x;   dY[6][1] = -2.0 * c2b * y;  dY[6][2] = 4.0 * c2b * z;
    dY[7][0] = -c2a * z;         dY[7][2] = -c2a * x;
    dY[8][0] = 2.0 * c2c * x;    dY[8][1] = -2.0 * c2c * y;
    if (deg < 3) return;
    const double c3a = 0.25 * sqrt(35.0 / (2.0 * pi)), c3b = 0.5 * sqrt(105.0 / pi);
    const double c3c = 0.25 * sqrt(21.0 / (2.0 * pi)), c3d = 0.25 * sqrt(7.0 / pi);
    const double c3e = 0.25 * sqrt(105.0 / pi);
    const double xx = x * x, yy = y * y, zz = z * z;
    /* Y9 = -c3a (3 x^2 y - y^3) */
    dY[9][0] = -c3a * 6.0 * x * y;           dY[9][1] = -c3a * (3.0 * xx - 3.0 * yy);
    /* Y10 = c3b x y z */
    dY[10][0] = c3b * y * z;                 dY[10][1] = c3b * x * z;               dY[10][2] = c3b * x * y;
    /* Y11 = -c3c (4 y z^2 - x^2 y - y^3) */
    dY[11][0] = c3c * 2.0 * x * y;           dY[11][1] = -c3c * (4.0 * zz - xx - 3.0 * yy);
    dY[11][2] = -c3c * 8.0 * y * z;
    /* Y12 = c3d (2 z^3 - 3 x^2 z - 3 y^2 z) */
    dY[12][0] = -c3d * 6.0 * x * z;          dY[12][1] = -c3d * 6.0 * y * z;
    dY[12][2] = c3d * (6.0 * zz - 3.0 * xx - 3.0 * yy);
    /* Y13 = -c3c (4 x z^2 - x^3 - x y^2) */
    dY[13][0] = -c3c * (4.0 * zz - 3.0 * xx - yy);
    dY[13][1] = c3c * 2.0 * x * y;           dY[13][2] = -c3c * 8.0 * x * z;
    /* Y14 = c3e (x^2 z - y^2 z) */
    dY[14][0] = c3e * 2.0 * x * z;           dY[14][1] = -c3e * 2.0 * y * z;        dY[14][2] = c3e * (xx - yy);
    /* Y15 = -c3a (x^3 - 3 x y^2) */
    dY[15][0] = -c3a * (3.0 * xx - 3.0 * yy); dY[15][1] = c3a * 6.0 * x * y;
}

/* d(loss)/d(mean2d) at camera c -> d(loss)/d(mu). */
static void mean_backward(const orc_cam *c, const p64 *P, const double dm[2], double *gmu)
{
    const double tz = P->t[2];
    const double dux = c->fx * dm[0], duy = c->fy * dm[1];
    const double dt[3] = {dux / tz, duy / tz, -(dux * P->t[0] + duy * P->t[1]) / (tz * tz)};
    for (int k = 0; k < 3; ++k) gmu[k] += (c->R[0 * 3 + k] * dt[0] + c->R[1 * 3 + k] * dt[1]) + c->R[2 * 3 + k] * dt[2];
}

/* d(loss)/d(A', beta, G', colour) at camera c -> every scene parameter. */
static void full_backward(const orc_cam *c, const p64 *P, const float *sh, int nb, int deg,
                          const double dcon[3], const double dcol[3], double *gmu, double *gls,
                          double *gq, double *gsh)
{
    /* conic -> Sigma2D entries */
    const double det2 = P->det * P->det;
    const double dsa = dcon[0] * HALF_LOG2E * (-P->sc * P->sc / det2);
    const double dsb = dcon[0] * HALF_LOG2E * (2.0 * P->sb * P->sc / det2) + dcon[1] * (-1.0 / P->sc);
    const double dsc = dcon[0] * HALF_LOG2E * (-P->sb * P->sb / det2) + dcon[1] * (P->sb / (P->sc * P->sc))
                     + dcon[2] * HALF_LOG2E * (-1.0 / (P->sc * P->sc));
    /* Sigma2D = J Vc J^T: dJ = 2 Gs J Vc, dVc = J^T Gs J, Gs the symmetric
     * gradient [[dsa, dsb/2], [dsb/2, dsc]] */
    const double Gs[4] = {dsa, 0.5 * dsb, 0.5 * dsb, dsc};
    const double J[6] = {P->j00, 0.0, P->j02, 0.0, P->j11, P->j12};
    double JV[6], dJ[6], dVc[9];
    for (int a = 0; a < 2; ++a)
        for (int l = 0; l < 3; ++l) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += J[a * 3 + k] * P->Vc[k * 3 + l];
            JV[a * 3 + l] = acc;
        }
    for (int a = 0; a < 2; ++a)
        for (int l = 0; l < 3; ++l) dJ[a * 3 + l] = 2.0 * (Gs[a * 2 + 0] * JV[0 * 3 + l] + Gs[a * 2 + 1] * JV[1 * 3 + l]);
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
            double acc = 0.0;
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) acc += J[a * 3 + k] * Gs[a * 2 + b] * J[b * 3 + l];
            dVc[k * 3 + l] = acc;
        }
    /* J -> camera-space mean (only the entries that depend on it) */
    const double tz = P->t[2];
    double dt[3] = {0.0, 0.0, 0.0};
    const double dj00 = dJ[0], dj02 = dJ[2], dj11 = dJ[4], dj12 = dJ[5];
    dt[2] += -dj00 * c->fx / (tz * tz) + dj02 * c->fx * P->cxl / (tz * tz)
           - dj11 * c->fy / (tz * tz) + dj12 * c->fy * P->cyl / (tz * tz);
    const double dcxl = -dj02 * c->fx / tz, dcyl = -dj12 * c->fy / tz;
    if (!P->clx) {
        dt[0] += dcxl / tz;
        dt[2] += -dcxl * P->t[0] / (tz * tz);
    }
    if (!P->cly) {
        dt[1] += dcyl / tz;
        dt[2] += -dcyl * P->t[1] / (tz * tz);
    }
    for (int k = 0; k < 3; ++k) gmu[k] += (c->R[0 * 3 + k] * dt[0] + c->R[1 * 3 + k] * dt[1]) + c->R[2 * 3 + k] * dt[2];
    /* Vc = R Sigma R^T: dSigma = R^T dVc R */
    double Rt[9], tmp[9], dSig[9];
    mat3_transpose(c->R, Rt);
    mat3_mul(Rt, dVc, tmp);
    mat3_mul(tmp, c->R, dSig);
    /* Sigma = M M^T: dM = (dSig + dSig^T) M */
    double dM[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += (dSig[a * 3 + k] + dSig[k * 3 + a]) * P->M[k * 3 + b];
            dM[a * 3 + b] = acc;
        }
    /* M = Rq diag(s), s = exp(log_scale) */
    double dRq[9];
    for (int b = 0; b < 3; ++b) {
        double ds = 0.0;
        for (int a = 0; a < 3; ++a) {
            dRq[a * 3 + b] = dM[a * 3 + b] * P->s[b];
            ds += dM[a * 3 + b] * P->Rq[a * 3 + b];
        }
        gls[b] += ds * P->s[b];
    }
    /* Rq(w, x, y, z) of the unit quaternion */
    const double w = P->qh[0], x = P->qh[1], y = P->qh[2], z = P->qh[3];
    const double *g = dRq;
    double dqh[4];
    dqh[0] = 2.0 * (-z * g[1] + y * g[2] + z * g[3] - x * g[5] - y * g[6] + x * g[7]);
    dqh[1] = 2.0 * (y * g[1] + z * g[2] + y * g[3] - 2.0 * x * g[4] - w * g[5] + z * g[6] + w * g[7] - 2.0 * x * g[8]);
    dqh[2] = 2.0 * (-2.0 * y * g[0] + x * g[1] + w * g[2] + x * g[3] + z * g[5] - w * g[6] + z * g[7] - 2.0 * y * g[8]);
    dqh[3] = 2.0 * (-2.0 * z * g[0] - w * g[1] + x * g[2] + w * g[3] - 2.0 * z * g[4] + y * g[5] + x * g[6] + y * g[7]);
    /* q^ = q / |q| */
    const double dot = ((dqh[0] * w + dqh[1] * x) + dqh[2] * y) + dqh[3] * z;
    for (int k = 0; k < 4; ++k) gq[k] += (dqh[k] - P->qh[k] * dot) / P->qn;
    /* colour: SH coefficients and the viewing direction */
    double dY[16][3];
    sh_basis_grad(deg, P->dir, dY);
    double ddir[3] = {0.0, 0.0, 0.0};
    for (int u = 0; u < 3; ++u) {
        if (!(P->raw[u] > 0.0) || dcol[u] == 0.0) continue;
        for (int b = 0; b < nb; ++b) {
            gsh[b * 3 + u] += P->Y[b] * dcol[u];
            for (int k = 0; k < 3; ++k) ddir[k] += dcol[u] * (double)sh[b * 3 + u] * dY[b][k];
        }
    }
    const double dd = (ddir[0] * P->dir[0] + ddir[1] * P->dir[1]) + ddir[2] * P->dir[2];
    for (int k = 0; k < 3; ++k) gmu[k] += (ddir[k] - P->dir[k] * dd) / P->dn;
}

typedef struct { double d; int64_t i; } dkey64;

static int cmp_dkey64(const void *a, const void *b)
{
    const dkey64 *x = (const dkey64 *)a, *y = (const dkey64 *)b;
    if (x->d != y->d) return x->d < y->d ? -1 : 1;
    return x->i < y->i ? -1 : (x->i > y->i);
}

static uint64_t mix(uint64_t h, uint64_t v)
{
    h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    return h * 0x100000001B3ull;
}

/* One blended entry of a subpixel's list. */
typedef struct {
    int64_t i;
    int clamped;
    double a, T, ex, dx, dy, w;
} bent;

int orc_grad_subpixels(int64_t M, int32_t deg, const float *means, const float *log_scales,
                       const float *quats, const float *opac, const float *sh, const float *cams,
                       int32_t N, const int32_t *V, int32_t W, int32_t H, int32_t S, const float *bg,
                       int64_t n_samples, const int64_t *samples, const double *gout, int32_t mode,
                       double *out, uint64_t *sig, double *d_means, double *d_log_scales,
                       double *d_quats, double *d_opacities, double *d_sh)
{
    if (M < 0 || N <= 0 || S <= 0 || W <= 0 || H <= 0 || deg < 0 || deg > 3 || (mode != 0 && mode != 1))
        return -1;
    const int64_t total = 3 * (int64_t)W * H;
    for (int64_t s = 0; s < n_samples; ++s)
        if (samples[s] < 0 || samples[s] >= total) return -1;
    const int nb = (deg + 1) * (deg + 1);
    const int grads = d_means != NULL;
    if (grads) {
        memset(d_means, 0, sizeof(double) * 3 * (size_t)M);
        memset(d_log_scales, 0, sizeof(double) * 3 * (size_t)M);
        memset(d_quats, 0, sizeof(double) * 4 * (size_t)M);
        memset(d_opacities, 0, sizeof(double) * (size_t)M);
        memset(d_sh, 0, sizeof(double) * 3 * nb * (size_t)M);
    }
    const int32_t K = (N + S - 1) / S;
    int32_t *slots = (int32_t *)malloc(sizeof(int32_t) * (size_t)K * S);
    int32_t *rep = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    orc_cluster_table(N, S, slots, rep);
    const size_t mm = (size_t)(M > 0 ? M : 1);
    p64 *prep = (p64 *)malloc(sizeof(p64) * mm), *pview = (p64 *)malloc(sizeof(p64) * mm);
    orc_proj *frep = (orc_proj *)malloc(sizeof(orc_proj) * mm), *fview = (orc_proj *)malloc(sizeof(orc_proj) * mm);
    dkey64 *keys = (dkey64 *)malloc(sizeof(dkey64) * mm);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * mm);
    bent *list = (bent *)malloc(sizeof(bent) * mm);
    double *dcon = (double *)calloc(mm * 3, sizeof(double)), *dcol = (double *)calloc(mm * 3, sizeof(double));
    double *dop = (double *)calloc(mm, sizeof(double)), *dm2 = (double *)calloc(mm * 2, sizeof(double));
    char *need = (char *)malloc((size_t)N);

    for (int32_t k = 0; k < K; ++k) {
        int any = 0;
        memset(need, 0, (size_t)N);
        for (int64_t s = 0; s < n_samples; ++s) {
            const int32_t j = V[samples[s]];
            if (j / S == k) need[j] = any = 1;
        }
        if (!any) continue;
        const int32_t r = rep[k];
        orc_cam cr;
        orc_load_cam(cams + 16 * (int64_t)r, W, H, &cr);
        for (int64_t i = 0; i < M; ++i)
            project64(means + 3 * i, log_scales + 3 * i, quats + 4 * i, opac[i], sh + (int64_t)nb * 3 * i, nb, deg,
                      &cr, prep + i);
        if (mode == 1)
            orc_project(M, deg, means, log_scales, quats, opac, sh, cams + 16 * (int64_t)r, W, H, frep);
        /* depth order at the representative view (Eq. 7), ties by index */
        int64_t n = 0;
        for (int64_t i = 0; i < M; ++i) {
            const int ok = mode == 1 ? frep[i].valid : prep[i].valid;
            if (!ok) continue;
            keys[n].d = mode == 1 ? (double)frep[i].depth : prep[i].depth;
            keys[n].i = i;
            ++n;
        }
        qsort(keys, (size_t)n, sizeof(dkey64), cmp_dkey64);
        for (int64_t e = 0; e < n; ++e) order[e] = keys[e].i;
        if (grads) {
            memset(dcon, 0, sizeof(double) * 3 * mm);
            memset(dcol, 0, sizeof(double) * 3 * mm);
            memset(dop, 0, sizeof(double) * mm);
        }
        for (int32_t j = 0; j < N; ++j) {
            if (!need[j]) continue;
            const p64 *pv = prep;
            const orc_proj *fv = frep;
            orc_cam cj;
            orc_load_cam(cams + 16 * (int64_t)j, W, H, &cj);
            if (j != r) {
                for (int64_t i = 0; i < M; ++i)
                    project64(means + 3 * i, log_scales + 3 * i, quats + 4 * i, opac[i], sh + (int64_t)nb * 3 * i,
                              nb, deg, &cj, pview + i);
                pv = pview;
                if (mode == 1) {
                    orc_project(M, deg, means, log_scales, quats, opac, sh, cams + 16 * (int64_t)j, W, H, fview);
                    fv = fview;
                }
            }
            if (grads) memset(dm2, 0, sizeof(double) * 2 * mm);
            for (int64_t s = 0; s < n_samples; ++s) {
                const int64_t p = samples[s];
                if (V[p] != j) continue;
                const int u = (int)(p % 3);
                const int64_t pix = p / 3;
                const double px = (double)(pix % W) + 0.5, py = (double)(pix / W) + 0.5;
                /* decisions, front to back */
                int64_t nl = 0;
                double Td = 1.0;
                uint64_t h = 0xCBF29CE484222325ull;
                for (int64_t e = 0; e < n; ++e) {
                    const int64_t i = order[e];
                    double alpha;
                    int clamped;
                    if (mode == 1) {
                        const orc_proj *g = frep + i, *mv = fv + i;
                        if (!mv->valid_mean) continue;
                        const double dx = px - (double)mv->mean2d[0], dy = py - (double)mv->mean2d[1];
                        const double w = dx + (double)g->conic[1] * dy;
                        const double E = (double)g->conic[0] * w * w + (double)g->conic[2] * dy * dy;
                        alpha = (double)g->opacity * exp2(-E);
                        clamped = alpha > ALPHA_MAX;
                        if (clamped) alpha = ALPHA_MAX;
                        if ((float)alpha < ALPHA_MIN) continue;
                        const double Tn = Td * (1.0 - alpha);
                        if ((float)Tn < T_STOP) break;
                        Td = Tn;
                    } else {
                        const p64 *g = prep + i, *mv = pv + i;
                        if (!mv->valid_mean) continue;
                        const double dx = px - mv->m2d[0], dy = py - mv->m2d[1];
                        const double w = dx + g->beta * dy;
                        const double E = g->A * w * w + g->G * dy * dy;
                        alpha = (double)opac[i] * exp2(-E);
                        clamped = alpha > ALPHA_MAX;
                        if (clamped) alpha = ALPHA_MAX;
                        if (alpha < (double)ALPHA_MIN) continue;
                        const double Tn = Td * (1.0 - alpha);
                        if (Tn < (double)T_STOP) break;
                        Td = Tn;
                    }
                    list[nl].i = i;
                    list[nl].clamped = clamped;
                    ++nl;
                    h = mix(h, (uint64_t)i * 8u + (uint64_t)clamped * 4u + (uint64_t)(prep[i].raw[u] > 0.0) * 2u
                                   + (uint64_t)(prep[i].clx || prep[i].cly));
                }
                h = mix(h, (uint64_t)nl);
                /* values in double on the blended list */
                double T = 1.0, C = 0.0;
                for (int64_t e = 0; e < nl; ++e) {
                    bent *b = list + e;
                    const p64 *g = prep + b->i, *mv = pv + b->i;
                    b->dx = px - mv->m2d[0];
                    b->dy = py - mv->m2d[1];
                    b->w = b->dx + g->beta * b->dy;
                    const double E = g->A * b->w * b->w + g->G * b->dy * b->dy;
                    b->ex = exp2(-E);
                    b->a = b->clamped ? ALPHA_MAX : (double)opac[b->i] * b->ex;
                    b->T = T;
                    C = C + g->color[u] * b->a * T;
                    T = T * (1.0 - b->a);
                }
                if (out) out[s] = C + T * (double)bg[u];
                if (sig) sig[s] = h;
                if (!grads || gout[s] == 0.0) continue;
                /* reverse pass over the blended list */
                const double gs = gout[s];
                double rest = T * (double)bg[u];
                for (int64_t e = nl - 1; e >= 0; --e) {
                    const bent *b = list + e;
                    const int64_t i = b->i;
                    const p64 *g = prep + i;
                    const double c = g->color[u];
                    dcol[3 * i + u] += gs * b->a * b->T;
                    const double da = gs * (c * b->T - rest / (1.0 - b->a));
                    rest += c * b->a * b->T;
                    if (b->clamped) continue;
                    dop[i] += da * b->ex;
                    const double dE = -da * (double)opac[i] * b->ex * LN2;
                    dcon[3 * i + 0] += dE * b->w * b->w;
                    dcon[3 * i + 1] += dE * 2.0 * g->A * b->w * b->dy;
                    dcon[3 * i + 2] += dE * b->dy * b->dy;
                    const double ddx = dE * 2.0 * g->A * b->w;
                    const double ddy = dE * (2.0 * g->A * b->w * g->beta + 2.0 * g->G * b->dy);
                    dm2[2 * i + 0] -= ddx;
                    dm2[2 * i + 1] -= ddy;
                }
            }
            if (grads)
                for (int64_t i = 0; i < M; ++i)
                    if (dm2[2 * i] != 0.0 || dm2[2 * i + 1] != 0.0) mean_backward(&cj, pv + i, dm2 + 2 * i, d_means + 3 * i);
        }
        if (!grads) continue;
        for (int64_t i = 0; i < M; ++i) {
            const double *dc = dcon + 3 * i, *dk = dcol + 3 * i;
            if (dc[0] == 0.0 && dc[1] == 0.0 && dc[2] == 0.0 && dk[0] == 0.0 && dk[1] == 0.0 && dk[2] == 0.0 &&
                dop[i] == 0.0)
                continue;
            d_opacities[i] += dop[i];
            full_backward(&cr, prep + i, sh + (int64_t)nb * 3 * i, nb, deg, dc, dk, d_means + 3 * i,
                          d_log_scales + 3 * i, d_quats + 4 * i, d_sh + (int64_t)nb * 3 * i);
        }
    }
    free(slots); free(rep); free(prep); free(pview); free(frep); free(fview); free(keys); free(order);
    free(list); free(dcon); free(dcol); free(dop); free(dm2); free(need);
    return 0;
}
