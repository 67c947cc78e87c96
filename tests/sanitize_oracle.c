/*
 * Driver for the oracle's AddressSanitizer / UndefinedBehaviorSanitizer run
 * (tests/test_oracle_sanitizers.py builds it with gcc together with
 * oracle/lfr_oracle.c and oracle/lfr_oracle_grad.c).  It calls every oracle
 * entry point on a small seeded scene, single- and multi-threaded, with
 * ragged panels, degenerate Gaussians and near-threshold stacks, and checks
 * the results that must agree exactly (threads, ranges around the value).
 * Exit status 0 means every check held; the sanitizers abort on any fault.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/lfr_oracle.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

static double urand(void)   /* xorshift64*, uniform in [0, 1) */
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (double)((rng_state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

static void make_cam(float *c, double theta, double radius, int W, int H)
{
    double st = sin(theta), ct = cos(theta);
    double pos[3] = {radius * st, 0.0, radius - radius * ct};
    double R[9] = {ct, 0.0, st, 0.0, 1.0, 0.0, -st, 0.0, ct};
    for (int k = 0; k < 9; ++k) c[k] = (float)R[k];
    for (int a = 0; a < 3; ++a) c[9 + a] = (float)(-(R[3 * a] * pos[0] + R[3 * a + 1] * pos[1] + R[3 * a + 2] * pos[2]));
    c[12] = c[13] = (float)(0.5 * W / tan(0.5236));
    c[14] = 0.5f * (float)W;
    c[15] = 0.5f * (float)H;
}

#define CHECK(cond)                                                     \
    do {                                                                \
        if (!(cond)) {                                                  \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            return 1;                                                   \
        }                                                               \
    } while (0)

int main(void)
{
    const int W = 37, H = 23, N = 5, deg = 3, nb = 16;
    const int64_t M = 300;
    float *means = malloc(sizeof(float) * 3 * M), *ls = malloc(sizeof(float) * 3 * M);
    float *q = malloc(sizeof(float) * 4 * M), *op = malloc(sizeof(float) * M);
    float *sh = malloc(sizeof(float) * 3 * nb * M);
    for (int64_t i = 0; i < M; ++i) {
        means[3 * i] = (float)(urand() * 2 - 1);
        means[3 * i + 1] = (float)(urand() * 1.2 - 0.6);
        means[3 * i + 2] = (float)(2.5 + urand() * 3);
        for (int a = 0; a < 3; ++a) ls[3 * i + a] = (float)(-3.5 + urand() * 2.5);
        for (int a = 0; a < 4; ++a) q[4 * i + a] = (float)(urand() * 2 - 1);
        op[i] = (float)urand();
        for (int b = 0; b < 3 * nb; ++b) sh[3 * nb * i + b] = (float)(b < 3 ? urand() : 0.2 * (urand() - 0.5));
    }
    /* degenerate entries: behind the camera, zero quaternion, NaN, opaque stack */
    means[2] = -3.0f;
    q[4] = q[5] = q[6] = q[7] = 0.0f;
    means[6] = NAN;
    for (int i = 10; i < 16; ++i) {
        means[3 * i] = 0.0f;
        means[3 * i + 1] = 0.0f;
        means[3 * i + 2] = 3.0f + 0.01f * (float)i;
        op[i] = 0.999f;
        for (int a = 0; a < 3; ++a) ls[3 * i + a] = -0.7f;
    }
    op[20] = 1.0f / 255.0f;
    float cams[5 * 16];
    for (int j = 0; j < N; ++j) make_cam(cams + 16 * j, (-10.0 + 5.0 * j) * 3.14159265358979 / 180.0, 4.0, W, H);

    int32_t *V = malloc(sizeof(int32_t) * 3 * W * H);
    CHECK(orc_view_map(W, H, N, 1, 6, 5, 2, -1, 3, V) == 0);
    for (int s = 0; s < 3 * W * H; ++s) CHECK(V[s] >= 0 && V[s] < N);
    int32_t slots[16], rep[16];
    CHECK(orc_cluster_table(N, 2, slots, rep) == 3);
    uint32_t *psi = malloc(sizeof(uint32_t) * 3 * W * H);
    CHECK(orc_remap(W, H, 16, 8, V, psi) == 0);
    orc_proj *pr = malloc(sizeof(orc_proj) * M);
    orc_project(M, deg, means, ls, q, op, sh, cams + 32, W, H, pr);
    double Y[16], dir[3] = {0.6, 0.0, 0.8};
    orc_sh_basis(3, dir, Y);

    const int64_t n = 3 * (int64_t)W * H;
    int64_t *samples = malloc(sizeof(int64_t) * n);
    for (int64_t s = 0; s < n; ++s) samples[s] = s;
    float *out1 = malloc(sizeof(float) * n), *out3 = malloc(sizeof(float) * n);
    float *lo = malloc(sizeof(float) * n), *hi = malloc(sizeof(float) * n);
    int32_t *fl1 = malloc(sizeof(int32_t) * n), *fl3 = malloc(sizeof(int32_t) * n), *paths = malloc(sizeof(int32_t) * n);
    double *tf1 = malloc(sizeof(double) * n), *tf3 = malloc(sizeof(double) * n);
    const float bg[3] = {0.1f, 0.2f, 0.3f};
    for (int S = 1; S <= 3; ++S) {
        orc_set_threads(1);
        CHECK(orc_render_subpixels(M, deg, means, ls, q, op, sh, cams, N, V, W, H, S, bg, n, samples, out1, fl1, tf1) == 0);
        orc_set_threads(3);
        CHECK(orc_render_subpixels_ex(M, deg, means, ls, q, op, sh, cams, N, V, W, H, S, bg, n, samples, out3, fl3,
                                      tf3, lo, hi, paths) == 0);
        for (int64_t s = 0; s < n; ++s) {
            CHECK(out1[s] == out3[s] && fl1[s] == fl3[s] && tf1[s] == tf3[s]);
            CHECK(lo[s] <= out1[s] && out1[s] <= hi[s] && paths[s] != 0);
        }
    }
    float *img = malloc(sizeof(float) * n);
    int32_t *pfl = malloc(sizeof(int32_t) * W * H);
    double *ptf = malloc(sizeof(double) * W * H);
    orc_set_threads(4);
    orc_render_view(M, deg, means, ls, q, op, sh, cams + 16, W, H, bg, img, pfl, ptf);
    orc_set_threads(1);

    double *gout = malloc(sizeof(double) * n), *val = malloc(sizeof(double) * n);
    uint64_t *sig = malloc(sizeof(uint64_t) * n);
    double *dm = malloc(sizeof(double) * 3 * M), *dl = malloc(sizeof(double) * 3 * M), *dq = malloc(sizeof(double) * 4 * M);
    double *dop = malloc(sizeof(double) * M), *dsh = malloc(sizeof(double) * 3 * nb * M);
    for (int64_t s = 0; s < n; ++s) gout[s] = urand() - 0.5;
    for (int mode = 0; mode < 2; ++mode)
        for (int S = 1; S <= 2; ++S)
            CHECK(orc_grad_subpixels(M, deg, means, ls, q, op, sh, cams, N, V, W, H, S, bg, n, samples, gout, mode,
                                     val, sig, dm, dl, dq, dop, dsh) == 0);
    /* invalid arguments are refused */
    int64_t bad = n;
    CHECK(orc_render_subpixels(M, deg, means, ls, q, op, sh, cams, N, V, W, H, 1, bg, 1, &bad, out1, fl1, tf1) == -1);
    CHECK(orc_view_map(W, H, N, 1, 0, 5, 2, 0, 1, V) == -1);

    free(means); free(ls); free(q); free(op); free(sh); free(V); free(psi); free(pr); free(samples);
    free(out1); free(out3); free(lo); free(hi); free(fl1); free(fl3); free(paths); free(tf1); free(tf3);
    free(img); free(pfl); free(ptf); free(gout); free(val); free(sig); free(dm); free(dl); free(dq); free(dop);
    free(dsh);
    printf("sanitized oracle run ok\n");
    return 0;
}
