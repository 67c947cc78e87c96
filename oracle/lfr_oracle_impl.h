/*
 * lfr_oracle_impl.h -- constants and camera helpers shared by the oracle's
 * translation units (lfr_oracle.c, lfr_oracle_grad.c).  TEST
 * INFRASTRUCTURE ONLY; not part of the HIP library.
 */
#ifndef LFR_ORACLE_IMPL_H
#define LFR_ORACLE_IMPL_H

#include <stdint.h>

#define ALPHA_MIN (1.0f / 255.0f)   /* alpha cutoff, decided in float32       */
#define T_STOP    1e-4f             /* transmittance stop, decided in float32 */
#define ALPHA_MAX 0.99              /* alpha clamp                            */
#define NEAR_Z    0.2f              /* near plane on the float32 depth        */
#define DILATION  0.3               /* added to the 2D covariance diagonal    */
#define CLAMP_FOV 1.3               /* Jacobian clamp, in units of tan(fov/2) */
#define U32 5.9604644775390625e-08  /* float32 unit roundoff 2^-24            */
#define HALF_LOG2E (0.5 * 1.44269504088896340736)

/* A pinhole camera in double precision. */
typedef struct {
    double R[9], t[3], fx, fy, cx, cy;
    double limx, limy;    /* Jacobian clamp on x/z and y/z */
    double campos[3];     /* camera centre = -R^T t        */
} orc_cam;

/* cam: 16 floats = world->camera R (row-major 3x3), t (3), fx, fy, cx, cy. */
void orc_load_cam(const float *c, int32_t W, int32_t H, orc_cam *o);
double orc_clampd(double v, double lo, double hi);

#endif
