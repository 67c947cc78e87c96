/*
 * lfr_oracle.h -- CPU oracle for subpixel-level 3D Gaussian rasterization of
 * one interlaced light-field image (CoherentRaster, arXiv 2605.04509).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow reference written from
 * the paper's equations.  It runs single-threaded unless orc_set_threads
 * asks for more; its parallel loops split independent items (Gaussians,
 * subpixels, rows), each computed by the same operations, so the results
 * are bit-identical for any thread count.  It shares no code with the
 * HIP library.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the product path never does.
 *
 * Arithmetic is IEEE double precision.  The only float32 roundings are the
 * ones the method's data layout defines: every projected attribute (2D mean,
 * factored conic, depth, colour) is stored as float32, and the discrete
 * decisions of the blend (alpha cutoff, transmittance stop) and the depth
 * sort key are taken on float32 values, i.e. in the precision of the
 * rasterizer being checked.
 */
#ifndef LFR_ORACLE_H
#define LFR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One projected Gaussian for one view (48 bytes). */
typedef struct {
    float mean2d[2];  /* pixel coordinates of the projected mean (Eq. 5)      */
    float conic[3];   /* A', beta, G': E = A'(dx + beta dy)^2 + G' dy^2 and
                         alpha = o * 2^-E  (the factored inverse 2D covariance,
                         pre-scaled by log2(e)/2)                            */
    float depth;      /* camera-space z of the mean (sort key of Eq. 7)      */
    float color[3];   /* max(0, SH(dir) + 0.5) per channel                   */
    float opacity;    /* o (copied)                                          */
    int32_t valid;      /* usable for covariance / colour / depth             */
    int32_t valid_mean; /* mean usable (finite and in front of the near plane) */
} orc_proj;

/* Eq. 1-3: view index of every subpixel, exact rational arithmetic.
 * V is [H][W][3] row-major.  Returns 0, -1 for invalid arguments. */
int orc_view_map(int32_t W, int32_t H, int32_t N,
                 int64_t tan_num, int64_t tan_den,
                 int64_t pitch_num, int64_t pitch_den,
                 int64_t off_num, int64_t off_den, int32_t *V);

/* Appendix B.1: contiguous clusters of S views; the last one is padded with
 * view N-1; representative = local index floor(S/2).
 * slots is [K][S], rep is [K], K = ceil(N/S).  Returns K. */
int32_t orc_cluster_table(int32_t N, int32_t S, int32_t *slots, int32_t *rep);

/* Section 4.3, Eq. 8: per tile (row-major tile order), the in-panel
 * subpixels listed in row-major order (y, x, u) and stably sorted by V.
 * psi receives 3*W*H panel-linear indices (y*W + x)*3 + u. */
int orc_remap(int32_t W, int32_t H, int32_t tile_w, int32_t tile_h,
              const int32_t *V, uint32_t *psi);

/* Eq. 4-6: project M Gaussians for one camera.
 * cam: 16 floats = world->camera R (row-major 3x3), t (3), fx, fy, cx, cy.
 * Scene arrays: means [M,3], log_scales [M,3], quats [M,4] (w,x,y,z),
 * opacities [M], sh [M,(deg+1)^2,3]. */
void orc_project(int64_t M, int32_t sh_degree, const float *means,
                 const float *log_scales, const float *quats,
                 const float *opacities, const float *sh, const float *cam,
                 int32_t W, int32_t H, orc_proj *out);

/* Real spherical-harmonic basis (degree <= 3) at a unit direction. */
void orc_sh_basis(int32_t degree, const double dir[3], double *out);

/* Eq. 9-10 for a list of subpixels, under the reuse rule with cluster size S
 * (S = 1 is the exact subpixel path).  samples are panel-linear indices.
 * cams: [N][16].  V: the full [H][W][3] view map.  For every sample:
 *   out    the rendered value (C + T * bg),
 *   flags  bit 0: some alpha was within the float32 error bound of 1/255,
 *          bit 1: some T' was within the float32 error bound of 1e-4
 *          (bounds: a first-order error analysis of the float32 evaluation
 *          of Eq. 10 and of the transmittance product, times 4),
 *   tflag  the transmittance T just before the first flagged event (0 if none).
 * Returns 0, or -1 for invalid arguments. */
int orc_render_subpixels(int64_t M, int32_t sh_degree, const float *means,
                         const float *log_scales, const float *quats,
                         const float *opacities, const float *sh,
                         const float *cams, int32_t N, const int32_t *V,
                         int32_t W, int32_t H, int32_t S, const float *bg,
                         int64_t n_samples, const int64_t *samples,
                         float *out, int32_t *flags, double *tflag);

/* orc_render_subpixels plus, per sample, the range of values reachable when
 * every flagged decision may go either way: the walk follows both outcomes
 * of each near-threshold alpha-cutoff or stop decision (at most 64 leaves)
 * and returns lo/hi, the smallest and largest leaf value (lo == hi == out
 * when nothing is flagged), and paths, the number of leaves (negated when
 * the 64-leaf limit cut some branch off).  lo, hi, paths: all NULL or all
 * non-NULL. */
int orc_render_subpixels_ex(int64_t M, int32_t sh_degree, const float *means,
                            const float *log_scales, const float *quats,
                            const float *opacities, const float *sh,
                            const float *cams, int32_t N, const int32_t *V,
                            int32_t W, int32_t H, int32_t S, const float *bg,
                            int64_t n_samples, const int64_t *samples,
                            float *out, int32_t *flags, double *tflag,
                            float *lo, float *hi, int32_t *paths);

/* Host threads used by orc_project, orc_render_subpixels(_ex) and
 * orc_render_view (1..256; 1 by default). */
void orc_set_threads(int32_t n);
int32_t orc_get_threads(void);

/* Standard single-view 3DGS render of a full W x H RGB image (section 3.3),
 * with the same blend rule; img is [H][W][3].  flags/tflag per pixel as
 * above (may be NULL). */
void orc_render_view(int64_t M, int32_t sh_degree, const float *means,
                     const float *log_scales, const float *quats,
                     const float *opacities, const float *sh, const float *cam,
                     int32_t W, int32_t H, const float *bg, float *img,
                     int32_t *flags, double *tflag);

/* Gradient oracle (lfr_oracle_grad.c).  The renderer of orc_render_subpixels
 * evaluated in double precision with no float32 rounding of the projected
 * attributes, and the analytic derivative of F = sum_s gout[s] * I[s] with
 * respect to every scene parameter (chain rule through Eq. 9-10, the reuse
 * rule of section 4.2, Eq. 4-6).  mode 0: the discrete decisions (validity,
 * depth order, 1/255 cutoff, 1e-4 stop, 0.99 clamp) are taken on the double
 * values; mode 1: as orc_render_subpixels takes them (float32 attributes).
 *   out   (may be NULL) the double-precision value of every sample,
 *   sig   (may be NULL) a 64-bit hash of every sample's decisions,
 *   d_*   (NULL = values only) dF/d(parameter), [M,3] [M,3] [M,4] [M] [M,B,3],
 *         overwritten.
 * Returns 0, or -1 for invalid arguments. */
int orc_grad_subpixels(int64_t M, int32_t sh_degree, const float *means,
                       const float *log_scales, const float *quats,
                       const float *opacities, const float *sh,
                       const float *cams, int32_t N, const int32_t *V,
                       int32_t W, int32_t H, int32_t S, const float *bg,
                       int64_t n_samples, const int64_t *samples,
                       const double *gout, int32_t mode, double *out,
                       uint64_t *sig, double *d_means, double *d_log_scales,
                       double *d_quats, double *d_opacities, double *d_sh);

#ifdef __cplusplus
}
#endif
#endif
