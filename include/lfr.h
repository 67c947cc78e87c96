/*
 * lfr.h -- C ABI of liblfr, a subpixel-level 3D Gaussian rasterizer for
 * lenticular light-field displays on AMD Instinct MI355X (gfx950).
 *
 * It renders one interlaced light-field image I_LF (W x H x 3 subpixels)
 * from a 3D Gaussian scene and a set of N views, following CoherentRaster
 * (arXiv 2605.04509):
 *   - each subpixel (x, y, u) belongs to view j = V[x, y, u] given by the
 *     lenticular slant / pitch / offset map (section 3.1, Eq. 1-3);
 *   - views are grouped into contiguous clusters of S views; each Gaussian's
 *     2D mean is projected per view, its 2D covariance, depth and SH colour
 *     once per cluster at the cluster's representative view (section 4.2,
 *     Eq. 5-6, appendix B.1);
 *   - (Gaussian, tile, cluster) pairs are keyed by (tile, cluster, depth)
 *     and sorted into per-(tile, cluster) lists (Eq. 7, appendix B.2);
 *   - subpixels are processed in the view-sorted order Psi of each tile so
 *     that a wavefront walks one list (section 4.3, Eq. 8), and blended front
 *     to back with Eq. 9-10 (alpha cutoff 1/255, clamp 0.99, stop when the
 *     transmittance would fall below 1e-4).
 * Cluster size 1 is the exact subpixel path; its result equals rendering
 * every view at full resolution and interlacing (section 4.1), which
 * lfr_render_fullframe_interlace computes the plain way.
 *
 * Conventions for every entry point:
 *   - Pointers named *_device are HIP device pointers on the context's
 *     device; every other pointer is host memory.  Device buffers passed in
 *     are borrowed for the duration of the call only.
 *   - Work is enqueued on the context's stream.  Calls return after
 *     enqueueing, except where a host readback is needed (noted per call);
 *     device outputs are valid after the stream is synchronized.
 *   - All arguments are validated before any launch.  On error nothing is
 *     written to outputs, a message is kept in the context (lfr_last_error),
 *     and a negative lfr_status is returned.
 *   - A context is bound to one stream and is not thread safe; use one
 *     context per host thread.
 */
#ifndef LFR_H
#define LFR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lfr_status;
#define LFR_OK               0
#define LFR_ERR_INVALID_ARG (-1)  /* bad pointer, size or parameter           */
#define LFR_ERR_OUT_OF_MEMORY (-2)/* device allocation failed                 */
#define LFR_ERR_HIP         (-3)  /* a HIP runtime call or launch failed      */
#define LFR_ERR_CAPACITY    (-4)  /* workspace limit set by the caller exceeded */
#define LFR_ERR_UNSUPPORTED (-5)  /* valid but outside what the library handles */

typedef struct lfr_context lfr_context;  /* device, stream, workspace, stats, last error */
typedef struct lfr_display lfr_display;  /* view map V, remap LUT Psi, per-tile tables  */

/* An exact rational number; den > 0. */
typedef struct { int64_t num, den; } lfr_rational;

/* Display description (section 3.1).  width/height in pixels (>= 1; three
 * subpixels per pixel), num_views N in [1, 65535], tan_slant = tan(alpha),
 * pitch = L_x in subpixels (> 0), offset = K_offset in subpixels, tile size
 * in pixels (tile_w, tile_h in {8, 16, 32, 64, 128}, tile_w * tile_h <= 8192).
 * The tile shape changes only the amount of work, never the image. */
typedef struct {
    int32_t width, height, num_views;
    lfr_rational tan_slant, pitch, offset;
    int32_t tile_w, tile_h;
} lfr_display_desc;

/* Pinhole camera, OpenCV axes (x right, y down, z forward).  R is the
 * row-major world->camera rotation, t the translation: X_cam = R X + t.
 * Pixel (x, y) is sampled at (x + 0.5, y + 0.5). */
typedef struct { float R[9]; float t[3]; float fx, fy, cx, cy; } lfr_camera;

/* An inward-facing arc of views (see lfr_make_view_cone). */
typedef struct {
    float orbit_center[3]; float radius; float span_deg; float fov_x_deg;
    float rig_offset[3]; int32_t num_views, width, height;
} lfr_view_cone;

/* A 3D Gaussian scene (section 3.3), float32 device arrays, C-contiguous:
 * means [M,3], log_scales [M,3] (per-axis log std), quats [M,4] (w,x,y,z;
 * normalized internally), opacities [M] (in [0,1]), sh [M,(d+1)^2,3]
 * (band-major, RGB innermost, real SH with the Condon-Shortley phase).
 * sh_degree d in [0,3].  num_gaussians may be 0. */
typedef struct {
    int64_t num_gaussians;
    int32_t sh_degree;
    int32_t reserved;
    const float *means, *log_scales, *quats, *opacities, *sh;
} lfr_scene;

/* Render options. */
#define LFR_REMAP             1u  /* view-coherent thread order (section 4.3) */
#define LFR_CULL_UNREFERENCED 2u  /* skip views/clusters no subpixel uses     */
#define LFR_TIMING            4u  /* record per-stage times into lfr_stats    */
#define LFR_SAVE_FOR_BACKWARD 8u  /* keep what lfr_render_backward needs      */
#define LFR_COUNT_WORK       16u  /* count blend evaluations (slower variant)  */
typedef struct {
    int32_t cluster_size;   /* S >= 1; 1 = exact path, no reuse           */
    uint32_t flags;         /* LFR_* bits above                            */
    float background[3];    /* added as T_final * background per channel   */
    int32_t first_chunk;    /* depth ranks per cluster in the first chunk;
                               later chunks grow 4x; 0 = max(32768, M/64).
                               Changes only the amount of work, never the
                               image.                                       */
    int32_t fullframe_tile; /* lfr_render_fullframe_interlace only: square
                               tile side of the per-view rasterizer, one of
                               8, 16, 32 (0 = 16)                           */
} lfr_render_opts;

/* Counters and timings of the last render on a context. */
typedef struct {
    uint64_t pairs;            /* Gaussian-(tile, cluster) pairs sorted, all chunks */
    uint64_t workspace_bytes;  /* device workspace currently held              */
    int32_t clusters;          /* clusters rendered (K')                       */
    int32_t views;             /* views whose means were projected (N')        */
    int32_t tasks;             /* blend work items (wavefronts or tiles)       */
    int32_t chunks;            /* depth chunks binned and blended              */
    float ms_project, ms_depth_sort, ms_keygen, ms_sort, ms_ranges, ms_blend, ms_total;
    uint64_t evals;            /* (subpixel, Gaussian) alphas evaluated (LFR_COUNT_WORK) */
    uint64_t blended;          /* of those, contributions blended               */
    float ms_sort_scatter;     /* LFR_TIMING: scatter launches of the tile sort */
    int32_t sort_scatter_launches;
    int32_t blend_launches;    /* blend kernel launches (one per blended chunk) */
    /* lfr_render_backward (timed when the forward had LFR_TIMING) */
    float ms_bwd_blend;        /* reverse blend into per-(Gaussian, cluster/view) grads */
    float ms_bwd_project;      /* projection backward into per-Gaussian grads  */
    float ms_bwd_total;
    /* lfr_render_batch */
    int32_t batch_frames;      /* frames in the last batch                     */
    int32_t batch_unplanned;   /* of those, rendered with host synchronization (first use of a frame slot) */
    int32_t batch_graphs;      /* of those, replayed from a captured hipGraph  */
    int32_t batch_rerendered;  /* planned frames whose pairs exceeded the plan and were rendered again */
    int32_t batch_groups;      /* renders the batch ran (merged groups and single frames) */
    /* LFR_COUNT_WORK, remapped blend only */
    uint64_t wave_steps;       /* wavefront steps (one staged Gaussian for 64 lanes) */
    uint64_t wave_steps_live;  /* of those, steps where some lane's alpha passed the cutoff */
    /* id of the forward the context keeps for lfr_render_backward (unique
     * per LFR_SAVE_FOR_BACKWARD render on the context), 0 if none */
    uint64_t saved_forward;
} lfr_stats;

/* One projected Gaussian (48 bytes), as returned by lfr_project:
 * E = conic[0] (dx + conic[1] dy)^2 + conic[2] dy^2 is (log2 e)/2 times the
 * Mahalanobis form of the inverse 2D covariance (its LDL^T factors), and a
 * subpixel's alpha is opacity * 2^-E.  The mean of an invalid view is NaN. */
typedef struct {
    float mean2d[2]; float conic[3]; float depth; float color[3]; float opacity;
    int32_t valid; int32_t valid_mean;
} lfr_proj_record;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  *out receives the
 * context (caller owns it; free with lfr_context_destroy). */
lfr_status lfr_context_create(int32_t device, void *hip_stream, lfr_context **out);
void lfr_context_destroy(lfr_context *ctx);
/* Switch the stream subsequent calls enqueue on. */
lfr_status lfr_context_set_stream(lfr_context *ctx, void *hip_stream);
/* Cap the device workspace (bytes; 0 = no cap).  A render that would need
 * more returns LFR_ERR_CAPACITY and leaves the workspace as it was. */
lfr_status lfr_context_set_limit(lfr_context *ctx, uint64_t max_workspace_bytes);
/* Release the workspace (it is regrown on demand). */
lfr_status lfr_context_trim(lfr_context *ctx);
lfr_status lfr_get_stats(const lfr_context *ctx, lfr_stats *out);
/* Message of the last error on this context ("" if none).  Owned by ctx. */
const char *lfr_last_error(const lfr_context *ctx);

/* ---- display (section 3.1 Eq. 1-3, section 4.3 Eq. 8) ------------------- */

/* Build V (exact integer evaluation of Eq. 1-3) and the per-tile
 * view-sorted LUT Psi on the device.  Synchronizes the stream.  The display
 * is owned by the caller (lfr_display_destroy) and may be used with any
 * context on the same device. */
lfr_status lfr_display_create(lfr_context *ctx, const lfr_display_desc *desc, lfr_display **out);
/* Same, from an explicit host view map view_map[H][W][3] (values in [0,N)). */
lfr_status lfr_display_create_from_map(lfr_context *ctx, int32_t width, int32_t height,
                                       int32_t num_views, const int32_t *view_map,
                                       int32_t tile_w, int32_t tile_h, lfr_display **out);
void lfr_display_destroy(lfr_display *display);
/* Copy V to host (int32 [H][W][3]).  Synchronizes. */
lfr_status lfr_display_get_view_map(const lfr_display *display, int32_t *host_out);
/* Copy Psi to host: 3*W*H panel-linear subpixel indices (y*W + x)*3 + u,
 * tiles in row-major tile order, each tile's subpixels in row-major order
 * stably sorted by view.  Synchronizes. */
lfr_status lfr_display_get_remap(const lfr_display *display, uint32_t *host_out);
/* Number of views that own at least one subpixel, and their mask
 * (host uint8 [N], may be NULL).  Synchronizes on first use. */
lfr_status lfr_display_referenced_views(const lfr_display *display, int32_t *count,
                                        uint8_t *host_mask);

/* ---- cameras -------------------------------------------------------------- */

/* num_views cameras on an inward arc: view j at angle
 * theta_j = -span/2 + span*j/(N-1) sits at center + radius*(sin, 0, -cos)
 * + rig_offset, looks along (-sin, 0, cos); fx = fy = (W/2)/tan(fov_x/2),
 * cx = W/2, cy = H/2.  host_out receives num_views cameras. */
lfr_status lfr_make_view_cone(const lfr_view_cone *cone, lfr_camera *host_out);

/* ---- rendering -------------------------------------------------------------- */

/* Render the interlaced image (section 4, appendix B.2 algorithm) into
 * out_device (float32 [H][W][3], caller-owned).  host_cams holds the N views
 * (num_cams == N).  One host readback (the pair count) synchronizes the
 * stream mid-call. */
lfr_status lfr_render(lfr_context *ctx, const lfr_display *display, const lfr_scene *scene,
                      const lfr_camera *host_cams, int32_t num_cams,
                      const lfr_render_opts *opts, float *out_device);

/* The plain baseline: render every needed view at full W x H resolution with
 * the standard single-view tile rasterizer (section 3.3), view_batch views
 * per pass, then gather I_LF[y][x][u] = I_{V[y,x,u]}[y][x][u].  With
 * LFR_CULL_UNREFERENCED only the views V references are rendered, otherwise
 * all N.  cluster_size and LFR_REMAP are ignored. */
lfr_status lfr_render_fullframe_interlace(lfr_context *ctx, const lfr_display *display,
                                          const lfr_scene *scene, const lfr_camera *host_cams,
                                          int32_t num_cams, const lfr_render_opts *opts,
                                          int32_t view_batch, float *out_device);

/* Project every Gaussian of `scene` for one camera on a W x H image with the
 * device projection kernel (section 4.1 Eq. 4): out_device receives
 * num_gaussians lfr_proj_record entries (caller-owned device memory). */
lfr_status lfr_project(lfr_context *ctx, const lfr_scene *scene, const lfr_camera *host_cam,
                       int32_t width, int32_t height, lfr_proj_record *out_device);

/* ---- differentiation ---------------------------------------------------- */

/* Gradients with respect to the scene parameters: float32 device arrays with
 * the shapes of the lfr_scene arrays (means [M,3], log_scales [M,3], quats
 * [M,4], opacities [M], sh [M,(d+1)^2,3]).  Caller-owned; every element is
 * overwritten. */
typedef struct {
    float *means, *log_scales, *quats, *opacities, *sh;
} lfr_scene_grads;

/* Backward of the last lfr_render on this context, which must have been
 * called with LFR_SAVE_FOR_BACKWARD (and no other call that renders,
 * projects, sorts, tunes or trims on this context in between; otherwise
 * LFR_ERR_INVALID_ARG).  saved_forward: the lfr_stats.saved_forward id read
 * right after that render, or 0 for "whichever forward is kept"; a non-zero
 * id that is no longer kept (another saving render came in between) is
 * refused with LFR_ERR_INVALID_ARG, so a caller that keeps several
 * forwards alive (e.g. two differentiable renders in one loss) cannot get
 * the gradients of the wrong one.  The paper defines the forward only; the backward
 * is its exact derivative with the forward's discrete decisions held fixed
 * (which Gaussians pass the 1/255 cutoff, where the 1e-4 transmittance stop
 * falls, the 0.99 alpha clamp, the colour clamp at 0 and the Jacobian
 * clamp; derivatives through an active clamp are 0), under the same reuse
 * rule (section 4.2 Eq. 5-6: the 2D mean per view, covariance and colour per
 * cluster).
 *
 * grad_out_device: float32 [H][W][3], dL/dI for the rendered image.
 * display and scene: the ones the forward used (the same display object and
 * the same scene arrays, unchanged since; refused otherwise).  grads: written with dL/d(parameter); the quaternion gradient is
 * with respect to the unnormalized input.  Per-(Gaussian, cluster) and
 * per-(Gaussian, view) sums use float32 atomics, so results vary in the
 * last bits between runs.  With LFR_SAVE_FOR_BACKWARD the forward bins all
 * Gaussians in one depth chunk (same image) and keeps 8 bytes per subpixel
 * (final transmittance, end of its blended list) plus its sorted lists. */
lfr_status lfr_render_backward(lfr_context *ctx, uint64_t saved_forward, const lfr_display *display,
                               const lfr_scene *scene, const float *grad_out_device,
                               const lfr_scene_grads *grads);

/* ---- batched frames (serving) --------------------------------------------- */

/* One frame of a batch: what lfr_render takes. */
typedef struct {
    const lfr_display *display;
    const lfr_scene *scene;
    const lfr_camera *host_cams;   /* num_cams == the display's num_views     */
    int32_t num_cams;
    lfr_render_opts opts;          /* LFR_SAVE_FOR_BACKWARD, LFR_COUNT_WORK not allowed; LFR_TIMING ignored */
    float *out_device;             /* float32 [H][W][3] of this frame's display */
} lfr_frame;

#define LFR_BATCH_GRAPH       1u  /* replay frames from captured hipGraphs      */
#define LFR_BATCH_TIGHT_PLANS 2u  /* plan exactly the pairs seen (no headroom)  */
#define LFR_BATCH_NO_MERGE    4u  /* render every frame on its own              */

/* Render num_frames frames on the context stream, each exactly as lfr_render
 * would (same image).  Consecutive frames with the same display, scene
 * arrays and options (the remapped blend) are merged into one render, up to
 * 16 at a time and within a device-workspace budget (32 GB, or half the
 * context limit when one is set): their clusters are numbered frame-major,
 * so the frame index travels in the (tile, cluster) keys and in the blend's
 * work items, and every stage (projection, depth sort, key generation, tile
 * sort, ranges, blend) runs once per depth chunk for the whole group
 * instead of once per frame (LFR_BATCH_NO_MERGE renders every frame on its
 * own).  Group g uses batch slot g of the context.  The first time a slot
 * sees its group (or after any of its frames' display, scene arrays,
 * options or outputs change) the group is rendered with the synchronizing
 * path and its per-depth-chunk pair counts become the slot's plan (x 1.25 +
 * 4096 capacity, exact with LFR_BATCH_TIGHT_PLANS).  Planned groups run with
 * no host synchronization and no allocation: buffers are sized by the plan
 * and every kernel reads its counts on the device.  With LFR_BATCH_GRAPH
 * each planned slot is captured once into a hipGraph and replayed afterwards
 * (cameras may change between batches; they are uploaded for all frames in
 * one copy before the groups run).  The call synchronizes once at the end,
 * checks every planned group's pair counts against its plan, and renders
 * any group that exceeded it again (synchronously) with a new plan;
 * lfr_stats reports how many frames took each path and how many renders
 * (groups) ran.  Display, scene and output buffers of planned slots must
 * stay allocated while the context keeps the slots (they are rebuilt when
 * a pointer changes). */
lfr_status lfr_render_batch(lfr_context *ctx, const lfr_frame *frames, int32_t num_frames, uint32_t flags);

/* ---- autotuning ------------------------------------------------------------- */

typedef struct {
    int32_t tile_w, tile_h;   /* display tile shape                         */
    int32_t cluster_size;     /* S                                          */
    float ms;                 /* median render time over the timed repetitions */
    uint64_t pairs;           /* Gaussian-(tile, cluster) pairs of one render */
} lfr_tune_result;

/* Time lfr_render for every (tile shape, cluster size) candidate and pick the
 * fastest.  For each tile shape a temporary display is built from `desc`
 * (its tile fields are replaced); renders use `opts` with cluster_size
 * replaced; one untimed render precedes `reps` timed ones (HIP events on the
 * context stream).  tiles: n_tiles (w, h) pairs; sizes: n_sizes cluster
 * sizes.  out_device: H*W*3 float32 scratch image (caller-owned).
 * results (host, may be NULL) receives n_tiles * n_sizes entries in
 * tile-major order; best (host) the fastest.  Tile shape never changes the
 * image; cluster size does (it sets the reuse approximation), so callers
 * that need a fixed image pass a single size.  Synchronizes. */
lfr_status lfr_autotune(lfr_context *ctx, const lfr_display_desc *desc, const lfr_scene *scene,
                        const lfr_camera *host_cams, int32_t num_cams, const lfr_render_opts *opts,
                        const int32_t *tiles, int32_t n_tiles, const int32_t *sizes, int32_t n_sizes,
                        int32_t reps, float *out_device, lfr_tune_result *results, lfr_tune_result *best);

/* ---- device sort (used by the binning stage, exposed for testing) ---------- */

/* Stable LSD radix sort of (key, value) pairs in place on the device, on key
 * bits [begin_bit, end_bit).  keys_device: uint32 [n] (or uint64 [n] for the
 * _u64 variant), values_device: uint32 [n]. */
lfr_status lfr_sort_pairs_u32(lfr_context *ctx, uint32_t *keys_device, uint32_t *values_device,
                              int64_t n, int32_t begin_bit, int32_t end_bit);
lfr_status lfr_sort_pairs_u64(lfr_context *ctx, uint64_t *keys_device, uint32_t *values_device,
                              int64_t n, int32_t begin_bit, int32_t end_bit);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sort as lfr_sort_pairs_u32 (identical output), with uint32 keys only and
 * n <= 4,194,304 (2^22; larger n returns LFR_ERR_CAPACITY and enqueues
 * nothing).  Its ping-pong buffers and histograms live in a fixed 36 MiB
 * device array that the library holds on each GPU it runs on until the
 * process ends; the call makes no hipMalloc, hipFree or other allocating
 * call (the first call on a device looks the array's address up).  Every
 * call on one GPU shares that array, from any context: calls that may
 * overlap on one GPU (other streams, other threads) race and must be
 * serialized by the caller. */
lfr_status lfr_sort_pairs_u32_noalloc(lfr_context *ctx, uint32_t *keys_device, uint32_t *values_device,
                                      int64_t n, int32_t begin_bit, int32_t end_bit);

#ifdef __cplusplus
}
#endif
#endif /* LFR_H */
