// Internal declarations shared by the liblfr HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "lfr.h"

namespace lfr {

// ---------------------------------------------------------------------------
// Method constants (paper section 4.3 Eq. 10 and the 3DGS conventions the
// paper inherits from gsplat).
// ---------------------------------------------------------------------------
constexpr float kAlphaMin = 1.0f / 255.0f;  // alpha cutoff
constexpr float kAlphaMax = 0.99f;          // alpha clamp
constexpr float kTStop = 1e-4f;             // transmittance stop
constexpr float kNearZ = 0.2f;              // near plane on the float32 depth
constexpr double kDilation = 0.3;           // 2D covariance dilation
constexpr double kClampFov = 1.3;           // Jacobian clamp (x tan(fov/2))
constexpr double kHalfLog2e = 0.5 * 1.44269504088896340736;
constexpr int kMaxClusterViews = 32;        // views unioned per cluster
constexpr int kMaxWaveViews = 4;            // distinct views in one blend wavefront
constexpr int kWave = 64;
// Stand-in for a 2D mean that is invalid in a view: far outside any panel,
// so E = +inf and alpha = 0 wherever it is evaluated, and no tile or row span
// contains it.
constexpr float kFarMean = 1e30f;

// Camera in double precision, with the derived clamp limits and centre.
struct DevCamera {
    double R[9];
    double t[3];
    double fx, fy, cx, cy;
    double limx, limy;
    double campos[3];
};

// Per (cluster, Gaussian) record, written by the projection and read by
// key generation and the blend: a = (A', beta, G', opacity), c = (r, g, b,
// cutoff exponent log2(255 o) + 0.01, beyond which alpha < 1/255), and m:
// for a cluster of at most kItemViews views the 2D mean in each of its views
// in view order (kFarMean where the mean is invalid and beyond the cluster's
// views), so that a blend lane's conic, colour and mean come from one cache
// line; for a larger cluster (whose blend reads the mean planes) m[0], m[1]
// are the smallest and largest x and y of the means of the views whose tile
// box is non-empty, for key generation.
constexpr int kItemViews = 4;
struct alignas(64) GaussRec {
    float4 a;
    float4 c;
    float2 m[kItemViews];
};
static_assert(sizeof(GaussRec) == 64, "GaussRec must be 64 bytes");

// Per-(cluster, Gaussian) gradient record of the reverse blend, the same
// layout as GaussRec: a = d(A', beta, G', opacity), c = d(r, g, b), unused.
struct GradRec {
    float4 a;
    float4 c;
};

// A blend work item: up to 64 subpixels of one tile that all belong to one
// cluster and to at most kMaxWaveViews distinct views, contiguous in Psi.
// Psi is sorted by view inside a tile, so the lanes of a task form at most
// kMaxWaveViews runs of one view each; the task records where each run
// starts and the compact mean slot of its view, so the blend needs neither
// the view map nor the slot table per lane.
struct alignas(16) Task {
    uint32_t tile;
    uint32_t cluster;      // compact cluster index
    uint32_t start;        // first position in Psi
    uint16_t count;        // 1..64
    uint16_t n_runs;       // distinct views, 1..kMaxWaveViews
    uint8_t run_start[4];  // first lane of run q; 64 for q >= n_runs
    uint16_t slot[4];      // compact mean slot of run q's view (0 for q >= n_runs)
    uint32_t frame;        // frame of a merged batch group (0 otherwise)
};
static_assert(sizeof(Task) == 32, "Task must be 32 bytes");

// Per-render cluster/view tables (device copies live in the context).
struct ViewTables {
    int n_clusters = 0;          // K'
    int n_views = 0;             // N' (views whose means are projected)
    std::vector<int32_t> cluster_rep;     // [K'] original view id of the representative
    std::vector<int32_t> cv_off;          // [K'+1] offsets into cv_list
    std::vector<int32_t> cv_list;         // compact view slots unioned per cluster
    std::vector<int32_t> view_ids;        // [N'] original view id per slot
    std::vector<int32_t> view_slot;       // [N] slot of view j (-1 if none)
    std::vector<int32_t> view_cluster;    // [N] compact cluster of view j (-1 if none)
};

// Per (display, cluster size, culling): blend work items and the number of
// subpixels of every (tile, cluster) list.
struct TaskSet {
    Task *d_tasks = nullptr;
    int n = 0;
    int32_t *d_view_cluster = nullptr;    // [N]
    uint32_t *d_tc_count = nullptr;       // [T << cluster_bits]
    int cluster_bits = 0;
    int xcd_shift = 4;                    // log2 of the blend's XCD task group (xcd_task)
};

// Stage timer: HIP events recorded on the working stream, summed per stage
// after the frame.
enum Stage {
    kStProject, kStDepthSort, kStKeygen, kStSort, kStRanges, kStBlend, kStScatter, kStTotal,
    kStBwdBlend, kStBwdProject, kStBwdTotal, kNumStages
};
struct Timer {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Span {
        int stage;
        size_t a, b;
    };
    std::vector<Span> spans;
    void reset(bool enable)
    {
        on = enable;
        used = 0;
        spans.clear();
    }
    size_t mark(hipStream_t s)
    {
        if (!on) return 0;
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) {
                on = false;
                return 0;
            }
            pool.push_back(e);
        }
        (void)hipEventRecord(pool[used], s);
        return used++;
    }
    void span(int stage, size_t a, size_t b)
    {
        if (on) spans.push_back(Span{stage, a, b});
    }
    // ms per stage; out[kNumStages]; the events must have completed
    void sum(float *out) const
    {
        for (int k = 0; k < kNumStages; ++k) out[k] = 0.f;
        for (const Span &sp : spans) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, pool[sp.a], pool[sp.b]) == hipSuccess) out[sp.stage] += ms;
            else (void)hipGetLastError();
        }
    }
    ~Timer()
    {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files).  All enqueue on `s`.
// ---------------------------------------------------------------------------
struct ViewMapParams {
    int32_t W, H, N;
    int64_t qa;   // Q           (multiplies 3x+u)
    int64_t qb;   // Q*3*tan     (multiplies y)
    int64_t qc;   // Q*K_offset
    int64_t P;    // Q*L_x
};
hipError_t launch_view_map(const ViewMapParams &p, uint16_t *V, hipStream_t s);
hipError_t launch_referenced_views(const uint16_t *V, int64_t n, uint32_t *mask, hipStream_t s);
hipError_t launch_remap(const uint16_t *V, int W, int H, int tw, int th, uint32_t *psi,
                        hipStream_t s);
hipError_t launch_task_count(const uint16_t *V, const uint32_t *psi, const int32_t *view_cluster,
                             int W, int H, int tw, int th, uint32_t *counts, hipStream_t s);
hipError_t launch_task_emit(const uint16_t *V, const uint32_t *psi, const int32_t *view_cluster,
                            const int32_t *view_slot, int W, int H, int tw, int th, const uint32_t *offsets,
                            Task *tasks, hipStream_t s);

struct SceneDev {
    int64_t M;
    int32_t deg;
    const float *means, *log_scales, *quats, *opac, *sh;
};
struct ProjectOut {
    GaussRec *rec;      // [K'][M]
    ushort4 *ibox;      // [K'][M]  the records' union tile boxes (read alone to skip saturated items)
    uint32_t *dkey;     // [K'][Mp] float32 depth bits, 0xFFFFFFFF if invalid or padding
    uint32_t *dval;     // [K'][Mp] Gaussian index; null: not written (a split depth order implies it)
    float2 *mean2d;     // [N'][M]  (kFarMean, kFarMean) if the mean is invalid; null: not written
    int64_t Mp;         // M rounded up to the sort's segment granule
};
struct TileGrid {
    int W, H;
    int tw_shift, th_shift;  // tile side = 1 << shift pixels
    const int32_t *cv_off;   // [K'+1] views of each cluster ...
    const int32_t *cv_list;  // ... as view slots
    const int32_t *cv_cam;   // camera (view id) of each cv_list entry
};
hipError_t launch_project(const SceneDev &sc, const DevCamera *cams, const TileGrid &tg,
                          int n_clusters, const int32_t *cluster_cam, const ProjectOut &out, hipStream_t s);
hipError_t launch_project_records(const SceneDev &sc, const DevCamera *cam, int W, int H,
                                  lfr_proj_record *out, hipStream_t s);

// Exclusive scan of uint32 -> uint32 with the 64-bit total written to *total.
size_t scan_temp_bytes(int64_t n);
hipError_t launch_exclusive_scan(const uint32_t *in, uint32_t *out, int64_t n, void *temp,
                                 uint64_t *total, hipStream_t s);

// Stable LSD radix sort on bits [b0, b1) in ceil((b1 - b0) / 8) passes of at
// most 8 bits each, the bits spread evenly; ping-pong between (k0, v0) and
// (k1, v1).  Returns in *result_in_alt whether the
// sorted data ended in (k1, v1).
size_t sort_temp_bytes(int64_t n);
// With a timer, every scatter launch is recorded as a kStScatter span.  With
// dn, the count is min(*dn, n) read on the device (n sizes the grid and temp).
// seg_len > 0: a segmented sort of n / seg_len independent segments of
// seg_len keys each (seg_len a multiple of sort_segment_granule()).
hipError_t radix_sort_u32(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n,
                          int b0, int b1, void *temp, bool *result_in_alt, hipStream_t s,
                          Timer *tm = nullptr, const uint64_t *dn = nullptr, int64_t seg_len = 0);
// seg_len > 0: a segmented sort of n / seg_len independent segments of
// seg_len keys each (seg_len a multiple of sort_segment_granule()).
hipError_t radix_sort_u64(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n,
                          int b0, int b1, void *temp, bool *result_in_alt, hipStream_t s, int64_t seg_len = 0,
                          Timer *tm = nullptr, const uint64_t *dn = nullptr);
int64_t sort_segment_granule();

// Split depth order (depth.hip): thresholds thr[k] (returned in *thr_out,
// inside temp) with at most R valid keys of cluster k's segment of dkey
// ([K'][Mp]) below them, and the keys below, in index order with their
// Gaussian index as value, copied into cluster k's segment of near_key /
// near_val ([K'][ncap], the rest of each segment invalid keys).  Mp and ncap
// are multiples of sort_segment_granule(), R <= ncap.
size_t split_temp_bytes(int n_clusters, int64_t Mp);
hipError_t launch_depth_split(const uint32_t *dkey, int n_clusters, int64_t Mp, int64_t R, int64_t ncap,
                              void *temp, uint32_t **thr_out, uint32_t *near_key, uint32_t *near_val,
                              hipStream_t s);

struct BinParams {
    int64_t M;
    int64_t Mp;               // stride of the per-cluster depth-sorted arrays
    int n_clusters;
    int W, H, tw_shift, th, TX, TY;  // tile width = 1 << tw_shift pixels
    int cluster_bits;
    const int32_t *cv_off;    // [K'+1]
    const int32_t *cv_list;   // compact view slots
    const uint32_t *alive;    // [K'][TY][alive_words] bit per (cluster, tile) list still needed
    int alive_words;          // 32-bit words per tile row
    const GaussRec *items;    // [K'][M] the projection's records
    const ushort4 *ibox;      // [K'][M] union tile box of each record
    const uint32_t *alive_total;  // unsaturated subpixels (planned frames exit early at 0), or null
    const uint32_t *alive_sat;    // [K'][TY+1][TX+1] summed-area table of alive lists, or null (all alive)
    const uint32_t *far_thr;      // [K'] depth-key thresholds of the far chunk (split depth order), or null
    const uint64_t *alive_mask;   // [K'][4] tile rows, columns 0..63, 64..127 with an alive list, or null
};
// Per wavefront of 64 items (K' * ceil(len / 64) of them): pair total wcnt
// and mask of the items with pairs wmask.  far: the far chunk of a split
// depth order (dkey_sorted is then the unsorted key array, dval_sorted
// unused, pair keys 64-bit).
hipError_t launch_chunk_count(const BinParams &bp, const uint32_t *dkey_sorted, const uint32_t *dval_sorted,
                              int64_t r0, int64_t len, uint32_t *wcnt, uint64_t *wmask, hipStream_t s,
                              bool far = false);
// wmask from the counting pass; woff: the exclusive scan of its wcnt.
hipError_t launch_chunk_emit(const BinParams &bp, const uint32_t *dkey_sorted, const uint32_t *dval_sorted,
                             int64_t r0, int64_t len, const uint64_t *wmask, const uint32_t *woff,
                             uint64_t n_pairs, void *pair_keys, uint32_t *pair_vals, hipStream_t s,
                             bool far = false);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
// With dP, the pair count is min(*dP, P) read on the device (P sizes the grid).
hipError_t launch_ranges(const uint32_t *keys, int64_t P, uint2 *ranges, hipStream_t s,
                         const uint64_t *dP = nullptr);
// The same for the far chunk's 64-bit keys (list in the upper half).
hipError_t launch_ranges_u64(const uint64_t *keys, int64_t P, uint2 *ranges, hipStream_t s,
                             const uint64_t *dP = nullptr);
hipError_t launch_copy_u32(uint32_t *dst, const uint32_t *src, int64_t n, hipStream_t s);
hipError_t launch_record_count(const uint64_t *src, uint64_t *dst, hipStream_t s);
hipError_t launch_alive_sat(const uint32_t *tc_alive, int n_clusters, int TX, int TY, int cluster_bits, uint32_t *sat,
                            hipStream_t s);
hipError_t launch_alive_bits(const uint32_t *tc_alive, int n_clusters, int TX, int TY, int words,
                             int cluster_bits, uint32_t *bits, hipStream_t s);
// Both: the alive bits and the summed-area table, in one launch where the
// table fits in LDS; then also, for grids of at most 64 tile rows and 128
// tile columns (alive_tables_have_masks), per cluster the masks of tile rows
// and tile columns holding an alive list (masks: [K'][4] u64).
bool alive_tables_have_masks(int TX, int TY);
hipError_t launch_alive_tables(const uint32_t *tc_alive, int n_clusters, int TX, int TY, int words,
                               int cluster_bits, uint32_t *bits, uint32_t *sat, uint64_t *masks, hipStream_t s);
hipError_t launch_tc_count(const uint16_t *V, const int32_t *view_cluster, int W, int H, int tw, int th,
                           int cluster_bits, uint32_t *counts, hipStream_t s);

struct BlendParams {
    int W, H, tw, th, TX;
    int64_t M;
    int cluster_bits;
    const uint16_t *V;
    const uint32_t *psi;
    const int32_t *view_slot;     // [N] compact mean slot of view j
    const int32_t *view_cluster;  // [N] compact cluster of view j
    const uint2 *ranges;
    const uint32_t *vals;         // sorted Gaussian indices
    const GaussRec *rec;          // [K'][M]
    const float2 *mean2d;         // [N'][M] (read for clusters of more than kItemViews views, and row-major)
    const int32_t *cv_off;        // [K'+1] first view slot of each cluster (slots are in view order)
    float bg[3];
    float *out;                   // [H][W][3]
    float *const *out_frames;     // merged batch group: output of each frame (null: out)
    int64_t n_sub;                // 3 W H: per-frame stride of the traversal state
    unsigned long long *work;     // [2] evals, blended (counting variant only)
    // resumable traversal over depth chunks
    float2 *state;                // per subpixel (T, C); saturated: T = 0 (remapped) or T < 0 (row-major)
    uint8_t *task_alive;          // per work item (remapped path)
    uint32_t *tc_alive;           // per (tile, cluster) list: unsaturated subpixels
    uint32_t *alive_total;        // unsaturated subpixels of the frame
    int first, last;              // first / last chunk of the frame
    // kept for the backward (single-chunk renders only; null otherwise):
    float *save_T;                // per subpixel: final transmittance
    uint32_t *save_end;           // per subpixel: 1 + position of its last blended pair (0: none)
};
hipError_t launch_blend_remap(const BlendParams &bp, const Task *tasks, int n_tasks, int xcd_shift,
                              hipStream_t s);

hipError_t launch_blend_rowmajor(const BlendParams &bp, hipStream_t s);

// Reverse blend over the remapped work items of a saved single-chunk render.
struct BwdParams {
    int W;
    int64_t M;
    int cluster_bits;
    const uint16_t *V;
    const uint32_t *psi;
    const int32_t *view_slot;     // [N] compact mean slot of view j
    const uint2 *ranges;
    const uint32_t *vals;
    const GaussRec *rec;          // [K'][M]
    const float2 *mean2d;         // [N'][M]
    const int32_t *cv_off;        // [K'+1] first view slot of each cluster
    float bg[3];
    const float *grad_out;        // [H][W][3] dL/dI
    const float *save_T;
    const uint32_t *save_end;
    GradRec *d_rec;               // [K'][M], zeroed by the caller
    float2 *d_mean2d;             // [N'][M], zeroed by the caller
};
hipError_t launch_blend_backward(const BwdParams &bp, const Task *tasks, int n_tasks, int xcd_shift, hipStream_t s);

// Projection backward: per Gaussian, the record gradients of every cluster
// and the mean gradients of every view -> parameter gradients.
struct SceneGrads {
    float *means, *log_scales, *quats, *opac, *sh;
};
hipError_t launch_project_backward(const SceneDev &sc, const DevCamera *cams, int n_clusters,
                                   const int32_t *cluster_cam, int n_views, const int32_t *view_cam,
                                   const GradRec *d_rec, const float2 *d_mean2d, const SceneGrads &out,
                                   hipStream_t s);

struct FullFrameParams {
    int W, H, tw, th, TX, TY;
    int64_t M;
    int n_views;                  // views in this batch
    int cluster_bits;
    const uint2 *ranges;
    const uint32_t *vals;
    const GaussRec *rec;          // [B][M]
    const float2 *mean2d;         // [B][M]
    float bg[3];
    float *images;                // [B][H][W][3]
};
hipError_t launch_blend_fullframe(const FullFrameParams &fp, hipStream_t s);
hipError_t launch_interlace(const uint16_t *V, int64_t n_sub, const int32_t *view_batch_slot,
                            const float *images, int64_t image_stride, float *out, hipStream_t s);

}  // namespace lfr
