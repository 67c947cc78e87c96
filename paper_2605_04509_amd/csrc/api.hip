// C ABI of liblfr: argument validation, workspace management and the stage
// sequence of the renderer (appendix B.2 algorithm), all enqueued on the
// context's stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <numeric>

#include "lfr_internal.h"

using namespace lfr;

// First depth chunk: max(kFirstChunk, M / kFirstChunkDiv) ranks per cluster;
// each following chunk is 4x longer.
constexpr int64_t kFirstChunk = 32768;
constexpr int64_t kFirstChunkDiv = 64;

namespace {

enum Slot {
    kRec, kDKey0, kDVal0, kDKey1, kDVal1, kMean2D, kCounts, kWaveMask, kOffsets, kScanTemp,
    kPairK0, kPairV0, kPairK1, kPairV1, kSortTemp, kRanges, kCams, kTables, kTotal, kImages, kBatchSlot,
    kWork, kAlive, kAliveBits, kState, kTaskAlive, kSaveT, kSaveEnd, kDRec, kDMean, kBatchTables, kBatchNeed,
    kAliveSat, kItemBox, kNearK0, kNearV0, kNearK1, kNearV1, kSplit, kFarK0, kFarK1, kAliveMask, kNumSlots
};

struct Buf {
    void *p = nullptr;
    size_t n = 0;
};

}  // namespace

// What lfr_render_backward needs from the last LFR_SAVE_FOR_BACKWARD render:
// pointers into the context workspace and the display's work items, valid
// until the next call that uses the workspace.
struct SavedForward {
    bool valid = false;
    uint64_t id = 0;                  // unique per saved forward on the context
    const void *display = nullptr;
    uint64_t display_uid = 0;
    lfr_scene scene{};                // the scene arrays the forward read
    int64_t M = 0;
    int deg = 0;
    bool timing = false;
    float bg[3] = {0.f, 0.f, 0.f};
    int n_clusters = 0, n_views = 0, cbits = 0;
    const DevCamera *cams = nullptr;
    const int32_t *cluster_cam = nullptr, *view_cam = nullptr, *view_slot = nullptr, *cv_off = nullptr;
    const GaussRec *rec = nullptr;
    const float2 *mean2d = nullptr;
    const uint2 *ranges = nullptr;
    const uint32_t *vals = nullptr;
    const Task *tasks = nullptr;
    int n_tasks = 0, xcd_shift = 4;
    const float *save_T = nullptr;
    const uint32_t *save_end = nullptr;
};

// A batch slot: the group of frames it was planned for (one frame, or frames
// merged into one render), its plan (pair capacity per depth chunk) and, with
// LFR_BATCH_GRAPH, the captured planned group.
struct FrameSlot {
    const void *display = nullptr;
    uint64_t display_uid = 0;
    lfr_scene scene{};
    lfr_render_opts opts{};
    std::vector<float *> outs;        // the group's frames' outputs
    bool tight = false;
    std::vector<uint64_t> caps;       // empty: not planned
    hipGraphExec_t graph = nullptr;
    uint64_t graph_gen = 0;           // workspace generation the graph was captured with
    size_t graph_table_off = 0;       // offset of the frame's tables it was captured with
};

struct lfr_context {
    int device = 0;
    hipStream_t stream = nullptr;
    uint64_t limit = 0;
    std::string err;
    lfr_stats stats{};
    Buf ws[kNumSlots];
    uint64_t ws_gen = 0;              // bumped whenever a workspace buffer moves
    bool capturing = false;           // a hipGraph capture is in progress: no allocation
    void *pinned = nullptr;
    size_t pinned_n = 0;
    void *batch_pinned = nullptr;     // staging of a batch's camera tables
    size_t batch_pinned_n = 0;
    hipStream_t cap_stream = nullptr; // non-blocking stream graphs are captured on
    std::vector<FrameSlot> slots;
    Timer timer;
    SavedForward saved;
    uint64_t next_saved_id = 1;
};

struct lfr_display {
    int device = 0;
    uint64_t uid = 0;                 // unique per display ever created
    int W = 0, H = 0, N = 0, tw = 0, th = 0, TX = 0, TY = 0, T = 0;
    uint16_t *d_V = nullptr;
    uint32_t *d_psi = nullptr;
    std::vector<uint8_t> ref;  // referenced-view mask
    int n_ref = 0;
    std::map<int64_t, TaskSet> tasks;
};

namespace {

lfr_status fail(lfr_context *ctx, lfr_status code, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

#define HIPCHK(ctx, expr)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail((ctx), LFR_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                       \
    } while (0)

#define CHK(expr)                    \
    do {                             \
        lfr_status s_ = (expr);      \
        if (s_ != LFR_OK) return s_; \
    } while (0)

uint64_t ws_total(const lfr_context *ctx)
{
    uint64_t t = 0;
    for (const Buf &b : ctx->ws) t += b.n;
    return t;
}

// Grow-only workspace slot.
lfr_status ws_get(lfr_context *ctx, Slot s, size_t bytes, void **out)
{
    Buf &b = ctx->ws[s];
    if (bytes == 0) bytes = 1;
    if (b.n < bytes) {
        if (ctx->capturing)
            return fail(ctx, LFR_ERR_CAPACITY, "workspace would grow during a graph capture");
        ++ctx->ws_gen;
        size_t want = bytes + bytes / 8 + 256;
        const uint64_t after = ws_total(ctx) - b.n + want;
        if (ctx->limit && after > ctx->limit) {
            want = bytes;
            if (ws_total(ctx) - b.n + want > ctx->limit)
                return fail(ctx, LFR_ERR_CAPACITY, "workspace limit %llu bytes exceeded (need %llu)",
                            (unsigned long long)ctx->limit, (unsigned long long)(ws_total(ctx) - b.n + want));
        }
        if (b.p) {
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
            HIPCHK(ctx, hipFree(b.p));
            b.p = nullptr;
            b.n = 0;
        }
        if (hipMalloc(&b.p, want) != hipSuccess) {
            (void)hipGetLastError();
            b.p = nullptr;
            return fail(ctx, LFR_ERR_OUT_OF_MEMORY, "hipMalloc of %llu bytes failed", (unsigned long long)want);
        }
        b.n = want;
    }
    *out = b.p;
    return LFR_OK;
}

template <typename T>
lfr_status ws_get_t(lfr_context *ctx, Slot s, size_t count, T **out)
{
    void *p = nullptr;
    CHK(ws_get(ctx, s, count * sizeof(T), &p));
    *out = (T *)p;
    return LFR_OK;
}

lfr_status pinned_get(lfr_context *ctx, size_t bytes, void **out)
{
    if (ctx->pinned_n < bytes) {
        if (ctx->pinned) {
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
            HIPCHK(ctx, hipHostFree(ctx->pinned));
            ctx->pinned = nullptr;
            ctx->pinned_n = 0;
        }
        const size_t want = std::max<size_t>(bytes, 1 << 16);
        HIPCHK(ctx, hipHostMalloc(&ctx->pinned, want, hipHostMallocDefault));
        ctx->pinned_n = want;
    }
    *out = ctx->pinned;
    return LFR_OK;
}

int bits_for(int64_t n)
{
    int b = 0;
    while (((int64_t)1 << b) < n) ++b;
    return b;
}

bool cam_ok(const lfr_camera &c)
{
    for (float v : c.R)
        if (!isfinite(v)) return false;
    for (float v : c.t)
        if (!isfinite(v)) return false;
    return isfinite(c.fx) && isfinite(c.fy) && isfinite(c.cx) && isfinite(c.cy) && c.fx > 0 && c.fy > 0;
}

DevCamera dev_camera(const lfr_camera &c, int W, int H)
{
    DevCamera d;
    for (int k = 0; k < 9; ++k) d.R[k] = c.R[k];
    for (int k = 0; k < 3; ++k) d.t[k] = c.t[k];
    d.fx = c.fx;
    d.fy = c.fy;
    d.cx = c.cx;
    d.cy = c.cy;
    d.limx = kClampFov * ((0.5 * (double)W) / d.fx);
    d.limy = kClampFov * ((0.5 * (double)H) / d.fy);
    for (int a = 0; a < 3; ++a)
        d.campos[a] = -((d.R[0 + a] * d.t[0] + d.R[3 + a] * d.t[1]) + d.R[6 + a] * d.t[2]);
    return d;
}

lfr_status check_scene(lfr_context *ctx, const lfr_scene *sc)
{
    if (!sc) return fail(ctx, LFR_ERR_INVALID_ARG, "scene is NULL");
    if (sc->num_gaussians < 0 || sc->num_gaussians > (int64_t)0x7FFFFFFF)
        return fail(ctx, LFR_ERR_INVALID_ARG, "num_gaussians %lld out of range", (long long)sc->num_gaussians);
    if (sc->sh_degree < 0 || sc->sh_degree > 3)
        return fail(ctx, LFR_ERR_INVALID_ARG, "sh_degree %d not in [0,3]", sc->sh_degree);
    if (sc->num_gaussians > 0 && (!sc->means || !sc->log_scales || !sc->quats || !sc->opacities || !sc->sh))
        return fail(ctx, LFR_ERR_INVALID_ARG, "scene array pointer is NULL");
    return LFR_OK;
}

SceneDev scene_dev(const lfr_scene *sc)
{
    return SceneDev{sc->num_gaussians, sc->sh_degree, sc->means, sc->log_scales, sc->quats, sc->opacities, sc->sh};
}

// Host tables of compact clusters / view slots for cluster size S.
ViewTables build_tables(const lfr_display *d, int S, bool cull)
{
    ViewTables vt;
    const int N = d->N;
    const int K = (N + S - 1) / S;
    vt.view_slot.assign(N, -1);
    vt.view_cluster.assign(N, -1);
    std::vector<int> slot_of(N, -1);
    // view slots: referenced views (cull) or all views
    for (int j = 0; j < N; ++j)
        if (!cull || d->ref[j]) {
            slot_of[j] = (int)vt.view_ids.size();
            vt.view_ids.push_back(j);
        }
    vt.cv_off.push_back(0);
    for (int k = 0; k < K; ++k) {
        std::vector<int> members;
        for (int l = 0; l < S; ++l) {
            const int j = std::min(k * S + l, N - 1);
            if (std::find(members.begin(), members.end(), j) == members.end()) members.push_back(j);
        }
        std::vector<int> used;
        for (int j : members)
            if (slot_of[j] >= 0) used.push_back(j);
        if (used.empty()) continue;
        const int c = (int)vt.cluster_rep.size();
        vt.cluster_rep.push_back(std::min(k * S + S / 2, N - 1));
        for (int j : used) vt.cv_list.push_back(slot_of[j]);
        vt.cv_off.push_back((int)vt.cv_list.size());
        for (int j : members) vt.view_cluster[j] = c;
    }
    for (int j = 0; j < N; ++j) vt.view_slot[j] = slot_of[j];
    vt.n_clusters = (int)vt.cluster_rep.size();
    vt.n_views = (int)vt.view_ids.size();
    return vt;
}

// The tables of F frames merged into one render (a batch group): frame f's
// view j is view f N + j, its view slot s is f N' + s and its cluster k is
// f K' + k.  Every stage then treats the group as one render with F K'
// clusters, and the cluster index carries the frame into the keys.
ViewTables merge_tables(const ViewTables &vt, int F, int N)
{
    if (F == 1) return vt;
    ViewTables g;
    const int K = vt.n_clusters, NV = vt.n_views;
    g.n_clusters = F * K;
    g.n_views = F * NV;
    g.cv_off.push_back(0);
    for (int f = 0; f < F; ++f) {
        for (int k = 0; k < K; ++k) {
            g.cluster_rep.push_back(f * N + vt.cluster_rep[k]);
            for (int e = vt.cv_off[k]; e < vt.cv_off[k + 1]; ++e) g.cv_list.push_back(f * NV + vt.cv_list[e]);
            g.cv_off.push_back((int)g.cv_list.size());
        }
        for (int v = 0; v < NV; ++v) g.view_ids.push_back(f * N + vt.view_ids[v]);
        for (int j = 0; j < N; ++j) {
            g.view_slot.push_back(vt.view_slot[j] < 0 ? -1 : f * NV + vt.view_slot[j]);
            g.view_cluster.push_back(vt.view_cluster[j] < 0 ? -1 : f * K + vt.view_cluster[j]);
        }
    }
    return g;
}

// Device copy of the small per-render tables, laid out in one buffer.
struct DevTables {
    DevCamera *cams = nullptr;
    int32_t *cluster_cam = nullptr, *view_cam = nullptr, *cv_off = nullptr, *cv_list = nullptr, *cv_cam = nullptr,
            *view_slot = nullptr, *view_cluster = nullptr;
    float **out_frames = nullptr;     // a batch group: the frames' outputs
};

// Bytes of the tables of vt (one frame or a merged group: vt.view_slot has
// one entry per view id) with room for `n_out` output pointers.
size_t tables_bytes(const ViewTables &vt, int n_out = 0)
{
    const size_t NT = vt.view_slot.size();
    const size_t n_int = vt.cluster_rep.size() + vt.view_ids.size() + vt.cv_off.size() + 2 * vt.cv_list.size() + 2 * NT;
    return sizeof(DevCamera) * NT + n_int * sizeof(int32_t) + (n_out > 0 ? 16 + sizeof(float *) * n_out : 0);
}

// Lay the tables out in host staging h for the device copy at dv.  cams[f]
// holds the N cameras of frame f of the group (F = vt's view ids / N); outs
// (n_out > 0) the frames' output pointers.
void write_tables(const lfr_display *d, const lfr_camera *const *cams, const ViewTables &vt, void *h, void *dv,
                  DevTables *out, float *const *outs = nullptr, int n_out = 0)
{
    const int N = d->N;
    const int NT = (int)vt.view_slot.size();
    const size_t cam_bytes = sizeof(DevCamera) * NT;
    DevCamera *hc = (DevCamera *)h;
    for (int g = 0; g < NT; ++g) hc[g] = dev_camera(cams[g / N][g % N], d->W, d->H);
    int32_t *hi = (int32_t *)((char *)h + cam_bytes);
    int32_t *di = (int32_t *)((char *)dv + cam_bytes);
    size_t o = 0;
    auto put = [&](const std::vector<int32_t> &v, int32_t **dst) {
        if (!v.empty()) memcpy(hi + o, v.data(), v.size() * sizeof(int32_t));
        *dst = di + o;
        o += v.size();
    };
    put(vt.cluster_rep, &out->cluster_cam);
    put(vt.view_ids, &out->view_cam);
    put(vt.cv_off, &out->cv_off);
    put(vt.cv_list, &out->cv_list);
    std::vector<int32_t> cv_cam(vt.cv_list.size());
    for (size_t e = 0; e < cv_cam.size(); ++e) cv_cam[e] = vt.view_ids[vt.cv_list[e]];
    put(cv_cam, &out->cv_cam);
    put(vt.view_slot, &out->view_slot);
    put(vt.view_cluster, &out->view_cluster);
    out->cams = (DevCamera *)dv;
    out->out_frames = nullptr;
    if (n_out > 0) {
        const size_t off = (cam_bytes + o * sizeof(int32_t) + 15) & ~(size_t)15;
        memcpy((char *)h + off, outs, sizeof(float *) * n_out);
        out->out_frames = (float **)((char *)dv + off);
    }
}

lfr_status upload_tables(lfr_context *ctx, const lfr_display *d, const lfr_camera *const *cams, const ViewTables &vt,
                         DevTables *out, float *const *outs = nullptr, int n_out = 0)
{
    const size_t bytes = tables_bytes(vt, n_out);
    void *h = nullptr, *dv = nullptr;
    CHK(pinned_get(ctx, bytes + 64, &h));
    CHK(ws_get(ctx, kTables, bytes + 64, &dv));
    write_tables(d, cams, vt, h, dv, out, outs, n_out);
    HIPCHK(ctx, hipMemcpyAsync(dv, h, bytes, hipMemcpyHostToDevice, ctx->stream));
    return LFR_OK;
}

// Project every Gaussian for the clusters and views of `vt`, then sort each
// cluster's Gaussians by depth (key = float32 depth bits, one sort segment
// per cluster).  With R > 0 the depth order is split (depth.hip): only the
// R nearest ranks of each cluster are sorted, the rest is the far chunk.
struct Projected {
    int64_t Mp = 0;             // stride of the unsorted per-cluster key segments (dkey)
    int64_t ns = 0;             // stride of the depth-sorted segments (dks, dvs)
    GaussRec *rec = nullptr;
    ushort4 *ibox = nullptr;
    float2 *mean2d = nullptr;
    const uint32_t *dkey = nullptr;  // unsorted depth keys [K'][Mp]
    const uint32_t *dks = nullptr;
    const uint32_t *dvs = nullptr;
    const uint32_t *thr = nullptr;   // split: [K'] far thresholds; else null
    int cbits = 0, tbits = 0;
};

// A tile grid over the W x H panel.
// (tile sides are powers of two, checked where displays and full-frame
// renders are set up, so a tile index is a shift of a pixel index)
struct Grid {
    int W, H, tw, th, TX, TY, T;
    int tw_shift, th_shift;
};
Grid make_grid(int W, int H, int tw, int th)
{
    Grid g{W, H, tw, th, (W + tw - 1) / tw, (H + th - 1) / th, 0, __builtin_ctz((unsigned)tw),
           __builtin_ctz((unsigned)th)};
    g.T = g.TX * g.TY;
    return g;
}
Grid grid_of(const lfr_display *d) { return make_grid(d->W, d->H, d->tw, d->th); }

lfr_status project_and_sort(lfr_context *ctx, const Grid &d_, const lfr_scene *scene, const DevTables &dt,
                            const ViewTables &vt, bool planes, int64_t R, Projected *out)
{
    const Grid *d = &d_;
    hipStream_t s = ctx->stream;
    Timer &tm = ctx->timer;
    const int64_t M = scene->num_gaussians;
    const int KC = vt.n_clusters, NV = vt.n_views;
    const int64_t MK = M * KC;
    const int cbits = bits_for(KC);
    const int tbits = bits_for(d->T);
    if (cbits + tbits > 32)
        return fail(ctx, LFR_ERR_UNSUPPORTED, "tile (%d bits) + cluster (%d bits) keys exceed 32 bits", tbits, cbits);
    if (MK > (int64_t)0xFFFFFFFFll)
        return fail(ctx, LFR_ERR_UNSUPPORTED, "Gaussians x clusters = %lld exceeds 2^32", (long long)MK);
    // depth keys: one segment of Mp >= M entries per cluster, padded to the
    // sort's granule, so the depth sort is a segmented sort on 32 bits
    const int64_t G = sort_segment_granule();
    const int64_t Mp = (M + G - 1) / G * G, MKp = Mp * KC;
    const bool split = R > 0;
    ProjectOut po;
    po.Mp = Mp;
    uint32_t *dkey1 = nullptr;
    uint32_t *dval1 = nullptr;
    void *sort_temp;
    CHK(ws_get_t(ctx, kRec, MK, &po.rec));
    CHK(ws_get_t(ctx, kItemBox, MK, &po.ibox));
    CHK(ws_get_t(ctx, kDKey0, MKp, &po.dkey));
    po.dval = nullptr;  // a split order needs no index array: items are read in index order
    if (!split) {
        CHK(ws_get_t(ctx, kDVal0, MKp, &po.dval));
        CHK(ws_get_t(ctx, kDKey1, MKp, &dkey1));
        CHK(ws_get_t(ctx, kDVal1, MKp, &dval1));
    }
    // (the per-view mean planes only when something reads them)
    po.mean2d = nullptr;
    if (planes) CHK(ws_get_t(ctx, kMean2D, std::max<int64_t>(M * NV, 1), &po.mean2d));
    CHK(ws_get(ctx, kSortTemp, sort_temp_bytes(MKp), &sort_temp));
    const size_t e0 = tm.mark(s);
    const TileGrid tg{d->W, d->H, d->tw_shift, d->th_shift, dt.cv_off, dt.cv_list, dt.cv_cam};
    HIPCHK(ctx, launch_project(scene_dev(scene), dt.cams, tg, KC, dt.cluster_cam, po, s));
    const size_t e1 = tm.mark(s);
    tm.span(kStProject, e0, e1);
    bool alt = false;
    out->thr = nullptr;
    if (!split) {
        HIPCHK(ctx, radix_sort_u32(po.dkey, po.dval, dkey1, dval1, MKp, 0, 32, sort_temp, &alt, s, nullptr, nullptr,
                                   Mp));
        out->dks = alt ? dkey1 : po.dkey;
        out->dvs = alt ? dval1 : po.dval;
        out->ns = Mp;
    } else {
        // the near set: at most R items per cluster, in segments of ns
        const int64_t ns = (std::min<int64_t>(R, M) + G - 1) / G * G, nKs = ns * KC;
        uint32_t *nk0, *nv0, *nk1, *nv1, *thr = nullptr;
        void *split_temp;
        CHK(ws_get_t(ctx, kNearK0, nKs, &nk0));
        CHK(ws_get_t(ctx, kNearV0, nKs, &nv0));
        CHK(ws_get_t(ctx, kNearK1, nKs, &nk1));
        CHK(ws_get_t(ctx, kNearV1, nKs, &nv1));
        CHK(ws_get(ctx, kSplit, split_temp_bytes(KC, Mp), &split_temp));
        HIPCHK(ctx, launch_depth_split(po.dkey, KC, Mp, std::min<int64_t>(R, M), ns, split_temp, &thr, nk0, nv0, s));
        HIPCHK(ctx, radix_sort_u32(nk0, nv0, nk1, nv1, nKs, 0, 32, sort_temp, &alt, s, nullptr, nullptr, ns));
        out->dks = alt ? nk1 : nk0;
        out->dvs = alt ? nv1 : nv0;
        out->ns = ns;
        out->thr = thr;
    }
    tm.span(kStDepthSort, e1, tm.mark(s));
    out->rec = po.rec;
    out->ibox = po.ibox;
    out->mean2d = po.mean2d;
    out->dkey = po.dkey;
    out->cbits = cbits;
    out->tbits = tbits;
    out->Mp = Mp;
    return LFR_OK;
}

BinParams bin_params(const Grid &d_, const DevTables &dt, const ViewTables &vt, int64_t M, int64_t Mp, int cbits,
                     const uint32_t *alive, const GaussRec *items, const ushort4 *ibox)
{
    const Grid *d = &d_;
    BinParams bp;
    bp.M = M;
    bp.Mp = Mp;
    bp.n_clusters = vt.n_clusters;
    bp.W = d->W;
    bp.H = d->H;
    bp.tw_shift = d->tw_shift;
    bp.th = d->th;
    bp.TX = d->TX;
    bp.TY = d->TY;
    bp.cluster_bits = cbits;
    bp.cv_off = dt.cv_off;
    bp.cv_list = dt.cv_list;
    bp.alive = alive;
    bp.alive_words = (d->TX + 31) / 32;
    bp.items = items;
    bp.ibox = ibox;
    bp.alive_total = nullptr;
    bp.alive_sat = nullptr;
    bp.far_thr = nullptr;
    bp.alive_mask = nullptr;
    return bp;
}

// Device-side totals: [0] pair count of the last scan (u64), [1] low word:
// unsaturated subpixels of the frame (u32).
struct Totals {
    uint64_t pairs;
    uint32_t alive;
    uint32_t pad;
};

// Start rank of the last depth chunk for M Gaussians and a first chunk of
// len0 ranks (each next chunk 4x longer); 0 when there is only one chunk.
int64_t last_chunk_start(int64_t M, int64_t len0)
{
    int64_t r0 = 0, len = len0;
    for (;;) {
        len = std::min(len, M - r0);
        if (r0 + len >= M) return r0;
        r0 += len;
        len *= 4;
    }
}

// One depth chunk: pair count -> scan -> (host readback) -> emit -> stable
// sort on the tile bits -> list ranges.  With cap > 0 (a planned frame) there
// is no readback: buffers hold cap pairs, the emit, sort and ranges kernels
// read the count from the device (clamped to cap), and the count is copied to
// *d_need for the host to check after the frame.
struct Chunk {
    uint64_t P = 0;        // pairs (unplanned chunks only)
    uint32_t alive = 0;    // unsaturated subpixels before the chunk (unplanned only)
    const uint32_t *vals = nullptr;
    uint2 *ranges = nullptr;
};

// far: the far chunk of a split depth order (items: every Gaussian in index
// order, len = M; 64-bit pair keys with the depth below the list key).
lfr_status bin_chunk(lfr_context *ctx, const BinParams &bp_in, const Projected &pr, int64_t r0, int64_t len,
                     Totals *d_tot, Chunk *out, uint64_t cap = 0, uint64_t *d_need = nullptr, bool far = false)
{
    BinParams bp = bp_in;
    if (far) {
        bp.Mp = pr.Mp;
        bp.far_thr = pr.thr;
    }
    const uint32_t *dk = far ? pr.dkey : pr.dks;
    hipStream_t s = ctx->stream;
    Timer &tm = ctx->timer;
    // per wavefront of 64 items: pair total, its exclusive scan, item mask
    const int64_t nw = (len + 63) / 64 * bp.n_clusters;
    uint32_t *wcnt, *woff;
    uint64_t *wmask;
    void *scan_temp;
    CHK(ws_get_t(ctx, kCounts, nw, &wcnt));
    CHK(ws_get_t(ctx, kOffsets, nw, &woff));
    CHK(ws_get_t(ctx, kWaveMask, nw, &wmask));
    CHK(ws_get(ctx, kScanTemp, scan_temp_bytes(nw), &scan_temp));
    const size_t e0 = tm.mark(s);
    HIPCHK(ctx, launch_chunk_count(bp, dk, pr.dvs, r0, len, wcnt, wmask, s, far));
    HIPCHK(ctx, launch_exclusive_scan(wcnt, woff, nw, scan_temp, &d_tot->pairs, s));
    uint64_t P = cap;
    const uint64_t *dP = nullptr;
    Totals ht{};
    if (cap > 0) {
        dP = &d_tot->pairs;
        if (d_need) HIPCHK(ctx, launch_record_count(dP, d_need, s));
    } else {
        void *h = nullptr;
        CHK(pinned_get(ctx, sizeof(Totals), &h));
        HIPCHK(ctx, hipMemcpyAsync(h, d_tot, sizeof(Totals), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        ht = *(const Totals *)h;
        if (ht.pairs >= 0xFFFFFFFFull)
            return fail(ctx, LFR_ERR_UNSUPPORTED, "%llu Gaussian-tile pairs in one chunk exceed 2^32",
                        (unsigned long long)ht.pairs);
        P = ht.pairs;
    }
    uint32_t *pk0 = nullptr, *pv0, *pk1 = nullptr, *pv1;
    uint64_t *fk0 = nullptr, *fk1 = nullptr;
    void *sort_temp;
    if (far) {
        CHK(ws_get_t(ctx, kFarK0, P, &fk0));
        CHK(ws_get_t(ctx, kFarK1, P, &fk1));
    } else {
        CHK(ws_get_t(ctx, kPairK0, P, &pk0));
        CHK(ws_get_t(ctx, kPairK1, P, &pk1));
    }
    CHK(ws_get_t(ctx, kPairV0, P, &pv0));
    CHK(ws_get_t(ctx, kPairV1, P, &pv1));
    CHK(ws_get(ctx, kSortTemp, sort_temp_bytes((int64_t)std::max<uint64_t>(P, (uint64_t)(pr.Mp * bp.n_clusters))),
               &sort_temp));
    HIPCHK(ctx, launch_chunk_emit(bp, dk, pr.dvs, r0, len, wmask, woff, P, far ? (void *)fk0 : (void *)pk0, pv0, s,
                                  far));
    const size_t e1 = tm.mark(s);
    tm.span(kStKeygen, e0, e1);
    bool palt = false;
    const int list_bits = bp.cluster_bits + bits_for((int64_t)bp.TX * bp.TY);
    if (far)
        HIPCHK(ctx, radix_sort_u64(fk0, pv0, fk1, pv1, (int64_t)P, 0, 32 + list_bits, sort_temp, &palt, s, 0, &tm,
                                   dP));
    else
        HIPCHK(ctx, radix_sort_u32(pk0, pv0, pk1, pv1, (int64_t)P, bp.cluster_bits, list_bits, sort_temp, &palt, s,
                                   &tm, dP));
    const size_t e2 = tm.mark(s);
    tm.span(kStSort, e1, e2);
    const int64_t n_ranges = ((int64_t)bp.TX * bp.TY) << bp.cluster_bits;
    uint2 *ranges;
    CHK(ws_get_t(ctx, kRanges, n_ranges, &ranges));
    HIPCHK(ctx, launch_fill_u32((uint32_t *)ranges, 0u, 2 * n_ranges, s));
    if (far)
        HIPCHK(ctx, launch_ranges_u64(palt ? fk1 : fk0, (int64_t)P, ranges, s, dP));
    else
        HIPCHK(ctx, launch_ranges(palt ? pk1 : pk0, (int64_t)P, ranges, s, dP));
    tm.span(kStRanges, e2, tm.mark(s));
    out->P = cap > 0 ? 0 : P;
    out->alive = ht.alive;
    out->vals = palt ? pv1 : pv0;
    out->ranges = ranges;
    return LFR_OK;
}

// Launch order of the blend work items: cluster by cluster, and inside a
// cluster by blocks of kTaskBlock x kTaskBlock tiles (row-major blocks,
// row-major tiles inside a block), so that the items that read the same
// Gaussians' records (one cluster, neighbouring tiles) run close together.
constexpr int kTaskBlock = 4;

lfr_status order_tasks(lfr_context *ctx, const lfr_display *d, Task *d_tasks, int n, std::vector<Task> *out)
{
    std::vector<Task> &h = *out;
    h.resize(n);
    if (n == 0) return LFR_OK;
    HIPCHK(ctx, hipMemcpy(h.data(), d_tasks, sizeof(Task) * n, hipMemcpyDeviceToHost));
    if (n == 1) return LFR_OK;
    const int nbx = (d->TX + kTaskBlock - 1) / kTaskBlock;
    auto key = [&](const Task &t) {
        const int ty = (int)t.tile / d->TX, tx = (int)t.tile % d->TX;
        const uint64_t blk = (uint64_t)(ty / kTaskBlock) * nbx + (uint64_t)(tx / kTaskBlock);
        const uint64_t in = (uint64_t)(ty % kTaskBlock) * kTaskBlock + (uint64_t)(tx % kTaskBlock);
        return ((uint64_t)t.cluster << 48) | (blk << 16) | in;
    };
    std::stable_sort(h.begin(), h.end(), [&](const Task &a, const Task &b) { return key(a) < key(b); });
    HIPCHK(ctx, hipMemcpy(d_tasks, h.data(), sizeof(Task) * n, hipMemcpyHostToDevice));
    return LFR_OK;
}

// Size of the blend's XCD task groups (log2): about the work items of one
// kTaskBlock x kTaskBlock block of tiles of one cluster (16 times the mean
// items per (tile, cluster) list, to the nearest power of two, 16 .. 512),
// so that the items reading the records of neighbouring tiles run on one
// XCD.  Measured on the outdoor frame (8 items per list: flat from 16 to
// 128) and the paper's display shapes (about 25 per list: the blend 10-17%
// faster at 512 than at 16).
int xcd_group_shift(const std::vector<Task> &h)
{
    if (h.empty()) return 4;
    int64_t lists = 1;
    for (size_t e = 1; e < h.size(); ++e)
        lists += (h[e].tile != h[e - 1].tile || h[e].cluster != h[e - 1].cluster) ? 1 : 0;
    const double g = (double)(kTaskBlock * kTaskBlock) * (double)h.size() / (double)lists;
    const int sh = (int)std::lround(std::log2(std::max(g, 1.0)));
    return std::min(9, std::max(4, sh));
}

// Blend work items and per-(tile, cluster) subpixel counts for cluster
// size S, built once per display.
lfr_status get_layout(lfr_context *ctx, lfr_display *d, int S, bool cull, const ViewTables &vt, TaskSet **out)
{
    const int64_t key = (int64_t)S * 2 + (cull ? 1 : 0);
    auto it = d->tasks.find(key);
    if (it != d->tasks.end()) {
        *out = &it->second;
        return LFR_OK;
    }
    hipStream_t s = ctx->stream;
    TaskSet ts;
    ts.cluster_bits = bits_for(vt.n_clusters);
    // device memory of this call: the temporaries are freed on every return,
    // the task set's arrays on an error return
    struct Guard {
        std::vector<void *> tmp, owned;
        bool keep = false;
        ~Guard()
        {
            for (void *p : tmp) (void)hipFree(p);
            if (!keep)
                for (void *p : owned) (void)hipFree(p);
        }
    } guard;
    auto dev_alloc = [&](void **p, size_t bytes, bool owned) -> hipError_t {
        const hipError_t e = hipMalloc(p, bytes);
        if (e == hipSuccess) (owned ? guard.owned : guard.tmp).push_back(*p);
        return e;
    };
    const int64_t n_tc = (int64_t)d->T << ts.cluster_bits;
    HIPCHK(ctx, dev_alloc((void **)&ts.d_view_cluster, sizeof(int32_t) * d->N, true));
    HIPCHK(ctx, hipMemcpy(ts.d_view_cluster, vt.view_cluster.data(), sizeof(int32_t) * d->N, hipMemcpyHostToDevice));
    HIPCHK(ctx, dev_alloc((void **)&ts.d_tc_count, sizeof(uint32_t) * n_tc, true));
    HIPCHK(ctx, launch_fill_u32(ts.d_tc_count, 0u, n_tc, s));
    HIPCHK(ctx, launch_tc_count(d->d_V, ts.d_view_cluster, d->W, d->H, d->tw, d->th, ts.cluster_bits,
                                ts.d_tc_count, s));
    uint32_t *cnt = nullptr, *off = nullptr;
    uint64_t *tot = nullptr;
    void *tmp = nullptr;
    HIPCHK(ctx, dev_alloc((void **)&cnt, sizeof(uint32_t) * d->T, false));
    HIPCHK(ctx, dev_alloc((void **)&off, sizeof(uint32_t) * d->T, false));
    HIPCHK(ctx, dev_alloc((void **)&tot, sizeof(uint64_t), false));
    HIPCHK(ctx, dev_alloc(&tmp, scan_temp_bytes(d->T), false));
    HIPCHK(ctx, launch_task_count(d->d_V, d->d_psi, ts.d_view_cluster, d->W, d->H, d->tw, d->th, cnt, s));
    HIPCHK(ctx, launch_exclusive_scan(cnt, off, d->T, tmp, tot, s));
    uint64_t n = 0;
    HIPCHK(ctx, hipMemcpyAsync(&n, tot, sizeof n, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    HIPCHK(ctx, dev_alloc((void **)&ts.d_tasks, sizeof(Task) * std::max<uint64_t>(n, 1), true));
    int32_t *vslot = nullptr;
    HIPCHK(ctx, dev_alloc((void **)&vslot, sizeof(int32_t) * d->N, false));
    HIPCHK(ctx, hipMemcpy(vslot, vt.view_slot.data(), sizeof(int32_t) * d->N, hipMemcpyHostToDevice));
    HIPCHK(ctx, launch_task_emit(d->d_V, d->d_psi, ts.d_view_cluster, vslot, d->W, d->H, d->tw, d->th, off,
                                 ts.d_tasks, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    ts.n = (int)n;
    std::vector<Task> h;
    CHK(order_tasks(ctx, d, ts.d_tasks, ts.n, &h));
    ts.xcd_shift = xcd_group_shift(h);
    guard.keep = true;
    auto ins = d->tasks.emplace(key, ts);
    *out = &ins.first->second;
    return LFR_OK;
}

// The work items and per-(tile, cluster) subpixel counts of F frames merged
// into one render (a batch group): F copies of the display's items with
// cluster f K' + k, mean slots f N' + s and the frame index, laid out frame
// after frame; counts under the group's cluster bits.  Built once per
// display, cluster size, culling and F.
lfr_status get_group_layout(lfr_context *ctx, lfr_display *d, int S, bool cull, const ViewTables &vt, int F,
                            TaskSet **out)
{
    TaskSet *base = nullptr;
    CHK(get_layout(ctx, d, S, cull, vt, &base));
    if (F == 1) {
        *out = base;
        return LFR_OK;
    }
    const int64_t key = ((int64_t)F << 32) | ((int64_t)S * 2 + (cull ? 1 : 0));
    auto it = d->tasks.find(key);
    if (it != d->tasks.end()) {
        *out = &it->second;
        return LFR_OK;
    }
    const int K = vt.n_clusters, NV = vt.n_views;
    const int cb1 = base->cluster_bits, cbg = bits_for((int64_t)F * K);
    std::vector<Task> h1(std::max(base->n, 1));
    std::vector<uint32_t> c1((size_t)d->T << cb1);
    if (base->n) HIPCHK(ctx, hipMemcpy(h1.data(), base->d_tasks, sizeof(Task) * base->n, hipMemcpyDeviceToHost));
    HIPCHK(ctx, hipMemcpy(c1.data(), base->d_tc_count, sizeof(uint32_t) * c1.size(), hipMemcpyDeviceToHost));
    std::vector<Task> hg((size_t)F * base->n);
    std::vector<uint32_t> cg((size_t)d->T << cbg, 0u);
    for (int f = 0; f < F; ++f) {
        for (int e = 0; e < base->n; ++e) {
            Task t = h1[e];
            t.cluster += (uint32_t)(f * K);
            for (int q = 0; q < (int)t.n_runs; ++q) t.slot[q] = (uint16_t)(t.slot[q] + f * NV);
            t.frame = (uint32_t)f;
            hg[(size_t)f * base->n + e] = t;
        }
        for (int64_t t = 0; t < d->T; ++t)
            for (int k = 0; k < K; ++k) cg[(size_t)(t << cbg) | (size_t)(f * K + k)] = c1[(size_t)(t << cb1) | k];
    }
    TaskSet ts;
    ts.cluster_bits = cbg;
    ts.n = F * base->n;
    ts.xcd_shift = base->xcd_shift;
    struct Guard {
        std::vector<void *> p;
        bool keep = false;
        ~Guard()
        {
            if (!keep)
                for (void *q : p) (void)hipFree(q);
        }
    } guard;
    HIPCHK(ctx, hipMalloc((void **)&ts.d_tasks, sizeof(Task) * std::max<size_t>(hg.size(), 1)));
    guard.p.push_back(ts.d_tasks);
    HIPCHK(ctx, hipMalloc((void **)&ts.d_tc_count, sizeof(uint32_t) * cg.size()));
    guard.p.push_back(ts.d_tc_count);
    if (!hg.empty()) HIPCHK(ctx, hipMemcpy(ts.d_tasks, hg.data(), sizeof(Task) * hg.size(), hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMemcpy(ts.d_tc_count, cg.data(), sizeof(uint32_t) * cg.size(), hipMemcpyHostToDevice));
    guard.keep = true;
    auto ins = d->tasks.emplace(key, ts);
    *out = &ins.first->second;
    return LFR_OK;
}

// Every entry point starts here.  Calls that use the workspace drop the
// saved forward (keep_saved = false).
lfr_status begin(lfr_context *ctx, bool keep_saved = false)
{
    if (!ctx) return LFR_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!keep_saved) ctx->saved.valid = false;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    return LFR_OK;
}

lfr_status check_render_args(lfr_context *ctx, const lfr_display *d, const lfr_scene *scene,
                             const lfr_camera *cams, int32_t num_cams, const lfr_render_opts *opts, const float *out)
{
    if (!d) return fail(ctx, LFR_ERR_INVALID_ARG, "display is NULL");
    if (d->device != ctx->device) return fail(ctx, LFR_ERR_INVALID_ARG, "display lives on another device");
    CHK(check_scene(ctx, scene));
    if (!cams) return fail(ctx, LFR_ERR_INVALID_ARG, "cameras are NULL");
    if (num_cams != d->N) return fail(ctx, LFR_ERR_INVALID_ARG, "num_cams %d != num_views %d", num_cams, d->N);
    for (int j = 0; j < num_cams; ++j)
        if (!cam_ok(cams[j])) return fail(ctx, LFR_ERR_INVALID_ARG, "camera %d is not finite or has f <= 0", j);
    if (!opts) return fail(ctx, LFR_ERR_INVALID_ARG, "opts is NULL");
    if (opts->cluster_size < 1) return fail(ctx, LFR_ERR_INVALID_ARG, "cluster_size must be >= 1");
    if (opts->first_chunk < 0) return fail(ctx, LFR_ERR_INVALID_ARG, "first_chunk must be >= 0");
    if (opts->fullframe_tile < 0) return fail(ctx, LFR_ERR_INVALID_ARG, "fullframe_tile must be >= 0");
    if (opts->cluster_size > kMaxClusterViews)
        return fail(ctx, LFR_ERR_UNSUPPORTED, "cluster_size %d > %d", opts->cluster_size, kMaxClusterViews);
    for (float b : opts->background)
        if (!isfinite(b)) return fail(ctx, LFR_ERR_INVALID_ARG, "background is not finite");
    if (!out) return fail(ctx, LFR_ERR_INVALID_ARG, "output is NULL");
    return LFR_OK;
}

lfr_status finish_timing(lfr_context *ctx)
{
    const Timer &tm = ctx->timer;
    if (!tm.on || tm.used == 0) return LFR_OK;
    HIPCHK(ctx, hipEventSynchronize(tm.pool[tm.used - 1]));
    float ms[kNumStages];
    tm.sum(ms);
    lfr_stats &st = ctx->stats;
    st.ms_project = ms[kStProject];
    st.ms_depth_sort = ms[kStDepthSort];
    st.ms_keygen = ms[kStKeygen];
    st.ms_sort = ms[kStSort];
    st.ms_ranges = ms[kStRanges];
    st.ms_blend = ms[kStBlend];
    st.ms_sort_scatter = ms[kStScatter];
    st.ms_total = ms[kStTotal];
    int n = 0;
    for (const auto &sp : tm.spans) n += sp.stage == kStScatter;
    st.sort_scatter_launches = n;
    return LFR_OK;
}

lfr_status finish_backward_timing(lfr_context *ctx)
{
    const Timer &tm = ctx->timer;
    if (!tm.on || tm.used == 0) return LFR_OK;
    HIPCHK(ctx, hipEventSynchronize(tm.pool[tm.used - 1]));
    float ms[kNumStages];
    tm.sum(ms);
    ctx->stats.ms_bwd_blend = ms[kStBwdBlend];
    ctx->stats.ms_bwd_project = ms[kStBwdProject];
    ctx->stats.ms_bwd_total = ms[kStBwdTotal];
    return LFR_OK;
}

// How render_frame runs one frame.
//  - tables: camera tables already on the device (batched frames upload all
//    frames' tables at once), else they are uploaded here;
//  - caps (planned frame): pair capacity of every depth chunk.  Nothing is
//    read back and nothing synchronizes; every chunk runs; each chunk's pair
//    count is recorded to d_need[chunk] for the caller to compare with caps
//    afterwards (a count above its cap means the frame must be re-rendered);
//  - chunk_pairs (unplanned frame): receives each chunk's pair count.
constexpr int kMaxPlannedChunks = 16;
constexpr uint64_t kUnplannedChunkCap = 1u << 16;
struct FrameRun {
    const DevTables *tables = nullptr;
    const std::vector<uint64_t> *caps = nullptr;
    uint64_t *d_need = nullptr;
    std::vector<uint64_t> *chunk_pairs = nullptr;
};

// F frames of the subpixel renderer (appendix B.2 algorithm) as one render:
// frames that share the display, the scene and the options and differ only
// in their cameras (cams[f], outs[f]).  With F > 1 the frames are merged:
// their clusters are numbered f K' + k (merge_tables), so one launch of each
// stage serves every frame.  F > 1 needs the remapped blend and neither
// saving nor counting.  Arguments are already validated.  `run` (may be
// null) selects how it runs: see FrameRun.
lfr_status render_group(lfr_context *ctx, const lfr_display *display, const lfr_scene *scene, int F,
                        const lfr_camera *const *cams, const lfr_render_opts *opts, float *const *outs,
                        const FrameRun *run)
{
    lfr_display *d = const_cast<lfr_display *>(display);
    const bool planned = run && run->caps;
    hipStream_t s = ctx->stream;
    const bool cull = (opts->flags & LFR_CULL_UNREFERENCED) != 0;
    const bool remap = (opts->flags & LFR_REMAP) != 0;
    const bool count = (opts->flags & LFR_COUNT_WORK) != 0;
    const bool save = (opts->flags & LFR_SAVE_FOR_BACKWARD) != 0;
    if (F < 1 || (F > 1 && (!remap || count || save)))
        return fail(ctx, LFR_ERR_INVALID_ARG, "merged frames need the remapped blend, without saving or counting");
    const int S = opts->cluster_size;
    const int64_t M = scene->num_gaussians;
    const int64_t nsub = 3ll * d->W * d->H, nsub_all = nsub * F;
    ctx->stats = lfr_stats{};
    Timer &tm = ctx->timer;
    const ViewTables vt1 = build_tables(d, S, cull);
    const ViewTables vt = merge_tables(vt1, F, d->N);
    // the records index a cluster's means by slot - cv_off[k]: view slots are
    // numbered in view order, cluster by cluster
    for (size_t e = 0; e < vt.cv_list.size(); ++e)
        if (vt.cv_list[e] != (int32_t)e) return fail(ctx, LFR_ERR_UNSUPPORTED, "view slots out of cluster order");
    TaskSet *ts = nullptr;
    CHK(get_group_layout(ctx, d, S, cull, vt1, F, &ts));
    tm.reset(!planned && (opts->flags & LFR_TIMING) != 0);
    const size_t t0 = tm.mark(s);
    DevTables dt;
    if (run && run->tables)
        dt = *run->tables;
    else
        CHK(upload_tables(ctx, d, cams, vt, &dt, outs, F > 1 ? F : 0));
    Projected pr;
    // the mean planes are read by the row-major blend and for clusters whose
    // means do not fit in the record
    bool planes = !remap;
    for (int k = 0; k < vt.n_clusters; ++k) planes = planes || vt.cv_off[k + 1] - vt.cv_off[k] > kItemViews;
    // depth chunks: ranks [r0, r0 + len) of every cluster, len growing 4x
    // from len0.  With more than one chunk and no lists to keep, the depth
    // order is split: only the ranks before the last chunk are sorted, and
    // the last chunk is the far set, binned in index order.
    const int64_t len0 = opts->first_chunk > 0
                             ? (int64_t)opts->first_chunk
                             : std::max<int64_t>(kFirstChunk, (M + kFirstChunkDiv - 1) / kFirstChunkDiv);
    const int64_t R = save ? 0 : last_chunk_start(M, len0);
    CHK(project_and_sort(ctx, grid_of(d), scene, dt, vt, planes, R, &pr));

    // traversal state: unsaturated subpixels per (tile, cluster) list and in
    // total, the lists' alive bits, per-subpixel (T, C), per-item flags
    const int words = (d->TX + 31) / 32;
    const int64_t n_tc = (int64_t)d->T << pr.cbits;
    uint32_t *tc_alive, *alive_bits;
    float2 *state;
    uint8_t *task_alive;
    Totals *d_tot;
    CHK(ws_get_t(ctx, kAlive, n_tc, &tc_alive));
    CHK(ws_get_t(ctx, kAliveBits, (int64_t)vt.n_clusters * d->TY * words, &alive_bits));
    CHK(ws_get_t(ctx, kState, nsub_all, &state));
    CHK(ws_get_t(ctx, kTaskAlive, (size_t)std::max(ts->n, 1) + 4, &task_alive));
    CHK(ws_get_t(ctx, kTotal, 1, &d_tot));
    // per-frame traversal state: every list and subpixel unsaturated
    auto reset_state = [&]() -> lfr_status {
        HIPCHK(ctx, launch_copy_u32(tc_alive, ts->d_tc_count, n_tc, s));
        HIPCHK(ctx, launch_fill_u32(&d_tot->alive, (uint32_t)nsub_all, 1, s));
        HIPCHK(ctx, launch_fill_u32((uint32_t *)task_alive, 0x01010101u, (std::max(ts->n, 1) + 3) / 4, s));
        HIPCHK(ctx, launch_alive_bits(tc_alive, vt.n_clusters, d->TX, d->TY, words, pr.cbits, alive_bits, s));
        return LFR_OK;
    };
    CHK(reset_state());
    uint32_t *alive_sat;
    uint64_t *alive_mask;
    CHK(ws_get_t(ctx, kAliveSat, (size_t)vt.n_clusters * (d->TY + 1) * (d->TX + 1) + 1, &alive_sat));
    CHK(ws_get_t(ctx, kAliveMask, (size_t)vt.n_clusters * 4, &alive_mask));

    BlendParams bp;
    bp.W = d->W;
    bp.H = d->H;
    bp.tw = d->tw;
    bp.th = d->th;
    bp.TX = d->TX;
    bp.M = M;
    bp.cluster_bits = pr.cbits;
    bp.V = d->d_V;
    bp.psi = d->d_psi;
    bp.view_slot = dt.view_slot;
    bp.view_cluster = dt.view_cluster;
    bp.rec = pr.rec;
    bp.mean2d = pr.mean2d;
    bp.cv_off = dt.cv_off;
    for (int k = 0; k < 3; ++k) bp.bg[k] = opts->background[k];
    bp.out = outs[0];
    bp.out_frames = F > 1 ? dt.out_frames : nullptr;
    bp.n_sub = nsub;
    bp.work = nullptr;
    bp.state = state;
    bp.task_alive = task_alive;
    bp.tc_alive = tc_alive;
    bp.alive_total = &d_tot->alive;
    if (count) {
        CHK(ws_get_t(ctx, kWork, 4, &bp.work));
        HIPCHK(ctx, launch_fill_u32((uint32_t *)bp.work, 0u, 8, s));
    }
    bp.save_T = nullptr;
    bp.save_end = nullptr;
    if (save) {
        CHK(ws_get_t(ctx, kSaveT, nsub, &bp.save_T));
        CHK(ws_get_t(ctx, kSaveEnd, nsub, &bp.save_end));
    }
    BinParams bin = bin_params(grid_of(d), dt, vt, M, pr.ns, pr.cbits, alive_bits, pr.rec, pr.ibox);
    if (planned) bin.alive_total = &d_tot->alive;


    // The backward needs each subpixel's whole list in one chunk: a render
    // that keeps its lists first tries the first chunk alone and keeps it if
    // every subpixel saturated there (the lists then hold every entry any
    // subpixel reached); otherwise it renders again with one chunk holding
    // every rank.
    int64_t r0 = 0, len = len0;
    Chunk saved_chunk;
    bool blend_ran = false;
    uint64_t pairs = 0;
    int chunks = 0;
    bool single = save && len0 >= M;  // saving with one chunk of every rank
    for (int c = 0;; ++c) {
        if (single && c == 0) len = std::max<int64_t>(M, 1);
        len = std::min(len, M - r0);
        const bool last = r0 + len >= M;
        // the far chunk: every Gaussian, in index order, beyond the thresholds
        const bool far = pr.thr && r0 >= R;
        const int64_t cr0 = far ? 0 : r0, clen = far ? M : len;
        Chunk ch;
        if (planned) {
            const uint64_t cap = c < (int)run->caps->size() ? (*run->caps)[c] : kUnplannedChunkCap;
            CHK(bin_chunk(ctx, bin, pr, cr0, clen, d_tot, &ch, std::max<uint64_t>(cap, 1),
                          run->d_need ? run->d_need + std::min(c, kMaxPlannedChunks - 1) : nullptr, far));
        } else {
            CHK(bin_chunk(ctx, bin, pr, cr0, clen, d_tot, &ch, 0, nullptr, far));
            if (run && run->chunk_pairs) run->chunk_pairs->push_back(ch.P);
        }
        saved_chunk = ch;
        // every subpixel saturated: all outputs written (a planned frame
        // runs every chunk; its kernels see the saturation on the device)
        if (!planned && blend_ran && ch.alive == 0) break;
        ++chunks;
        pairs += ch.P;
        if (planned || ch.P > 0 || last) {
            bp.ranges = ch.ranges;
            bp.vals = ch.vals;
            bp.first = blend_ran ? 0 : 1;
            bp.last = last ? 1 : 0;
            const size_t e0 = tm.mark(s);
            if (remap)
                HIPCHK(ctx, launch_blend_remap(bp, ts->d_tasks, ts->n, ts->xcd_shift, s));
            else
                HIPCHK(ctx, launch_blend_rowmajor(bp, s));
            const size_t e1 = tm.mark(s);
            tm.span(kStBlend, e0, e1);
            ++ctx->stats.blend_launches;
            if (!last) {
                HIPCHK(ctx, launch_alive_tables(tc_alive, vt.n_clusters, d->TX, d->TY, words, pr.cbits, alive_bits,
                                                alive_sat, alive_mask, s));
                bin.alive_sat = alive_sat;   // later chunks skip items whose tiles are all saturated
                bin.alive_mask = alive_tables_have_masks(d->TX, d->TY) ? alive_mask : nullptr;
                tm.span(kStRanges, e1, tm.mark(s));
            }
            blend_ran = true;
        }
        if (last) break;
        if (save && !single) {
            // after the first chunk: keep it if every subpixel saturated
            void *h = nullptr;
            CHK(pinned_get(ctx, sizeof(Totals), &h));
            HIPCHK(ctx, hipMemcpyAsync(h, d_tot, sizeof(Totals), hipMemcpyDeviceToHost, s));
            HIPCHK(ctx, hipStreamSynchronize(s));
            if (((const Totals *)h)->alive == 0) break;
            // not saturated: start again with one chunk of every rank
            single = true;
            CHK(reset_state());
            bin.alive_sat = nullptr;
            bin.alive_mask = nullptr;
            if (bp.work) HIPCHK(ctx, launch_fill_u32((uint32_t *)bp.work, 0u, 8, s));
            ctx->stats.blend_launches = 0;
            blend_ran = false;
            pairs = 0;
            chunks = 0;
            r0 = 0;
            c = -1;
            continue;
        }
        r0 += len;
        len *= 4;
    }
    tm.span(kStTotal, t0, tm.mark(s));
    if (save) {
        SavedForward &sv = ctx->saved;
        sv.id = ctx->next_saved_id++;
        sv.display = d;
        sv.display_uid = d->uid;
        sv.scene = *scene;
        sv.M = M;
        sv.deg = scene->sh_degree;
        sv.timing = (opts->flags & LFR_TIMING) != 0;
        for (int k = 0; k < 3; ++k) sv.bg[k] = opts->background[k];
        sv.n_clusters = vt.n_clusters;
        sv.n_views = vt.n_views;
        sv.cbits = pr.cbits;
        sv.cams = dt.cams;
        sv.cluster_cam = dt.cluster_cam;
        sv.view_cam = dt.view_cam;
        sv.view_slot = dt.view_slot;
        sv.rec = pr.rec;
        sv.mean2d = pr.mean2d;
        sv.cv_off = dt.cv_off;
        sv.ranges = saved_chunk.ranges;
        sv.vals = saved_chunk.vals;
        sv.tasks = ts->d_tasks;
        sv.n_tasks = ts->n;
        sv.xcd_shift = ts->xcd_shift;
        sv.save_T = bp.save_T;
        sv.save_end = bp.save_end;
        sv.valid = true;
    }
    ctx->stats.pairs = pairs;
    ctx->stats.chunks = chunks;  // blend_launches was counted in the loop
    ctx->stats.clusters = vt.n_clusters;
    ctx->stats.views = vt.n_views;
    ctx->stats.tasks = remap ? ts->n : d->T;
    ctx->stats.workspace_bytes = ws_total(ctx);
    if (planned) return LFR_OK;
    if (count) {
        unsigned long long w[4] = {0, 0, 0, 0};
        HIPCHK(ctx, hipMemcpyAsync(w, bp.work, sizeof w, hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        ctx->stats.evals = w[0];
        ctx->stats.blended = w[1];
        ctx->stats.wave_steps = w[2];
        ctx->stats.wave_steps_live = w[3];
    }
    return finish_timing(ctx);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

lfr_status lfr_context_create(int32_t device, void *hip_stream, lfr_context **out)
{
    if (!out) return LFR_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return LFR_ERR_INVALID_ARG;
    }
    if (hipSetDevice(device) != hipSuccess) return LFR_ERR_HIP;
    lfr_context *ctx = new lfr_context();
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    *out = ctx;
    return LFR_OK;
}

void lfr_context_destroy(lfr_context *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (FrameSlot &sl : ctx->slots)
        if (sl.graph) (void)hipGraphExecDestroy(sl.graph);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    for (Buf &b : ctx->ws)
        if (b.p) (void)hipFree(b.p);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->batch_pinned) (void)hipHostFree(ctx->batch_pinned);
    delete ctx;
}

lfr_status lfr_context_set_stream(lfr_context *ctx, void *hip_stream)
{
    if (!ctx) return LFR_ERR_INVALID_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return LFR_OK;
}

lfr_status lfr_context_set_limit(lfr_context *ctx, uint64_t max_workspace_bytes)
{
    if (!ctx) return LFR_ERR_INVALID_ARG;
    ctx->limit = max_workspace_bytes;
    return LFR_OK;
}

lfr_status lfr_context_trim(lfr_context *ctx)
{
    CHK(begin(ctx));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (Buf &b : ctx->ws) {
        if (b.p) HIPCHK(ctx, hipFree(b.p));
        b.p = nullptr;
        b.n = 0;
    }
    ++ctx->ws_gen;
    return LFR_OK;
}

lfr_status lfr_get_stats(const lfr_context *ctx, lfr_stats *out)
{
    if (!ctx || !out) return LFR_ERR_INVALID_ARG;
    *out = ctx->stats;
    out->workspace_bytes = ws_total(ctx);
    out->saved_forward = ctx->saved.valid ? ctx->saved.id : 0;
    return LFR_OK;
}

const char *lfr_last_error(const lfr_context *ctx) { return ctx ? ctx->err.c_str() : "context is NULL"; }

static lfr_status display_finish(lfr_context *ctx, lfr_display *d, lfr_display **out)
{
    hipStream_t s = ctx->stream;
    HIPCHK(ctx, hipMalloc(&d->d_psi, sizeof(uint32_t) * 3 * (size_t)d->W * d->H));
    HIPCHK(ctx, launch_remap(d->d_V, d->W, d->H, d->tw, d->th, d->d_psi, s));
    uint32_t *mask = nullptr;
    HIPCHK(ctx, hipMalloc(&mask, sizeof(uint32_t) * d->N));
    struct FreeMask {
        uint32_t *p;
        ~FreeMask() { (void)hipFree(p); }
    } free_mask{mask};  // on every return below
    HIPCHK(ctx, launch_fill_u32(mask, 0u, d->N, s));
    HIPCHK(ctx, launch_referenced_views(d->d_V, 3ll * d->W * d->H, mask, s));
    std::vector<uint32_t> hm(d->N);
    HIPCHK(ctx, hipMemcpyAsync(hm.data(), mask, sizeof(uint32_t) * d->N, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    d->ref.assign(d->N, 0);
    d->n_ref = 0;
    for (int j = 0; j < d->N; ++j)
        if (hm[j]) {
            d->ref[j] = 1;
            ++d->n_ref;
        }
    *out = d;
    return LFR_OK;
}

// Tile sides 8..128 (powers of two) with at most 8192 pixels per tile (the
// remap LUT sorts a tile's subpixels in up to 128 KB of LDS).
static bool tile_ok(int t) { return t == 8 || t == 16 || t == 32 || t == 64 || t == 128; }
static bool tile_shape_ok(int tw, int th) { return tile_ok(tw) && tile_ok(th) && tw * th <= 8192; }

static lfr_display *new_display(lfr_context *ctx, int W, int H, int N, int tw, int th)
{
    static std::atomic<uint64_t> next_uid{1};
    lfr_display *d = new lfr_display();
    d->device = ctx->device;
    d->uid = next_uid++;
    d->W = W;
    d->H = H;
    d->N = N;
    d->tw = tw;
    d->th = th;
    d->TX = (W + tw - 1) / tw;
    d->TY = (H + th - 1) / th;
    d->T = d->TX * d->TY;
    return d;
}

lfr_status lfr_display_create(lfr_context *ctx, const lfr_display_desc *desc, lfr_display **out)
{
    CHK(begin(ctx, true));
    if (!desc || !out) return fail(ctx, LFR_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    const lfr_display_desc &D = *desc;
    if (D.width < 1 || D.height < 1 || (int64_t)D.width * D.height > (int64_t)1 << 30)
        return fail(ctx, LFR_ERR_INVALID_ARG, "panel %d x %d out of range", D.width, D.height);
    if (D.num_views < 1 || D.num_views > 65535)
        return fail(ctx, LFR_ERR_INVALID_ARG, "num_views %d not in [1, 65535]", D.num_views);
    if (D.tan_slant.den <= 0 || D.pitch.den <= 0 || D.offset.den <= 0 || D.pitch.num <= 0)
        return fail(ctx, LFR_ERR_INVALID_ARG, "rational parameters need den > 0 and pitch > 0");
    if (!tile_shape_ok(D.tile_w, D.tile_h))
        return fail(ctx, LFR_ERR_INVALID_ARG, "tile %d x %d: sides must be 8, 16, 32, 64 or 128, area <= 8192",
                    D.tile_w, D.tile_h);
    if ((D.width + D.tile_w - 1) / D.tile_w > 65535 || (D.height + D.tile_h - 1) / D.tile_h > 65535)
        return fail(ctx, LFR_ERR_UNSUPPORTED, "more than 65535 tiles per panel row or column");
    // Exact-integer form of Eq. 1-3; every intermediate must fit in int64.
    typedef __int128 i128;
    auto g = [](i128 a, i128 b) {
        if (a < 0) a = -a;
        if (b < 0) b = -b;
        while (b) {
            i128 t = a % b;
            a = b;
            b = t;
        }
        return a;
    };
    i128 Q = D.tan_slant.den;
    Q = Q / g(Q, D.pitch.den) * D.pitch.den;
    Q = Q / g(Q, D.offset.den) * D.offset.den;
    const i128 lim = (i128)1 << 62;
    const i128 qa = Q, qb = Q * 3 * D.tan_slant.num / D.tan_slant.den, qc = (i128)D.offset.num * (Q / D.offset.den),
               P = (i128)D.pitch.num * (Q / D.pitch.den);
    const i128 absq = qb < 0 ? -qb : qb, absc = qc < 0 ? -qc : qc;
    const i128 maxD = (i128)3 * D.width * qa + (i128)D.height * absq + absc;
    if (Q > lim || maxD > lim || P > lim || P * D.num_views > lim)
        return fail(ctx, LFR_ERR_UNSUPPORTED, "lens parameters too large for 64-bit exact arithmetic");
    lfr_display *d = new_display(ctx, D.width, D.height, D.num_views, D.tile_w, D.tile_h);
    ViewMapParams vp{D.width, D.height, D.num_views, (int64_t)qa, (int64_t)qb, (int64_t)qc, (int64_t)P};
    lfr_status st = LFR_OK;
    if (hipMalloc(&d->d_V, sizeof(uint16_t) * 3 * (size_t)D.width * D.height) != hipSuccess) {
        st = fail(ctx, LFR_ERR_OUT_OF_MEMORY, "hipMalloc for the view map failed");
    } else if (launch_view_map(vp, d->d_V, ctx->stream) != hipSuccess) {
        st = fail(ctx, LFR_ERR_HIP, "view map launch failed");
    } else {
        st = display_finish(ctx, d, out);
    }
    if (st != LFR_OK) lfr_display_destroy(d);
    return st;
}

lfr_status lfr_display_create_from_map(lfr_context *ctx, int32_t W, int32_t H, int32_t N, const int32_t *view_map,
                                       int32_t tw, int32_t th, lfr_display **out)
{
    CHK(begin(ctx, true));
    if (!view_map || !out) return fail(ctx, LFR_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (W < 1 || H < 1 || (int64_t)W * H > (int64_t)1 << 30 || N < 1 || N > 65535)
        return fail(ctx, LFR_ERR_INVALID_ARG, "bad panel or view count");
    if (!tile_shape_ok(tw, th))
        return fail(ctx, LFR_ERR_INVALID_ARG, "tile sides must be 8, 16, 32, 64 or 128, area <= 8192");
    if ((W + tw - 1) / tw > 65535 || (H + th - 1) / th > 65535)
        return fail(ctx, LFR_ERR_UNSUPPORTED, "more than 65535 tiles per panel row or column");
    const size_t n = 3 * (size_t)W * H;
    std::vector<uint16_t> v16(n);
    for (size_t s = 0; s < n; ++s) {
        if (view_map[s] < 0 || view_map[s] >= N)
            return fail(ctx, LFR_ERR_INVALID_ARG, "view_map[%zu] = %d not in [0, %d)", s, view_map[s], N);
        v16[s] = (uint16_t)view_map[s];
    }
    lfr_display *d = new_display(ctx, W, H, N, tw, th);
    lfr_status st = LFR_OK;
    if (hipMalloc(&d->d_V, sizeof(uint16_t) * n) != hipSuccess) {
        st = fail(ctx, LFR_ERR_OUT_OF_MEMORY, "hipMalloc for the view map failed");
    } else if (hipMemcpy(d->d_V, v16.data(), sizeof(uint16_t) * n, hipMemcpyHostToDevice) != hipSuccess) {
        st = fail(ctx, LFR_ERR_HIP, "view map upload failed");
    } else {
        st = display_finish(ctx, d, out);
    }
    if (st != LFR_OK) lfr_display_destroy(d);
    return st;
}

void lfr_display_destroy(lfr_display *d)
{
    if (!d) return;
    (void)hipSetDevice(d->device);
    (void)hipDeviceSynchronize();
    if (d->d_V) (void)hipFree(d->d_V);
    if (d->d_psi) (void)hipFree(d->d_psi);
    for (auto &kv : d->tasks) {
        if (kv.second.d_tasks) (void)hipFree(kv.second.d_tasks);
        if (kv.second.d_view_cluster) (void)hipFree(kv.second.d_view_cluster);
        if (kv.second.d_tc_count) (void)hipFree(kv.second.d_tc_count);
    }
    delete d;
}

lfr_status lfr_display_get_view_map(const lfr_display *d, int32_t *host_out)
{
    if (!d || !host_out) return LFR_ERR_INVALID_ARG;
    if (hipSetDevice(d->device) != hipSuccess) return LFR_ERR_HIP;
    const size_t n = 3 * (size_t)d->W * d->H;
    std::vector<uint16_t> v(n);
    if (hipDeviceSynchronize() != hipSuccess) return LFR_ERR_HIP;
    if (hipMemcpy(v.data(), d->d_V, n * sizeof(uint16_t), hipMemcpyDeviceToHost) != hipSuccess) return LFR_ERR_HIP;
    for (size_t s = 0; s < n; ++s) host_out[s] = v[s];
    return LFR_OK;
}

lfr_status lfr_display_get_remap(const lfr_display *d, uint32_t *host_out)
{
    if (!d || !host_out) return LFR_ERR_INVALID_ARG;
    if (hipSetDevice(d->device) != hipSuccess) return LFR_ERR_HIP;
    if (hipDeviceSynchronize() != hipSuccess) return LFR_ERR_HIP;
    const size_t n = 3 * (size_t)d->W * d->H;
    if (hipMemcpy(host_out, d->d_psi, n * sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess) return LFR_ERR_HIP;
    return LFR_OK;
}

lfr_status lfr_display_referenced_views(const lfr_display *d, int32_t *count, uint8_t *host_mask)
{
    if (!d) return LFR_ERR_INVALID_ARG;
    if (count) *count = d->n_ref;
    if (host_mask) memcpy(host_mask, d->ref.data(), d->N);
    return LFR_OK;
}

lfr_status lfr_make_view_cone(const lfr_view_cone *c, lfr_camera *out)
{
    if (!c || !out || c->num_views < 1 || c->width < 1 || c->height < 1 || !(c->fov_x_deg > 0) ||
        !(c->fov_x_deg < 180))
        return LFR_ERR_INVALID_ARG;
    const double pi = 3.14159265358979323846;
    const double f = (0.5 * c->width) / tan(c->fov_x_deg * pi / 180.0 * 0.5);
    for (int j = 0; j < c->num_views; ++j) {
        double th = 0.0;
        if (c->num_views > 1)
            th = (-0.5 * c->span_deg + c->span_deg * (double)j / (double)(c->num_views - 1)) * pi / 180.0;
        const double st = sin(th), ct = cos(th);
        const double pos[3] = {c->orbit_center[0] + c->radius * st + c->rig_offset[0],
                               c->orbit_center[1] + c->rig_offset[1],
                               c->orbit_center[2] - c->radius * ct + c->rig_offset[2]};
        const double R[9] = {ct, 0.0, st, 0.0, 1.0, 0.0, -st, 0.0, ct};
        lfr_camera &o = out[j];
        for (int k = 0; k < 9; ++k) o.R[k] = (float)R[k];
        for (int a = 0; a < 3; ++a) o.t[a] = (float)(-(R[3 * a] * pos[0] + R[3 * a + 1] * pos[1] + R[3 * a + 2] * pos[2]));
        o.fx = o.fy = (float)f;
        o.cx = (float)(0.5 * c->width);
        o.cy = (float)(0.5 * c->height);
    }
    return LFR_OK;
}

lfr_status lfr_render(lfr_context *ctx, const lfr_display *display, const lfr_scene *scene,
                      const lfr_camera *host_cams, int32_t num_cams, const lfr_render_opts *opts, float *out_device)
{
    CHK(begin(ctx));
    CHK(check_render_args(ctx, display, scene, host_cams, num_cams, opts, out_device));
    return render_group(ctx, display, scene, 1, &host_cams, opts, &out_device, nullptr);
}

lfr_status lfr_render_backward(lfr_context *ctx, uint64_t saved_forward, const lfr_display *display,
                               const lfr_scene *scene, const float *grad_out_device, const lfr_scene_grads *grads)
{
    CHK(begin(ctx, true));
    const SavedForward &sv = ctx->saved;
    if (!sv.valid)
        return fail(ctx, LFR_ERR_INVALID_ARG,
                    "no saved forward: call lfr_render with LFR_SAVE_FOR_BACKWARD first (and nothing that uses "
                    "this context's workspace in between)");
    if (saved_forward != 0 && saved_forward != sv.id)
        return fail(ctx, LFR_ERR_INVALID_ARG,
                    "saved forward %llu is no longer kept (the context now keeps forward %llu): a later render "
                    "replaced it", (unsigned long long)saved_forward, (unsigned long long)sv.id);
    if (!display || (const void *)display != sv.display || display->uid != sv.display_uid)
        return fail(ctx, LFR_ERR_INVALID_ARG, "display differs from the saved forward's");
    CHK(check_scene(ctx, scene));
    if (scene->num_gaussians != sv.M || scene->sh_degree != sv.deg)
        return fail(ctx, LFR_ERR_INVALID_ARG, "scene (M %lld, degree %d) differs from the saved forward's (M %lld, "
                    "degree %d)", (long long)scene->num_gaussians, scene->sh_degree, (long long)sv.M, sv.deg);
    if (scene->means != sv.scene.means || scene->log_scales != sv.scene.log_scales ||
        scene->quats != sv.scene.quats || scene->opacities != sv.scene.opacities || scene->sh != sv.scene.sh)
        return fail(ctx, LFR_ERR_INVALID_ARG, "scene arrays differ from the ones the saved forward read");
    if (!grad_out_device) return fail(ctx, LFR_ERR_INVALID_ARG, "grad_out is NULL");
    if (!grads) return fail(ctx, LFR_ERR_INVALID_ARG, "grads is NULL");
    const int64_t M = sv.M;
    if (M > 0 && (!grads->means || !grads->log_scales || !grads->quats || !grads->opacities || !grads->sh))
        return fail(ctx, LFR_ERR_INVALID_ARG, "a gradient array pointer is NULL");
    hipStream_t s = ctx->stream;
    GradRec *d_rec;
    float2 *d_mean;
    CHK(ws_get_t(ctx, kDRec, (size_t)std::max<int64_t>(M * sv.n_clusters, 1), &d_rec));
    CHK(ws_get_t(ctx, kDMean, (size_t)std::max<int64_t>(M * sv.n_views, 1), &d_mean));
    Timer &tm = ctx->timer;
    tm.reset(sv.timing);
    const size_t t0 = tm.mark(s);
    HIPCHK(ctx, launch_fill_u32((uint32_t *)d_rec, 0u, M * sv.n_clusters * 8, s));
    HIPCHK(ctx, launch_fill_u32((uint32_t *)d_mean, 0u, M * sv.n_views * 2, s));
    BwdParams bp;
    bp.W = display->W;
    bp.M = M;
    bp.cluster_bits = sv.cbits;
    bp.V = display->d_V;
    bp.psi = display->d_psi;
    bp.view_slot = sv.view_slot;
    bp.ranges = sv.ranges;
    bp.vals = sv.vals;
    bp.rec = sv.rec;
    bp.mean2d = sv.mean2d;
    bp.cv_off = sv.cv_off;
    for (int k = 0; k < 3; ++k) bp.bg[k] = sv.bg[k];
    bp.grad_out = grad_out_device;
    bp.save_T = sv.save_T;
    bp.save_end = sv.save_end;
    bp.d_rec = d_rec;
    bp.d_mean2d = d_mean;
    const size_t e0 = tm.mark(s);
    if (M > 0 && sv.ranges) HIPCHK(ctx, launch_blend_backward(bp, sv.tasks, sv.n_tasks, sv.xcd_shift, s));
    const size_t e1 = tm.mark(s);
    tm.span(kStBwdBlend, e0, e1);
    SceneGrads sg{grads->means, grads->log_scales, grads->quats, grads->opacities, grads->sh};
    HIPCHK(ctx, launch_project_backward(scene_dev(scene), sv.cams, sv.n_clusters, sv.cluster_cam, sv.n_views,
                                        sv.view_cam, d_rec, d_mean, sg, s));
    const size_t e2 = tm.mark(s);
    tm.span(kStBwdProject, e1, e2);
    tm.span(kStBwdTotal, t0, e2);
    ctx->stats.ms_bwd_blend = ctx->stats.ms_bwd_project = ctx->stats.ms_bwd_total = 0.0f;
    return finish_backward_timing(ctx);
}

lfr_status lfr_render_fullframe_interlace(lfr_context *ctx, const lfr_display *display, const lfr_scene *scene,
                                          const lfr_camera *host_cams, int32_t num_cams,
                                          const lfr_render_opts *opts, int32_t view_batch, float *out_device)
{
    CHK(begin(ctx));
    CHK(check_render_args(ctx, display, scene, host_cams, num_cams, opts, out_device));
    if (view_batch < 1) return fail(ctx, LFR_ERR_INVALID_ARG, "view_batch must be >= 1");
    if (opts->flags & LFR_SAVE_FOR_BACKWARD)
        return fail(ctx, LFR_ERR_INVALID_ARG, "LFR_SAVE_FOR_BACKWARD applies to lfr_render only");
    const int ft = opts->fullframe_tile ? opts->fullframe_tile : 16;
    if (ft != 8 && ft != 16 && ft != 32)
        return fail(ctx, LFR_ERR_INVALID_ARG, "fullframe_tile must be 8, 16 or 32");
    const Grid fg = make_grid(display->W, display->H, ft, ft);
    lfr_display *d = const_cast<lfr_display *>(display);
    hipStream_t s = ctx->stream;
    const bool cull = (opts->flags & LFR_CULL_UNREFERENCED) != 0;
    const int64_t M = scene->num_gaussians;
    ctx->stats = lfr_stats{};
    Timer &tm = ctx->timer;
    tm.reset((opts->flags & LFR_TIMING) != 0);
    std::vector<int> views;
    for (int j = 0; j < d->N; ++j)
        if (!cull || d->ref[j]) views.push_back(j);
    const int64_t nsub = 3ll * d->W * d->H;
    const int words = (fg.TX + 31) / 32;
    const size_t t0 = tm.mark(s);
    uint64_t pairs = 0;
    for (size_t b0 = 0; b0 < views.size(); b0 += (size_t)view_batch) {
        const int B = (int)std::min<size_t>((size_t)view_batch, views.size() - b0);
        // every view of the batch is its own "cluster" (S = 1) and view slot
        ViewTables vt;
        vt.n_clusters = vt.n_views = B;
        vt.view_slot.assign(d->N, -1);
        vt.view_cluster.assign(d->N, -1);
        vt.cv_off.push_back(0);
        for (int b = 0; b < B; ++b) {
            const int j = views[b0 + b];
            vt.cluster_rep.push_back(j);
            vt.view_ids.push_back(j);
            vt.cv_list.push_back(b);
            vt.cv_off.push_back(b + 1);
            vt.view_slot[j] = b;
            vt.view_cluster[j] = b;
        }
        DevTables dt;
        CHK(upload_tables(ctx, d, &host_cams, vt, &dt));
        Projected pr;
        CHK(project_and_sort(ctx, fg, scene, dt, vt, true, 0, &pr));
        // one chunk with every tile of every view alive
        uint32_t *alive_bits;
        Totals *d_tot;
        CHK(ws_get_t(ctx, kAliveBits, (int64_t)B * fg.TY * words, &alive_bits));
        CHK(ws_get_t(ctx, kTotal, 1, &d_tot));
        HIPCHK(ctx, launch_fill_u32(alive_bits, 0xFFFFFFFFu, (int64_t)B * fg.TY * words, s));
        const BinParams bin = bin_params(fg, dt, vt, M, pr.ns, pr.cbits, alive_bits, pr.rec, pr.ibox);
        Chunk ch;
        CHK(bin_chunk(ctx, bin, pr, 0, M, d_tot, &ch));
        pairs += ch.P;
        float *images;
        CHK(ws_get_t(ctx, kImages, (size_t)B * nsub, &images));
        FullFrameParams fp;
        fp.W = d->W;
        fp.H = d->H;
        fp.tw = fg.tw;
        fp.th = fg.th;
        fp.TX = fg.TX;
        fp.TY = fg.TY;
        fp.M = M;
        fp.n_views = B;
        fp.cluster_bits = pr.cbits;
        fp.ranges = ch.ranges;
        fp.vals = ch.vals;
        fp.rec = pr.rec;
        fp.mean2d = pr.mean2d;
        for (int k = 0; k < 3; ++k) fp.bg[k] = opts->background[k];
        fp.images = images;
        const size_t e0 = tm.mark(s);
        HIPCHK(ctx, launch_blend_fullframe(fp, s));
        HIPCHK(ctx, launch_interlace(d->d_V, nsub, dt.view_slot, images, nsub, out_device, s));
        tm.span(kStBlend, e0, tm.mark(s));
    }
    tm.span(kStTotal, t0, tm.mark(s));
    ctx->stats.pairs = pairs;
    ctx->stats.chunks = 1;
    ctx->stats.views = (int)views.size();
    ctx->stats.clusters = (int)views.size();
    ctx->stats.workspace_bytes = ws_total(ctx);
    return finish_timing(ctx);
}

lfr_status lfr_autotune(lfr_context *ctx, const lfr_display_desc *desc, const lfr_scene *scene,
                        const lfr_camera *host_cams, int32_t num_cams, const lfr_render_opts *opts,
                        const int32_t *tiles, int32_t n_tiles, const int32_t *sizes, int32_t n_sizes, int32_t reps,
                        float *out_device, lfr_tune_result *results, lfr_tune_result *best)
{
    CHK(begin(ctx));
    if (!desc || !opts || !tiles || !sizes || !best || n_tiles < 1 || n_sizes < 1 || reps < 1 || reps > 1000)
        return fail(ctx, LFR_ERR_INVALID_ARG, "bad autotune arguments");
    for (int a = 0; a < n_tiles; ++a)
        if (!tile_shape_ok(tiles[2 * a], tiles[2 * a + 1]))
            return fail(ctx, LFR_ERR_INVALID_ARG, "candidate tile %d x %d not supported", tiles[2 * a],
                        tiles[2 * a + 1]);
    for (int b = 0; b < n_sizes; ++b)
        if (sizes[b] < 1 || sizes[b] > kMaxClusterViews)
            return fail(ctx, LFR_ERR_INVALID_ARG, "candidate cluster size %d not supported", sizes[b]);
    hipStream_t s = ctx->stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    lfr_tune_result bestr{0, 0, 0, 3.0e38f, 0};
    lfr_status st = LFR_OK;
    for (int a = 0; a < n_tiles && st == LFR_OK; ++a) {
        lfr_display_desc dd = *desc;
        dd.tile_w = tiles[2 * a];
        dd.tile_h = tiles[2 * a + 1];
        lfr_display *disp = nullptr;
        st = lfr_display_create(ctx, &dd, &disp);
        for (int b = 0; b < n_sizes && st == LFR_OK; ++b) {
            lfr_render_opts o = *opts;
            o.cluster_size = sizes[b];
            o.flags &= ~(uint32_t)(LFR_TIMING | LFR_COUNT_WORK);
            st = lfr_render(ctx, disp, scene, host_cams, num_cams, &o, out_device);
            const uint64_t pairs = ctx->stats.pairs;
            std::vector<float> ms(reps);
            for (int r = 0; r < reps && st == LFR_OK; ++r) {
                (void)hipEventRecord(e0, s);
                st = lfr_render(ctx, disp, scene, host_cams, num_cams, &o, out_device);
                (void)hipEventRecord(e1, s);
                if (st == LFR_OK && hipEventSynchronize(e1) == hipSuccess) (void)hipEventElapsedTime(&ms[r], e0, e1);
            }
            if (st != LFR_OK) break;
            std::sort(ms.begin(), ms.end());
            const lfr_tune_result res{dd.tile_w, dd.tile_h, sizes[b], ms[reps / 2], pairs};
            if (results) results[a * n_sizes + b] = res;
            if (res.ms < bestr.ms) bestr = res;
        }
        if (disp) lfr_display_destroy(disp);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != LFR_OK) return st;
    *best = bestr;
    return LFR_OK;
}

lfr_status lfr_project(lfr_context *ctx, const lfr_scene *scene, const lfr_camera *cam, int32_t W, int32_t H,
                       lfr_proj_record *out)
{
    CHK(begin(ctx));
    CHK(check_scene(ctx, scene));
    if (!cam || !out) return fail(ctx, LFR_ERR_INVALID_ARG, "NULL argument");
    if (!cam_ok(*cam)) return fail(ctx, LFR_ERR_INVALID_ARG, "camera is not finite or has f <= 0");
    if (W < 1 || H < 1) return fail(ctx, LFR_ERR_INVALID_ARG, "bad image size");
    void *h = nullptr, *dv = nullptr;
    CHK(pinned_get(ctx, sizeof(DevCamera), &h));
    CHK(ws_get(ctx, kCams, sizeof(DevCamera), &dv));
    *(DevCamera *)h = dev_camera(*cam, W, H);
    HIPCHK(ctx, hipMemcpyAsync(dv, h, sizeof(DevCamera), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, launch_project_records(scene_dev(scene), (const DevCamera *)dv, W, H, out, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));  // the pinned camera may be reused by the next call
    return LFR_OK;
}

}  // extern "C"

template <typename K>
static lfr_status sort_pairs(lfr_context *ctx, K *keys, uint32_t *vals, int64_t n, int32_t b0, int32_t b1)
{
    CHK(begin(ctx));
    const int kb = (int)(8 * sizeof(K));
    if (n < 0 || (n > 0 && (!keys || !vals)) || b0 < 0 || b1 > kb || b0 > b1)
        return fail(ctx, LFR_ERR_INVALID_ARG, "bad sort arguments");
    if (n > (int64_t)0xFFFFFFFFll) return fail(ctx, LFR_ERR_UNSUPPORTED, "n exceeds 2^32");
    if (n <= 1 || b0 == b1) return LFR_OK;
    K *k1;
    uint32_t *v1;
    void *tmp;
    CHK(ws_get_t(ctx, kPairK1, (size_t)n * sizeof(K) / sizeof(uint32_t) + 2, (uint32_t **)&k1));
    CHK(ws_get_t(ctx, kPairV1, (size_t)n, &v1));
    CHK(ws_get(ctx, kSortTemp, sort_temp_bytes(n), &tmp));
    bool alt = false;
    hipError_t e;
    if (sizeof(K) == 4)
        e = radix_sort_u32((uint32_t *)keys, vals, (uint32_t *)k1, v1, n, b0, b1, tmp, &alt, ctx->stream);
    else
        e = radix_sort_u64((uint64_t *)keys, vals, (uint64_t *)k1, v1, n, b0, b1, tmp, &alt, ctx->stream);
    HIPCHK(ctx, e);
    if (alt) {
        HIPCHK(ctx, hipMemcpyAsync(keys, k1, (size_t)n * sizeof(K), hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(vals, v1, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, ctx->stream));
    }
    return LFR_OK;
}

extern "C" {

lfr_status lfr_sort_pairs_u32(lfr_context *ctx, uint32_t *keys, uint32_t *vals, int64_t n, int32_t b0, int32_t b1)
{
    return sort_pairs<uint32_t>(ctx, keys, vals, n, b0, b1);
}

lfr_status lfr_sort_pairs_u64(lfr_context *ctx, uint64_t *keys, uint32_t *vals, int64_t n, int32_t b0, int32_t b1)
{
    return sort_pairs<uint64_t>(ctx, keys, vals, n, b0, b1);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free sort
// ---------------------------------------------------------------------------
namespace {

// The largest n lfr_sort_pairs_u32_noalloc takes, and the fixed device
// scratch it uses in place of the context workspace: the second key and
// value buffers of the ping-pong, then the radix histograms, their offsets
// and the scan's partial sums.
constexpr int64_t kNoAllocMaxPairs = int64_t(1) << 22;
constexpr size_t kNoAllocPingBytes = (size_t)kNoAllocMaxPairs * sizeof(uint32_t);
constexpr size_t kNoAllocTempBytes = size_t(4) << 20;
constexpr size_t kNoAllocScratchBytes = 2 * kNoAllocPingBytes + kNoAllocTempBytes;

// One copy per GPU, kept until the process ends (36 MiB).  In host code the
// name is a host-side stand-in, not a device address: host code only uses
// the per-device address that noalloc_scratch() resolves.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kNoAllocMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kNoAllocMaxDevices];

// The device address of `scratch` on the context's device (current after
// begin()), looked up on the first call on that device.
lfr_status noalloc_scratch(lfr_context *ctx, void **out)
{
    if (ctx->device < 0 || ctx->device >= kNoAllocMaxDevices)
        return fail(ctx, LFR_ERR_UNSUPPORTED, "device %d is beyond the allocation-free scratch table", ctx->device);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[ctx->device]) {
        void *p = nullptr;
        HIPCHK(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(ctx, LFR_ERR_HIP, "no device address for the allocation-free scratch");
        g_scratch_ptr[ctx->device] = p;
    }
    *out = g_scratch_ptr[ctx->device];
    return LFR_OK;
}

}  // namespace

extern "C" {

lfr_status lfr_sort_pairs_u32_noalloc(lfr_context *ctx, uint32_t *keys, uint32_t *vals, int64_t n, int32_t b0,
                                      int32_t b1)
{
    CHK(begin(ctx));
    if (n < 0 || (n > 0 && (!keys || !vals)) || b0 < 0 || b1 > 32 || b0 > b1)
        return fail(ctx, LFR_ERR_INVALID_ARG, "bad sort arguments");
    if (n > kNoAllocMaxPairs)
        return fail(ctx, LFR_ERR_CAPACITY, "n = %lld exceeds the allocation-free sort's limit of %lld pairs",
                    (long long)n, (long long)kNoAllocMaxPairs);
    if (n <= 1 || b0 == b1) return LFR_OK;
    if (sort_temp_bytes(n) > kNoAllocTempBytes)
        return fail(ctx, LFR_ERR_CAPACITY, "sort temporaries exceed the allocation-free scratch");
    void *base = nullptr;
    CHK(noalloc_scratch(ctx, &base));
    uint32_t *k1 = (uint32_t *)base;
    uint32_t *v1 = (uint32_t *)((char *)base + kNoAllocPingBytes);
    void *tmp = (char *)base + 2 * kNoAllocPingBytes;
    // every histogram, offset and partial the passes read is written by the
    // same pass first, so nothing in the scratch needs clearing
    bool alt = false;
    HIPCHK(ctx, radix_sort_u32(keys, vals, k1, v1, n, b0, b1, tmp, &alt, ctx->stream));
    if (alt) {
        HIPCHK(ctx, hipMemcpyAsync(keys, k1, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(vals, v1, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, ctx->stream));
    }
    return LFR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched frames
// ---------------------------------------------------------------------------
namespace {

// Frames merged into one render at most, and the device workspace a merged
// group may plan for (its per-(Gaussian, cluster) and per-(Gaussian, view)
// planes; half the context limit when one is set).
constexpr int kMaxGroupFrames = 16;
constexpr uint64_t kGroupBudget = 32ull << 30;

// Number of depth chunks render_group runs for M Gaussians.
int chunk_count(int64_t M, int32_t first_chunk)
{
    int64_t r0 = 0, len = first_chunk > 0 ? (int64_t)first_chunk
                                          : std::max<int64_t>(kFirstChunk, (M + kFirstChunkDiv - 1) / kFirstChunkDiv);
    int n = 0;
    for (;;) {
        len = std::min(len, M - r0);
        ++n;
        if (r0 + len >= M) return n;
        r0 += len;
        len *= 4;
    }
}

lfr_status batch_pinned_get(lfr_context *ctx, size_t bytes, void **out)
{
    if (ctx->batch_pinned_n < bytes) {
        if (ctx->batch_pinned) {
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
            HIPCHK(ctx, hipHostFree(ctx->batch_pinned));
            ctx->batch_pinned = nullptr;
            ctx->batch_pinned_n = 0;
        }
        const size_t want = std::max<size_t>(bytes, 1 << 16);
        HIPCHK(ctx, hipHostMalloc(&ctx->batch_pinned, want, hipHostMallocDefault));
        ctx->batch_pinned_n = want;
    }
    *out = ctx->batch_pinned;
    return LFR_OK;
}

void drop_graph(FrameSlot &sl)
{
    if (sl.graph) (void)hipGraphExecDestroy(sl.graph);
    sl.graph = nullptr;
}

// Frames a and b render with the same display, scene arrays and options.
bool mergeable(const lfr_frame &a, const lfr_frame &b)
{
    return a.display == b.display && a.display->uid == b.display->uid &&
           memcmp(a.scene, b.scene, sizeof(lfr_scene)) == 0 && memcmp(&a.opts, &b.opts, sizeof(lfr_render_opts)) == 0;
}

// A batch group: frames [first, first + count) rendered as one render.
struct Group {
    int first = 0, count = 0;
};

bool same_group(const FrameSlot &sl, const lfr_frame *f, const Group &g, bool tight)
{
    if ((int)sl.outs.size() != g.count || sl.tight != tight) return false;
    const lfr_frame &a = f[g.first];
    if (sl.display != (const void *)a.display || sl.display_uid != a.display->uid ||
        memcmp(&sl.scene, a.scene, sizeof(lfr_scene)) != 0 || memcmp(&sl.opts, &a.opts, sizeof(lfr_render_opts)) != 0)
        return false;
    for (int e = 0; e < g.count; ++e)
        if (sl.outs[e] != f[g.first + e].out_device) return false;
    return true;
}

// Plan from an unplanned render's per-chunk pair counts.
void set_plan(FrameSlot &sl, const std::vector<uint64_t> &pairs, bool tight)
{
    sl.caps.resize(pairs.size());
    for (size_t c = 0; c < pairs.size(); ++c)
        sl.caps[c] = tight ? pairs[c] : pairs[c] + pairs[c] / 4 + 4096;
}

// The cameras and outputs of a group, as render_group takes them.
struct GroupArgs {
    std::vector<const lfr_camera *> cams;
    std::vector<float *> outs;
};
GroupArgs group_args(const lfr_frame *f, const Group &g)
{
    GroupArgs a;
    for (int e = 0; e < g.count; ++e) {
        a.cams.push_back(f[g.first + e].host_cams);
        a.outs.push_back(f[g.first + e].out_device);
    }
    return a;
}

lfr_status run_group(lfr_context *ctx, const lfr_frame *f, const Group &g, const FrameRun &run)
{
    const GroupArgs a = group_args(f, g);
    const lfr_frame &h = f[g.first];
    return render_group(ctx, h.display, h.scene, g.count, a.cams.data(), &h.opts, a.outs.data(), &run);
}

// Capture one planned group into a graph.  On failure (e.g. the workspace
// would have to grow) the capture is discarded and *exec stays null.
lfr_status capture_group(lfr_context *ctx, const lfr_frame *f, const Group &g, const FrameRun &run,
                         hipGraphExec_t *exec)
{
    *exec = nullptr;
    if (!ctx->cap_stream) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    HIPCHK(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
    const hipStream_t user = ctx->stream;
    ctx->stream = ctx->cap_stream;
    ctx->capturing = true;
    const lfr_status st = run_group(ctx, f, g, run);
    ctx->capturing = false;
    ctx->stream = user;
    hipGraph_t gr = nullptr;
    const hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &gr);
    if (st != LFR_OK || ec != hipSuccess || !gr) {
        if (gr) (void)hipGraphDestroy(gr);
        (void)hipGetLastError();
        ctx->err.clear();
        return LFR_OK;
    }
    const hipError_t ei = hipGraphInstantiate(exec, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (ei != hipSuccess) {
        *exec = nullptr;
        (void)hipGetLastError();
    }
    return LFR_OK;
}

}  // namespace

extern "C" lfr_status lfr_render_batch(lfr_context *ctx, const lfr_frame *frames, int32_t num_frames, uint32_t flags)
{
    CHK(begin(ctx));
    if (num_frames < 0 || (num_frames > 0 && !frames))
        return fail(ctx, LFR_ERR_INVALID_ARG, "bad frame list");
    if (flags & ~(LFR_BATCH_GRAPH | LFR_BATCH_TIGHT_PLANS | LFR_BATCH_NO_MERGE))
        return fail(ctx, LFR_ERR_INVALID_ARG, "unknown batch flags");
    for (int i = 0; i < num_frames; ++i) {
        const lfr_frame &f = frames[i];
        CHK(check_render_args(ctx, f.display, f.scene, f.host_cams, f.num_cams, &f.opts, f.out_device));
        if (f.opts.flags & (LFR_SAVE_FOR_BACKWARD | LFR_COUNT_WORK))
            return fail(ctx, LFR_ERR_INVALID_ARG, "frame %d: LFR_SAVE_FOR_BACKWARD and LFR_COUNT_WORK are not "
                        "available in a batch", i);
    }
    const bool use_graph = (flags & LFR_BATCH_GRAPH) != 0, tight = (flags & LFR_BATCH_TIGHT_PLANS) != 0;
    const bool merge = (flags & LFR_BATCH_NO_MERGE) == 0;
    hipStream_t s = ctx->stream;

    // groups: runs of consecutive frames with the same display, scene and
    // options (remapped blend), as many as the key bits and the workspace
    // budget allow; every other frame is a group of one
    const uint64_t budget = ctx->limit ? ctx->limit / 2 : kGroupBudget;
    std::vector<Group> groups;
    std::vector<ViewTables> vt1s;
    for (int i = 0; i < num_frames;) {
        const lfr_frame &f = frames[i];
        lfr_display *d = const_cast<lfr_display *>(f.display);
        const bool cull = (f.opts.flags & LFR_CULL_UNREFERENCED) != 0;
        ViewTables vt1 = build_tables(d, f.opts.cluster_size, cull);
        const uint64_t M = (uint64_t)f.scene->num_gaussians;
        const uint64_t per_frame = M * (120ull * vt1.n_clusters + 8ull * vt1.n_views) + 16ull * d->W * d->H * 3;
        const int tbits = bits_for(d->T);
        Group g{i, 1};
        if (merge && (f.opts.flags & LFR_REMAP))
            while (g.count < kMaxGroupFrames && i + g.count < num_frames && mergeable(f, frames[i + g.count]) &&
                   per_frame * (uint64_t)(g.count + 1) <= budget &&
                   bits_for((int64_t)(g.count + 1) * vt1.n_clusters) + tbits <= 32)
                ++g.count;
        groups.push_back(g);
        vt1s.push_back(std::move(vt1));
        i += g.count;
    }
    const int n_groups = (int)groups.size();
    if ((int)ctx->slots.size() < n_groups) ctx->slots.resize(n_groups);
    int n_unplanned = 0, n_graphs = 0, n_rerendered = 0;

    // every group's tables (cameras, cluster/view tables, output pointers),
    // uploaded in one copy
    std::vector<ViewTables> vts(n_groups);
    std::vector<size_t> offs(n_groups);
    size_t total = 0;
    for (int gi = 0; gi < n_groups; ++gi) {
        const Group &g = groups[gi];
        const lfr_frame &f = frames[g.first];
        lfr_display *d = const_cast<lfr_display *>(f.display);
        const bool cull = (f.opts.flags & LFR_CULL_UNREFERENCED) != 0;
        TaskSet *ts = nullptr;
        CHK(get_group_layout(ctx, d, f.opts.cluster_size, cull, vt1s[gi], g.count, &ts));
        vts[gi] = merge_tables(vt1s[gi], g.count, d->N);
        offs[gi] = total;
        total += (tables_bytes(vts[gi], g.count > 1 ? g.count : 0) + 255) & ~(size_t)255;
    }
    void *dtab = nullptr, *htab = nullptr;
    uint64_t *need = nullptr;
    CHK(ws_get(ctx, kBatchTables, std::max<size_t>(total, 256), &dtab));
    CHK(ws_get_t(ctx, kBatchNeed, (size_t)std::max(n_groups, 1) * kMaxPlannedChunks, &need));
    CHK(batch_pinned_get(ctx, std::max<size_t>(total, 256), &htab));
    std::vector<DevTables> dts(n_groups);
    for (int gi = 0; gi < n_groups; ++gi) {
        const GroupArgs a = group_args(frames, groups[gi]);
        const int n_out = groups[gi].count > 1 ? groups[gi].count : 0;
        write_tables(frames[groups[gi].first].display, a.cams.data(), vts[gi], (char *)htab + offs[gi],
                     (char *)dtab + offs[gi], &dts[gi], a.outs.data(), n_out);
    }
    if (total) HIPCHK(ctx, hipMemcpyAsync(dtab, htab, total, hipMemcpyHostToDevice, s));

    std::vector<int> planned;
    for (int gi = 0; gi < n_groups; ++gi) {
        const Group &g = groups[gi];
        const lfr_frame &f = frames[g.first];
        FrameSlot &sl = ctx->slots[gi];
        if (!same_group(sl, frames, g, tight)) {
            drop_graph(sl);
            sl.caps.clear();
            sl.display = f.display;
            sl.display_uid = f.display->uid;
            sl.scene = *f.scene;
            sl.opts = f.opts;
            sl.outs = group_args(frames, g).outs;
            sl.tight = tight;
        }
        FrameRun run;
        run.tables = &dts[gi];
        if (sl.caps.empty() || chunk_count(f.scene->num_gaussians, f.opts.first_chunk) > kMaxPlannedChunks) {
            std::vector<uint64_t> pairs;
            run.chunk_pairs = &pairs;
            CHK(run_group(ctx, frames, g, run));
            set_plan(sl, pairs, tight);
            n_unplanned += g.count;
            continue;
        }
        run.caps = &sl.caps;
        run.d_need = need + (size_t)gi * kMaxPlannedChunks;
        if (use_graph) {
            if (sl.graph && (sl.graph_gen != ctx->ws_gen || sl.graph_table_off != offs[gi])) drop_graph(sl);
            if (!sl.graph) {
                CHK(capture_group(ctx, frames, g, run, &sl.graph));
                sl.graph_gen = ctx->ws_gen;
                sl.graph_table_off = offs[gi];
            }
            if (sl.graph) {
                HIPCHK(ctx, hipGraphLaunch(sl.graph, s));
                n_graphs += g.count;
                planned.push_back(gi);
                continue;
            }
        }
        CHK(run_group(ctx, frames, g, run));
        planned.push_back(gi);
    }

    // one synchronization: check the planned groups' pair counts
    std::vector<uint64_t> hneed((size_t)std::max(n_groups, 1) * kMaxPlannedChunks);
    if (!planned.empty())
        HIPCHK(ctx, hipMemcpyAsync(hneed.data(), need, hneed.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    for (int gi : planned) {
        const Group &g = groups[gi];
        const lfr_frame &f = frames[g.first];
        FrameSlot &sl = ctx->slots[gi];
        const int nc = chunk_count(f.scene->num_gaussians, f.opts.first_chunk);
        bool over = false;
        for (int c = 0; c < nc; ++c) {
            const uint64_t cap = c < (int)sl.caps.size() ? sl.caps[c] : kUnplannedChunkCap;
            over = over || hneed[(size_t)gi * kMaxPlannedChunks + c] > std::max<uint64_t>(cap, 1);
        }
        if (!over) continue;
        drop_graph(sl);
        FrameRun run;
        run.tables = &dts[gi];
        std::vector<uint64_t> pairs;
        run.chunk_pairs = &pairs;
        CHK(run_group(ctx, frames, g, run));
        set_plan(sl, pairs, tight);
        n_rerendered += g.count;
    }
    if (n_rerendered) HIPCHK(ctx, hipStreamSynchronize(s));
    ctx->stats = lfr_stats{};
    ctx->stats.batch_frames = num_frames;
    ctx->stats.batch_unplanned = n_unplanned;
    ctx->stats.batch_graphs = n_graphs;
    ctx->stats.batch_rerendered = n_rerendered;
    ctx->stats.batch_groups = n_groups;
    ctx->stats.workspace_bytes = ws_total(ctx);
    return LFR_OK;
}
