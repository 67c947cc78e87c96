// Key generation with reuse (section 4.2 "Key Generation", appendix B.2
// GenerateKeys): for each (Gaussian i, cluster k) the tiles touched by the
// union over the cluster's views j of the box around mean2d(i, j) with the
// cluster's half extents; one (key, i) pair per tile of that union, key =
// (tile << cluster_bits) | k.
//
// The Gaussians of every cluster are first sorted by depth; pairs are then
// generated chunk by chunk in that order (a chunk is a range of depth ranks,
// the same for every cluster), so a stable sort on the tile bits alone
// leaves every (tile, cluster) list sorted by (depth, i): the order of the
// 64-bit key (t, k, depth) of Eq. 7 / appendix B.2.  A tile is skipped when
// its (tile, cluster) list has no unsaturated subpixel left (`alive` bits,
// maintained by the blend between chunks): those lists would never be read.
//
// Tile coverage is conservative (the box bounds the alpha >= 1/255 region
// with margins), so the rendered result does not depend on the tiling.
#include <algorithm>
#include <type_traits>

#include "lfr_internal.h"

namespace lfr {

// Units of an item: (tile row, 32-tile word) cells of its union tile box b.
__device__ inline int item_units(ushort4 b)
{
    return ((int)b.w - (int)b.z + 1) * (((int)b.y >> 5) - ((int)b.x >> 5) + 1);
}

// Whether any (tile, cluster k) list inside the tile rectangle b (inclusive
// x0, x1, y0, y1) still has unsaturated subpixels: four lookups in the
// cluster's summed-area table of alive lists.
__device__ inline bool rect_alive(const BinParams &bp, int k, ushort4 b)
{
    const int64_t pitch = bp.TX + 1;
    const uint32_t *S = bp.alive_sat + (int64_t)k * (bp.TY + 1) * pitch;
    const int64_t y0 = b.z, y1 = (int64_t)b.w + 1, x0 = b.x, x1 = (int64_t)b.y + 1;
    return S[y1 * pitch + x1] - S[y0 * pitch + x1] - S[y1 * pitch + x0] + S[y0 * pitch + x0] != 0u;
}

// Tiles [lo, hi] (0 <= lo <= hi < 64) as a 64-bit mask.
__device__ __forceinline__ uint64_t span64(int lo, int hi)
{
    return (hi >= 63 ? ~0ull : ((2ull << hi) - 1ull)) & (~0ull << lo);
}

// What key generation reads per cluster, kept in scalar registers while a
// wavefront's runs stay in one cluster: whether any of its lists is still
// alive (the summed-area table's total), the last chunk's depth threshold,
// and the masks of tile rows and tile columns with an alive list (all ones
// without masks).
struct ClusterInfo {
    bool alive;
    uint32_t thr;
    uint64_t rows, c0, c1;
};

template <bool kFar>
__device__ inline ClusterInfo cluster_info(const BinParams &bp, int k)
{
    ClusterInfo c;
    c.alive = !bp.alive_sat || bp.alive_sat[((int64_t)k * (bp.TY + 1) + bp.TY) * (bp.TX + 1) + bp.TX] != 0u;
    c.thr = kFar ? bp.far_thr[k] : 0u;
    c.rows = c.c0 = c.c1 = ~0ull;
    if (bp.alive_mask) {
        const uint64_t *m = bp.alive_mask + 4 * (int64_t)k;
        c.rows = m[0];
        c.c0 = m[1];
        c.c1 = m[2];
    }
    return c;
}

// Whether the tile rectangle b (inside 64 x 128 tiles when the masks are
// real) can hold an alive list by the cluster's row and column masks
// (registers only; rect_alive then decides).
__device__ inline bool box_may_live(const ClusterInfo &c, ushort4 b)
{
    if (c.rows == ~0ull && c.c0 == ~0ull && c.c1 == ~0ull) return true;
    const int x0 = b.x, x1 = b.y;
    const uint64_t lo = x0 < 64 ? span64(x0, min(x1, 63)) : 0ull;
    const uint64_t hi = x1 >= 64 ? span64(max(x0, 64) - 64, x1 - 64) : 0ull;
    return (span64(b.z, b.w) & c.rows) != 0ull && ((lo & c.c0) | (hi & c.c1)) != 0ull;
}

// The x-range [xl, xr] (relative to the mean, padded) of the cutoff ellipse
// E <= E_c of record r, E = a (dx + beta dy)^2 + g dy^2, over the rows dy in
// [dlo, dhi]; false when no such row meets it.  For dy in an interval inside
// |dy| <= sqrt(E_c / g), the ellipse's right edge -beta dy + sqrt((E_c - g
// dy^2) / a) is concave and peaks at dy* = -beta sqrt(E_c / S) / g, S = 1/a
// + beta^2/g (where the edge reaches the full half width sqrt(E_c S)); the
// left edge is its mirror image.  So the extremes over the band are at dy*
// clamped into it.  E_c is the record's cutoff widened by 0.1% and 1e-3, and
// the range by 1e-4 relative and 0.02 px: margins far above the float32
// error of this evaluation (hardware reciprocals and square roots, about
// one ulp each) and of the blend's.
//
// What does not depend on the row band is computed once per record
// (ellipse_of): E_c, 1/a, 1/g, the half height sqrt(E_c / g) and dy*.
struct Ellipse {
    float beta, g, ec, ia, hy, ds;
};
__device__ inline Ellipse ellipse_of(const GaussRec &r)
{
    Ellipse e;
    e.beta = r.a.y;
    e.g = r.a.z;
    e.ec = r.c.w * 1.001f + 1e-3f;
    e.ia = __builtin_amdgcn_rcpf(r.a.x);
    const float ig = __builtin_amdgcn_rcpf(r.a.z);
    e.hy = __builtin_amdgcn_sqrtf(e.ec * ig);
    const float S = e.ia + (e.beta * e.beta) * ig;
    e.ds = -e.beta * __builtin_amdgcn_sqrtf(e.ec * __builtin_amdgcn_rcpf(S)) * ig;
    return e;
}
__device__ inline bool ellipse_xrange(const Ellipse &e, float dlo, float dhi, float &xl, float &xr)
{
    const float lo = fmaxf(dlo, -e.hy), hi = fminf(dhi, e.hy);
    if (!(lo <= hi)) return false;
    const float t1 = fminf(fmaxf(e.ds, lo), hi), t2 = fminf(fmaxf(e.ds, -hi), -lo);
    xr = -e.beta * t1 + __builtin_amdgcn_sqrtf(fmaxf(e.ec - e.g * t1 * t1, 0.0f) * e.ia);
    xl = e.beta * t2 - __builtin_amdgcn_sqrtf(fmaxf(e.ec - e.g * t2 * t2, 0.0f) * e.ia);
    const float pad = 1e-4f * fmaxf(fabsf(xr), fabsf(xl)) + 0.02f;
    xl -= pad;
    xr += pad;
    return true;
}

// Pixel columns [c0, c1] of the panel whose centres x + 0.5 lie in [xa, xb].
__device__ inline bool centre_cols(float xa, float xb, int W, int &c0, int &c1)
{
    const float f0 = fmaxf(ceilf(xa - 0.5f), 0.0f);
    const float f1 = fminf(floorf(xb - 0.5f), (float)(W - 1));
    if (!(f0 <= f1)) return false;
    c0 = (int)f0;
    c1 = (int)f1;
    return true;
}

// Pixel columns [c0, c1] whose centres in pixel rows [y0, y1] can lie in the
// cutoff ellipse e at mean m.
__device__ inline bool row_span(const Ellipse &e, float2 m, int y0, int y1, int W, int &c0, int &c1)
{
    float xl, xr;
    if (!ellipse_xrange(e, (float)y0 + 0.5f - m.y, (float)y1 + 0.5f - m.y, xl, xr)) return false;
    return centre_cols(m.x + xl, m.x + xr, W, c0, c1);
}

// The same for the union over several views whose means lie in the box
// [lo, hi]: each view's span lies in [m.x + xl, m.x + xr] with xl, xr taken
// over its own rows dy in [y0 + 0.5 - m.y, y1 + 0.5 - m.y], a sub-band of
// [y0 + 0.5 - hi.y, y1 + 0.5 - lo.y]; so [lo.x + xl, hi.x + xr] over that
// band holds all of them.
__device__ inline bool hull_span(const Ellipse &e, float2 lo, float2 hi, int y0, int y1, int W, int &c0, int &c1)
{
    float xl, xr;
    if (!ellipse_xrange(e, (float)y0 + 0.5f - hi.y, (float)y1 + 0.5f - lo.y, xl, xr)) return false;
    return centre_cols(lo.x + xl, hi.x + xr, W, c0, c1);
}

// Tiles of the item (Gaussian i, cluster k, union tile box b) in unit u: the
// OR over the cluster's views of the tiles in the unit's row and word that
// the view's ellipse span covers, restricted to alive lists.  The record
// holds the means of a cluster with up to kItemViews views (an invalid
// view's far stand-in mean covers nothing); for a larger cluster it holds
// the bounding box of the means of the views whose tile box is non-empty,
// and the row's span is that of the whole box (hull_span).  Also returns
// the unit's row and word.
__device__ inline uint32_t unit_mask(const BinParams &bp, int k, uint32_t i, const GaussRec &r, ushort4 b, int u,
                                     int &ty, int &w)
{
    const int w0 = (int)b.x >> 5;
    const int nw = ((int)b.y >> 5) - w0 + 1;
    // (most items span one or two words: no integer division for those)
    const int uq = nw == 1 ? u : (nw == 2 ? u >> 1 : u / nw);
    ty = (int)b.z + uq;
    w = w0 + (u - uq * nw);
    const int xb = w << 5;
    auto bits = [&](int lo, int hi) -> uint32_t {  // tiles [lo, hi] within the word
        lo -= xb;
        hi -= xb;
        if (hi < 0 || lo > 31) return 0u;
        const uint32_t mh = hi >= 31 ? 0xFFFFFFFFu : ((2u << hi) - 1u);
        const uint32_t ml = lo <= 0 ? 0xFFFFFFFFu : (0xFFFFFFFFu << lo);
        return mh & ml;
    };
    // the unit's word clipped to the item's box
    const uint32_t box = bits((int)b.x, (int)b.y);
    uint32_t m = 0;
    const int y0 = ty * bp.th, y1 = min(y0 + bp.th, bp.H) - 1;
    const int v0 = bp.cv_off[k], nvk = bp.cv_off[k + 1] - v0;
    const Ellipse el = ellipse_of(r);
    if (nvk > kItemViews) {
        int c0, c1;
        if (hull_span(el, r.m[0], r.m[1], y0, y1, bp.W, c0, c1)) m |= bits(c0 >> bp.tw_shift, c1 >> bp.tw_shift);
    } else {
#pragma unroll
        for (int v = 0; v < kItemViews; ++v) {
            int c0, c1;
            if (v < nvk && row_span(el, r.m[v], y0, y1, bp.W, c0, c1)) m |= bits(c0 >> bp.tw_shift, c1 >> bp.tw_shift);
        }
    }
    const uint32_t *alive_k = bp.alive + (int64_t)k * bp.TY * bp.alive_words;
    return m & box & alive_k[(int64_t)ty * bp.alive_words + w];
}

// The record of lane `owner`, handed over through lane exchanges (the lanes
// that work on an item's units read it from the lane that loaded it, not
// from memory).
__device__ __forceinline__ GaussRec shfl_item(const GaussRec &own, int owner)
{
    uint32_t w[16];
    __builtin_memcpy(w, &own, sizeof(GaussRec));
#pragma unroll
    for (int k = 0; k < 16; ++k) w[k] = (uint32_t)__shfl((int)w[k], owner, 64);
    GaussRec r;
    __builtin_memcpy(&r, w, sizeof(GaussRec));
    return r;
}

__device__ __forceinline__ ushort4 shfl_box(ushort4 own, int owner)
{
    uint32_t w[2];
    __builtin_memcpy(w, &own, sizeof(ushort4));
    w[0] = (uint32_t)__shfl((int)w[0], owner, 64);
    w[1] = (uint32_t)__shfl((int)w[1], owner, 64);
    ushort4 b;
    __builtin_memcpy(&b, w, sizeof(ushort4));
    return b;
}

// Position of the k-th set bit of m (k < popcount(m)).
__device__ inline int select_bit(uint32_t m, int k)
{
    int pos = 0, c;
    c = __popc(m & 0xFFFFu);
    if (k >= c) { k -= c; m >>= 16; pos += 16; }
    c = __popc(m & 0xFFu);
    if (k >= c) { k -= c; m >>= 8; pos += 8; }
    c = __popc(m & 0xFu);
    if (k >= c) { k -= c; m >>= 4; pos += 4; }
    c = __popc(m & 0x3u);
    if (k >= c) { k -= c; m >>= 2; pos += 2; }
    if (k >= (int)(m & 1u)) pos += 1;
    return pos;
}

__device__ inline uint32_t wave_incl_scan(uint32_t v, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Largest lane l with key[l] <= x, for a key that is non-decreasing over the
// lanes and key[0] <= x.
__device__ inline int wave_search(uint32_t key, uint32_t x)
{
    int l = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
        if ((uint32_t)__shfl((int)key, l + step, 64) <= x) l += step;
    return l;
}

// Items of one chunk: depth ranks [r0, r0 + len) of every cluster; item
// (k, r) sits at k * Mp + r of the depth-sorted arrays and at k * len + (r - r0)
// of the chunk's count / offset arrays.  The far chunk (kFar) is the last
// chunk of a split depth order: its items are every Gaussian r < len = M in
// index order, read from the unsorted key array at k * Mp + r, those with a
// valid key >= far_thr[k] taking part; its pair keys are 64-bit, the
// (tile, cluster) key above the depth key, so that one stable sort orders
// each list by (depth, i).
//
// Load balancing: each wavefront enumerates the units of its 64 consecutive
// items in item order and hands them out 64 at a time, so an item covering
// thousands of tiles is spread over the whole wavefront.  The counting pass
// adds each unit's tile count to its item (LDS) and writes, per wavefront w
// (k * ceil(len / 64) + r / 64), its pair total wcnt[w] and the mask of its
// items with pairs wmask[w]; the emitting pass starts at the wavefront's
// slot woff[w] (the exclusive scan of wcnt), lays the wavefront's pairs out
// in item order and writes them with consecutive lanes on consecutive
// slots.  A wavefront whose mask is empty emits nothing and reads no item.
// One run of 64 items (run wk of cluster k, run w of the chunk) on one
// wavefront; s_cnt: the wavefront's 64 counters in LDS.
template <bool kEmit, bool kFar>
__device__ __forceinline__ void chunk_run(const BinParams &bp, const uint32_t *__restrict__ dkey_sorted,
                                          const uint32_t *__restrict__ dval_sorted, int64_t r0, int64_t len, int k,
                                          const ClusterInfo &ci, int64_t wk, int64_t w, uint32_t *__restrict__ wcnt,
                                          uint64_t *__restrict__ wmask, const uint32_t *__restrict__ woff,
                                          uint64_t n_pairs, void *__restrict__ pair_keys_v,
                                          uint32_t *__restrict__ pair_vals, uint32_t *s_cnt)
{
    using PairKey = typename std::conditional<kFar, uint64_t, uint32_t>::type;
    PairKey *pair_keys = (PairKey *)pair_keys_v;
    const int lane = threadIdx.x & 63;
    const int64_t rl = wk * 64 + lane;
    const bool in = rl < len;
    // the emitting pass: only the items the counting pass found pairs for
    const uint64_t wm = kEmit ? wmask[w] : ~0ull;
    if (kEmit && wm == 0ull) return;
    const GaussRec *items_k = bp.items + (int64_t)k * bp.M;
    uint32_t i = 0, dkey_own = 0;
    int U = 0;
    // this lane's item record and union tile box (when it has units; only
    // such lanes' are ever read, by the unit lanes' exchanges, so the record
    // is not cleared: clearing it would wait for the previous run's loads)
    GaussRec own;
    ushort4 obox = make_ushort4(0, 0, 0, 0);
    // a cluster without any list that still has unsaturated subpixels emits
    // nothing (ci.alive: the summed-area table's total)
    if (in && ((wm >> lane) & 1ull)) {
        const int64_t e = (int64_t)k * bp.Mp + r0 + rl;
        const uint32_t dk = dkey_sorted[e], dv = kFar ? (uint32_t)rl : dval_sorted[e];
        // (far items sit at their index: the box is loaded with the key)
        ushort4 fbox = make_ushort4(0, 0, 0, 0);
        if (kFar) fbox = bp.ibox[(int64_t)k * bp.M + rl];
        // (the index is tested too, though never all ones, so that its load
        // is issued with the key's instead of after the key is known; so is a
        // far item's box, whose x0 <= x1 holds for every binned item)
        bool take = ci.alive & (dk != 0xFFFFFFFFu) & (dv != 0xFFFFFFFFu);
        if (kFar) take = take & (dk >= ci.thr) & (fbox.x <= fbox.y);
        if (take) {
            i = dv;
            dkey_own = dk;
            // items whose tiles are all saturated emit nothing: the counting
            // pass tests the 8-byte union box before it reads the record
            // (the emitting pass only sees items with pairs)
            obox = kFar ? fbox : bp.ibox[(int64_t)k * bp.M + i];
            if (kEmit || !bp.alive_sat || (box_may_live(ci, obox) && rect_alive(bp, k, obox))) {
                own = items_k[i];
                U = item_units(obox);
            }
        }
    }
    // a counting run without units: nothing to count
    if (!kEmit && __ballot(U > 0) == 0ull) {
        if (lane == 0) {
            wcnt[w] = 0u;
            wmask[w] = 0ull;
        }
        return;
    }
    const uint32_t uincl = wave_incl_scan((uint32_t)U, lane);
    const uint32_t ubase = uincl - (uint32_t)U;
    const uint32_t utot = (uint32_t)__shfl((int)uincl, 63, 64);
    if (!kEmit) s_cnt[lane] = 0;
    uint64_t out = 0;  // next pair slot of this wavefront
    if (kEmit && utot > 0) out = (uint64_t)woff[w];
    for (uint32_t ub = 0; ub < utot; ub += 64) {
        const uint32_t u = ub + (uint32_t)lane;
        const bool has = u < utot;
        const int owner = wave_search(ubase, has ? u : utot - 1);
        const uint32_t iown = (uint32_t)__shfl((int)i, owner, 64);
        const uint32_t down = kFar ? (uint32_t)__shfl((int)dkey_own, owner, 64) : 0u;
        const uint32_t uloc = (has ? u : utot - 1) - (uint32_t)__shfl((int)ubase, owner, 64);
        int ty = 0, w = 0;
        uint32_t m = 0;
        const GaussRec rown = shfl_item(own, owner);
        const ushort4 bown = shfl_box(obox, owner);
        if (has) m = unit_mask(bp, k, iown, rown, bown, (int)uloc, ty, w);
        const uint32_t c = (uint32_t)__popc(m);
        if (!kEmit) {
            if (c) atomicAdd(&s_cnt[owner], c);
        } else {
            // spread this round's pairs over the lanes
            const uint32_t cincl = wave_incl_scan(c, lane);
            const uint32_t cbase = cincl - c;
            const uint32_t ctot = (uint32_t)__shfl((int)cincl, 63, 64);
            const uint32_t tilebase = (uint32_t)ty * (uint32_t)bp.TX + ((uint32_t)w << 5);
            for (uint32_t pb = 0; pb < ctot; pb += 64) {
                const uint32_t pidx = pb + (uint32_t)lane;
                const uint32_t px = pidx < ctot ? pidx : ctot - 1;
                const int q = wave_search(cbase, px);
                const uint32_t mq = (uint32_t)__shfl((int)m, q, 64);
                const uint32_t kth = px - (uint32_t)__shfl((int)cbase, q, 64);
                const uint32_t tb = (uint32_t)__shfl((int)tilebase, q, 64);
                const uint32_t iq = (uint32_t)__shfl((int)iown, q, 64);
                const uint32_t dq = kFar ? (uint32_t)__shfl((int)down, q, 64) : 0u;
                const uint64_t slot = out + pidx;
                if (pidx < ctot && slot < n_pairs) {
                    const uint32_t t = tb + (uint32_t)select_bit(mq, (int)kth);
                    const uint32_t list = (t << bp.cluster_bits) | (uint32_t)k;
                    if (kFar)
                        pair_keys[slot] = (PairKey)(((uint64_t)list << 32) | dq);
                    else
                        pair_keys[slot] = (PairKey)list;
                    pair_vals[slot] = iq;
                }
            }
            out += ctot;
        }
    }
    if (!kEmit) {
        const uint32_t c = s_cnt[lane];
        const uint64_t m = __ballot(c != 0u);
        const uint32_t tot = (uint32_t)__shfl((int)wave_incl_scan(c, lane), 63, 64);
        if (lane == 0) {
            wcnt[w] = tot;
            wmask[w] = m;
        }
    }
}

// Wavefronts take the chunk's runs of 64 items in turn (run w = k *
// ceil(len / 64) + r / 64), so a long chunk runs on a few thousand blocks.
template <bool kEmit, bool kFar>
__global__ void __launch_bounds__(256) chunk_tiles_kernel(BinParams bp, const uint32_t *__restrict__ dkey_sorted,
                                                           const uint32_t *__restrict__ dval_sorted, int64_t r0,
                                                           int64_t len, uint32_t *__restrict__ wcnt,
                                                           uint64_t *__restrict__ wmask,
                                                           const uint32_t *__restrict__ woff, uint64_t n_pairs,
                                                           void *__restrict__ pair_keys_v,
                                                           uint32_t *__restrict__ pair_vals)
{
    __shared__ uint32_t s_cnt[4][64];
    // (the wavefront index through readfirstlane: uniform, so the run and
    // cluster arithmetic and the per-cluster loads are scalar)
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // (run counts fit 32 bits: K' M < 2^32 items)
    const uint32_t nwk = (uint32_t)((len + 63) >> 6), nw = nwk * (uint32_t)bp.n_clusters;
    // every subpixel saturated (chunks planned ahead of time): no pairs
    const bool done = bp.alive_total && *bp.alive_total == 0u;
    uint32_t kc = 0xFFFFFFFFu;  // the cluster whose values ci holds
    ClusterInfo ci = {};
    for (uint32_t w = blockIdx.x * 4u + (uint32_t)wave; w < nw; w += gridDim.x * 4u) {
        const uint32_t k = w / nwk;
        if (done) {
            if (!kEmit && lane == 0) {
                wcnt[w] = 0u;
                wmask[w] = 0ull;
            }
            continue;
        }
        if (k != kc) {
            kc = k;
            ci = cluster_info<kFar>(bp, (int)k);
        }
        chunk_run<kEmit, kFar>(bp, dkey_sorted, dval_sorted, r0, len, (int)k, ci, (int64_t)(w - k * nwk),
                               (int64_t)w, wcnt, wmask, woff, n_pairs, pair_keys_v, pair_vals, s_cnt[wave]);
    }
}

__global__ void __launch_bounds__(256) fill_kernel(uint32_t *p, uint32_t v, int64_t n)
{
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x)
        p[s] = v;
}

__global__ void __launch_bounds__(256) copy_kernel(uint32_t *__restrict__ dst, const uint32_t *__restrict__ src,
                                                    int64_t n)
{
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x)
        dst[s] = src[s];
}

// The (tile, cluster) list of a pair key: the key itself, or the upper half
// of a far-chunk key (list above depth).
__device__ __forceinline__ uint32_t list_of(uint32_t key) { return key; }
__device__ __forceinline__ uint32_t list_of(uint64_t key) { return (uint32_t)(key >> 32); }

// [start, end) of every (tile, cluster) list, indexed by the list's key.  The
// pair count is P, or min(*dP, P) when dP is given.
template <typename K>
__global__ void __launch_bounds__(256) ranges_kernel(const K *__restrict__ keys, int64_t P_cap,
                                                      const uint64_t *dP, uint2 *ranges)
{
    const int64_t P = dP ? (int64_t)min(*dP, (uint64_t)P_cap) : P_cap;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    // the three loads are independent (clamped indices), so none waits for another
    const uint32_t k = list_of(keys[p]);
    const uint32_t kb = list_of(keys[p > 0 ? p - 1 : p]);
    const uint32_t ka = list_of(keys[p + 1 < P ? p + 1 : p]);
    if (p == 0 || kb != k) ranges[k].x = (uint32_t)p;
    if (p == P - 1 || ka != k) ranges[k].y = (uint32_t)(p + 1);
}

// dst = *src (a device count recorded for the host to read later).
__global__ void record_count_kernel(const uint64_t *src, uint64_t *dst) { *dst = *src; }

// alive bit of (cluster k, tile t) = (number of unsaturated subpixels of the
// (t, k) list) > 0; one thread per 32-bit word of a tile row.
__global__ void __launch_bounds__(256) alive_bits_kernel(const uint32_t *__restrict__ tc_alive, int n_clusters,
                                                          int TX, int TY, int words, int cluster_bits,
                                                          uint32_t *__restrict__ bits)
{
    const int64_t wid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)n_clusters * TY * words;
    if (wid >= n) return;
    const int w = (int)(wid % words);
    const int64_t rowid = wid / words;
    const int ty = (int)(rowid % TY);
    const int k = (int)(rowid / TY);
    // all 32 loads first (columns past the row read its last tile and are
    // not counted)
    uint32_t v[32];
#pragma unroll
    for (int b = 0; b < 32; ++b) {
        const int tx = min((w << 5) + b, TX - 1);
        const uint32_t t = (uint32_t)(ty * TX + tx);
        v[b] = tc_alive[(t << cluster_bits) | (uint32_t)k];
    }
    uint32_t m = 0;
#pragma unroll
    for (int b = 0; b < 32; ++b)
        if ((w << 5) + b < TX && v[b] > 0) m |= 1u << b;
    bits[wid] = m;
}

// Summed-area table of alive (tile, cluster) lists, one block per cluster:
// sat[k][y][x] = number of lists with tile row < y and tile column < x whose
// unsaturated-subpixel count is non-zero.  Rows are prefixed by one wavefront
// each (64 tiles per step), then columns by one thread each.
__global__ void __launch_bounds__(256) alive_sat_kernel(const uint32_t *__restrict__ tc_alive, int TX, int TY,
                                                         int cluster_bits, uint32_t *__restrict__ sat)
{
    const int k = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n_waves = blockDim.x >> 6;
    const int64_t pitch = TX + 1;
    uint32_t *S = sat + (int64_t)k * (TY + 1) * pitch;
    for (int x = threadIdx.x; x <= TX; x += blockDim.x) S[x] = 0u;
    for (int ty = wave; ty < TY; ty += n_waves) {
        uint32_t *row = S + (int64_t)(ty + 1) * pitch;
        if (lane == 0) row[0] = 0u;
        uint32_t carry = 0;
        for (int x0 = 0; x0 < TX; x0 += 64) {
            const int tx = x0 + lane;
            uint32_t v = 0;
            if (tx < TX) {
                const uint32_t t = (uint32_t)(ty * TX + tx);
                v = tc_alive[(t << cluster_bits) | (uint32_t)k] > 0 ? 1u : 0u;
            }
            const uint32_t incl = wave_incl_scan(v, lane);
            if (tx < TX) row[tx + 1] = carry + incl;
            carry += (uint32_t)__shfl((int)incl, 63, 64);
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x <= TX; x += blockDim.x) {
        uint32_t run = 0;
        for (int y = 1; y <= TY; ++y) {
            run += S[(int64_t)y * pitch + x];
            S[(int64_t)y * pitch + x] = run;
        }
    }
}

// Both tables of one cluster at once, the summed-area table built in LDS
// (for grids whose table fits kSatLdsMax entries): each wavefront takes tile
// rows, 64 tiles at a time; the ballot of the row's alive flags gives two
// words of alive bits, their prefix sum the table's row; the columns are then
// prefixed in LDS by one thread each and the table written out whole.
constexpr int kSatBlock = 1024;
constexpr int kSatLdsMax = 12288;  // 48 KB
__global__ void __launch_bounds__(kSatBlock) alive_tables_kernel(const uint32_t *__restrict__ tc_alive, int TX,
                                                                  int TY, int words, int cluster_bits,
                                                                  uint32_t *__restrict__ bits,
                                                                  uint32_t *__restrict__ sat,
                                                                  uint64_t *__restrict__ masks)
{
    __shared__ uint32_t S[kSatLdsMax];
    __shared__ unsigned long long s_mask[3];  // rows, columns 0..63, columns 64..127 with an alive list
    if (threadIdx.x < 3) s_mask[threadIdx.x] = 0ull;
    __syncthreads();
    const int k = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int pitch = TX + 1, n = (TY + 1) * pitch;
    for (int x = threadIdx.x; x <= TX; x += kSatBlock) S[x] = 0u;
    for (int ty = wave; ty < TY; ty += kSatBlock / 64) {
        uint32_t *row = S + (ty + 1) * pitch;
        if (lane == 0) row[0] = 0u;
        uint32_t carry = 0;
        for (int x0 = 0; x0 < TX; x0 += 64) {
            const int tx = x0 + lane;
            const uint32_t t = (uint32_t)(ty * TX + min(tx, TX - 1));
            const uint32_t c = tc_alive[(t << cluster_bits) | (uint32_t)k];
            const uint32_t v = (tx < TX && c > 0u) ? 1u : 0u;
            const uint64_t b = __ballot(v != 0u);
            const int w0 = x0 >> 5;
            uint32_t *brow = bits + ((int64_t)k * TY + ty) * words;
            if (lane == 0) brow[w0] = (uint32_t)b;
            if (lane == 1 && w0 + 1 < words) brow[w0 + 1] = (uint32_t)(b >> 32);
            const uint32_t incl = wave_incl_scan(v, lane);
            if (tx < TX) row[tx + 1] = carry + incl;
            carry += (uint32_t)__popcll(b);
            if (lane == 0 && b != 0ull && x0 < 128) atomicOr(&s_mask[1 + (x0 >> 6)], (unsigned long long)b);
        }
        if (lane == 0 && carry != 0u && ty < 64) atomicOr(&s_mask[0], 1ull << ty);
    }
    __syncthreads();
    if (masks && threadIdx.x < 4) masks[4 * (int64_t)k + threadIdx.x] = threadIdx.x < 3 ? s_mask[threadIdx.x] : 0ull;
    for (int x = threadIdx.x; x <= TX; x += kSatBlock) {
        uint32_t run = 0;
        for (int y = 1; y <= TY; ++y) {
            run += S[y * pitch + x];
            S[y * pitch + x] = run;
        }
    }
    __syncthreads();
    uint32_t *out = sat + (int64_t)k * n;
    for (int e = threadIdx.x; e < n; e += kSatBlock) out[e] = S[e];
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// Blocks of 4 wavefronts for a chunk of len ranks per cluster: one per 4
// runs of 64 items, at most kChunkBlocks.
constexpr int64_t kChunkBlocks = 4096;
static unsigned chunk_blocks(int64_t len, int n_clusters)
{
    const int64_t runs = (len + 63) / 64 * n_clusters;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((runs + 3) / 4, kChunkBlocks));
}

hipError_t launch_chunk_count(const BinParams &bp, const uint32_t *dkey_sorted, const uint32_t *dval_sorted,
                              int64_t r0, int64_t len, uint32_t *wcnt, uint64_t *wmask, hipStream_t s, bool far)
{
    if (len == 0 || bp.n_clusters == 0) return hipSuccess;
    if (far && !bp.far_thr) return hipErrorInvalidValue;
    const dim3 grid(chunk_blocks(len, bp.n_clusters));
    if (far)
        hipLaunchKernelGGL((chunk_tiles_kernel<false, true>), grid, dim3(256), 0, s, bp, dkey_sorted, dval_sorted,
                           r0, len, wcnt, wmask, (const uint32_t *)nullptr, (uint64_t)0, (void *)nullptr,
                           (uint32_t *)nullptr);
    else
        hipLaunchKernelGGL((chunk_tiles_kernel<false, false>), grid, dim3(256), 0, s, bp, dkey_sorted, dval_sorted,
                           r0, len, wcnt, wmask, (const uint32_t *)nullptr, (uint64_t)0, (void *)nullptr,
                           (uint32_t *)nullptr);
    return hipGetLastError();
}

hipError_t launch_chunk_emit(const BinParams &bp, const uint32_t *dkey_sorted, const uint32_t *dval_sorted,
                             int64_t r0, int64_t len, const uint64_t *wmask, const uint32_t *woff,
                             uint64_t n_pairs, void *pair_keys, uint32_t *pair_vals, hipStream_t s, bool far)
{
    if (len == 0 || bp.n_clusters == 0 || n_pairs == 0) return hipSuccess;
    if (far && !bp.far_thr) return hipErrorInvalidValue;
    const dim3 grid(chunk_blocks(len, bp.n_clusters));
    if (far)
        hipLaunchKernelGGL((chunk_tiles_kernel<true, true>), grid, dim3(256), 0, s, bp, dkey_sorted, dval_sorted, r0,
                           len, (uint32_t *)nullptr, const_cast<uint64_t *>(wmask), woff, n_pairs, pair_keys,
                           pair_vals);
    else
        hipLaunchKernelGGL((chunk_tiles_kernel<true, false>), grid, dim3(256), 0, s, bp, dkey_sorted, dval_sorted,
                           r0, len, (uint32_t *)nullptr, const_cast<uint64_t *>(wmask), woff, n_pairs, pair_keys,
                           pair_vals);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)g), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_ranges(const uint32_t *keys, int64_t P, uint2 *ranges, hipStream_t s, const uint64_t *dP)
{
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(ranges_kernel<uint32_t>, dim3(blocks_for(P)), dim3(256), 0, s, keys, P, dP, ranges);
    return hipGetLastError();
}

hipError_t launch_ranges_u64(const uint64_t *keys, int64_t P, uint2 *ranges, hipStream_t s, const uint64_t *dP)
{
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(ranges_kernel<uint64_t>, dim3(blocks_for(P)), dim3(256), 0, s, keys, P, dP, ranges);
    return hipGetLastError();
}

hipError_t launch_copy_u32(uint32_t *dst, const uint32_t *src, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)g), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_record_count(const uint64_t *src, uint64_t *dst, hipStream_t s)
{
    hipLaunchKernelGGL(record_count_kernel, dim3(1), dim3(1), 0, s, src, dst);
    return hipGetLastError();
}

hipError_t launch_alive_sat(const uint32_t *tc_alive, int n_clusters, int TX, int TY, int cluster_bits, uint32_t *sat,
                            hipStream_t s)
{
    if (n_clusters == 0) return hipSuccess;
    hipLaunchKernelGGL(alive_sat_kernel, dim3((unsigned)n_clusters), dim3(256), 0, s, tc_alive, TX, TY, cluster_bits,
                       sat);
    return hipGetLastError();
}

bool alive_tables_have_masks(int TX, int TY)
{
    return (int64_t)(TY + 1) * (TX + 1) <= kSatLdsMax && TY <= 64 && TX <= 128;
}

hipError_t launch_alive_tables(const uint32_t *tc_alive, int n_clusters, int TX, int TY, int words, int cluster_bits,
                               uint32_t *bits, uint32_t *sat, uint64_t *masks, hipStream_t s)
{
    if (n_clusters == 0) return hipSuccess;
    if ((int64_t)(TY + 1) * (TX + 1) > kSatLdsMax) {
        const hipError_t e = launch_alive_bits(tc_alive, n_clusters, TX, TY, words, cluster_bits, bits, s);
        if (e != hipSuccess) return e;
        return launch_alive_sat(tc_alive, n_clusters, TX, TY, cluster_bits, sat, s);
    }
    hipLaunchKernelGGL(alive_tables_kernel, dim3((unsigned)n_clusters), dim3(kSatBlock), 0, s, tc_alive, TX, TY, words,
                       cluster_bits, bits, sat, alive_tables_have_masks(TX, TY) ? masks : nullptr);
    return hipGetLastError();
}

hipError_t launch_alive_bits(const uint32_t *tc_alive, int n_clusters, int TX, int TY, int words, int cluster_bits,
                             uint32_t *bits, hipStream_t s)
{
    const int64_t n = (int64_t)n_clusters * TY * words;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(alive_bits_kernel, dim3(blocks_for(n)), dim3(256), 0, s, tc_alive, n_clusters, TX, TY, words,
                       cluster_bits, bits);
    return hipGetLastError();
}

}  // namespace lfr
