// Stable LSD radix sort of (key, value) pairs, digits of at most 8 bits.
//
// Per pass: (1) every 4096-key tile builds a 256-bin digit histogram in LDS;
// (2) the [digit][tile] histogram matrix is exclusive-scanned, giving every
// (digit, tile) its first output slot; (3) every tile re-reads its keys,
// ranks them stably (wavefront ballots) and writes them out in digit runs.
#include "lfr_internal.h"

namespace lfr {

constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortBlock * kSortItems;
constexpr int kSortWaves = kSortBlock / 64;

// Histogram layout (nd = digit values of the pass): [digit][tile] for one
// segment; with segments of seg tiles each (seg > 0), [segment][digit][tile in
// segment], so that one linear exclusive scan keeps every segment's keys
// inside the segment (a segmented sort: keys never cross segment boundaries).
__device__ __forceinline__ int64_t hist_index(int d, int64_t tile, int64_t nb, int64_t seg, int nd)
{
    if (seg == 0) return (int64_t)d * nb + tile;
    return ((tile / seg) * nd + d) * seg + tile % seg;
}

// The element count is n, or min(*dn, n) when dn is given (a count known only
// on the device; the grid is sized for n).
__device__ __forceinline__ int64_t sort_count(int64_t n, const uint64_t *dn)
{
    if (!dn) return n;
    const uint64_t d = *dn;
    return d < (uint64_t)n ? (int64_t)d : n;
}

template <typename K>
__global__ void __launch_bounds__(kSortBlock) sort_hist_kernel(const K *__restrict__ keys, int64_t n_cap,
                                                                const uint64_t *dn, int shift, uint32_t mask,
                                                                uint32_t *hist, int64_t nb, int64_t seg)
{
    const int64_t n = sort_count(n_cap, dn);
    // four copies of the histogram, lane l counting into copy l & 3 (257
    // words apart: a digit's copies lie in different banks), so that lanes of
    // one atomic instruction collide four times less often on a digit that
    // many keys share (the top digit of float depths takes few values)
    __shared__ uint32_t h[4 * 257];
    uint32_t *hc = h + (threadIdx.x & 3) * 257;
    for (int b = threadIdx.x; b < 4 * 257; b += kSortBlock) h[b] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    // all of a thread's keys are loaded before the first is counted (a
    // load guarded by its own bounds test would wait for each in turn)
    // (indices past the count read element 0, which the grid's capacity
    // always holds, and are not counted)
    K k[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t idx = base + it * kSortBlock + threadIdx.x;
        k[it] = keys[idx < n ? idx : 0];
    }
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t idx = base + it * kSortBlock + threadIdx.x;
        if (idx < n) atomicAdd(&hc[(uint32_t)(k[it] >> shift) & mask], 1u);
    }
    __syncthreads();
    if (threadIdx.x <= mask)
        hist[hist_index(threadIdx.x, blockIdx.x, nb, seg, (int)mask + 1)] =
            h[threadIdx.x] + h[257 + threadIdx.x] + h[514 + threadIdx.x] + h[771 + threadIdx.x];
}

// Scatter of one 4096-key tile.  Wavefront w ranks the contiguous keys
// [tile + 1024 w, tile + 1024 (w + 1)) 64 at a time: eight ballots find the
// lanes with an equal digit, the lane's rank is the popcount of equal lanes
// below it plus the wavefront's running count of that digit (kept in LDS and
// advanced by the lowest equal lane).  Wavefront counts are then prefixed in
// wavefront order, which keeps the sort stable.  Keys are first placed into
// an LDS copy of the tile in digit order and then written out in that order,
// so each digit's run is written with consecutive addresses.
template <typename K>
__global__ void __launch_bounds__(kSortBlock) sort_scatter_kernel(const K *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                                   K *__restrict__ kout, uint32_t *__restrict__ vout,
                                                                   int64_t n_cap, const uint64_t *dn, int shift,
                                                                   uint32_t mask, const uint32_t *__restrict__ offs,
                                                                   const uint32_t *__restrict__ hist, int64_t nb,
                                                                   int64_t seg)
{
    const int64_t n = sort_count(n_cap, dn);
    constexpr int kPerWave = kSortTile / kSortWaves;  // 1024
    constexpr int kIt = kPerWave / 64;                // 16
    __shared__ K s_key[kSortTile];
    __shared__ uint32_t s_val[kSortTile];
    __shared__ uint32_t s_cnt[kSortWaves][256];
    __shared__ uint32_t s_dstart[256];  // first slot of each digit inside the tile
    __shared__ uint32_t s_gbase[256];   // first global slot of each digit for this tile
    __shared__ uint32_t s_wsum[kSortWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    const int64_t tile = (int64_t)blockIdx.x * kSortTile;

    // digit starts inside the tile: exclusive scan of this tile's histogram
    {
        const bool dig = (uint32_t)tid <= mask;  // a digit value of this pass
        const int64_t hi = dig ? hist_index(tid, blockIdx.x, nb, seg, (int)mask + 1) : 0;
        const uint32_t h = dig ? hist[hi] : 0u;
        uint32_t incl = h;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t t = (uint32_t)__shfl_up((int)incl, d, 64);
            if (lane >= d) incl += t;
        }
        if (lane == 63) s_wsum[wave] = incl;
        s_gbase[tid] = dig ? offs[hi] : 0u;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) s_cnt[w][tid] = 0;
        __syncthreads();
        uint32_t before = 0;
        for (int w = 0; w < wave; ++w) before += s_wsum[w];
        s_dstart[tid] = before + incl - h;
    }
    __syncthreads();

    K key[kIt];
    uint32_t val[kIt], rank[kIt];
    const int64_t wbase = tile + (int64_t)wave * kPerWave;
    // all loads first (see sort_hist_kernel), then the ranking
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int64_t idx = wbase + it * 64 + lane;
        const int64_t ci = idx < n ? idx : 0;
        key[it] = kin[ci];
        val[it] = vin[ci];
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int64_t idx = wbase + it * 64 + lane;
        const bool valid = idx < n;
        const uint32_t digit = (uint32_t)(key[it] >> shift) & mask;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (digit >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
        uint32_t old = 0;
        if (valid) old = s_cnt[wave][digit];
        rank[it] = old + below;
        if (valid && below == 0) s_cnt[wave][digit] = old + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) {
            const uint32_t c = s_cnt[w][tid];
            s_cnt[w][tid] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int64_t idx = wbase + it * 64 + lane;
        if (idx < n) {
            const uint32_t digit = (uint32_t)(key[it] >> shift) & mask;
            const uint32_t pos = s_dstart[digit] + s_cnt[wave][digit] + rank[it];
            s_key[pos] = key[it];
            s_val[pos] = val[it];
        }
    }
    __syncthreads();
    const int cnt = (int)min((int64_t)kSortTile, n - tile);
    for (int p = tid; p < cnt; p += kSortBlock) {
        const K k = s_key[p];
        const uint32_t digit = (uint32_t)(k >> shift) & mask;
        const uint32_t g = s_gbase[digit] + ((uint32_t)p - s_dstart[digit]);
        kout[g] = k;
        vout[g] = s_val[p];
    }
}

static int64_t sort_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

size_t sort_temp_bytes(int64_t n)
{
    const int64_t nb = sort_tiles(n) > 0 ? sort_tiles(n) : 1;
    const int64_t nh = 256 * nb;
    // hist + offsets + scan temp
    return (size_t)(2 * nh * sizeof(uint32_t)) + scan_temp_bytes(nh) + 64;
}

template <typename K>
static hipError_t radix_sort_impl(K *k0, uint32_t *v0, K *k1, uint32_t *v1, int64_t n, int b0, int b1,
                                  void *temp, bool *in_alt, hipStream_t s, Timer *tm = nullptr,
                                  const uint64_t *dn = nullptr, int64_t seg = 0)
{
    *in_alt = false;
    if (n <= 1 || b1 <= b0) return hipSuccess;
    const int64_t nb = sort_tiles(n);
    const int64_t nh = 256 * nb;  // room for 8-bit digits; a pass with fewer uses its first part
    uint32_t *hist = (uint32_t *)temp;
    uint32_t *offs = hist + nh;
    void *stemp = (void *)(((uintptr_t)(offs + nh) + 63) & ~(uintptr_t)63);
    K *ki = k0, *ko = k1;
    uint32_t *vi = v0, *vo = v1;
    // as few passes of at most 8 bits as the range needs, the bits spread
    // evenly over them (fewer digit values per pass give longer runs of
    // consecutive output slots in the scatter)
    const int passes = (b1 - b0 + 7) / 8;
    const int step = (b1 - b0 + passes - 1) / passes;
    for (int shift = b0; shift < b1; shift += step) {
        const int bits = (b1 - shift) < step ? (b1 - shift) : step;
        const uint32_t mask = (1u << bits) - 1u;
        hipLaunchKernelGGL(sort_hist_kernel<K>, dim3((unsigned)nb), dim3(kSortBlock), 0, s, ki, n, dn, shift,
                           mask, hist, nb, seg);
        hipError_t e = launch_exclusive_scan(hist, offs, (int64_t)(mask + 1) * nb, stemp, nullptr, s);
        if (e != hipSuccess) return e;
        const size_t ea = tm ? tm->mark(s) : 0;
        hipLaunchKernelGGL(sort_scatter_kernel<K>, dim3((unsigned)nb), dim3(kSortBlock), 0, s, ki, vi, ko, vo, n,
                           dn, shift, mask, offs, hist, nb, seg);
        if (tm) tm->span(kStScatter, ea, tm->mark(s));
        K *tk = ki;
        ki = ko;
        ko = tk;
        uint32_t *tv = vi;
        vi = vo;
        vo = tv;
        *in_alt = !*in_alt;
    }
    return hipGetLastError();
}

hipError_t radix_sort_u32(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n, int b0, int b1,
                          void *temp, bool *in_alt, hipStream_t s, Timer *tm, const uint64_t *dn, int64_t seg_len)
{
    if (seg_len > 0 && (seg_len % kSortTile != 0 || n % seg_len != 0)) return hipErrorInvalidValue;
    return radix_sort_impl<uint32_t>(k0, v0, k1, v1, n, b0, b1, temp, in_alt, s, tm, dn,
                                     seg_len > 0 ? seg_len / kSortTile : 0);
}

hipError_t radix_sort_u64(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n, int b0, int b1,
                          void *temp, bool *in_alt, hipStream_t s, int64_t seg_len, Timer *tm, const uint64_t *dn)
{
    if (seg_len > 0 && (seg_len % kSortTile != 0 || n % seg_len != 0)) return hipErrorInvalidValue;
    return radix_sort_impl<uint64_t>(k0, v0, k1, v1, n, b0, b1, temp, in_alt, s, tm, dn,
                                     seg_len > 0 ? seg_len / kSortTile : 0);
}

int64_t sort_segment_granule() { return kSortTile; }

}  // namespace lfr
