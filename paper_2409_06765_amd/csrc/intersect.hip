// Tile binning, key emission, stable LSD radix sort and tile ranges
// (Rasterization of Gaussians: 16x16 tiles, per-tile depth order).
//
// Two ways to the same per-tile lists:
//  * the general one: (tile << 32 | depth bits, id) pairs emitted in
//    (camera, Gaussian, row-major tile) order, stably radix-sorted on all
//    key bits;
//  * the binning path used by the pipeline: the projected Gaussians are
//    first stably sorted by depth bits (C*N 32-bit keys; the first pass
//    also drops the Gaussians of no tiles, so the later passes and
//    everything after them see only the visible ones), their binning records
//    (what the emission reads of a Gaussian, its tile count included) are
//    gathered into that order in one pass, their tiles are then
//    emitted in that order with 32-bit tile keys (each emit block also
//    counts the first tile-bit digits of its slots, the histogram the sort's
//    first pass needs), and a stable sort on the tile bits alone (two passes
//    at 1080p) finishes the job.  Stability makes the result (tile, depth
//    bits, id) order, identical bit for bit.
// Prefix sums and sorts use reduce-then-scan (no inter-block waiting), so
// every kernel finishes whatever the order in which blocks are scheduled.
#include <algorithm>
#include <mutex>

#include "common.hpp"

#pragma clang fp contract(off)

namespace gsr {
namespace {

// Keys equal to kDropKey (all ones, 32-bit keys) are left out of a sort pass
// run with drop set: the pass then also compacts, writing only the other pairs.
constexpr uint32_t kDropKey = 0xFFFFFFFFu;

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;   // elements per block

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T u = __shfl_up(v, d, kWave);
        if (lane >= d) v += u;
    }
    return v;
}

// Exclusive scan over a block of kScanThreads threads; returns the block total.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T &total) {
    __shared__ T wsum[kScanThreads / kWave];
    const int lane = __lane_id(), w = threadIdx.x / kWave;
    T inc = wave_inclusive_scan(v);
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    T before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kScanThreads / kWave; i++) {
        if (i < w) before += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    total = tot;
    return before + inc - v;
}

__device__ __forceinline__ int tile_count(const CamTable &cams, int N, int64_t g, const float *means2d,
                                          const int32_t *radii) {
    const int r = radii[g];
    if (r <= 0) return 0;
    const int c = (int)(g / N);
    int x0, x1, y0, y1;
    tile_rect(means2d[2 * g], means2d[2 * g + 1], r, cams.cam[c].TX, cams.cam[c].TY, x0, x1, y0, y1);
    return (x1 > x0 && y1 > y0) ? (x1 - x0) * (y1 - y0) : 0;
}

// What the binning needs to cull tiles (params tile_cull): the conics and the
// opacities the compositing kernels use (opacity times compensation when
// antialiased); on = 0 keeps whole rectangles.
struct CullIn {
    const float *conics;
    const float *opacities;
    const float *comps;
    float alpha_min;
    int on;
};

// The tile rectangle of projected Gaussian g (camera c) and its culling rule.
struct GaussTiles {
    int x0, x1, y0, y1;
    TileCull cull;
};

__device__ __forceinline__ GaussTiles gauss_tiles(const CamTable &cams, int N, int64_t g, const float *means2d,
                                                  const int32_t *radii, const CullIn &ci) {
    GaussTiles t;
    t.x0 = t.x1 = t.y0 = t.y1 = 0;
    t.cull.mode = 1;
    const int r = radii[g];
    if (r <= 0) return t;
    const int c = (int)(g / N);
    const float mx = means2d[2 * g], my = means2d[2 * g + 1];
    tile_rect(mx, my, r, cams.cam[c].TX, cams.cam[c].TY, t.x0, t.x1, t.y0, t.y1);
    if (!(t.x1 > t.x0 && t.y1 > t.y0)) { t.x1 = t.x0; t.y1 = t.y0; return t; }
    if (ci.on) {
        float o = ci.opacities[g % N];
        if (ci.comps) o *= ci.comps[g];
        t.cull = tile_cull_setup(mx, my, ci.conics[3 * g], ci.conics[3 * g + 1], ci.conics[3 * g + 2], o, ci.alpha_min, r);
    }
    return t;
}

// What the key emission needs of a projected Gaussian with tiles, packed by
// bin_keys_kernel into one 32-byte record, which gather_recs_kernel moves
// into depth order (the order the emission visits the Gaussians in) together
// with the tile count it holds: {mean x, mean y, conic a, conic b},
// {conic c, opacity (times the compensation), radius (int bits), tiles (int bits)}.
struct BinRec {
    float4 a;
    float4 b;
};

__device__ __forceinline__ GaussTiles gauss_tiles_rec(const CamTable &cams, int N, int64_t g, const BinRec &r,
                                                      const CullIn &ci) {
    GaussTiles t;
    t.x0 = t.x1 = t.y0 = t.y1 = 0;
    t.cull.mode = 1;
    const int rad = __float_as_int(r.b.z);
    if (rad <= 0) return t;
    const int c = (int)(g / N);
    tile_rect(r.a.x, r.a.y, rad, cams.cam[c].TX, cams.cam[c].TY, t.x0, t.x1, t.y0, t.y1);
    if (!(t.x1 > t.x0 && t.y1 > t.y0)) { t.x1 = t.x0; t.y1 = t.y0; return t; }
    if (ci.on) t.cull = tile_cull_setup(r.a.x, r.a.y, r.a.z, r.a.w, r.b.x, r.b.y, ci.alpha_min, rad);
    return t;
}

// Tiles of a Gaussian: the rectangle's area, or the sum of its rows' runs.
__device__ __forceinline__ int gauss_tile_count(const GaussTiles &t) {
    if (t.cull.mode == 1) return (t.x1 - t.x0) * (t.y1 - t.y0);
    int n = 0;
#pragma clang loop unroll(disable) vectorize(disable) interleave(disable)
    for (int ty = t.y0; ty < t.y1; ty++) {
        int xa, xb;
        tile_cull_row(t.cull, ty, t.x0, t.x1, xa, xb);
        n += xb - xa;
    }
    return n;
}

// First row at or after ty with a non-empty run (t.y1 if none) and its run.
__device__ __forceinline__ int next_row(const GaussTiles &t, int ty, int &xa, int &xb) {
#pragma clang loop unroll(disable) vectorize(disable) interleave(disable)
    for (; ty < t.y1; ty++) {
        tile_cull_row(t.cull, ty, t.x0, t.x1, xa, xb);
        if (xb > xa) return ty;
    }
    xa = xb = t.x0;
    return t.y1;
}

// ---- prefix sums ----------------------------------------------------------
// Tiles per Gaussian and per-block sums.
__global__ void __launch_bounds__(kScanThreads) count_kernel(CamTable cams, int N, int64_t n_total,
        const float *__restrict__ means2d, const int32_t *__restrict__ radii, int32_t *__restrict__ counts,
        int64_t *__restrict__ block_sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t local = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        const int64_t g = base + i;
        if (g < n_total) {
            const int k = tile_count(cams, N, g, means2d, radii);
            counts[g] = k;
            local += k;
        }
    }
    int64_t total;
    block_exclusive_scan<int64_t>(local, total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// Per-block sums of an int32 array.
__global__ void __launch_bounds__(kScanThreads) block_sums_kernel(int64_t n_total, const int32_t *__restrict__ vals,
                                                                  int64_t *__restrict__ block_sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t local = 0;
    if (base + kScanItems <= n_total) {          // one 16-byte load (base is a multiple of 4)
        const int4 q = *reinterpret_cast<const int4 *>(vals + base);
        local = ((int64_t)q.x + q.y) + ((int64_t)q.z + q.w);
    } else {
#pragma unroll
        for (int i = 0; i < kScanItems; i++)
            if (base + i < n_total) local += vals[base + i];
    }
    int64_t total;
    block_exclusive_scan<int64_t>(local, total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// The emission records gathered into depth order (recs_sorted[i] =
// recs[order[i]]), their tile counts (kept in the record) as counts_sorted,
// and the per-block sums of those counts, in one pass: the one random read of
// the binning path, after which the emission reads its records in order.
// Positions at or past *n_kept (the Gaussians the depth order kept) become
// entries of no tiles, their order set to Gaussian 0 (their records are not
// read); Gaussians of no tiles inside it (the one-block sort keeps them) carry
// records of count 0.
__global__ void __launch_bounds__(kScanThreads) gather_recs_kernel(int64_t n_total,
        const int64_t *__restrict__ n_kept, int32_t *__restrict__ order, const BinRec *__restrict__ recs,
        BinRec *__restrict__ recs_sorted, int32_t *__restrict__ counts_sorted, int64_t *__restrict__ block_sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
    const int64_t kept = min(n_total, *n_kept);
    int64_t local = 0;
    // the loads first (clamped to slot 0 past the end, which always exists), then the rest
    int32_t gs[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        const int64_t j = base + (int64_t)i * kScanThreads;
        const int32_t g = order[j < kept ? j : 0];
        gs[i] = (g >= 0 && g < n_total) ? g : -1;
    }
    BinRec rs[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; i++) rs[i] = recs[gs[i] >= 0 ? gs[i] : 0];
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        const int64_t j = base + (int64_t)i * kScanThreads;   // block sums only: any split of the block's slots
        if (j < kept) {
            BinRec r = rs[i];
            if (gs[i] < 0) {                     // radius 0, count 0: a bad order entry emits nothing
                r.a = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                r.b = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
            recs_sorted[j] = r;
            const int32_t c = __float_as_int(r.b.w);
            counts_sorted[j] = c;
            local += c;
        } else if (j < n_total) {
            order[j] = 0;
            counts_sorted[j] = 0;
        }
    }
    int64_t total;
    block_exclusive_scan<int64_t>(local, total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// One block turns the block sums into exclusive block offsets, kSumItems
// consecutive sums per thread per round (one round up to 4,096 sums).
constexpr int kSumItems = 16;

__global__ void __launch_bounds__(kScanThreads) scan_sums_kernel(int64_t *__restrict__ sums, int64_t nb,
                                                                 int64_t *__restrict__ total_out,
                                                                 int64_t *__restrict__ total_copy) {
    int64_t carry = 0;
    for (int64_t start = 0; start < nb; start += (int64_t)kScanThreads * kSumItems) {
        const int64_t i0 = start + (int64_t)threadIdx.x * kSumItems;
        int64_t v[kSumItems], local = 0;
#pragma unroll
        for (int k = 0; k < kSumItems; k++) {
            v[k] = i0 + k < nb ? sums[i0 + k] : 0;
            local += v[k];
        }
        int64_t tot;
        int64_t run = carry + block_exclusive_scan<int64_t>(local, tot);
#pragma unroll
        for (int k = 0; k < kSumItems; k++) {
            if (i0 + k < nb) sums[i0 + k] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) {
        *total_out = carry;
        if (total_copy) *total_copy = carry;
    }
}

// Per-element exclusive offsets.
__global__ void __launch_bounds__(kScanThreads) offsets_kernel(int64_t n_total, const int32_t *__restrict__ counts,
        const int64_t *__restrict__ block_off, int64_t *__restrict__ offsets) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    if (base + kScanItems <= n_total) {          // one 16-byte load (base is a multiple of 4)
        const int4 q = *reinterpret_cast<const int4 *>(counts + base);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
#pragma unroll
        for (int i = 0; i < kScanItems; i++) v[i] = (base + i < n_total) ? counts[base + i] : 0;
    }
    int64_t local = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) local += v[i];
    int64_t total;
    int64_t run = block_exclusive_scan<int64_t>(local, total) + block_off[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        if (base + i < n_total) offsets[base + i] = run;
        run += v[i];
    }
}

// ---- key emission ------------------------------------------------------------
// The output is cut into fixed slices of kEmitChunk entries, one slice per
// wave, so the work per wave is bounded whatever the tile counts are (a few
// Gaussians covering thousands of tiles, clustered in depth order, would
// otherwise keep single waves busy long after the rest finished).  A wave
// finds the entry owning its first slot with a 64-way search over the
// exclusive offsets, then walks windows of consecutive entries of the
// emission sequence (projected Gaussians in id order, or in depth order when
// `order` is given).  Each lane takes one entry and writes the runs of its
// tile rows (whole rectangle rows, or the culled runs) into an LDS table of
// up to kEmitRows rows: slot of the run's first tile, that tile, run length,
// entry.  An entry with more rows than fit is continued in the next window.
// The culling records, when given, are in emission order (recs[q] for entry q).
// Then each lane writes a run of at most 8 consecutive slots of the wave's
// slice, finding its row by binary search over the table.  The slice is
// staged in LDS and written out coalesced.  Keys are tile << 32 | depth bits
// (uint64) or the tile id alone (uint32).
constexpr int kEmitThreads = 256;
constexpr int kBinsEmit = 256;      // the radix sort's digit bins (one per thread of an emit block)
constexpr int kEmitChunk = 512;
constexpr int kEmitRows = 256;

template <typename K>
__device__ __forceinline__ K make_key(uint32_t tile, uint32_t dbits);
template <>
__device__ __forceinline__ uint64_t make_key<uint64_t>(uint32_t tile, uint32_t dbits) {
    return ((uint64_t)tile << 32) | (uint64_t)dbits;
}
template <>
__device__ __forceinline__ uint32_t make_key<uint32_t>(uint32_t tile, uint32_t) { return tile; }

// Largest s in [0, n) with offsets[s] <= pos (offsets non-decreasing, offsets[0] = 0 <= pos);
// wave-cooperative: every lane returns the same value.
__device__ __forceinline__ int64_t owner_search(const int64_t *__restrict__ offsets, int64_t n, int64_t pos) {
    const int lane = __lane_id();
    int64_t lo = 0, hi = n;                    // answer in [lo, hi)
    while (hi - lo > 1) {
        const int64_t step = (hi - lo + kWave - 1) / kWave;
        const int64_t q = lo + (int64_t)lane * step;
        const bool le = q < hi && offsets[q] <= pos;
        const uint64_t m = __ballot(le);       // lane 0 is always set: offsets[lo] <= pos
        const int L = 63 - __builtin_clzll(m);
        lo = lo + (int64_t)L * step;
        hi = min(lo + step, hi);
    }
    return lo;
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename K>
__global__ void __launch_bounds__(kEmitThreads) emit_kernel(CamTable cams, int N, int64_t n_total,
        const float *__restrict__ means2d, const int32_t *__restrict__ radii, const float *__restrict__ depths,
        CullIn cull, const int32_t *__restrict__ order, const int64_t *__restrict__ offsets, int64_t cap,
        const int64_t *__restrict__ count_dev, K *__restrict__ keys, int32_t *__restrict__ ids,
        int32_t *__restrict__ hist, int hist_bits, int hist_stride, const BinRec *__restrict__ recs) {
    constexpr int kWaves = kEmitThreads / kWave;
    const int64_t total = count_dev ? *count_dev : cap;   // end of the last entry
    cap = min(cap, total);                       // capacity mode: the true count lives on the device
    __shared__ int32_t s_rslot[kWaves][kEmitRows];   // slot of the row run's first tile, from the window start
    __shared__ int32_t s_rtile[kWaves][kEmitRows];   // that tile
    __shared__ uint8_t s_rent[kWaves][kEmitRows];    // entry (lane) of the row
    __shared__ uint32_t s_dbits[kWaves][kWave];
    __shared__ int32_t s_g[kWaves][kWave];
    __shared__ K s_okey[kWaves][kEmitChunk];     // the wave's slice, written out coalesced at the end
    __shared__ int32_t s_oid[kWaves][kEmitChunk];
    const int lane = __lane_id(), w = threadIdx.x / kWave;
    const int64_t c0 = ((int64_t)blockIdx.x * kWaves + w) * kEmitChunk;
    const bool active = c0 < cap;                // wave-uniform
    const int64_t c1 = min(c0 + (int64_t)kEmitChunk, cap);
    if (active) {
    int64_t s = owner_search(offsets, n_total, c0);
    int r0 = 0;                                  // rows of entry s emitted by earlier windows
    int64_t so = 0;                              // and their slots
    while (s < n_total) {
        // ---- the window: lane i takes entry s + i, from row r0 for lane 0
        const int64_t q = s + lane;
        int64_t g = 0, start = 0;
        GaussTiles t;
        t.x0 = t.x1 = t.y0 = t.y1 = 0;
        t.cull.mode = 1;
        int nr = 0, base = 0, TX = 0;
        // the window's loads first, from in-bounds positions (the last entry past the end), so that they
        // are in flight together
        const int64_t qc = min(q, n_total - 1);
        const int64_t g_ld = order ? (int64_t)order[qc] : qc;
        const int64_t off_q = offsets[qc];
        const int64_t off_n = offsets[min(qc + 1, n_total - 1)];
        BinRec rq;
        if (recs) rq = recs[qc];
        if (q < n_total) {
            g = g_ld;
            if (g < 0 || g >= n_total) g = 0;    // order comes from the depth sort; this only bounds a bad input
            start = off_q + (lane == 0 ? so : 0);
            const int64_t end = q + 1 < n_total ? off_n : total;
            if (end > start) {
                t = recs ? gauss_tiles_rec(cams, N, g, rq, cull) : gauss_tiles(cams, N, g, means2d, radii, cull);
                nr = t.y1 - t.y0 - (lane == 0 ? r0 : 0);
                base = cams.cam[g / N].tile_base;
                TX = cams.cam[g / N].TX;
            }
            if constexpr (sizeof(K) == 8) s_dbits[w][lane] = __float_as_uint(depths[g]);   // 32-bit keys: tile only
            s_g[w][lane] = (int32_t)g;
        }
        const int ry0 = t.y0 + (lane == 0 ? r0 : 0);   // first row of this lane's entry in the table
        // rows of the lanes before this one; lanes that fit whole, and a partial last one
        int rb = nr;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int u = __shfl_up(rb, d, kWave);
            if (lane >= d) rb += u;
        }
        rb -= nr;
        const int nfit = __popcll(__ballot(q < n_total && rb + nr <= kEmitRows));   // a prefix of the lanes
        const int take = lane < nfit ? nr : (lane == nfit ? max(0, min(nr, kEmitRows - rb)) : 0);
        const int nrows = __shfl(rb + take, min(nfit, kWave - 1), kWave);
        // ---- the table's rows, four consecutive ones per lane: owner entry, tile run, length.  Each lane
        // first marks its own rows with its lane index, so a row finds its owner with one LDS read
        for (int r = 0; r < take; r++) s_rent[w][rb + r] = (uint8_t)lane;
        wave_sync_lds();
        constexpr int kPer = kEmitRows / kWave;
        int len[kPer], tile[kPer], own[kPer];
#pragma unroll
        for (int k = 0; k < kPer; k++) {
            const int i = lane * kPer + k;
            const int lo = i < nrows ? (int)s_rent[w][i] : 0;
            own[k] = lo;
            GaussTiles ot;
            ot.x0 = __shfl(t.x0, lo, kWave);
            ot.x1 = __shfl(t.x1, lo, kWave);
            ot.cull.mode = __shfl(t.cull.mode, lo, kWave);
            ot.cull.mx = __shfl(t.cull.mx, lo, kWave);
            ot.cull.my = __shfl(t.cull.my, lo, kWave);
            ot.cull.B = __shfl(t.cull.B, lo, kWave);
            ot.cull.det = __shfl(t.cull.det, lo, kWave);
            ot.cull.L4A = __shfl(t.cull.L4A, lo, kWave);
            ot.cull.vmax = __shfl(t.cull.vmax, lo, kWave);
            ot.cull.vr = __shfl(t.cull.vr, lo, kWave);
            ot.cull.inv2A = __shfl(t.cull.inv2A, lo, kWave);
            ot.cull.su = __shfl(t.cull.su, lo, kWave);
            const int ty = __shfl(ry0, lo, kWave) + (i - __shfl(rb, lo, kWave));
            int xa = ot.x0, xb = ot.x0;
            if (i < nrows) tile_cull_row(ot.cull, ty, ot.x0, ot.x1, xa, xb);
            len[k] = xb - xa;
            tile[k] = __shfl(base, lo, kWave) + ty * __shfl(TX, lo, kWave) + xa;
        }
        // slots of the rows: the window's first slot plus the lengths of the rows before
        int sum = 0;
#pragma unroll
        for (int k = 0; k < kPer; k++) sum += len[k];
        int ex = sum;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int u = __shfl_up(ex, d, kWave);
            if (lane >= d) ex += u;
        }
        const int wlen = __shfl(ex, kWave - 1, kWave);   // slots of the window
        ex -= sum;
        const int64_t wbeg = __shfl(start, 0, kWave);
        const int64_t wend = wbeg + wlen;
#pragma unroll
        for (int k = 0; k < kPer; k++) {
            const int i = lane * kPer + k;
            if (i < nrows) {
                s_rslot[w][i] = (int32_t)(wbeg - c0) + ex;     // may be negative: rows before the slice
                s_rtile[w][i] = tile[k];
            }
            ex += len[k];
        }
        const bool partial = nfit < kWave && s + nfit < n_total;   // lane nfit stopped inside its entry (or at 0 rows)
        const int taken = partial ? __shfl(take, nfit, kWave) : 0;
        wave_sync_lds();
        // ---- write the slice's slots of this window
        const int64_t p0 = max(c0, wbeg), p1 = min(c1, wend);
        if (p0 < p1) {
            const int run = (int)((p1 - p0 + kWave - 1) / kWave);
            int64_t pos = p0 + (int64_t)lane * run;
            const int64_t pend = min(pos + run, p1);
            if (pos < pend) {
                int rel = (int)(pos - c0);
                int lo = 0, hi = nrows - 1;      // the last row whose first slot is <= rel
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_rslot[w][mid] <= rel) lo = mid; else hi = mid - 1;
                }
#pragma clang loop unroll(disable) vectorize(disable) interleave(disable)
                for (; pos < pend; pos++, rel++) {
                    while (lo + 1 < nrows && s_rslot[w][lo + 1] <= rel) lo++;
                    const int e = s_rent[w][lo];
                    s_okey[w][rel] = make_key<K>((uint32_t)(s_rtile[w][lo] + (rel - s_rslot[w][lo])), s_dbits[w][e]);
                    s_oid[w][rel] = s_g[w][e];
                }
            }
        }
        if (wend >= c1) break;
        // the next window
        if (partial && nfit == 0) {              // lane 0's entry continues
            r0 += taken;
            so = wend - offsets[s];
        } else if (partial) {
            s += nfit;
            r0 = taken;
            so = wend - offsets[s];
        } else {
            s += kWave;
            r0 = 0;
            so = 0;
        }
        wave_sync_lds();                         // the window's LDS is rewritten next
    }
    wave_sync_lds();
    const int n_out = (int)(c1 - c0);             // every slot of [c0, c1) was written above
    for (int i = lane; i < n_out; i += kWave) {
        keys[c0 + i] = s_okey[w][i];
        ids[c0 + i] = s_oid[w][i];
    }
    }
    if (hist) {
        // the block's slots are one tile of the radix sort that follows: its histogram of the first
        // pass's digits (the low hist_bits bits), as radix_hist_kernel would count them
        __shared__ int32_t s_hist[kBinsEmit];
        s_hist[threadIdx.x] = 0;
        __syncthreads();
        if (active) {
            const uint32_t mask = (1u << hist_bits) - 1u;
            for (int i = lane; i < (int)(c1 - c0); i += kWave) atomicAdd(&s_hist[(uint32_t)s_okey[w][i] & mask], 1);
        }
        __syncthreads();
        if ((int)threadIdx.x < (1 << hist_bits)) hist[(int64_t)threadIdx.x * hist_stride + blockIdx.x] = s_hist[threadIdx.x];
    }
}

int64_t emit_blocks(int64_t cap) {
    const int64_t per_block = (int64_t)kEmitChunk * (kEmitThreads / kWave);
    return (cap + per_block - 1) / per_block;
}

__global__ void fill_zero_kernel(uint32_t *__restrict__ p, int64_t n_words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Up to kFillMax buffers zeroed by one launch: blockIdx.y picks the buffer.
constexpr int kFillMax = 8;
struct FillList {
    uint32_t *p[kFillMax];
    int64_t words[kFillMax];
};

__global__ void fill_zero_multi_kernel(FillList f) {
    const int b = blockIdx.y;
    uint32_t *p = f.p[b];
    const int64_t n = f.words[b];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

template <typename K>
__device__ __forceinline__ int32_t tile_of(K key) { return (int32_t)(sizeof(K) == 8 ? (uint64_t)key >> 32 : key); }

// Each thread takes kRangeItems consecutive keys (and the one on each side).
constexpr int kRangeItems = 8;

template <typename K>
__global__ void __launch_bounds__(256) ranges_kernel(int64_t M, const int64_t *__restrict__ count_dev,
                                                     const K *__restrict__ keys, int32_t total_tiles,
                                                     int32_t *__restrict__ ranges) {
    if (count_dev) M = min(M, *count_dev);
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRangeItems;
    if (i0 >= M) return;
    int32_t t[kRangeItems + 2];
    bool loaded = false;
    if constexpr (sizeof(K) == 4) {
        static_assert(kRangeItems == 8, "two 16-byte loads of 32-bit keys");
        if (i0 + kRangeItems <= M) {   // i0 is a multiple of 8 and the key buffer 256-byte aligned
            const uint4 *q = reinterpret_cast<const uint4 *>(keys + i0);
            const uint4 lo = q[0], hi = q[1];
            t[1] = (int32_t)lo.x; t[2] = (int32_t)lo.y; t[3] = (int32_t)lo.z; t[4] = (int32_t)lo.w;
            t[5] = (int32_t)hi.x; t[6] = (int32_t)hi.y; t[7] = (int32_t)hi.z; t[8] = (int32_t)hi.w;
            t[0] = i0 > 0 ? tile_of<K>(keys[i0 - 1]) : -1;
            t[kRangeItems + 1] = i0 + kRangeItems < M ? tile_of<K>(keys[i0 + kRangeItems]) : -1;
            loaded = true;
        }
    }
    if (!loaded) {
#pragma unroll
        for (int k = 0; k < kRangeItems + 2; k++) {
            const int64_t i = i0 - 1 + k;
            t[k] = (i >= 0 && i < M) ? tile_of<K>(keys[i]) : -1;
        }
    }
#pragma unroll
    for (int k = 1; k <= kRangeItems; k++) {
        const int64_t i = i0 - 1 + k;
        const int32_t tk = t[k];
        if (i >= M || tk < 0 || tk >= total_tiles) continue;
        if (t[k - 1] != tk) ranges[2 * tk] = (int32_t)i;
        if (t[k + 1] != tk) ranges[2 * tk + 1] = (int32_t)(i + 1);
    }
}

int64_t range_blocks(int64_t M) { return (M + 256 * kRangeItems - 1) / (256 * kRangeItems); }

// ---- binning-path helpers -------------------------------------------------------
// Depth-sort keys of the projected Gaussians and their emission records (tile
// count included); a Gaussian of no tiles gets kDropKey, which the first sort
// pass leaves out (the one-block sort keeps it, last), and a record of count 0
// whose other fields are not read.
__global__ void __launch_bounds__(256) bin_keys_kernel(CamTable cams, int N, int64_t n_total,
        const float *__restrict__ means2d, const int32_t *__restrict__ radii, const float *__restrict__ depths,
        CullIn cull, uint32_t *__restrict__ dkeys, BinRec *__restrict__ recs) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_total) return;
    // every input of the Gaussian loaded up front (all in bounds), then the tiles from the record
    const int rad = radii[g];
    const float mx = means2d[2 * g], my = means2d[2 * g + 1], dep = depths[g];
    float o = 0.0f, ca = 0.0f, cb = 0.0f, cc = 0.0f;
    if (cull.on) {
        o = cull.opacities[g % N];
        if (cull.comps) o *= cull.comps[g];
        ca = cull.conics[3 * g]; cb = cull.conics[3 * g + 1]; cc = cull.conics[3 * g + 2];
    }
    BinRec r;
    r.a = make_float4(mx, my, ca, cb);
    r.b = make_float4(cc, o, __int_as_float(rad), 0.0f);
    const int k = gauss_tile_count(gauss_tiles_rec(cams, N, g, r, cull));
    dkeys[g] = k > 0 ? __float_as_uint(dep) : kDropKey;
    if (k > 0) {
        r.b.w = __int_as_float(k);
        recs[g] = r;
    } else {
        recs[g].b.w = __int_as_float(0);
    }
}

// 64-bit keys of the sorted lists (only when a caller asks for them).
__global__ void __launch_bounds__(256) keys64_kernel(int64_t M, const int64_t *__restrict__ count_dev,
                                                     const uint32_t *__restrict__ tkeys,
                                                     const int32_t *__restrict__ ids, const float *__restrict__ depths,
                                                     int64_t n_total, uint64_t *__restrict__ keys) {
    if (count_dev) M = min(M, *count_dev);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int32_t g = ids[i];
    const uint32_t db = (g >= 0 && g < n_total) ? __float_as_uint(depths[g]) : 0u;
    keys[i] = ((uint64_t)tkeys[i] << 32) | db;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (uint64 or uint32 key, int32 id), up to 8 bits per
// pass (an even number of passes; where the bits do not split evenly the low
// passes take the narrower digits).  Per pass: (1) per-block digit histograms
// (LDS atomics), stored digit-major;
// (2) one block per digit scans its row over the blocks; (3) each block
// ranks its elements stably (wave-level match on the digit bits, then wave
// and block prefixes), reorders them in LDS and writes digit runs out.
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kBins = 256;

// Lanes (among `active`) holding the same digit as this lane.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t active) {
    uint64_t m = active;
#pragma unroll
    for (int b = 0; b < 8; b++) {   // all eight bits: a narrower digit's upper bits are 0 in every lane
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        m &= bit ? bal : ~bal;
    }
    return m;
}


template <typename K>
__global__ void __launch_bounds__(kSortThreads) radix_hist_kernel(const K *__restrict__ keys, int64_t M,
        const int64_t *__restrict__ count_dev, int shift, int bits, int nblocks, int stride,
        int32_t *__restrict__ hist, int drop) {
    __shared__ int32_t cnt[kBins];
    if (count_dev) M = min(M, *count_dev);      // blocks past the count write zero histograms
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t mask = (1u << bits) - 1u;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    // every load first, from in-bounds positions (slot 0 past the count; the buffers hold at least one
    // pair), so that a wave has all its loads in flight at once; then the counts
    const int64_t last = M > 0 ? M - 1 : 0;
    K kv[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; i++) kv[i] = keys[min(base + (int64_t)i * kSortThreads + threadIdx.x, last)];
#pragma unroll
    for (int i = 0; i < kSortItems; i++) {
        const int64_t idx = base + (int64_t)i * kSortThreads + threadIdx.x;
        const bool valid = idx < M && !(drop && (uint64_t)kv[i] == kDropKey);
        if (valid) atomicAdd(&cnt[(uint32_t)(kv[i] >> shift) & mask], 1);   // counts need no order: LDS atomics
    }
    __syncthreads();
    if (threadIdx.x < (1 << bits)) hist[(int64_t)threadIdx.x * stride + blockIdx.x] = cnt[threadIdx.x];
}

// One block per digit: exclusive scan of hist[d][0..nblocks) in place; the
// row total goes to digit_tot[d].  Rows are `stride` entries apart (a
// multiple of 4, so they are read and written as int4), and each thread
// takes kRowItems consecutive entries per round: a row of a few thousand
// blocks takes one or two rounds of a block scan.
constexpr int kRowItems = 16;

__global__ void __launch_bounds__(kScanThreads) radix_rowscan_kernel(int32_t *__restrict__ hist, int nblocks,
                                                                     int stride, int32_t *__restrict__ digit_tot) {
    int32_t *row = hist + (int64_t)blockIdx.x * stride;
    int32_t carry = 0;
    for (int start = 0; start < nblocks; start += kScanThreads * kRowItems) {
        const int base = start + (int)threadIdx.x * kRowItems;
        int32_t v[kRowItems];
        int32_t local = 0;
#pragma unroll
        for (int i = 0; i < kRowItems; i += 4) {
            int4 q = make_int4(0, 0, 0, 0);
            if (base + i < stride) q = *reinterpret_cast<const int4 *>(row + base + i);
            v[i] = base + i < nblocks ? q.x : 0;
            v[i + 1] = base + i + 1 < nblocks ? q.y : 0;
            v[i + 2] = base + i + 2 < nblocks ? q.z : 0;
            v[i + 3] = base + i + 3 < nblocks ? q.w : 0;
            local += (v[i] + v[i + 1]) + (v[i + 2] + v[i + 3]);
        }
        int32_t tot;
        int32_t run = carry + block_exclusive_scan<int32_t>(local, tot);
#pragma unroll
        for (int i = 0; i < kRowItems; i += 4) {
            int4 q;
            q.x = run; run += v[i];
            q.y = run; run += v[i + 1];
            q.z = run; run += v[i + 2];
            q.w = run; run += v[i + 3];
            if (base + i < stride) *reinterpret_cast<int4 *>(row + base + i) = q;
        }
        carry += tot;
    }
    if (threadIdx.x == 0) digit_tot[blockIdx.x] = carry;
}

// ids_in NULL: the ids are the input positions.  drop: pairs with kDropKey
// are left out, and block 0 writes the number of pairs kept to kept_out.
template <typename K>
__global__ void __launch_bounds__(kSortThreads) radix_scatter_kernel(const K *__restrict__ keys_in,
        const int32_t *__restrict__ ids_in, K *__restrict__ keys_out, int32_t *__restrict__ ids_out,
        int64_t M, const int64_t *__restrict__ count_dev, int shift, int bits, int nblocks, int stride,
        const int32_t *__restrict__ hist, const int32_t *__restrict__ digit_tot, int drop,
        int64_t *__restrict__ kept_out) {
    if (count_dev) M = min(M, *count_dev);
    __shared__ K s_keys[kSortTile];
    __shared__ int32_t s_ids[kSortTile];
    __shared__ int32_t s_wcnt[kSortWaves][kBins];
    __shared__ int32_t s_dstart[kBins];
    __shared__ int32_t s_gout[kBins];
    __shared__ int32_t s_nkept;
    const int t = threadIdx.x, lane = __lane_id(), w = t / kWave;
    const uint32_t mask = (1u << bits) - 1u;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;

    // global start of each digit's run for this block (digits past 2^bits never occur)
    {
        const bool used = t < (1 << bits);
        int32_t tot;
        const int32_t before = block_exclusive_scan<int32_t>(used ? digit_tot[t] : 0, tot);
        s_gout[t] = before + (used ? hist[(int64_t)t * stride + blockIdx.x] : 0);
        if (kept_out && blockIdx.x == 0 && t == 0) *kept_out = tot;
    }
#pragma unroll
    for (int k = 0; k < kSortWaves; k++) s_wcnt[k][t] = 0;
    __syncthreads();

    // load, wave-striped: wave w owns [w*64*ITEMS, (w+1)*64*ITEMS) of the tile
    K key[kSortItems];
    int32_t val[kSortItems];
    int32_t rank[kSortItems];
    const uint64_t lt = lanemask_lt();
    // every load first, from in-bounds positions (as in radix_hist_kernel), then the ranking
    const int64_t last = M > 0 ? M - 1 : 0;
#pragma unroll
    for (int i = 0; i < kSortItems; i++) {
        const int64_t idx = min(base + (int64_t)w * (kWave * kSortItems) + i * kWave + lane, last);
        key[i] = keys_in[idx];
        val[i] = ids_in ? ids_in[idx] : (int32_t)idx;
    }
#pragma unroll
    for (int i = 0; i < kSortItems; i++) {
        const int64_t idx = base + (int64_t)w * (kWave * kSortItems) + i * kWave + lane;
        const bool valid = idx < M && !(drop && (uint64_t)key[i] == kDropKey);
        if (!valid) val[i] = 0;
        const uint32_t d = (uint32_t)(key[i] >> shift) & mask;
        const uint64_t active = __ballot(valid);
        const uint64_t peers = match_digit(d, active);
        rank[i] = -1;
        if (valid) {
            const int32_t before = s_wcnt[w][d];
            rank[i] = before + (int32_t)__popcll(peers & lt);
            if ((peers & lt) == 0) s_wcnt[w][d] = before + (int32_t)__popcll(peers);
        }
    }
    __syncthreads();
    // per digit: exclusive prefix over the waves, then over the digits
    {
        int32_t c[kSortWaves], run = 0;
#pragma unroll
        for (int k = 0; k < kSortWaves; k++) { c[k] = s_wcnt[k][t]; s_wcnt[k][t] = run; run += c[k]; }
        int32_t tot;
        s_dstart[t] = block_exclusive_scan<int32_t>(run, tot);
        if (t == 0) s_nkept = tot;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kSortItems; i++) {
        if (rank[i] >= 0) {
            const uint32_t d = (uint32_t)(key[i] >> shift) & mask;
            const int pos = s_dstart[d] + s_wcnt[w][d] + rank[i];
            if (pos >= 0 && pos < kSortTile) {   // always true; keeps a ranking bug from writing out of bounds
                s_keys[pos] = key[i];
                s_ids[pos] = val[i];
            }
        }
    }
    __syncthreads();
    const int n_valid = s_nkept;                 // pairs of this block kept (0 past the count)
    for (int j = t; j < n_valid; j += kSortThreads) {
        const K k = s_keys[j];
        const uint32_t d = (uint32_t)(k >> shift) & mask;
        const int64_t gpos = (int64_t)s_gout[d] + (j - s_dstart[d]);
        if (gpos >= 0 && gpos < M) {
            keys_out[gpos] = k;
            ids_out[gpos] = s_ids[j];
        }
    }
}

// Small inputs (up to kSmallSort pairs of 32-bit keys): every pass in one block, the pairs in
// LDS between passes, the same stable ranking as radix_scatter_kernel (wave-striped positions,
// per-wave digit counts, prefix over waves then digits), so one launch replaces three per pass.
constexpr int kSmallThreads = 1024;
constexpr int kSmallItems = 16;
constexpr int kSmallSort = kSmallThreads * kSmallItems;
constexpr int kSmallWaves = kSmallThreads / kWave;

__global__ void __launch_bounds__(kSmallThreads) radix_sort_small_kernel(uint32_t *__restrict__ keys,
                                                                         int32_t *__restrict__ ids, int M,
                                                                         int key_bits, int iota,
                                                                         int64_t *__restrict__ kept_out) {
    __shared__ uint32_t s_keys[kSmallSort];
    __shared__ int32_t s_ids[kSmallSort];
    __shared__ int32_t s_wcnt[kSmallWaves][kBins];
    __shared__ int32_t s_dstart[kBins];
    __shared__ int32_t s_wtot[kBins / kWave];
    const int t = threadIdx.x, lane = __lane_id(), w = t / kWave;
    const uint64_t lt = lanemask_lt();
    uint32_t key[kSmallItems];
    int32_t val[kSmallItems];
    // position of item i of this lane: w * 1024 + i * 64 + lane (wave-striped)
#pragma unroll
    for (int i = 0; i < kSmallItems; i++) {      // every load first, clamped in bounds (M >= 1 here)
        const int idx = min(w * (kWave * kSmallItems) + i * kWave + lane, M - 1);
        key[i] = keys[idx];
        val[i] = iota ? idx : ids[idx];
    }
#pragma unroll
    for (int i = 0; i < kSmallItems; i++) {
        const int idx = w * (kWave * kSmallItems) + i * kWave + lane;
        if (idx >= M) { key[i] = 0u; val[i] = 0; }
    }
    if (kept_out && t == 0) *kept_out = M;        // every pair kept (dropped keys sort last)
    for (int shift = 0; shift < key_bits; shift += 8) {
        const int bits = min(8, key_bits - shift);
        const uint32_t mask = (1u << bits) - 1u;
        for (int k = t; k < kSmallWaves * kBins; k += kSmallThreads) (&s_wcnt[0][0])[k] = 0;
        __syncthreads();
        int32_t rank[kSmallItems];
#pragma unroll
        for (int i = 0; i < kSmallItems; i++) {
            const int idx = w * (kWave * kSmallItems) + i * kWave + lane;
            const bool valid = idx < M;
            const uint32_t d = (key[i] >> shift) & mask;
            const uint64_t peers = match_digit(d, __ballot(valid));
            rank[i] = -1;
            if (valid) {
                const int32_t before = s_wcnt[w][d];
                rank[i] = before + (int32_t)__popcll(peers & lt);
                if ((peers & lt) == 0) s_wcnt[w][d] = before + (int32_t)__popcll(peers);
            }
        }
        __syncthreads();
        // per digit: exclusive prefix over the waves, then over the digits (threads 0..255)
        int32_t run = 0;
        if (t < kBins) {
#pragma unroll
            for (int k = 0; k < kSmallWaves; k++) {
                const int32_t c = s_wcnt[k][t];
                s_wcnt[k][t] = run;
                run += c;
            }
        }
        const int32_t inc = wave_inclusive_scan<int32_t>(run);
        if (lane == kWave - 1 && w < kBins / kWave) s_wtot[w] = inc;
        __syncthreads();
        if (t < kBins) {
            int32_t before = 0;
            for (int k = 0; k < w; k++) before += s_wtot[k];
            s_dstart[t] = before + inc - run;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kSmallItems; i++) {
            if (rank[i] >= 0) {
                const uint32_t d = (key[i] >> shift) & mask;
                const int pos = s_dstart[d] + s_wcnt[w][d] + rank[i];
                if (pos >= 0 && pos < kSmallSort) {   // always true; keeps a ranking bug from writing out of bounds
                    s_keys[pos] = key[i];
                    s_ids[pos] = val[i];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kSmallItems; i++) {
            const int idx = w * (kWave * kSmallItems) + i * kWave + lane;
            if (idx < M) {
                key[i] = s_keys[idx];
                val[i] = s_ids[idx];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < kSmallItems; i++) {
        const int idx = w * (kWave * kSmallItems) + i * kWave + lane;
        if (idx < M) {
            keys[idx] = key[i];
            ids[idx] = val[i];
        }
    }
}

// ---- dispatch order of the compositing blocks ---------------------------------
// Tiles sorted by list length, longest first, so that the blocks that run
// longest start first and the short ones fill in behind them (longest
// processing time first).  Lengths are grouped in buckets of an eighth of an
// octave (bucket = 1 + 8 floor(log2 len) + the next three bits of len, 0 for
// an empty list); the order within a bucket is whatever the atomics give.
constexpr int kOrderBuckets = 256;
constexpr int kOrderThreads = 256;
static_assert(kOrderThreads == kOrderBuckets, "one thread per bucket");

__device__ __forceinline__ int order_bucket(int len) {
    if (len <= 0) return 0;
    const int o = 31 - __clz(len);
    const int m = o >= 3 ? (len >> (o - 3)) & 7 : (len << (3 - o)) & 7;
    return min(kOrderBuckets - 1, 1 + 8 * o + m);
}

// hist[b] += tiles of bucket b (one block-local histogram per block).
__global__ void __launch_bounds__(kOrderThreads) order_hist_kernel(int32_t T, const int32_t *__restrict__ ranges,
                                                                   int32_t *__restrict__ hist) {
    __shared__ int32_t s_hist[kOrderBuckets];
    s_hist[threadIdx.x] = 0;
    __syncthreads();
    const int t = blockIdx.x * kOrderThreads + threadIdx.x;
    if (t < T) atomicAdd(&s_hist[order_bucket(ranges[2 * t + 1] - ranges[2 * t])], 1);
    __syncthreads();
    if (s_hist[threadIdx.x] > 0) atomicAdd(&hist[threadIdx.x], s_hist[threadIdx.x]);
}

// order[pos] = tile with pos = (tiles in longer buckets) + (slot of this
// block within the bucket, from cursor) + (rank within the block).
__global__ void __launch_bounds__(kOrderThreads) order_scatter_kernel(int32_t T, const int32_t *__restrict__ ranges,
                                                                      const int32_t *__restrict__ hist,
                                                                      int32_t *__restrict__ cursor,
                                                                      int32_t *__restrict__ order) {
    __shared__ int32_t s_base[kOrderBuckets];
    __shared__ int32_t s_cnt[kOrderBuckets];
    const int b = threadIdx.x;
    s_base[b] = hist[b];
    s_cnt[b] = 0;
    __syncthreads();
    // s_base[b] = tiles in buckets above b (inclusive suffix scan minus own count)
    const int own = s_base[b];
    for (int off = 1; off < kOrderBuckets; off <<= 1) {
        const int v = b + off < kOrderBuckets ? s_base[b + off] : 0;
        __syncthreads();
        s_base[b] += v;
        __syncthreads();
    }
    s_base[b] -= own;
    const int t = blockIdx.x * kOrderThreads + threadIdx.x;
    int bk = 0, rank = 0;
    if (t < T) {
        bk = order_bucket(ranges[2 * t + 1] - ranges[2 * t]);
        rank = atomicAdd(&s_cnt[bk], 1);
    }
    __syncthreads();
    __shared__ int32_t s_off[kOrderBuckets];
    s_off[b] = s_cnt[b] > 0 ? atomicAdd(&cursor[b], s_cnt[b]) : 0;
    __syncthreads();
    if (t < T) {
        const int pos = s_base[bk] + s_off[bk] + rank;
        if (pos >= 0 && pos < T) order[pos] = t;
    }
}

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

constexpr int hist_stride(int64_t nb) { return (int)((nb + 3) & ~(int64_t)3); }

constexpr size_t radix_ws_bytes(int64_t M) {
    const int64_t nb = (M + kSortTile - 1) / kSortTile;
    return align256((size_t)kBins * (size_t)hist_stride(nb > 0 ? nb : 1) * sizeof(int32_t)) +
           align256(kBins * sizeof(int32_t));
}

// Sorts M pairs by the low key_bits bits; an even number of passes leaves
// the result in keys/ids.  count_dev (nullable): the true number of pairs,
// at most M, read on the device (the grids are sized for M).
// kept (with 32-bit keys, count_dev NULL): the first pass leaves out the
// pairs whose key is kDropKey, takes the ids from the input positions (ids is
// not read), and writes the number of pairs kept to *kept; later passes sort
// those alone, and the result is in keys/ids [0, *kept).  A sort small enough
// for one block keeps every pair (the dropped keys sort last) and writes M.
// hist0_ready: the first pass's block histograms are already in the
// workspace (written by the kernel that produced the keys).
template <typename K>
int radix_sort(int64_t M, int key_bits, K *keys, int32_t *ids, K *keys_alt, int32_t *ids_alt, void *ws,
               hipStream_t s, const int64_t *count_dev = nullptr, int64_t *kept = nullptr, bool hist0_ready = false) {
    if (kept && M == 0) return launch_fill_zero(kept, sizeof(int64_t), s);
    if (M <= 1 && !kept) return GSR_OK;
    if constexpr (sizeof(K) == 4) {
        if (!count_dev && M <= kSmallSort) {   // the whole sort in one block
            radix_sort_small_kernel<<<1, kSmallThreads, 0, s>>>(keys, ids, (int)M, key_bits, kept ? 1 : 0, kept);
            return launch_check("radix_sort");
        }
    }
    int passes = (key_bits + 7) / 8;
    if (passes % 2) passes++;
    const int nb = (int)((M + kSortTile - 1) / kSortTile);
    const int stride = hist_stride(nb);
    int32_t *hist = (int32_t *)ws;
    int32_t *dtot = (int32_t *)((char *)ws + align256((size_t)kBins * stride * sizeof(int32_t)));
    K *kin = keys, *kout = keys_alt;
    int32_t *iin = ids, *iout = ids_alt;
    for (int ps = 0; ps < passes; ps++) {
        // the lower passes take the narrower digits (fewer buckets: longer runs in the scattered writes)
        const int shift = (key_bits * ps) / passes;
        const int bits = (key_bits * (ps + 1)) / passes - shift;   // 0: a padding pass, a stable copy
        const int drop = kept && ps == 0;
        const int64_t *cnt = kept && ps > 0 ? kept : count_dev;
        if (!(hist0_ready && ps == 0))
            radix_hist_kernel<K><<<nb, kSortThreads, 0, s>>>(kin, M, cnt, shift, bits, nb, stride, hist, drop);
        radix_rowscan_kernel<<<1 << bits, kScanThreads, 0, s>>>(hist, nb, stride, dtot);
        radix_scatter_kernel<K><<<nb, kSortThreads, 0, s>>>(kin, drop ? nullptr : iin, kout, iout, M, cnt, shift,
                                                           bits, nb, stride, hist, dtot, drop,
                                                           drop ? kept : nullptr);
        K *tk = kin; kin = kout; kout = tk;
        int32_t *ti = iin; iin = iout; iout = ti;
    }
    return launch_check("radix_sort");
}

// Binning workspace layout: prepare part (C*N sized, kept until finish).
struct BinPrep {
    BinRec *recs;            // [n] what the emission reads of each Gaussian with tiles, by Gaussian
    BinRec *recs_sorted;     // [n] the same in depth order
    int64_t *kept;           // [1] projected Gaussians with at least one tile
    uint32_t *dkeys, *dkeys_alt;
    int32_t *order, *order_alt;   // depth order of the projected Gaussians
    int32_t *counts_sorted;  // [n]
    int64_t *offsets_sorted; // [n]
    int64_t *block_sums;     // scan partials
    int64_t *total;          // [1]
    void *sort_ws;
};

BinPrep carve_prep(void *ws, int64_t n) {
    BinPrep b;
    char *p = (char *)ws;
    auto take = [&](size_t bytes) { void *q = p; p += align256(bytes); return q; };
    const size_t nn = (size_t)(n > 0 ? n : 1);
    b.recs = (BinRec *)take(nn * sizeof(BinRec));
    b.recs_sorted = (BinRec *)take(nn * sizeof(BinRec));
    b.kept = (int64_t *)take(8);
    b.dkeys = (uint32_t *)take(nn * 4);
    b.dkeys_alt = (uint32_t *)take(nn * 4);
    b.order = (int32_t *)take(nn * 4);
    b.order_alt = (int32_t *)take(nn * 4);
    b.counts_sorted = (int32_t *)take(nn * 4);
    b.offsets_sorted = (int64_t *)take(nn * 8);
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    b.block_sums = (int64_t *)take((size_t)(nb > 0 ? nb : 1) * 8);
    b.total = (int64_t *)take(8);
    b.sort_ws = (void *)take(radix_ws_bytes(n));
    return b;
}

size_t prep_bytes(int64_t n) {
    const size_t nn = (size_t)(n > 0 ? n : 1);
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    return 2 * align256(nn * sizeof(BinRec)) + align256(8) + 5 * align256(nn * 4) + align256(nn * 8) +
           align256((size_t)(nb > 0 ? nb : 1) * 8) + align256(8) + radix_ws_bytes(n);
}

struct BinFin {
    uint32_t *tkeys, *tkeys_alt;
    int32_t *ids_alt;
    void *sort_ws;
};

BinFin carve_fin(void *ws, int64_t M) {
    BinFin b;
    char *p = (char *)ws;
    auto take = [&](size_t bytes) { void *q = p; p += align256(bytes); return q; };
    const size_t mm = (size_t)(M > 0 ? M : 1);
    b.tkeys = (uint32_t *)take(mm * 4);
    b.tkeys_alt = (uint32_t *)take(mm * 4);
    b.ids_alt = (int32_t *)take(mm * 4);
    b.sort_ws = (void *)take(radix_ws_bytes(M));
    return b;
}

size_t fin_bytes(int64_t M) {
    const size_t mm = (size_t)(M > 0 ? M : 1);
    return 3 * align256(mm * 4) + radix_ws_bytes(M);
}

int scan_counts(int64_t n, const int32_t *counts, int64_t *block_sums, int64_t *offsets, int64_t *total,
                hipStream_t s, int64_t *total_copy = nullptr) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    block_sums_kernel<<<dim3((unsigned)nb), dim3(kScanThreads), 0, s>>>(n, counts, block_sums);
    scan_sums_kernel<<<1, kScanThreads, 0, s>>>(block_sums, nb, total, total_copy);
    offsets_kernel<<<dim3((unsigned)nb), dim3(kScanThreads), 0, s>>>(n, counts, block_sums, offsets);
    return launch_check("scan");
}

}  // namespace

size_t count_workspace_bytes(int64_t n) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    return align256((size_t)(nb > 0 ? nb : 1) * sizeof(int64_t));
}

int launch_intersect_count(const gsr_params &p, const CamTable &cams, int N, const float *means2d,
                           const int32_t *radii, int32_t *counts, int64_t *offsets, int64_t *total_dev,
                           void *ws, hipStream_t s) {
    (void)p;
    const int64_t n = (int64_t)cams.C * N;
    if (n == 0) return launch_fill_zero(total_dev, sizeof(int64_t), s);
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    int64_t *sums = (int64_t *)ws;
    count_kernel<<<dim3((unsigned)nb), dim3(kScanThreads), 0, s>>>(cams, N, n, means2d, radii, counts, sums);
    scan_sums_kernel<<<1, kScanThreads, 0, s>>>(sums, nb, total_dev, nullptr);
    offsets_kernel<<<dim3((unsigned)nb), dim3(kScanThreads), 0, s>>>(n, counts, sums, offsets);
    return launch_check("intersect_count");
}

int launch_intersect_emit(const gsr_params &p, const CamTable &cams, int N, const float *means2d,
                          const int32_t *radii, const float *depths, const int64_t *offsets, int64_t cap,
                          uint64_t *keys, int32_t *ids, hipStream_t s) {
    (void)p;
    const int64_t n = (int64_t)cams.C * N;
    if (n == 0 || cap == 0) return GSR_OK;
    const int64_t nb = emit_blocks(cap);
    const CullIn none{nullptr, nullptr, nullptr, 0.0f, 0};   // this route keeps whole rectangles
    emit_kernel<uint64_t><<<dim3((unsigned)nb), dim3(kEmitThreads), 0, s>>>(cams, N, n, means2d, radii, depths,
                                                                           none, nullptr, offsets, cap, nullptr, keys,
                                                                           ids, nullptr, 0, 0, nullptr);
    return launch_check("intersect_emit");
}

int launch_fill_zero(void *ptr, size_t bytes, hipStream_t s) {
    const int64_t words = (int64_t)(bytes / 4);
    if (words == 0) return GSR_OK;
    int64_t blocks = (words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    fill_zero_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>((uint32_t *)ptr, words);
    return launch_check("fill_zero");
}

int launch_fill_zero_multi(int n, void *const *ptrs, const size_t *bytes, hipStream_t s) {
    FillList f;
    int k = 0;
    int64_t most = 0;
    for (int i = 0; i < n; i++) {
        const int64_t words = (int64_t)(bytes[i] / 4);
        if (!ptrs[i] || words == 0) continue;
        if (k == kFillMax) return fail(GSR_EINVAL, "fill_zero_multi: more than %d buffers", kFillMax);
        f.p[k] = (uint32_t *)ptrs[i];
        f.words[k] = words;
        most = words > most ? words : most;
        k++;
    }
    if (k == 0) return GSR_OK;
    int64_t blocks = (most + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    fill_zero_multi_kernel<<<dim3((unsigned)blocks, (unsigned)k), dim3(256), 0, s>>>(f);
    return launch_check("fill_zero");
}

int launch_tile_ranges(int64_t M, const uint64_t *keys, int32_t total_tiles, int32_t *ranges, hipStream_t s) {
    int rc = launch_fill_zero(ranges, (size_t)total_tiles * 2 * sizeof(int32_t), s);
    if (rc != GSR_OK || M == 0) return rc;
    ranges_kernel<uint64_t><<<dim3((unsigned)range_blocks(M)), dim3(256), 0, s>>>(M, nullptr, keys, total_tiles,
                                                                                  ranges);
    return launch_check("tile_ranges");
}

size_t tile_order_bytes() { return 2 * kOrderBuckets * sizeof(int32_t); }

int launch_tile_order(int32_t T, const int32_t *ranges, int32_t *order, void *ws, hipStream_t s) {
    int32_t *hist = (int32_t *)ws, *cursor = hist + kOrderBuckets;
    int rc = launch_fill_zero(ws, tile_order_bytes(), s);
    if (rc != GSR_OK || T == 0) return rc;
    const dim3 grid((unsigned)((T + kOrderThreads - 1) / kOrderThreads)), block(kOrderThreads);
    order_hist_kernel<<<grid, block, 0, s>>>(T, ranges, hist);
    order_scatter_kernel<<<grid, block, 0, s>>>(T, ranges, hist, cursor, order);
    return launch_check("tile_order");
}

size_t sort_workspace_bytes(int64_t M) { return radix_ws_bytes(M); }

int launch_sort_pairs(int64_t M, int key_bits, uint64_t *keys, int32_t *ids, uint64_t *keys_alt,
                      int32_t *ids_alt, void *ws, hipStream_t s) {
    return radix_sort<uint64_t>(M, key_bits, keys, ids, keys_alt, ids_alt, ws, s);
}

// ---- the sort without a workspace argument ------------------------------------
// For callers that cannot allocate (graph capture, serving loops): the digit
// histograms and totals live in a file-scope device array, one copy per GPU,
// sized for kStaticSortMax pairs (16 MiB + 1 KiB).  Its device address is
// looked up once per device, with that device current, and kept; host code
// hands the kernels that address, never the array's own (host-side) name.
// Every slot the sort reads is first written by the same call's kernels
// (histograms by radix_hist_kernel, totals by radix_rowscan_kernel), so
// nothing needs clearing; calls that overlap on one GPU share the array and
// race.
namespace {
constexpr int64_t kStaticSortMax = (int64_t)1 << 25;
constexpr size_t kStaticSortBytes = radix_ws_bytes(kStaticSortMax);
constexpr int kStaticDevices = 64;
__device__ __align__(256) unsigned char scratch[kStaticSortBytes];
void *g_scratch[kStaticDevices];
std::mutex g_scratch_mu;

int static_scratch(void **ptr) {
    int dev = -1;
    int rc = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (rc != GSR_OK) return rc;
    if (dev < 0 || dev >= kStaticDevices) return fail(GSR_EINVAL, "device %d beyond the %d supported", dev, kStaticDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (rc != GSR_OK) return rc;
        if (!p) return fail(GSR_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch[dev] = p;
    }
    *ptr = g_scratch[dev];
    return GSR_OK;
}
}  // namespace

int64_t sort_static_max_pairs() { return kStaticSortMax; }

int launch_sort_pairs_static(int64_t M, int key_bits, uint64_t *keys, int32_t *ids, uint64_t *keys_alt,
                             int32_t *ids_alt, hipStream_t s) {
    if (M > kStaticSortMax) return fail(GSR_EINVAL, "%lld pairs exceed the %lld of the static sort", (long long)M,
                                        (long long)kStaticSortMax);
    void *ws = nullptr;
    const int rc = static_scratch(&ws);
    if (rc != GSR_OK) return rc;
    static_assert(radix_ws_bytes(kStaticSortMax) <= kStaticSortBytes, "static sort space too small");
    return radix_sort<uint64_t>(M, key_bits, keys, ids, keys_alt, ids_alt, ws, s);
}

size_t bin_prepare_bytes(int64_t n) { return prep_bytes(n); }
size_t bin_finish_bytes(int64_t M) { return fin_bytes(M); }
const int64_t *bin_total_ptr(void *ws_prep, int64_t n) { return carve_prep(ws_prep, n).total; }

namespace {
CullIn cull_inputs(const gsr_params &p, const float *conics, const float *opacities, const float *comps) {
    return CullIn{conics, opacities, p.antialiased ? comps : nullptr, p.alpha_min, p.tile_cull ? 1 : 0};
}
}  // namespace

size_t scan_workspace_bytes(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile + 1) * sizeof(int64_t); }

int launch_scan_i32(int64_t n, const int32_t *counts, int64_t *offsets, int64_t *total, void *ws, hipStream_t s) {
    if (n == 0) return launch_fill_zero(total, sizeof(int64_t), s);
    return scan_counts(n, counts, (int64_t *)ws, offsets, total, s);
}

int launch_bin_prepare(const gsr_params &p, const CamTable &cams, int N, const float *means2d,
                       const int32_t *radii, const float *depths, const float *conics, const float *opacities,
                       const float *comps, void *ws_prep, int64_t *total_dev, hipStream_t s) {
    const int64_t n = (int64_t)cams.C * N;
    BinPrep b = carve_prep(ws_prep, n);
    if (n == 0) {
        int rc = launch_fill_zero(b.total, sizeof(int64_t), s);
        if (rc == GSR_OK && total_dev) rc = launch_fill_zero(total_dev, sizeof(int64_t), s);
        return rc;
    }
    const unsigned nb = (unsigned)((n + 255) / 256);
    bin_keys_kernel<<<nb, 256, 0, s>>>(cams, N, n, means2d, radii, depths, cull_inputs(p, conics, opacities, comps),
                                       b.dkeys, b.recs);
    // the depth order of the Gaussians that have tiles (the first pass drops the others)
    int rc = radix_sort<uint32_t>(n, 32, b.dkeys, b.order, b.dkeys_alt, b.order_alt, b.sort_ws, s, nullptr, b.kept);
    if (rc != GSR_OK) return rc;
    // gather + block sums, then the scan of the block sums, which writes the count into the workspace
    // and, when asked, into total_dev (no copy node), then the offsets
    const int64_t nbs = (n + kScanTile - 1) / kScanTile;
    gather_recs_kernel<<<dim3((unsigned)nbs), dim3(kScanThreads), 0, s>>>(n, b.kept, b.order, b.recs, b.recs_sorted,
                                                                       b.counts_sorted, b.block_sums);
    scan_sums_kernel<<<1, kScanThreads, 0, s>>>(b.block_sums, nbs, b.total, total_dev);
    offsets_kernel<<<dim3((unsigned)nbs), dim3(kScanThreads), 0, s>>>(n, b.counts_sorted, b.block_sums,
                                                                    b.offsets_sorted);
    return launch_check("bin_prepare");
}

int launch_bin_finish(const gsr_params &p, const CamTable &cams, int N, const float *means2d,
                      const int32_t *radii, const float *depths, const float *conics, const float *opacities,
                      const float *comps, int64_t M, void *ws_prep, void *ws_fin, int32_t *ids, int32_t *ranges,
                      uint64_t *keys64, hipStream_t s) {
    const int64_t n = (int64_t)cams.C * N;
    BinPrep b = carve_prep(ws_prep, n);
    BinFin f = carve_fin(ws_fin, M);
    int rc = launch_fill_zero(ranges, (size_t)cams.total_tiles * 2 * sizeof(int32_t), s);
    if (rc != GSR_OK || n == 0 || M == 0) return rc;
    const int64_t ne = emit_blocks(M);
    const int tile_bits = cams.total_tiles > 1 ? 32 - __builtin_clz((unsigned)(cams.total_tiles - 1)) : 1;
    // the sort's first-pass digit width (as radix_sort splits tile_bits) and histogram layout: each emit block
    // fills one sort tile, so it counts that tile's first digits on the way
    static_assert(kEmitChunk * (kEmitThreads / kWave) == kSortTile, "an emit block fills one sort tile");
    int passes = (tile_bits + 7) / 8;
    if (passes % 2) passes++;
    const int width0 = tile_bits / passes;
    const bool fuse = M > 1;
    // M is the capacity; the true count (b.total, from the prepare step) is read on the device
    emit_kernel<uint32_t><<<dim3((unsigned)ne), dim3(kEmitThreads), 0, s>>>(
        cams, N, n, means2d, radii, depths, cull_inputs(p, conics, opacities, comps), b.order, b.offsets_sorted, M,
        b.total, f.tkeys, ids, fuse ? (int32_t *)f.sort_ws : nullptr, width0, hist_stride(ne), b.recs_sorted);
    rc = radix_sort<uint32_t>(M, tile_bits, f.tkeys, ids, f.tkeys_alt, f.ids_alt, f.sort_ws, s, b.total, nullptr,
                              fuse);
    if (rc != GSR_OK) return rc;
    ranges_kernel<uint32_t><<<dim3((unsigned)range_blocks(M)), dim3(256), 0, s>>>(M, b.total, f.tkeys,
                                                                                  cams.total_tiles, ranges);
    if (keys64)
        keys64_kernel<<<dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s>>>(M, b.total, f.tkeys, ids, depths, n,
                                                                             keys64);
    return launch_check("bin_finish");
}

}  // namespace gsr
