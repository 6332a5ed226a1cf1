// Tile binning, key emission, stable LSD radix sort and tile ranges
// (Rasterization of Gaussians: 16x16 tiles, per-tile depth order).
//
// Prefix sums and the sort use reduce-then-scan (no inter-block waiting), so
// every kernel finishes regardless of the order in which blocks are scheduled.
#include "common.hpp"

#pragma clang fp contract(off)

namespace gsr {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;   // elements per block

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Inclusive scan across the 64 lanes of a wave.
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

// Pass 1: tiles per Gaussian and per-block sums.
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

// Pass 2: one block turns the block sums into exclusive block offsets.
__global__ void __launch_bounds__(kScanThreads) scan_sums_kernel(int64_t *__restrict__ sums, int64_t nb,
                                                                 int64_t *__restrict__ total_out) {
    int64_t carry = 0;
    for (int64_t start = 0; start < nb; start += kScanThreads) {
        const int64_t i = start + threadIdx.x;
        const int64_t v = i < nb ? sums[i] : 0;
        int64_t tot;
        const int64_t ex = block_exclusive_scan<int64_t>(v, tot);
        if (i < nb) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

// Pass 3: per-element exclusive offsets.
__global__ void __launch_bounds__(kScanThreads) offsets_kernel(int64_t n_total, const int32_t *__restrict__ counts,
        const int64_t *__restrict__ block_off, int64_t *__restrict__ offsets) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int64_t local = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        v[i] = (base + i < n_total) ? counts[base + i] : 0;
        local += v[i];
    }
    int64_t total;
    int64_t run = block_exclusive_scan<int64_t>(local, total) + block_off[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        if (base + i < n_total) offsets[base + i] = run;
        run += v[i];
    }
}

// Key emission, one wave per 64 consecutive projected Gaussians: the wave's
// output range is contiguous, so lanes stride over it and each finds the
// Gaussian owning its slot by binary search; writes are fully coalesced and
// a Gaussian covering thousands of tiles is spread over the whole wave.
constexpr int kEmitThreads = 256;
__global__ void __launch_bounds__(kEmitThreads) emit_kernel(CamTable cams, int N, int64_t n_total,
        const float *__restrict__ means2d, const int32_t *__restrict__ radii, const float *__restrict__ depths,
        const int64_t *__restrict__ offsets, int64_t cap, uint64_t *__restrict__ keys, int32_t *__restrict__ ids) {
    __shared__ int32_t s_rel[kEmitThreads];   // slot of the lane's first entry, relative to the wave
    __shared__ int32_t s_x0[kEmitThreads], s_y0[kEmitThreads], s_w[kEmitThreads];
    __shared__ int32_t s_row[kEmitThreads];   // tile_base + y0 * TX + x0 of the lane's camera
    __shared__ int32_t s_TX[kEmitThreads];
    __shared__ uint32_t s_dbits[kEmitThreads];
    const int lane = __lane_id(), w = threadIdx.x / kWave;
    const int64_t g = (int64_t)blockIdx.x * kEmitThreads + threadIdx.x;
    const int64_t g0 = (int64_t)blockIdx.x * kEmitThreads + (int64_t)w * kWave;
    if (g0 >= n_total) return;                // whole wave past the end (wave-uniform)
    int cnt = 0, x0 = 0, x1 = 0, y0 = 0, y1 = 0, TX = 0, row = 0;
    int64_t off = 0;
    uint32_t dbits = 0;
    if (g < n_total) {
        off = offsets[g];
        const int r = radii[g];
        if (r > 0) {
            const int c = (int)(g / N);
            TX = cams.cam[c].TX;
            tile_rect(means2d[2 * g], means2d[2 * g + 1], r, TX, cams.cam[c].TY, x0, x1, y0, y1);
            if (x1 > x0 && y1 > y0) cnt = (x1 - x0) * (y1 - y0);
            row = cams.cam[c].tile_base + y0 * TX + x0;
            dbits = __float_as_uint(depths[g]);
        }
    }
    const int64_t wbase = __shfl(off, 0, kWave);
    int64_t end = off + cnt;
    // wave end = the largest end (offsets are non-decreasing)
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const int64_t o2 = __shfl_xor(end, d, kWave);
        end = o2 > end ? o2 : end;
    }
    const int total = (int)(end - wbase);
    s_rel[threadIdx.x] = (g < n_total) ? (int)(off - wbase) : 0x7fffffff;
    s_x0[threadIdx.x] = x0; s_y0[threadIdx.x] = y0; s_w[threadIdx.x] = x1 - x0;
    s_row[threadIdx.x] = row; s_TX[threadIdx.x] = TX; s_dbits[threadIdx.x] = dbits;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int wb = w * kWave;
    for (int j = lane; j < total; j += kWave) {
        // largest L with s_rel[L] <= j (always a lane with a non-empty rectangle)
        int lo = 0, hi = kWave - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_rel[wb + mid] <= j) lo = mid; else hi = mid - 1;
        }
        const int k = wb + lo;
        const int local = j - s_rel[k];
        const int wdt = s_w[k];
        const int dy = local / wdt;
        const int dx = local - dy * wdt;
        const uint32_t tile = (uint32_t)(s_row[k] + dy * s_TX[k] + dx);
        const int64_t pos = wbase + j;
        if (pos < cap) {
            keys[pos] = ((uint64_t)tile << 32) | (uint64_t)s_dbits[k];
            ids[pos] = (int32_t)(g0 + lo);
        }
    }
}

__global__ void fill_zero_kernel(uint32_t *__restrict__ p, int64_t n_words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void ranges_kernel(int64_t M, const uint64_t *__restrict__ keys, int32_t total_tiles,
                              int32_t *__restrict__ ranges) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int32_t t = (int32_t)(keys[i] >> 32);
    if (t < 0 || t >= total_tiles) return;
    if (i == 0 || (int32_t)(keys[i - 1] >> 32) != t) ranges[2 * t] = (int32_t)i;
    if (i == M - 1 || (int32_t)(keys[i + 1] >> 32) != t) ranges[2 * t + 1] = (int32_t)(i + 1);
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (uint64 key, int32 id), up to 8 bits per pass.
// Per pass: (1) per-block digit histograms, stored digit-major;
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
__device__ __forceinline__ uint64_t match_digit(uint32_t d, int bits, uint64_t active) {
    uint64_t m = active;
    for (int b = 0; b < bits; b++) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        m &= bit ? bal : ~bal;
    }
    return m;
}

__global__ void __launch_bounds__(kSortThreads) radix_hist_kernel(const uint64_t *__restrict__ keys, int64_t M,
        int shift, int bits, int nblocks, int32_t *__restrict__ hist) {
    __shared__ int32_t cnt[kBins];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t mask = (1u << bits) - 1u;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const int lane = __lane_id();
#pragma unroll
    for (int i = 0; i < kSortItems; i++) {
        const int64_t idx = base + (int64_t)i * kSortThreads + threadIdx.x;
        const bool valid = idx < M;
        const uint32_t d = valid ? (uint32_t)(keys[idx] >> shift) & mask : 0u;
        const uint64_t active = __ballot(valid);
        const uint64_t peers = match_digit(d, bits, active);
        if (valid && (peers & lanemask_lt()) == 0) atomicAdd(&cnt[d], (int32_t)__popcll(peers));
        (void)lane;
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// One block per digit: exclusive scan of hist[d][0..nblocks) in place; the
// row total goes to digit_tot[d].
__global__ void __launch_bounds__(kScanThreads) radix_rowscan_kernel(int32_t *__restrict__ hist, int nblocks,
                                                                     int32_t *__restrict__ digit_tot) {
    int32_t *row = hist + (int64_t)blockIdx.x * nblocks;
    int32_t carry = 0;
    for (int start = 0; start < nblocks; start += kScanThreads) {
        const int i = start + threadIdx.x;
        const int32_t v = i < nblocks ? row[i] : 0;
        int32_t tot;
        const int32_t ex = block_exclusive_scan<int32_t>(v, tot);
        if (i < nblocks) row[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) digit_tot[blockIdx.x] = carry;
}

__global__ void __launch_bounds__(kSortThreads) radix_scatter_kernel(const uint64_t *__restrict__ keys_in,
        const int32_t *__restrict__ ids_in, uint64_t *__restrict__ keys_out, int32_t *__restrict__ ids_out,
        int64_t M, int shift, int bits, int nblocks, const int32_t *__restrict__ hist,
        const int32_t *__restrict__ digit_tot) {
    __shared__ uint64_t s_keys[kSortTile];
    __shared__ int32_t s_ids[kSortTile];
    __shared__ int32_t s_wcnt[kSortWaves][kBins];
    __shared__ int32_t s_dstart[kBins];
    __shared__ int32_t s_gout[kBins];
    const int t = threadIdx.x, lane = __lane_id(), w = t / kWave;
    const uint32_t mask = (1u << bits) - 1u;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;

    // global start of each digit's run for this block
    {
        int32_t tot;
        const int32_t before = block_exclusive_scan<int32_t>(digit_tot[t], tot);
        s_gout[t] = before + hist[(int64_t)t * nblocks + blockIdx.x];
    }
#pragma unroll
    for (int k = 0; k < kSortWaves; k++) s_wcnt[k][t] = 0;
    __syncthreads();

    // load, wave-striped: wave w owns [w*64*ITEMS, (w+1)*64*ITEMS) of the tile
    uint64_t key[kSortItems];
    int32_t val[kSortItems];
    int32_t rank[kSortItems];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int i = 0; i < kSortItems; i++) {
        const int64_t idx = base + (int64_t)w * (kWave * kSortItems) + i * kWave + lane;
        const bool valid = idx < M;
        key[i] = valid ? keys_in[idx] : 0ull;
        val[i] = valid ? ids_in[idx] : 0;
        const uint32_t d = (uint32_t)(key[i] >> shift) & mask;
        const uint64_t active = __ballot(valid);
        const uint64_t peers = match_digit(d, bits, active);
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
    const int n_valid = (int)((M - base) < kSortTile ? (M - base) : kSortTile);
    for (int j = t; j < n_valid; j += kSortThreads) {
        const uint64_t k = s_keys[j];
        const uint32_t d = (uint32_t)(k >> shift) & mask;
        const int64_t gpos = (int64_t)s_gout[d] + (j - s_dstart[d]);
        if (gpos >= 0 && gpos < M) {
            keys_out[gpos] = k;
            ids_out[gpos] = s_ids[j];
        }
    }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

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
    scan_sums_kernel<<<1, kScanThreads, 0, s>>>(sums, nb, total_dev);
    offsets_kernel<<<dim3((unsigned)nb), dim3(kScanThreads), 0, s>>>(n, counts, sums, offsets);
    return launch_check("intersect_count");
}

int launch_intersect_emit(const gsr_params &p, const CamTable &cams, int N, const float *means2d,
                          const int32_t *radii, const float *depths, const int64_t *offsets, int64_t cap,
                          uint64_t *keys, int32_t *ids, hipStream_t s) {
    (void)p;
    const int64_t n = (int64_t)cams.C * N;
    if (n == 0 || cap == 0) return GSR_OK;
    const int64_t nb = (n + kEmitThreads - 1) / kEmitThreads;
    emit_kernel<<<dim3((unsigned)nb), dim3(kEmitThreads), 0, s>>>(cams, N, n, means2d, radii, depths, offsets,
                                                                 cap, keys, ids);
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

int launch_tile_ranges(int64_t M, const uint64_t *keys, int32_t total_tiles, int32_t *ranges, hipStream_t s) {
    int rc = launch_fill_zero(ranges, (size_t)total_tiles * 2 * sizeof(int32_t), s);
    if (rc != GSR_OK || M == 0) return rc;
    ranges_kernel<<<dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s>>>(M, keys, total_tiles, ranges);
    return launch_check("tile_ranges");
}

size_t sort_workspace_bytes(int64_t M) {
    const int64_t nb = (M + kSortTile - 1) / kSortTile;
    return align256((size_t)kBins * (size_t)(nb > 0 ? nb : 1) * sizeof(int32_t)) + align256(kBins * sizeof(int32_t));
}

int launch_sort_pairs(int64_t M, int key_bits, uint64_t *keys, int32_t *ids, uint64_t *keys_alt,
                      int32_t *ids_alt, void *ws, hipStream_t s) {
    if (M <= 1) return GSR_OK;
    // An even number of passes leaves the result in keys/ids.
    int passes = (key_bits + 7) / 8;
    if (passes % 2) passes++;
    const int width = (key_bits + passes - 1) / passes;
    const int nb = (int)((M + kSortTile - 1) / kSortTile);
    int32_t *hist = (int32_t *)ws;
    int32_t *dtot = (int32_t *)((char *)ws + align256((size_t)kBins * nb * sizeof(int32_t)));
    uint64_t *kin = keys, *kout = keys_alt;
    int32_t *iin = ids, *iout = ids_alt;
    for (int ps = 0; ps < passes; ps++) {
        const int shift = ps * width;
        int bits = key_bits - shift;
        if (bits > width) bits = width;
        if (bits < 1) bits = 1;   // only when passes were padded to an even count
        radix_hist_kernel<<<nb, kSortThreads, 0, s>>>(kin, M, shift, bits, nb, hist);
        radix_rowscan_kernel<<<kBins, kScanThreads, 0, s>>>(hist, nb, dtot);
        radix_scatter_kernel<<<nb, kSortThreads, 0, s>>>(kin, iin, kout, iout, M, shift, bits, nb, hist, dtot);
        uint64_t *tk = kin; kin = kout; kout = tk;
        int32_t *ti = iin; iin = iout; iout = ti;
    }
    return launch_check("sort_pairs");
}

}  // namespace gsr
