// Backward pass of the compositing (Depth Compositing Gradients).
//
// Same tiling as the forward: a 256-thread block per 16x16 tile, an 8x8
// quad per wave, LDS-staged batches walked back to front over the same
// per-quad lists.  Each pixel restores T from final_T by T_k = T_{k+1} /
// (1 - alpha_k) and carries the dot product of v_C with S, the colour
// accumulated behind the current entry plus final_T times the background
// (the alpha gradient needs S only through it).  A wave starts at the
// largest last_ids among its own pixels.
//
// The nine per-pixel gradients of one Gaussian are summed over the 64 lanes
// by a transposing butterfly on DPP lane swizzles: three exchange steps halve
// the number of values per lane (8 -> 4 -> 2 -> 1, pairing lanes that differ
// in bit 0, 1 and 2), three more finish the sums, so lane i ends up with the
// total of value i & 7.  Lanes 0..8 (0..10 with the absolute mean gradient)
// then issue one hardware float atomic instruction.
//
// Plain RGB runs raster_bwd_rgb_kernel, one wave per tile with four pixels
// per lane (one per quad), which sums each entry's gradients over the quads
// it reaches before that reduction; other channel sets run
// raster_bwd_kernel, four waves per tile, a quad each.
#include "common.hpp"

namespace gsr {
namespace {

constexpr int kThreads = 256;
// Fewer tiles than the 1024 SIMDs of an MI355X (256 CUs x 4): the RGB
// backward then runs the four-waves-per-tile kernel.
constexpr int kFewTiles = 1024;
constexpr int kBatch = 256;

// DPP controls (GFX9 encoding): quad_perm [1,0,3,2] and [2,3,0,1], rotate a
// 16-lane row by 4 and by 8.
constexpr int kDppXor1 = 0xB1;
constexpr int kDppXor2 = 0x4E;
constexpr int kDppRor4 = 0x124;
constexpr int kDppRor8 = 0x128;

struct RasterBwdArgs {
    gsr_params p;
    int N;
    int CN;
    int D;                                // feature channels of colors
    int Dt;                               // channels composited: D, plus one for depth; at most the kernel's DM
    const float *__restrict__ feat;       // colors [C,N,D] or [N,D] (read here unless plain RGB)
    const float *__restrict__ depths;     // [C,N], channel D when a depth mode is set
    const PackedGauss *__restrict__ gauss;
    const float *__restrict__ background;
    const int32_t *__restrict__ ranges;
    const int32_t *__restrict__ ids;
    const int32_t *__restrict__ order;     // dispatch order of the tiles (nullable)
    const float *__restrict__ image;      // the forward's image (expected depth reads its depth channel)
    const float *__restrict__ final_T;
    const int32_t *__restrict__ last_ids;
    const float *__restrict__ v_image;
    const float *__restrict__ v_alpha;
    float *__restrict__ v_means2d;
    float *__restrict__ v_conics;
    float *__restrict__ v_colors;         // [C,N,D] or [N,D] as colors
    float *__restrict__ v_depths;         // [C,N], gradient of the depth channel
    float *__restrict__ v_opac;
    float *__restrict__ v_means2d_abs;
};

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

// Keep the half selected by this lane's bit and add the partner's copy of it.
template <int CTRL>
__device__ __forceinline__ float bfly(float a, float b, bool hi) {
    const float keep = hi ? b : a;
    const float send = hi ? a : b;
    return keep + dpp<CTRL>(send);
}

// v plus the value of lane i ^ 16 (i ^ 32): v_permlane16_swap exchanges the
// odd 16-lane rows of one register with the even rows of the other,
// v_permlane32_swap the upper half of one with the lower half of the other;
// given v twice, each lane ends with its own value in one register and its
// partner's in the other, so their sum is the pair total, with no LDS trip.
// Written as inline assembly because the compiler's builtin returns the
// first register for both results; the leading s_nop gives the two wait
// states a VALU write needs before these instructions read it.
__device__ __forceinline__ float add_xor16(float v) {
    float a = v, b = v;
    asm volatile("s_nop 1\n\tv_permlane16_swap_b32 %0, %1" : "+v"(a), "+v"(b));
    return a + b;
}
__device__ __forceinline__ float add_xor32(float v) {
    float a = v, b = v;
    asm volatile("s_nop 1\n\tv_permlane32_swap_b32 %0, %1" : "+v"(a), "+v"(b));
    return a + b;
}

// Sum over the lane's 16-lane row, result in every lane of the row.
__device__ __forceinline__ float row_total(float v) {
    v += dpp<kDppXor1>(v);
    v += dpp<kDppXor2>(v);
    v += dpp<kDppRor4>(v);
    return v + dpp<kDppRor8>(v);
}

// Sum over all 64 lanes, result in every lane.
__device__ __forceinline__ float wave_total(float v) { return add_xor32(add_xor16(row_total(v))); }

// Where the gradient of composited channel d of Gaussian g (id n within its
// camera) goes: a feature channel of v_colors, or v_depths for the depth
// channel.
template <typename Args>
__device__ __forceinline__ float *channel_dst(const Args &a, int d, int &mul, bool &by_n) {
    if (d < a.D) { mul = a.D; by_n = a.p.colors_shared != 0; return a.v_colors + d; }
    mul = 1; by_n = false;
    return a.v_depths;
}

// DM: channel capacity as in the forward (3: RGB from the packed records;
// otherwise a.Dt <= DM channels staged into LDS).  Channels 0..2 ride in the
// transposing butterfly, further channels get a wave sum each.
template <int DM>
__global__ void __launch_bounds__(kThreads) raster_bwd_kernel(RasterBwdArgs a, CamTable cams) {
    constexpr bool kRGB = DM == 3;
    __shared__ float4 s_xyo[kBatch];   // mean x, mean y, opacity, -
    __shared__ float4 s_con[kBatch];   // conic a, b, c, -
    __shared__ float4 s_col[kBatch];   // colour r, g, b, log2(opacity / alpha_min)
    __shared__ float s_feat[kRGB ? 1 : DM * kBatch];
    __shared__ int32_t s_id[kBatch];
    __shared__ uint8_t s_qlist[4][kBatch];
    __shared__ int32_t s_wcnt[4][4];
    __shared__ int32_t s_qcnt[4];
    __shared__ int32_t s_wmax[kThreads / kWave];

    const int tile = block_tile(a.order, cams.total_tiles);
    if (tile < 0) return;
    const int c = camera_of_tile(cams, tile);
    const CamInfo ci = cams.cam[c];
    const int lt = tile - ci.tile_base;
    const int ty = lt / ci.TX, tx = lt - ty * ci.TX;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
    const int xi = tx * kTile + (w & 1) * 8 + (lane & 7);
    const int yi = ty * kTile + (w >> 1) * 8 + (lane >> 3);
    const bool inside = xi < ci.W && yi < ci.H;
    const float px = (float)xi + 0.5f, py = (float)yi + 0.5f;
    const float tile_x0 = (float)(tx * kTile), tile_y0 = (float)(ty * kTile);
    const int start = a.ranges[2 * tile];
    const float amin = a.p.alpha_min, amax = a.p.alpha_max;

    // Per pixel: T restored back to front, and SV = (S . v_C) with S the colour accumulated behind the
    // current entry (plus final_T times the background): dL/dalpha only needs S through that dot
    // product, and S . v_C advances by (colour . v_C) alpha T_k per composited entry.
    const int D = kRGB ? 3 : a.D, Dt = kRGB ? 3 : a.Dt;
    int last = -1;
    float T = 1.0f, vC[DM], vATf = 0.0f, SV = 0.0f;
#pragma unroll
    for (int d = 0; d < DM; d++) vC[d] = 0.0f;
    if (inside) {
        const int64_t pix = ci.pix_off + (int64_t)yi * ci.W + xi;
        last = a.last_ids[pix];
        const float Tf = a.final_T[pix];
        T = Tf;
#pragma unroll
        for (int d = 0; d < DM; d++) vC[d] = d < Dt ? a.v_image[(int64_t)Dt * pix + d] : 0.0f;
        float v_alpha = a.v_alpha ? a.v_alpha[pix] : 0.0f;
        if (!kRGB && Dt > D && a.p.render_depth == GSR_DEPTH_EXPECTED) {
            // E = A / W with A the composited depth and W = sum alpha T = 1 - final_T: the gradient
            // reaches A as v_E / W and W as -v_E E / W, which is an alpha-output gradient
            const float Wn = 1.0f - Tf;
            float vE = 0.0f;
#pragma unroll
            for (int d = 0; d < DM; d++) vE = d == D ? vC[d] : vE;
            const float gA = Wn > 0.0f ? vE / Wn : 0.0f;
#pragma unroll
            for (int d = 0; d < DM; d++) vC[d] = d == D ? gA : vC[d];
            v_alpha -= gA * a.image[(int64_t)Dt * pix + D];
        }
        vATf = v_alpha * Tf;
        if (a.background) {
            float bv = 0.0f;
#pragma unroll
            for (int d = 0; d < DM; d++) bv += d < D ? a.background[D * c + d] * vC[d] : 0.0f;
            SV = Tf * bv;
        }
    }
    // largest last index of the wave and of the block
    int m = last;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m = max(m, __shfl_xor(m, d, kWave));
    const int wave_last = __builtin_amdgcn_readfirstlane(m);
    if (lane == 0) s_wmax[w] = wave_last;
    __syncthreads();
    int stop = s_wmax[0];
    for (int i = 1; i < kThreads / kWave; i++) stop = max(stop, s_wmax[i]);
    const bool want_abs = a.v_means2d_abs != nullptr;
    const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;

    // After the reduction lane i < 8 holds the total of value i (mean x, y;
    // conic a, b, c; channels 0..2), lane 8 the opacity gradient, lanes
    // 9 .. 8 + extra channels 3 .. Dt - 1, the next two the absolute mean
    // gradient.  Each of these lanes adds its total at dst_base + i * dst_mul
    // with i the Gaussian's list id g, or its id n within the camera for
    // features shared by all cameras.
    const int extra = Dt > 3 ? Dt - 3 : 0;
    const int nslots = 9 + extra + (want_abs ? 2 : 0);
    float *dst_base = nullptr;
    int dst_mul = 0;
    bool dst_by_n = false;
    if (a.p.grad_records) {   // plain RGB: lanes 0..8 are the fields of the Gaussian's record, in order
        if (lane < 9) { dst_base = a.v_means2d + lane; dst_mul = GSR_GRAD_RECORD; }
        else if (lane < 11 && want_abs) { dst_base = a.v_means2d_abs + (lane - 9); dst_mul = 2; }
    }
    else if (lane < 2) { dst_base = a.v_means2d + lane; dst_mul = 2; }
    else if (lane < 5) { dst_base = a.v_conics + (lane - 2); dst_mul = 3; }
    else if (lane < 8) { if (lane - 5 < Dt) dst_base = channel_dst(a, lane - 5, dst_mul, dst_by_n); }
    else if (lane == 8) { dst_base = a.v_opac; dst_mul = 1; }
    else if (lane < 9 + extra) { dst_base = channel_dst(a, lane - 6, dst_mul, dst_by_n); }
    else if (lane < 11 + extra && want_abs) { dst_base = a.v_means2d_abs + (lane - 9 - extra); dst_mul = 2; }
    const int cam_base = c * a.N;

    for (int hi = stop + 1; hi > start; hi -= kBatch) {
        const int base = max(start, hi - kBatch);
        __syncthreads();
        const int k = base + (int)threadIdx.x;
        uint32_t qm = 0u;
        if (k < hi) {
            int g = a.ids[k];
            if ((unsigned)g >= (unsigned)a.CN) g = 0;   // ids come from the sort; this only bounds a bad input
            const PackedGauss r = a.gauss[g];
            qm = refine_quad_mask(quad_mask(r.xyoh.x, r.xyoh.y, r.xyoh.w, r.conh.w, tile_x0, tile_y0), r.xyoh,
                                  r.conh, r.col.w, tile_x0, tile_y0);
            s_xyo[threadIdx.x] = r.xyoh;
            s_con[threadIdx.x] = r.conh;
            s_col[threadIdx.x] = r.col;
            s_id[threadIdx.x] = g;
            if (!kRGB) stage_features<DM, kBatch>(a, c, g, threadIdx.x, s_feat);
        }
        compact_quads(qm, s_qlist, s_wcnt, s_qcnt);
        for (int j = s_qcnt[w] - 1; j >= 0; j--) {
            const int e = __builtin_amdgcn_readfirstlane(s_qlist[w][j]);
            const int kk = base + e;
            if (kk > wave_last) continue;               // past every pixel's last composited entry
            const float4 xyo = s_xyo[e];
            const float4 con = s_con[e];
            const float dx = xyo.x - px, dy = xyo.y - py;
            const float sig = scaled_sigma(con, dx, dy);          // log2(e) sigma, as in the forward
            const float ex = __builtin_amdgcn_exp2f(-sig);
            const float araw = xyo.z * ex;
            const float al = min_alpha(araw, amax);
            const bool use = kk <= last && sig >= 0.0f && al >= amin;
            if (__ballot(use) == 0ull) continue;
            const float inv = __builtin_amdgcn_rcpf(1.0f - al);
            const float Tk = T * inv;
            const float wgt = use ? al * Tk : 0.0f;
            // dL/dalpha = (colour T_k - S / (1 - alpha)) . v_C + v_alpha final_T / (1 - alpha)
            float cv;
            if (kRGB) {
                const float4 col = s_col[e];
                cv = (col.x * vC[0] + col.y * vC[1]) + col.z * vC[2];
            } else {
                cv = 0.0f;
#pragma unroll
                for (int d = 0; d < DM; d++) cv = fmaf(s_feat[d * kBatch + e], vC[d], cv);
            }
            float v_al = fmaf(Tk, cv, inv * (vATf - SV));
            SV = fmaf(wgt, cv, SV);
            T = use ? Tk : T;
            v_al = (use && araw <= amax) ? v_al : 0.0f;   // clamped alpha: no gradient to o or sigma
            const float v_sig = -araw * v_al;
            const float h = 0.5f * v_sig;
            // d sigma / d mean = (a dx + b dy, b dx + c dy) = (a u_c, b u_c + (c - b^2/a) dy) with
            // u_c = dx + (b/a) dy: in the record's terms (2 A u_c, 2 A r u_c + 2 Q dy) / log2(e)
            const float u = v_sig * (2.0f / kLog2e);
            const float uc = fmaf(con.y, dy, dx);
            const float g_mx = u * (con.x * uc);
            const float g_my = u * fmaf(con.x * con.y, uc, con.z * dy);
            // transposing butterfly: 8 values -> lane holds value (lane & 7)
            const float w0 = bfly<kDppXor1>(g_mx, g_my, b0);
            const float w1 = bfly<kDppXor1>(h * dx * dx, v_sig * dx * dy, b0);
            const float w2 = bfly<kDppXor1>(h * dy * dy, wgt * vC[0], b0);
            const float w3 = bfly<kDppXor1>(wgt * vC[1], DM > 2 ? wgt * vC[DM > 2 ? 2 : 0] : 0.0f, b0);
            const float x0 = bfly<kDppXor2>(w0, w1, b1);
            const float x1 = bfly<kDppXor2>(w2, w3, b1);
            float y = bfly<kDppRor4>(x0, x1, b2);
            y += dpp<kDppRor8>(y);
            y = add_xor32(add_xor16(y));
            const float zo = wave_total(ex * v_al);
            float val = lane < 8 ? y : zo;
#pragma unroll
            for (int d = 3; d < DM; d++) {
                if (d < Dt) {                            // uniform: Dt is the same for every lane
                    const float zc = wave_total(wgt * vC[d]);
                    val = lane == 6 + d ? zc : val;
                }
            }
            if (want_abs) {
                const float zx = wave_total(fabsf(g_mx)), zy = wave_total(fabsf(g_my));
                val = lane == 9 + extra ? zx : lane == 10 + extra ? zy : val;
            }
            if (lane < nslots && dst_base) {
                const int g = __builtin_amdgcn_readfirstlane(s_id[e]);   // uniform: scalar index arithmetic
                int n = g - cam_base;
                if ((unsigned)n >= (unsigned)a.N) n = 0;   // only a bad id can leave the tile's camera
                unsafeAtomicAdd(dst_base + (int64_t)(dst_by_n ? n : g) * dst_mul, val);
            }
        }
    }
}

// Plain RGB: one wave per 16x16 tile.  Lane l owns pixel (l & 7, l >> 3) of
// each of the four 8x8 quads, so an entry's per-pixel gradients are first
// summed in registers over the quads it reaches (its quad mask is uniform
// across the wave) and then reduced and added to memory once per (tile,
// entry) instead of once per (quad, entry): fewer butterfly reductions and
// fewer atomics for the same per-pixel work.  Batches of 64 entries are
// staged in LDS, compacted: entries that reach no quad (or only quads past
// their last composited entry) are dropped at staging time, and the rest are
// stored in list order, so the walk reads its records at consecutive slots
// with no index lookup in between.
constexpr int kTileBatch = 128;   // two entries per lane

// The gradient outputs are global memory.  An address formed from an integer
// would make the atomic a flat instruction, which also counts on the LDS
// counter, so the next entry's LDS reads would wait for it to complete; the
// explicit address space keeps it a global atomic.
using global_float = __attribute__((address_space(1))) float;

template <bool kStd, bool kAbs>
__global__ void __launch_bounds__(kWave) raster_bwd_rgb_kernel(RasterBwdArgs a, CamTable cams) {
    __shared__ float4 s_xyo[kTileBatch];
    __shared__ float4 s_con[kTileBatch];
    __shared__ float4 s_col[kTileBatch];

    const int tile = block_tile(a.order, cams.total_tiles);
    if (tile < 0) return;
    const int c = camera_of_tile(cams, tile);
    const CamInfo ci = cams.cam[c];
    const int lt = tile - ci.tile_base;
    const int ty = lt / ci.TX, tx = lt - ty * ci.TX;
    const int lane = threadIdx.x;
    const float tile_x0 = (float)(tx * kTile), tile_y0 = (float)(ty * kTile);
    // pixel centre of this lane in quad 0; quad q adds (8 (q & 1), 8 (q >> 1))
    const float px0 = tile_x0 + (float)(lane & 7) + 0.5f, py0 = tile_y0 + (float)(lane >> 3) + 0.5f;
    const int start = a.ranges[2 * tile];
    // kStd: the thresholds are the defaults, compiled in as constants
    const float amin = kStd ? kStdAlphaMin : a.p.alpha_min, amax = kStd ? kStdAlphaMax : a.p.alpha_max;

    // per pixel (one per quad): T restored back to front, R = v_alpha final_T - S . v_C with S the colour
    // composited behind the current entry (background included), v_C, last index
    float T[4], R[4], vC[4][3];
    int last[4], qlast[4];
    int stop = -1;
    // every pixel's inputs loaded first (a pixel outside the image reads the camera's first pixel and
    // is then reset), so that the four quads' loads are in flight together
    bool ins[4];
    float va[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int xi = tx * kTile + (q & 1) * 8 + (lane & 7), yi = ty * kTile + (q >> 1) * 8 + (lane >> 3);
        ins[q] = xi < ci.W && yi < ci.H;
        const int64_t pix = ci.pix_off + (ins[q] ? (int64_t)yi * ci.W + xi : 0);
        last[q] = a.last_ids[pix];
        T[q] = a.final_T[pix];
        vC[q][0] = a.v_image[3 * pix]; vC[q][1] = a.v_image[3 * pix + 1]; vC[q][2] = a.v_image[3 * pix + 2];
        va[q] = a.v_alpha ? a.v_alpha[pix] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
        R[q] = 0.0f;
        if (ins[q]) {
            const float Tf = T[q];
            if (a.v_alpha) R[q] = va[q] * Tf;
            if (a.background) {
                const float *bg = a.background + 3 * c;
                R[q] -= Tf * ((bg[0] * vC[q][0] + bg[1] * vC[q][1]) + bg[2] * vC[q][2]);
            }
        } else {
            T[q] = 1.0f; vC[q][0] = vC[q][1] = vC[q][2] = 0.0f;
            last[q] = -1;
        }
        int m = last[q];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) m = max(m, __shfl_xor(m, d, kWave));
        qlast[q] = __builtin_amdgcn_readfirstlane(m);       // largest last index of quad q
        stop = max(stop, qlast[q]);
    }
    constexpr bool want_abs = kAbs;   // v_means2d_abs given: compiled in only where it is asked for
    const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4, b3 = lane & 8;
    const int nslots = want_abs ? 11 : 9;
    float *dst_base = nullptr;
    uint32_t dst_stride = 0;      // bytes between consecutive Gaussians' values of this lane's output
    bool dst_by_n = false;
    if (a.p.grad_records) {   // lanes 0..8 are the fields of the Gaussian's record, in order
        if (lane < 9) { dst_base = a.v_means2d + lane; dst_stride = 4 * GSR_GRAD_RECORD; }
        else if (lane < 11 && want_abs) { dst_base = a.v_means2d_abs + (lane - 9); dst_stride = 8; }
    }
    else if (lane < 2) { dst_base = a.v_means2d + lane; dst_stride = 8; }
    else if (lane < 5) { dst_base = a.v_conics + (lane - 2); dst_stride = 12; }
    else if (lane < 8) { dst_base = a.v_colors + (lane - 5); dst_stride = 12; dst_by_n = a.p.colors_shared != 0; }
    else if (lane == 8) { dst_base = a.v_opac; dst_stride = 4; }
    else if (lane < 11 && want_abs) { dst_base = a.v_means2d_abs + (lane - 9); dst_stride = 8; }
    const bool dst_lane = lane < nslots && dst_base != nullptr;
    const bool recs = a.p.grad_records != 0;
    const uint64_t dst_addr = (uint64_t)dst_base;
    const int cam_base = c * a.N;
    // lanes 2, 4: dL/da, dL/dc are half the dx^2, dy^2 moments; lanes 9, 10: |dL/dmu'| carries log2(e)
    const float lscale = lane < 2 ? 2.0f / kLog2e : (lane == 2 || lane == 4) ? 0.5f
                       : (lane == 9 || lane == 10) ? 1.0f / kLog2e : 1.0f;

    for (int hi = stop + 1; hi > start; hi -= kTileBatch) {
        const int base = max(start, hi - kTileBatch);
        // two entries per lane, the batch's first and second halves: both ids loaded first (clamped,
        // in-bounds positions), then each half's records
        int gh[2];
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int g = a.ids[min(base + h * kWave + lane, hi - 1)];
            gh[h] = (unsigned)g < (unsigned)a.CN ? g : 0;   // ids come from the sort; this only bounds a bad input
        }
        // the entries that reach a quad, compacted in list order; the records' spare words carry the list
        // index, the quad mask and the id
        int nslot = 0;
        const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int k = base + h * kWave + lane;
            const PackedGauss r = a.gauss[gh[h]];
            uint32_t qm = 0u;
            if (k < hi) {
                qm = refine_quad_mask(quad_mask(r.xyoh.x, r.xyoh.y, r.xyoh.w, r.conh.w, tile_x0, tile_y0), r.xyoh,
                                      r.conh, r.col.w, tile_x0, tile_y0);
#pragma unroll
                for (int q = 0; q < 4; q++)
                    if (k > qlast[q]) qm &= ~(1u << q);      // past every pixel of the quad's last entry
            }
            const uint64_t bal = __ballot(qm != 0u);
            if (qm != 0u) {
                const int slot = nslot + __popcll(bal & below);
                s_xyo[slot] = make_float4(r.xyoh.x, r.xyoh.y, r.xyoh.z, __int_as_float(k));
                s_con[slot] = make_float4(r.conh.x, r.conh.y, r.conh.z, __uint_as_float(qm));
                s_col[slot] = make_float4(r.col.x, r.col.y, r.col.z, __int_as_float(gh[h]));
            }
            nslot += __popcll(bal);
        }
        __syncthreads();
        for (int j = nslot - 1; j >= 0; j--) {
            const float4 xyo = s_xyo[j];
            const float4 con = s_con[j];
            const float4 col = s_col[j];
            const int kk = __builtin_amdgcn_readfirstlane(__float_as_int(xyo.w));
            const uint32_t qme = __builtin_amdgcn_readfirstlane(__float_as_uint(con.w));
            // Per-lane sums over this lane's pixels of v_sigma times (dx, dy, dx^2, dx dy, dy^2), of the
            // colour gradients, of v_sigma, and of |dL/dmu'|: the conic and the opacity are the same for
            // every pixel, so the mean gradient (d sigma / d mu' is linear in dx, dy) and the opacity
            // gradient (v_sigma = -o e^-sigma dL/dalpha) follow from these sums after the reduction.
            // started at -0, the identity of float addition (0 + x is not x for x = -0), so the first
            // quad's terms are taken as they are instead of being added to zero
            float acc[8] = {-0.0f, -0.0f, -0.0f, -0.0f, -0.0f, -0.0f, -0.0f, -0.0f};
            float acc_o = -0.0f, acc_ax = -0.0f, acc_ay = -0.0f;
            bool any = false;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                if (!((qme >> q) & 1u)) continue;                  // uniform
                const float dx = xyo.x - (px0 + (float)((q & 1) * 8)), dy = xyo.y - (py0 + (float)((q >> 1) * 8));
                const float sig = scaled_sigma(con, dx, dy);      // log2(e) sigma, as in the forward
                const float ex = __builtin_amdgcn_exp2f(-sig);
                const float araw = xyo.z * ex;
                const float al = min_alpha(araw, amax);
                const bool use = kk <= last[q] && sig >= 0.0f && al >= amin;
                if (__ballot(use) == 0ull) continue;               // uniform
                any = true;
                const float inv = __builtin_amdgcn_rcpf(1.0f - al);
                const float Tk = T[q] * inv;
                const float cv = (col.x * vC[q][0] + col.y * vC[q][1]) + col.z * vC[q][2];
                const float v_al = fmaf(Tk, cv, inv * R[q]);
                // lanes that do not composite the entry (and clamped alphas: no gradient to o or sigma) get
                // zero weights through selects, so the wave never branches on them
                const float wgt = use ? al * Tk : 0.0f;
                const float m_sig = (use && araw <= amax) ? -araw : 0.0f;
                R[q] = fmaf(-wgt, cv, R[q]);
                T[q] = use ? Tk : T[q];
                const float v_sig = m_sig * v_al;
                const float t = v_sig * dx, sy = v_sig * dy;
                acc[0] += t;
                acc[1] += sy;
                acc[2] = fmaf(t, dx, acc[2]);
                acc[3] = fmaf(t, dy, acc[3]);
                acc[4] = fmaf(sy, dy, acc[4]);
                acc[5] = fmaf(wgt, vC[q][0], acc[5]);
                acc[6] = fmaf(wgt, vC[q][1], acc[6]);
                acc[7] = fmaf(wgt, vC[q][2], acc[7]);
                acc_o += v_sig;
                if (want_abs) {                                   // per-pixel |dL/dmu'|, log2(e) folded in
                    const float tc = fmaf(con.y, sy, t);          // v_sigma u_c, u_c = dx + r dy
                    acc_ax += fabsf(2.0f * con.x * tc);
                    acc_ay += fabsf(2.0f * fmaf(con.x * con.y, tc, con.z * sy));
                }
            }
            if (!any) continue;
            {   // the mean gradient is linear in the first moments with this entry's coefficients: form it per
                // lane before the reduction, so lanes 0 and 1 take their totals as they are
                const float sc = fmaf(con.y, acc[1], acc[0]);
                acc[1] = fmaf(con.x * con.y, sc, con.z * acc[1]);
                acc[0] = con.x * sc;
            }
            // Transposing butterfly: lanes 0-7 of each 16-lane row end with the row's total of value
            // (lane & 7); lanes 8-15 then take the row totals of the v_sigma sum (lane 8) and of the two
            // |dL/dmu'| sums (lanes 9, 10), and one pair of cross-row exchanges finishes all of them.
            const float w0 = bfly<kDppXor1>(acc[0], acc[1], b0);
            const float w1 = bfly<kDppXor1>(acc[2], acc[3], b0);
            const float w2 = bfly<kDppXor1>(acc[4], acc[5], b0);
            const float w3 = bfly<kDppXor1>(acc[6], acc[7], b0);
            const float x0 = bfly<kDppXor2>(w0, w1, b1);
            const float x1 = bfly<kDppXor2>(w2, w3, b1);
            float y = bfly<kDppRor4>(x0, x1, b2);
            y += dpp<kDppRor8>(y);
            float side = row_total(acc_o);
            if (want_abs) {
                const float zx = row_total(acc_ax), zy = row_total(acc_ay);
                side = b0 ? zx : b1 ? zy : side;          // lane 9 (1001b), lane 10 (1010b), lane 8
            }
            y = b3 ? side : y;
            y = add_xor32(add_xor16(y));
            // lanes 0, 1: dL/dmu' = (2 A' S_dx + B' S_dy, B' S_dx + 2 C' S_dy) / log2(e) with the scaled
            // conic (A', B', C') = (A, 2 A r, Q + A r^2), i.e. 2 (A s_c, A r s_c + Q S_dy) / log2(e) with
            // s_c = S_dx + r S_dy; lane 8: dL/do = -(sum of v_sigma) / o
            const float val = y * (lane == 8 ? -__builtin_amdgcn_rcpf(xyo.z) : lscale);
            const int ge = __builtin_amdgcn_readfirstlane(__float_as_int(col.w));   // uniform: scalar index arithmetic
            if (!want_abs && recs) {
                // the nine lanes add to one record: a base shared by the wave plus the lane's field
                // (one address multiply-add per entry instead of a per-lane 64-bit product)
                global_float *rec = (global_float *)a.v_means2d + (uint64_t)(uint32_t)ge * GSR_GRAD_RECORD;
                if (lane < GSR_GRAD_RECORD) __builtin_amdgcn_global_atomic_fadd_f32(rec + lane, val);
            } else {
                int n = ge - cam_base;
                if ((unsigned)n >= (unsigned)a.N) n = 0;   // only a bad id can leave the tile's camera
                const uint32_t gi = dst_by_n ? (uint32_t)n : (uint32_t)ge;
                if (dst_lane)
                    __builtin_amdgcn_global_atomic_fadd_f32((global_float *)(dst_addr + (uint64_t)gi * dst_stride), val);
            }
        }
        __syncthreads();
    }
}

}  // namespace

int launch_rasterize_bwd(const gsr_params &p, const CamTable &cams, int N, int D, const float *means2d,
                         const float *conics, const float *colors, const float *depths, const float *opacities,
                         const float *comps, const float *background, const int32_t *ranges,
                         const int32_t *ids, const int32_t *tile_order, const float *image, const float *final_T,
                         const int32_t *last_ids,
                         const float *v_image, const float *v_alpha, float *v_means2d, float *v_conics,
                         float *v_colors, float *v_depths, float *v_opac, float *v_means2d_abs, void *ws, int flags,
                         hipStream_t s) {
    const size_t CN = (size_t)cams.C * (size_t)N;
    const size_t FN = p.colors_shared ? (size_t)N : CN;
    int rc = GSR_OK;
    if (!(flags & GSR_BWD_ACCUMULATE)) {   // one launch zeroes every output
        const bool rec = p.grad_records != 0;
        void *const ptrs[6] = {v_means2d, rec ? nullptr : v_conics, (D > 0 && !rec) ? v_colors : nullptr,
                               p.render_depth != GSR_DEPTH_NONE ? v_depths : nullptr, rec ? nullptr : v_opac,
                               v_means2d_abs};
        const size_t bytes[6] = {CN * (rec ? GSR_GRAD_RECORD : 2) * sizeof(float), CN * 3 * sizeof(float),
                                 FN * (size_t)D * sizeof(float), CN * sizeof(float), CN * sizeof(float),
                                 CN * 2 * sizeof(float)};
        rc = launch_fill_zero_multi(6, ptrs, bytes, s);
    }
    if (rc != GSR_OK || cams.total_tiles == 0 || N == 0) return rc;
    const int cn = cams.C * N;
    PackedGauss *gauss = (PackedGauss *)ws;
    if (!(flags & GSR_BWD_PACKED)) {
        rc = launch_pack(p, cn, N, D, means2d, conics, colors, opacities, p.antialiased ? comps : nullptr, gauss,
                         s);
        if (rc != GSR_OK) return rc;
    }
    RasterBwdArgs a{p, N, cn, D, composited_channels(p, D), colors, depths, gauss, background, ranges, ids, tile_order,
                    image,
                    final_T, last_ids, v_image, v_alpha, v_means2d, v_conics, v_colors, v_depths, v_opac,
                    v_means2d_abs};
    const dim3 grid((unsigned)cams.total_tiles), block(kThreads);
    switch (channel_capacity(p, D)) {
        case 3:
            // one wave per tile leaves SIMDs idle when the views have fewer tiles than the GPU has
            // SIMDs; then a block of four quad waves per tile finishes sooner
            if (cams.total_tiles < kFewTiles)
                raster_bwd_kernel<4><<<grid, block, 0, s>>>(a, cams);
            else if (standard_thresholds(p) && !v_means2d_abs)
                raster_bwd_rgb_kernel<true, false><<<grid, dim3(kWave), 0, s>>>(a, cams);
            else if (standard_thresholds(p))
                raster_bwd_rgb_kernel<true, true><<<grid, dim3(kWave), 0, s>>>(a, cams);
            else if (!v_means2d_abs)
                raster_bwd_rgb_kernel<false, false><<<grid, dim3(kWave), 0, s>>>(a, cams);
            else
                raster_bwd_rgb_kernel<false, true><<<grid, dim3(kWave), 0, s>>>(a, cams);
            break;
        case 4: raster_bwd_kernel<4><<<grid, block, 0, s>>>(a, cams); break;
        case 8: raster_bwd_kernel<8><<<grid, block, 0, s>>>(a, cams); break;
        case 16: raster_bwd_kernel<16><<<grid, block, 0, s>>>(a, cams); break;
        default: raster_bwd_kernel<32><<<grid, block, 0, s>>>(a, cams); break;
    }
    return launch_check("rasterize_bwd");
}

}  // namespace gsr
