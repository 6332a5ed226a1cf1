// Backward pass of the compositing (Depth Compositing Gradients).
//
// Same tiling as the forward: a 256-thread block per 16x16 tile, an 8x8
// quad per wave, LDS-staged batches walked back to front, with the same
// quad culling.  Each pixel restores T from final_T by T_k = T_{k+1} /
// (1 - alpha_k) and carries S, the colour accumulated behind the current
// entry plus final_T times the background.  A wave starts at the largest
// last_ids among its own pixels.
//
// The nine per-pixel gradients of one Gaussian are summed over the 64 lanes
// by a transposing butterfly on DPP lane swizzles: three exchange steps halve
// the number of values per lane (8 -> 4 -> 2 -> 1, pairing lanes that differ
// in bit 0, 1 and 2), three more finish the sums, so lane i ends up with the
// total of value i & 7.  Lanes 0..8 (0..10 with the absolute mean gradient)
// then issue one hardware float atomic instruction.
#include "common.hpp"

namespace gsr {
namespace {

constexpr int kThreads = 256;
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
    const PackedGauss *__restrict__ gauss;
    const float *__restrict__ background;
    const int32_t *__restrict__ ranges;
    const int32_t *__restrict__ ids;
    const float *__restrict__ final_T;
    const int32_t *__restrict__ last_ids;
    const float *__restrict__ v_image;
    const float *__restrict__ v_alpha;
    float *__restrict__ v_means2d;
    float *__restrict__ v_conics;
    float *__restrict__ v_colors;
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

// Sum over all 64 lanes, result in every lane.
__device__ __forceinline__ float wave_total(float v) {
    v += dpp<kDppXor1>(v);
    v += dpp<kDppXor2>(v);
    v += dpp<kDppRor4>(v);
    v += dpp<kDppRor8>(v);
    v += __shfl_xor(v, 16, kWave);
    v += __shfl_xor(v, 32, kWave);
    return v;
}

__global__ void __launch_bounds__(kThreads) raster_bwd_kernel(RasterBwdArgs a, CamTable cams) {
    __shared__ float4 s_xyo[kBatch];   // mean x, mean y, opacity, quad mask bits
    __shared__ float4 s_con[kBatch];   // conic a, b, c, -
    __shared__ float4 s_col[kBatch];   // colour r, g, b, -
    __shared__ int32_t s_id[kBatch];
    __shared__ int32_t s_wmax[kThreads / kWave];

    const int tile = blockIdx.x;
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

    int last = -1;
    float T = 1.0f, Tf = 1.0f, vC0 = 0.0f, vC1 = 0.0f, vC2 = 0.0f, vA = 0.0f;
    float S0 = 0.0f, S1 = 0.0f, S2 = 0.0f;
    if (inside) {
        const int64_t pix = ci.pix_off + (int64_t)yi * ci.W + xi;
        last = a.last_ids[pix];
        Tf = a.final_T[pix];
        T = Tf;
        vC0 = a.v_image[3 * pix]; vC1 = a.v_image[3 * pix + 1]; vC2 = a.v_image[3 * pix + 2];
        if (a.v_alpha) vA = a.v_alpha[pix];
        if (a.background) {
            S0 = Tf * a.background[3 * c]; S1 = Tf * a.background[3 * c + 1]; S2 = Tf * a.background[3 * c + 2];
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

    // destination of the value this lane holds after the reduction
    const int slot = lane < 11 ? lane : -1;

    for (int hi = stop + 1; hi > start; hi -= kBatch) {
        const int base = max(start, hi - kBatch);
        __syncthreads();
        const int k = base + (int)threadIdx.x;
        if (k < hi) {
            int g = a.ids[k];
            if ((unsigned)g >= (unsigned)a.CN) g = 0;   // ids come from the sort; this only bounds a bad input
            const PackedGauss r = a.gauss[g];
            const uint32_t qm = quad_mask(r.xyoh.x, r.xyoh.y, r.xyoh.w, r.conh.w, tile_x0, tile_y0);
            s_xyo[threadIdx.x] = make_float4(r.xyoh.x, r.xyoh.y, r.xyoh.z, __uint_as_float(qm));
            s_con[threadIdx.x] = r.conh;
            s_col[threadIdx.x] = r.col;
            s_id[threadIdx.x] = g;
        }
        __syncthreads();
        const int jtop = min(hi, wave_last + 1) - 1 - base;   // entries past the wave's last index carry nothing
        for (int j = jtop; j >= 0; j--) {
            const float4 xyo = s_xyo[j];
            const uint32_t qm = __builtin_amdgcn_readfirstlane(__float_as_uint(xyo.w));
            if (!((qm >> w) & 1u)) continue;            // below alpha_min at every pixel of this quad
            const int kk = base + j;
            const float4 con = s_con[j];
            const float dx = xyo.x - px, dy = xyo.y - py;
            const float sigma = 0.5f * (con.x * dx * dx + con.z * dy * dy) + con.y * dx * dy;
            const float e = __expf(-sigma);
            const float araw = xyo.z * e;
            const float al = fminf(amax, araw);
            const bool use = kk <= last && sigma >= 0.0f && al >= amin;
            if (__ballot(use) == 0ull) continue;
            const float4 col = s_col[j];
            const float inv = __builtin_amdgcn_rcpf(1.0f - al);
            const float Tk = T * inv;
            const float wgt = use ? al * Tk : 0.0f;
            float v_al = (col.x * Tk - S0 * inv) * vC0 + (col.y * Tk - S1 * inv) * vC1 +
                         (col.z * Tk - S2 * inv) * vC2 + vA * (Tf * inv);
            S0 += col.x * wgt; S1 += col.y * wgt; S2 += col.z * wgt;
            T = use ? Tk : T;
            v_al = (use && araw <= amax) ? v_al : 0.0f;   // clamped alpha: no gradient to o or sigma
            const float v_sig = -araw * v_al;
            const float g_mx = v_sig * (con.x * dx + con.y * dy);
            const float g_my = v_sig * (con.y * dx + con.z * dy);
            // transposing butterfly: 8 values -> lane holds value (lane & 7)
            const float w0 = bfly<kDppXor1>(g_mx, g_my, b0);
            const float w1 = bfly<kDppXor1>(v_sig * (0.5f * dx * dx), v_sig * (dx * dy), b0);
            const float w2 = bfly<kDppXor1>(v_sig * (0.5f * dy * dy), wgt * vC0, b0);
            const float w3 = bfly<kDppXor1>(wgt * vC1, wgt * vC2, b0);
            const float x0 = bfly<kDppXor2>(w0, w1, b1);
            const float x1 = bfly<kDppXor2>(w2, w3, b1);
            float y = bfly<kDppRor4>(x0, x1, b2);
            y += dpp<kDppRor8>(y);
            y += __shfl_xor(y, 16, kWave);
            y += __shfl_xor(y, 32, kWave);
            const float zo = wave_total(e * v_al);
            float zx = 0.0f, zy = 0.0f;
            if (want_abs) { zx = wave_total(fabsf(g_mx)); zy = wave_total(fabsf(g_my)); }
            if (slot >= 0 && (slot < 9 || want_abs)) {
                const int g = s_id[j];
                float *dst = slot < 2 ? a.v_means2d + 2 * g + slot
                           : slot < 5 ? a.v_conics + 3 * g + (slot - 2)
                           : slot < 8 ? a.v_colors + 3 * g + (slot - 5)
                           : slot == 8 ? a.v_opac + g
                                       : a.v_means2d_abs + 2 * g + (slot - 9);
                const float val = slot < 8 ? y : slot == 8 ? zo : slot == 9 ? zx : zy;
                unsafeAtomicAdd(dst, val);
            }
        }
    }
}

}  // namespace

int launch_rasterize_bwd(const gsr_params &p, const CamTable &cams, int N, const float *means2d,
                         const float *conics, const float *colors, const float *opacities,
                         const float *comps, const float *background, const int32_t *ranges,
                         const int32_t *ids, const float *final_T, const int32_t *last_ids,
                         const float *v_image, const float *v_alpha, float *v_means2d, float *v_conics,
                         float *v_colors, float *v_opac, float *v_means2d_abs, void *ws, hipStream_t s) {
    const size_t CN = (size_t)cams.C * (size_t)N;
    int rc = launch_fill_zero(v_means2d, CN * 2 * sizeof(float), s);
    if (rc == GSR_OK) rc = launch_fill_zero(v_conics, CN * 3 * sizeof(float), s);
    if (rc == GSR_OK) rc = launch_fill_zero(v_colors, CN * 3 * sizeof(float), s);
    if (rc == GSR_OK) rc = launch_fill_zero(v_opac, CN * sizeof(float), s);
    if (rc == GSR_OK && v_means2d_abs) rc = launch_fill_zero(v_means2d_abs, CN * 2 * sizeof(float), s);
    if (rc != GSR_OK || cams.total_tiles == 0 || N == 0) return rc;
    const int cn = cams.C * N;
    PackedGauss *gauss = (PackedGauss *)ws;
    rc = launch_pack(p, cn, N, means2d, conics, colors, opacities, p.antialiased ? comps : nullptr, gauss, s);
    if (rc != GSR_OK) return rc;
    RasterBwdArgs a{p, N, cn, gauss, background, ranges, ids, final_T, last_ids, v_image, v_alpha, v_means2d,
                    v_conics, v_colors, v_opac, v_means2d_abs};
    raster_bwd_kernel<<<dim3((unsigned)cams.total_tiles), dim3(kThreads), 0, s>>>(a, cams);
    return launch_check("rasterize_bwd");
}

}  // namespace gsr
