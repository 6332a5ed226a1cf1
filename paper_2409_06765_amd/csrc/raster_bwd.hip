// Backward pass of the compositing (Depth Compositing Gradients).
//
// Same tiling as the forward: a 256-thread block per 16x16 tile, an 8x8
// quad per wave.  The tile's list is walked back to front in LDS-staged
// batches, starting at the largest last_ids of the block.  Each pixel
// restores T from final_T by T_k = T_{k+1} / (1 - alpha_k) and carries the
// colour S accumulated behind the current entry.  The per-pixel gradients
// of one Gaussian are summed over the wave's 64 lanes before a single lane
// issues hardware float atomics, so a (Gaussian, wave) pair costs at most
// nine atomics (eleven with the absolute mean gradient).
#include "common.hpp"

namespace gsr {
namespace {

constexpr int kThreads = 256;
constexpr int kBatch = 256;

struct RasterBwdArgs {
    gsr_params p;
    int N;
    int CN;
    const float *__restrict__ means2d;
    const float *__restrict__ conics;
    const float *__restrict__ colors;
    const float *__restrict__ opacities;
    const float *__restrict__ comps;
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

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

__global__ void __launch_bounds__(kThreads) raster_bwd_kernel(RasterBwdArgs a, CamTable cams) {
    __shared__ float4 s_xyo[kBatch];   // mean x, mean y, opacity, -
    __shared__ float4 s_con[kBatch];   // conic a, b, c, -
    __shared__ float4 s_col[kBatch];   // colour r, g, b, -
    __shared__ int32_t s_id[kBatch];
    __shared__ int32_t s_wmax[kThreads / kWave];

    const int tile = blockIdx.x;
    const int c = camera_of_tile(cams, tile);
    const CamInfo ci = cams.cam[c];
    const int lt = tile - ci.tile_base;
    const int ty = lt / ci.TX, tx = lt - ty * ci.TX;
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int xi = tx * kTile + (w & 1) * 8 + (lane & 7);
    const int yi = ty * kTile + (w >> 1) * 8 + (lane >> 3);
    const bool inside = xi < ci.W && yi < ci.H;
    const float px = (float)xi + 0.5f, py = (float)yi + 0.5f;
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
    // one past the largest last index in the block
    int m = last;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m = max(m, __shfl_xor(m, d, kWave));
    if (lane == 0) s_wmax[w] = m;
    __syncthreads();
    int stop = s_wmax[0];
    for (int i = 1; i < kThreads / kWave; i++) stop = max(stop, s_wmax[i]);
    const int hi_end = stop + 1;   // entries [start, hi_end) can have gradients
    const bool want_abs = a.v_means2d_abs != nullptr;

    for (int b1 = hi_end; b1 > start; b1 -= kBatch) {
        const int b0 = max(start, b1 - kBatch);
        __syncthreads();
        const int k = b0 + (int)threadIdx.x;
        if (k < b1) {
            int g = a.ids[k];
            if ((unsigned)g >= (unsigned)a.CN) g = 0;   // ids come from the sort; this only bounds a bad input
            const int n = g % a.N;
            float o = a.opacities[n];
            if (a.comps) o *= a.comps[g];
            s_xyo[threadIdx.x] = make_float4(a.means2d[2 * g], a.means2d[2 * g + 1], o, 0.0f);
            s_con[threadIdx.x] = make_float4(a.conics[3 * g], a.conics[3 * g + 1], a.conics[3 * g + 2], 0.0f);
            s_col[threadIdx.x] = make_float4(a.colors[3 * g], a.colors[3 * g + 1], a.colors[3 * g + 2], 0.0f);
            s_id[threadIdx.x] = g;
        }
        __syncthreads();
        for (int j = b1 - 1 - b0; j >= 0; j--) {
            const int kk = b0 + j;
            float g_mx = 0.0f, g_my = 0.0f, g_ca = 0.0f, g_cb = 0.0f, g_cc = 0.0f;
            float g_r = 0.0f, g_g = 0.0f, g_b = 0.0f, g_o = 0.0f;
            bool contrib = false;
            if (kk <= last) {
                const float4 xyo = s_xyo[j];
                const float4 con = s_con[j];
                const float dx = xyo.x - px, dy = xyo.y - py;
                const float sigma = 0.5f * (con.x * dx * dx + con.z * dy * dy) + con.y * dx * dy;
                if (sigma >= 0.0f) {
                    const float e = __expf(-sigma);
                    const float araw = xyo.z * e;
                    const float al = fminf(amax, araw);
                    if (al >= amin) {
                        contrib = true;
                        const float4 col = s_col[j];
                        const float one_m = 1.0f - al;
                        const float inv = 1.0f / one_m;
                        const float Tk = T * inv;
                        const float wgt = al * Tk;
                        g_r = wgt * vC0; g_g = wgt * vC1; g_b = wgt * vC2;
                        float v_al = (col.x * Tk - S0 * inv) * vC0 + (col.y * Tk - S1 * inv) * vC1 +
                                     (col.z * Tk - S2 * inv) * vC2;
                        v_al += vA * (Tf * inv);
                        S0 += col.x * wgt; S1 += col.y * wgt; S2 += col.z * wgt;
                        T = Tk;
                        if (araw <= amax) {
                            g_o = e * v_al;
                            const float v_sig = -araw * v_al;
                            g_mx = v_sig * (con.x * dx + con.y * dy);
                            g_my = v_sig * (con.y * dx + con.z * dy);
                            g_ca = v_sig * (0.5f * dx * dx);
                            g_cb = v_sig * (dx * dy);
                            g_cc = v_sig * (0.5f * dy * dy);
                        }
                    }
                }
            }
            if (__ballot(contrib) == 0ull) continue;
            const float a_mx = fabsf(g_mx), a_my = fabsf(g_my);
            g_mx = wave_sum(g_mx); g_my = wave_sum(g_my);
            g_ca = wave_sum(g_ca); g_cb = wave_sum(g_cb); g_cc = wave_sum(g_cc);
            g_r = wave_sum(g_r); g_g = wave_sum(g_g); g_b = wave_sum(g_b);
            g_o = wave_sum(g_o);
            float s_ax = 0.0f, s_ay = 0.0f;
            if (want_abs) { s_ax = wave_sum(a_mx); s_ay = wave_sum(a_my); }
            if (lane == 0) {
                const int g = s_id[j];
                unsafeAtomicAdd(&a.v_means2d[2 * g], g_mx);
                unsafeAtomicAdd(&a.v_means2d[2 * g + 1], g_my);
                unsafeAtomicAdd(&a.v_conics[3 * g], g_ca);
                unsafeAtomicAdd(&a.v_conics[3 * g + 1], g_cb);
                unsafeAtomicAdd(&a.v_conics[3 * g + 2], g_cc);
                unsafeAtomicAdd(&a.v_colors[3 * g], g_r);
                unsafeAtomicAdd(&a.v_colors[3 * g + 1], g_g);
                unsafeAtomicAdd(&a.v_colors[3 * g + 2], g_b);
                unsafeAtomicAdd(&a.v_opac[g], g_o);
                if (want_abs) {
                    unsafeAtomicAdd(&a.v_means2d_abs[2 * g], s_ax);
                    unsafeAtomicAdd(&a.v_means2d_abs[2 * g + 1], s_ay);
                }
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
                         float *v_colors, float *v_opac, float *v_means2d_abs, hipStream_t s) {
    const size_t CN = (size_t)cams.C * (size_t)N;
    int rc = launch_fill_zero(v_means2d, CN * 2 * sizeof(float), s);
    if (rc == GSR_OK) rc = launch_fill_zero(v_conics, CN * 3 * sizeof(float), s);
    if (rc == GSR_OK) rc = launch_fill_zero(v_colors, CN * 3 * sizeof(float), s);
    if (rc == GSR_OK) rc = launch_fill_zero(v_opac, CN * sizeof(float), s);
    if (rc == GSR_OK && v_means2d_abs) rc = launch_fill_zero(v_means2d_abs, CN * 2 * sizeof(float), s);
    if (rc != GSR_OK || cams.total_tiles == 0 || N == 0) return rc;
    RasterBwdArgs a{p, N, cams.C * N, means2d, conics, colors, opacities, p.antialiased ? comps : nullptr, background,
                    ranges, ids, final_T, last_ids, v_image, v_alpha, v_means2d, v_conics, v_colors, v_opac,
                    v_means2d_abs};
    raster_bwd_kernel<<<dim3((unsigned)cams.total_tiles), dim3(kThreads), 0, s>>>(a, cams);
    return launch_check("rasterize_bwd");
}

}  // namespace gsr
