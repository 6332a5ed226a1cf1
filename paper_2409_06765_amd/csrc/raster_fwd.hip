// Front-to-back alpha compositing of 16x16 tiles (Rasterization of Gaussians).
//
// One 256-thread block per tile; each of the four wave64s owns an 8x8 pixel
// quad (compact quads keep a wave's lanes on the same side of a Gaussian's
// support).  The tile's sorted list is walked in batches of 256 Gaussians
// staged in LDS with one coalesced gather per batch; every lane then reads
// the same LDS entry (broadcast).  A pixel stops when its next composite
// would take T below T_min; the block leaves the list as soon as all its
// pixels have stopped (counted at each batch boundary).
#include "common.hpp"

namespace gsr {
namespace {

constexpr int kThreads = 256;
constexpr int kBatch = 256;

struct RasterArgs {
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
    float *__restrict__ image;
    float *__restrict__ alpha;
    float *__restrict__ final_T;
    int32_t *__restrict__ last_ids;
    int32_t *__restrict__ n_eval;
};

__global__ void __launch_bounds__(kThreads) raster_fwd_kernel(RasterArgs a, CamTable cams) {
    __shared__ float4 s_xyo[kBatch];   // mean x, mean y, opacity, -
    __shared__ float4 s_con[kBatch];   // conic a, b, c, -
    __shared__ float4 s_col[kBatch];   // colour r, g, b, -

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
    const int start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    const float amin = a.p.alpha_min, amax = a.p.alpha_max, tmin = a.p.T_min;

    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    int last = -1, nev = 0, ncomp = 0;
    bool done = !inside;
    for (int b0 = start; b0 < end; b0 += kBatch) {
        if (__syncthreads_count(done) == kThreads) break;
        const int k = b0 + (int)threadIdx.x;
        if (k < end) {
            int g = a.ids[k];
            if ((unsigned)g >= (unsigned)a.CN) g = 0;   // ids come from the sort; this only bounds a bad input
            const int n = g % a.N;
            float o = a.opacities[n];
            if (a.comps) o *= a.comps[g];
            s_xyo[threadIdx.x] = make_float4(a.means2d[2 * g], a.means2d[2 * g + 1], o, 0.0f);
            s_con[threadIdx.x] = make_float4(a.conics[3 * g], a.conics[3 * g + 1], a.conics[3 * g + 2], 0.0f);
            s_col[threadIdx.x] = make_float4(a.colors[3 * g], a.colors[3 * g + 1], a.colors[3 * g + 2], 0.0f);
        }
        __syncthreads();
        const int cnt = min(kBatch, end - b0);
        if (!done) {
            for (int j = 0; j < cnt; j++) {
                const float4 xyo = s_xyo[j];
                const float4 con = s_con[j];
                const float dx = xyo.x - px, dy = xyo.y - py;
                const float sigma = 0.5f * (con.x * dx * dx + con.z * dy * dy) + con.y * dx * dy;
                nev++;
                if (sigma < 0.0f) continue;
                const float al = fminf(amax, xyo.z * __expf(-sigma));
                if (al < amin) continue;
                const float Tn = T * (1.0f - al);
                if (Tn < tmin) { done = true; break; }
                const float wgt = al * T;
                const float4 col = s_col[j];
                C0 += col.x * wgt; C1 += col.y * wgt; C2 += col.z * wgt;
                T = Tn;
                last = b0 + j;
                ncomp++;
            }
        }
    }
    if (!inside) return;
    const int64_t pix = ci.pix_off + (int64_t)yi * ci.W + xi;
    float bg0 = 0.0f, bg1 = 0.0f, bg2 = 0.0f;
    if (a.background) { bg0 = a.background[3 * c]; bg1 = a.background[3 * c + 1]; bg2 = a.background[3 * c + 2]; }
    a.image[3 * pix] = C0 + T * bg0;
    a.image[3 * pix + 1] = C1 + T * bg1;
    a.image[3 * pix + 2] = C2 + T * bg2;
    a.alpha[pix] = 1.0f - T;
    a.final_T[pix] = T;
    a.last_ids[pix] = last;
    if (a.n_eval) {
        a.n_eval[2 * pix] = nev;
        a.n_eval[2 * pix + 1] = ncomp;
    }
}

}  // namespace

int launch_rasterize_fwd(const gsr_params &p, const CamTable &cams, int N, const float *means2d,
                         const float *conics, const float *colors, const float *opacities,
                         const float *comps, const float *background, const int32_t *ranges,
                         const int32_t *ids, float *image, float *alpha, float *final_T, int32_t *last_ids,
                         int32_t *n_eval, hipStream_t s) {
    if (cams.total_tiles == 0) return GSR_OK;
    RasterArgs a{p, N, cams.C * N, means2d, conics, colors, opacities, p.antialiased ? comps : nullptr, background, ranges,
                 ids, image, alpha, final_T, last_ids, n_eval};
    raster_fwd_kernel<<<dim3((unsigned)cams.total_tiles), dim3(kThreads), 0, s>>>(a, cams);
    return launch_check("rasterize_fwd");
}

}  // namespace gsr
