// Front-to-back alpha compositing of 16x16 tiles (Rasterization of Gaussians).
//
// One 256-thread block per tile; each of the four wave64s owns an 8x8 pixel
// quad.  The tile's sorted list is walked in batches of 256 Gaussians staged
// in LDS by one coalesced gather.  While staging, the batch is also split
// into four per-quad index lists (compact_quads) of the entries whose
// alpha >= alpha_min support box (precomputed per projected Gaussian by
// pack_kernel) reaches the quad, so a wave only visits entries that can
// change one of its pixels; the rest are below alpha_min everywhere in the
// quad and would be skipped by every pixel anyway.  The per-pixel update is
// branch-free (selects), so the wave never splits on skip/stop decisions.
// The block leaves the list once every pixel has stopped.
#include "common.hpp"

namespace gsr {
namespace {

constexpr int kThreads = 256;
constexpr int kBatch = 256;

// Colours go into the record only for plain RGB (D = 3, no depth channel);
// other channel sets are staged from the feature array by the compositing
// kernels.  shared: colours are [N,D], one row per Gaussian for all cameras.
__global__ void __launch_bounds__(256) pack_kernel(int CN, int N, bool rgb, bool shared, float alpha_min,
        const float *__restrict__ means2d, const float *__restrict__ conics, const float *__restrict__ colors,
        const float *__restrict__ opacities, const float *__restrict__ comps, PackedGauss *__restrict__ out) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= CN) return;
    const int n = g % N;
    float o = opacities[n];
    if (comps) o *= comps[g];
    const float ca = conics[3 * g], cb = conics[3 * g + 1], cc = conics[3 * g + 2];
    const float2 h = support_extent(ca, cb, cc, o, alpha_min);
    PackedGauss r;
    r.xyoh = make_float4(means2d[2 * g], means2d[2 * g + 1], o, h.x);
    // the completed square of sigma (see PackedGauss): A, r, Q in double, each rounded once
    float A = 0.5f * kLog2e * ca, rb = 0.0f, Q = 0.5f * kLog2e * cc;
    if (ca > 0.0f) {
        const double ad = ca, bd = cb, cd = cc;
        A = (float)(0.5 * kLog2eD * ad);
        rb = cb / ca;
        Q = (float)(0.5 * kLog2eD * ((ad * cd - bd * bd) / ad));
    }
    r.conh = make_float4(A, rb, Q, h.y);
    const float Lq = o >= alpha_min ? log2f(o / alpha_min) : -1.0f;
    const int f = shared ? n : g;
    r.col = rgb ? make_float4(colors[3 * f], colors[3 * f + 1], colors[3 * f + 2], Lq)
                : make_float4(0.0f, 0.0f, 0.0f, Lq);
    out[g] = r;
}

struct RasterArgs {
    gsr_params p;
    int N;
    int CN;
    int D;                                // feature channels of colors
    int Dt;                               // channels composited: D, plus one for depth; at most the kernel's DM
    const float *__restrict__ feat;       // colors [C,N,D] or [N,D] (read here unless plain RGB)
    const float *__restrict__ depths;     // [C,N], composited as channel D when a depth mode is set
    const PackedGauss *__restrict__ gauss;
    const float *__restrict__ background;
    const int32_t *__restrict__ ranges;
    const int32_t *__restrict__ ids;
    const int32_t *__restrict__ order;     // dispatch order of the tiles (nullable)
    float *__restrict__ image;
    float *__restrict__ alpha;
    float *__restrict__ final_T;
    int32_t *__restrict__ last_ids;
    int32_t *__restrict__ n_eval;
};

// kCount: also count the entries each pixel evaluates and composites.
// DM: channel capacity; DM = 3 takes RGB from the packed records, any other
// DM stages a.Dt <= DM channels per entry into LDS.
template <bool kCount, int DM, bool kStd>
__global__ void __launch_bounds__(kThreads) raster_fwd_kernel(RasterArgs a, CamTable cams) {
    constexpr bool kRGB = DM == 3;
    __shared__ float4 s_xyo[kBatch];   // mean x, mean y, opacity, list position (int bits)
    __shared__ float4 s_con[kBatch];   // conic a, b, c, -
    __shared__ float4 s_col[kBatch];   // colour r, g, b, log2(opacity / alpha_min)
    __shared__ float s_feat[kRGB ? 1 : DM * kBatch];
    // the plain RGB walk's lists hold byte offsets (16-bit), the others slots (8-bit)
    constexpr bool kFast = kRGB && kStd && !kCount;
    using QL = std::conditional_t<kFast, uint16_t, uint8_t>;
    __shared__ __align__(16) QL s_qlist[4][kBatch];
    __shared__ int32_t s_wcnt[4][4];
    __shared__ int32_t s_qcnt[4];

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
    const int start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    // kStd: the thresholds are the defaults, compiled in as constants (no per-entry canonicalisation)
    const float amin = kStd ? kStdAlphaMin : a.p.alpha_min, amax = kStd ? kStdAlphaMax : a.p.alpha_max;
    const float tmin = kStd ? kStdTMin : a.p.T_min;

    float T = 1.0f, Wacc = 0.0f, Cacc[DM];   // Wacc: sum of alpha T, the expected-depth normaliser
#pragma unroll
    for (int d = 0; d < DM; d++) Cacc[d] = 0.0f;
    int last = -1, ncomp = 0, stop_at = -1;
    int nq = 0, nq_last = 0, nit = 0;        // counts: quad-list entries evaluated live, up to the last, stepped
    bool done = !inside;
    float live = inside ? 1.0f : 0.0f;       // the plain RGB walk's form of !done
    for (int b0 = start; b0 < end; b0 += kBatch) {
        if (__syncthreads_count(done) == kThreads) break;
        const int k = b0 + (int)threadIdx.x;
        uint32_t qm = 0u;
        bool rec_ok = true;
        if (k < end) {
            int g = a.ids[k];
            if ((unsigned)g >= (unsigned)a.CN) g = 0;   // ids come from the sort; this only bounds a bad input
            const PackedGauss r = a.gauss[g];
            qm = refine_quad_mask(quad_mask(r.xyoh.x, r.xyoh.y, r.xyoh.w, r.conh.w, tile_x0, tile_y0), r.xyoh,
                                  r.conh, r.col.w, tile_x0, tile_y0);
            // the fourth word (the support extent, used above) takes the entry's list position, which the
            // plain RGB walk records for the last composited entry without scalar arithmetic
            s_xyo[threadIdx.x] = make_float4(r.xyoh.x, r.xyoh.y, r.xyoh.z, __int_as_float(k));
            s_con[threadIdx.x] = r.conh;
            rec_ok = isfinite(r.xyoh.x) && isfinite(r.xyoh.y) && isfinite(r.conh.y) && r.conh.x >= 0.0f &&
                     r.conh.z >= 0.0f && r.conh.x < INFINITY && r.conh.z < INFINITY;
            s_col[threadIdx.x] = r.col;
            if (!kRGB) stage_features<DM, kBatch>(a, c, g, threadIdx.x, s_feat);
        }
        compact_quads(qm, s_qlist, s_wcnt, s_qcnt);
        const int cnt = __builtin_amdgcn_readfirstlane(s_qcnt[w]);   // entries that can reach this wave's quad
        // a batch whose records are all finite with A, Q >= 0 has sigma >= 0 at every pixel (a sum of
        // two non-negative terms): its walk needs no sign test
        bool sig_free = true;
        if constexpr (kRGB && kStd && !kCount) sig_free = __syncthreads_and(rec_ok) != 0;
        if (__all(done)) continue;
        if constexpr (kRGB && kStd && !kCount) {
            // The timed instance: the same decisions with the per-lane state in vector registers and
            // every condition applied by a select, so no lane mask is combined by scalar instructions
            // (the scalar unit, shared by the waves of a compute unit, limits this loop more than the
            // vector units); the list entries are the records' byte offsets, eight per LDS read, kept in
            // vector registers; the list position of the last composited entry comes with the record;
            // the all-stopped test runs once per eight entries.  With the default thresholds an entry
            // that reaches a live pixel has alpha >= 1/255 and T >= 1e-4 before it, so it composites
            // exactly where its weight alpha T is positive.
            auto walk = [&](auto check) {
            constexpr bool CHECK_SIG = decltype(check)::value;
            for (int j0 = 0; j0 < cnt; j0 += 8) {
                const int jn = min(cnt - j0, 8);
                const uint4 o8 = *reinterpret_cast<const uint4 *>(&s_qlist[w][j0]);
                const uint32_t o2[4] = {o8.x, o8.y, o8.z, o8.w};
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    if (u >= jn) break;
                    const uint32_t off = (o2[u >> 1] >> (16 * (u & 1))) & 0xFFFFu;   // 16 x slot
                    const float4 xyo = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(s_xyo) + off);
                    const float4 con = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(s_con) + off);
                    const float dx = xyo.x - px, dy = xyo.y - py;
                    const float sig = scaled_sigma(con, dx, dy);
                    const float al = min_alpha(xyo.z * __builtin_amdgcn_exp2f(-sig), amax);
                    float ae = (CHECK_SIG && sig < 0.0f) ? 0.0f : al;   // alpha where the entry is used, else 0
                    ae = ae >= amin ? ae : 0.0f;
                    ae *= live;
                    const float Tn = T * (1.0f - ae);
                    const bool keep = Tn >= tmin;                 // false only where this entry stops the pixel
                    const float wgt = keep ? ae * T : 0.0f;
                    const float4 col = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(s_col) + off);
                    Cacc[0] = fmaf(col.x, wgt, Cacc[0]);
                    Cacc[1] = fmaf(col.y, wgt, Cacc[1]);
                    Cacc[2] = fmaf(col.z, wgt, Cacc[2]);
                    T = keep ? Tn : T;
                    live = keep ? live : 0.0f;
                    last = wgt > 0.0f ? __float_as_int(xyo.w) : last;
                }
                if (__all(live == 0.0f)) break;
            }
            };
            if (sig_free) walk(std::false_type{});
            else walk(std::true_type{});
            done = live == 0.0f;
            continue;
        }
        for (int j = 0; j < cnt; j++) {
            const int e = __builtin_amdgcn_readfirstlane(s_qlist[w][j]);
            const float4 xyo = s_xyo[e];
            const float4 con = s_con[e];
            const float dx = xyo.x - px, dy = xyo.y - py;
            const float sig = scaled_sigma(con, dx, dy);          // log2(e) sigma
            const float al = min_alpha(xyo.z * __builtin_amdgcn_exp2f(-sig), amax);
            const float Tn = T * (1.0f - al);
            const bool use = !done && sig >= 0.0f && al >= amin;
            const bool stop = use && Tn < tmin;
            const bool comp = use && !stop;
            if (kCount) {
                stop_at = stop ? b0 + e : stop_at;
                nit++;
                nq += done ? 0 : 1;
                nq_last = comp ? nq : nq_last;
            }
            done = done || stop;
            const float wgt = comp ? al * T : 0.0f;
            if (kRGB) {
                const float4 col = s_col[e];
                Cacc[0] += col.x * wgt; Cacc[1] += col.y * wgt; Cacc[2] += col.z * wgt;
            } else {
#pragma unroll
                for (int d = 0; d < DM; d++) Cacc[d] += s_feat[d * kBatch + e] * wgt;
                Wacc += wgt;
            }
            T = comp ? Tn : T;
            last = comp ? b0 + e : last;
            if (kCount) ncomp += comp ? 1 : 0;
            if ((j & 7) == 7 && __all(done)) break;
        }
    }
    if (!inside) return;
    const int64_t pix = ci.pix_off + (int64_t)yi * ci.W + xi;
    const int D = kRGB ? 3 : a.D, Dt = kRGB ? 3 : a.Dt;
#pragma unroll
    for (int d = 0; d < DM; d++) {
        if (d < D) {
            a.image[(int64_t)Dt * pix + d] = Cacc[d] + T * (a.background ? a.background[D * c + d] : 0.0f);
        } else if (d < Dt) {                         // depth: no background; expected depth divides by sum alpha T
            a.image[(int64_t)Dt * pix + d] =
                a.p.render_depth == GSR_DEPTH_EXPECTED ? (Wacc > 0.0f ? Cacc[d] / Wacc : 0.0f) : Cacc[d];
        }
    }
    a.alpha[pix] = 1.0f - T;
    a.final_T[pix] = T;
    a.last_ids[pix] = last;
    if (kCount) {
        // entries evaluated: up to and including the one that stopped the pixel, else the whole list
        int32_t *ne = a.n_eval + 5 * pix;
        ne[0] = stop_at >= 0 ? stop_at - start + 1 : end - start;
        ne[1] = ncomp;
        ne[2] = nq;          // entries of the quad's list this pixel evaluated (the stopping one included)
        ne[3] = nq_last;     // entries of the quad's list up to its last composited one (a backward's walk)
        ne[4] = nit;         // entries its wave stepped through (evaluations issued for this lane)
    }
}

}  // namespace

size_t pack_workspace_bytes(int64_t cn) { return ((size_t)(cn > 0 ? cn : 1) * sizeof(PackedGauss) + 255) & ~(size_t)255; }

int launch_pack(const gsr_params &p, int CN, int N, int D, const float *means2d, const float *conics,
                const float *colors, const float *opacities, const float *comps, PackedGauss *out, hipStream_t s) {
    pack_kernel<<<dim3((unsigned)((CN + 255) / 256)), dim3(256), 0, s>>>(
        CN, N, channel_capacity(p, D) == 3, p.colors_shared != 0, p.alpha_min, means2d, conics, colors, opacities,
        comps, out);
    return launch_check("pack");
}

int composited_channels(const gsr_params &p, int D) { return D + (p.render_depth != GSR_DEPTH_NONE ? 1 : 0); }

int channel_capacity(const gsr_params &p, int D) {
    if (D == 3 && p.render_depth == GSR_DEPTH_NONE) return 3;
    const int Dt = composited_channels(p, D);
    return Dt <= 4 ? 4 : Dt <= 8 ? 8 : Dt <= 16 ? 16 : 32;
}

int launch_rasterize_fwd(const gsr_params &p, const CamTable &cams, int N, int D, const float *means2d,
                         const float *conics, const float *colors, const float *depths, const float *opacities,
                         const float *comps, const float *background, const int32_t *ranges,
                         const int32_t *ids, const int32_t *tile_order, float *image, float *alpha,
                         float *final_T, int32_t *last_ids, int32_t *n_eval, void *ws, hipStream_t s) {
    if (cams.total_tiles == 0) return GSR_OK;
    const int CN = cams.C * N;
    PackedGauss *gauss = (PackedGauss *)ws;
    if (CN > 0) {
        int rc = launch_pack(p, CN, N, D, means2d, conics, colors, opacities, p.antialiased ? comps : nullptr,
                             gauss, s);
        if (rc != GSR_OK) return rc;
    }
    RasterArgs a{p, N, CN, D, composited_channels(p, D), colors, depths, gauss, background, ranges, ids, tile_order,
                 image, alpha, final_T, last_ids, n_eval};
    const dim3 grid((unsigned)cams.total_tiles), block(kThreads);
    const bool std_thr = standard_thresholds(p);
#define GSR_RF(DM) do { if (n_eval) raster_fwd_kernel<true, DM, false><<<grid, block, 0, s>>>(a, cams); \
                        else if (std_thr) raster_fwd_kernel<false, DM, true><<<grid, block, 0, s>>>(a, cams); \
                        else raster_fwd_kernel<false, DM, false><<<grid, block, 0, s>>>(a, cams); } while (0)
    switch (channel_capacity(p, D)) {
        case 3: GSR_RF(3); break;
        case 4: GSR_RF(4); break;
        case 8: GSR_RF(8); break;
        case 16: GSR_RF(16); break;
        default: GSR_RF(32); break;
    }
#undef GSR_RF
    return launch_check("rasterize_fwd");
}

}  // namespace gsr
