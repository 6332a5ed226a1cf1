// The C ABI (include/gsraster.h): argument checks, per-camera layout tables,
// workspace sizing and status codes around the kernel launchers.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "common.hpp"

namespace gsr {

static thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return GSR_OK;
    return fail(GSR_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int launch_check(const char *what) { return hip_check(hipGetLastError(), what); }

}  // namespace gsr

using namespace gsr;

namespace {

constexpr int kMaxSide = 16384;

int check_params(const gsr_params *p) {
    if (!p) return fail(GSR_EINVAL, "params is NULL");
    if (p->tile != kTile) return fail(GSR_EINVAL, "tile must be %d (got %d)", kTile, p->tile);
    if (p->sh_degree < -1 || p->sh_degree > 3) return fail(GSR_EINVAL, "sh_degree must be in -1..3");
    if (!(p->near_plane > 0.0f) || !(p->far_plane > p->near_plane))
        return fail(GSR_EINVAL, "need 0 < near_plane < far_plane");
    if (!(p->eps2d >= 0.0f) || !(p->jac_clamp >= 0.0f)) return fail(GSR_EINVAL, "eps2d and jac_clamp must be >= 0");
    if (!(p->alpha_min > 0.0f) || !(p->alpha_max < 1.0f) || !(p->alpha_min < p->alpha_max))
        return fail(GSR_EINVAL, "need 0 < alpha_min < alpha_max < 1");
    if (!(p->T_min > 0.0f) || !(p->T_min < 1.0f)) return fail(GSR_EINVAL, "need 0 < T_min < 1");
    if (p->render_depth < GSR_DEPTH_NONE || p->render_depth > GSR_DEPTH_EXPECTED)
        return fail(GSR_EINVAL, "render_depth must be 0, 1 or 2 (got %d)", p->render_depth);
    if (p->colors_shared != 0 && p->colors_shared != 1) return fail(GSR_EINVAL, "colors_shared must be 0 or 1");
    if (p->tile_cull != 0 && p->tile_cull != 1) return fail(GSR_EINVAL, "tile_cull must be 0 or 1");
    return GSR_OK;
}

// Builds the per-camera layout; validates C, N, W, H.
int make_cams(int C, int N, const int32_t *W, const int32_t *H, CamTable &t) {
    if (C < 0 || C > GSR_MAX_CAMERAS) return fail(GSR_EINVAL, "C must be in 0..%d (got %d)", GSR_MAX_CAMERAS, C);
    if (N < 0) return fail(GSR_EINVAL, "N must be >= 0 (got %d)", N);
    if ((int64_t)C * N >= (int64_t)INT32_MAX) return fail(GSR_EINVAL, "C*N must be below 2^31");
    if (C > 0 && (!W || !H)) return fail(GSR_EINVAL, "W and H must be host arrays of C sizes");
    memset(&t, 0, sizeof(t));
    t.C = C;
    int64_t po = 0, to = 0;
    for (int c = 0; c < C; c++) {
        if (W[c] < 1 || W[c] > kMaxSide || H[c] < 1 || H[c] > kMaxSide)
            return fail(GSR_EINVAL, "camera %d: image size %dx%d out of range", c, W[c], H[c]);
        CamInfo &ci = t.cam[c];
        ci.W = W[c];
        ci.H = H[c];
        ci.TX = (W[c] + kTile - 1) / kTile;
        ci.TY = (H[c] + kTile - 1) / kTile;
        ci.pix_off = po;
        ci.tile_base = (int32_t)to;
        po += (int64_t)W[c] * H[c];
        to += (int64_t)ci.TX * ci.TY;
    }
    if (to >= (int64_t)INT32_MAX) return fail(GSR_EINVAL, "too many tiles");
    t.total_tiles = (int32_t)to;
    t.total_pix = po;
    return GSR_OK;
}

#define GSR_NEED(ptr)                                                               \
    do {                                                                            \
        if (!(ptr)) return fail(GSR_EINVAL, "%s: %s must not be NULL", fn, #ptr);  \
    } while (0)

}  // namespace

extern "C" {

int gsr_abi_version(void) { return GSR_ABI_VERSION; }

const char *gsr_last_error(void) { return g_err; }

void gsr_default_params(gsr_params *p) {
    if (!p) return;
    p->near_plane = 0.01f;
    p->far_plane = INFINITY;
    p->eps2d = 0.3f;
    p->jac_clamp = 1.3f;
    p->alpha_min = 1.0f / 255.0f;
    p->alpha_max = 0.99f;
    p->T_min = 1e-4f;
    p->tile = kTile;
    p->sh_degree = -1;
    p->antialiased = 0;
    p->render_depth = GSR_DEPTH_NONE;
    p->colors_shared = 0;
    p->tile_cull = 1;
}

size_t gsr_workspace_bytes(int op, int C, int N, int64_t M) {
    switch (op) {
        case GSR_OP_INTERSECT_COUNT: return count_workspace_bytes((int64_t)(C > 0 ? C : 0) * (N > 0 ? N : 0));
        case GSR_OP_SORT: return sort_workspace_bytes(M > 0 ? M : 0);
        case GSR_OP_RASTERIZE: return pack_workspace_bytes((int64_t)(C > 0 ? C : 0) * (N > 0 ? N : 0));
        case GSR_OP_BIN_PREPARE: return bin_prepare_bytes((int64_t)(C > 0 ? C : 0) * (N > 0 ? N : 0));
        case GSR_OP_BIN_FINISH: return bin_finish_bytes(M > 0 ? M : 0);
        case GSR_OP_PROJECT_BWD: return pose_workspace_bytes(C > 0 ? C : 0, N > 0 ? N : 0);
        case GSR_OP_TILE_ORDER: return tile_order_bytes();
        default: return 0;
    }
}

int gsr_project_fwd(const gsr_params *p, int C, int N, const int32_t *W, const int32_t *H,
                    const float *means, const float *quats, const float *scales, const float *opacities,
                    const float *sh_or_colors, const float *viewmats, const float *Ks,
                    float *means2d, float *conics, int32_t *radii, float *depths, float *colors,
                    float *compensations, gsr_stream_t stream) {
    static const char *fn = "gsr_project_fwd";
    (void)opacities;
    int rc = check_params(p);
    CamTable cams;
    if (rc == GSR_OK) rc = make_cams(C, N, W, H, cams);
    if (rc != GSR_OK) return rc;
    if ((int64_t)C * N == 0) return GSR_OK;
    GSR_NEED(means); GSR_NEED(quats); GSR_NEED(scales); GSR_NEED(viewmats); GSR_NEED(Ks);
    GSR_NEED(means2d); GSR_NEED(conics); GSR_NEED(radii); GSR_NEED(depths);
    if (p->sh_degree >= 0 || colors) { GSR_NEED(sh_or_colors); GSR_NEED(colors); }
    if (p->antialiased) GSR_NEED(compensations);
    return launch_project_fwd(*p, cams, N, means, quats, scales, sh_or_colors, viewmats, Ks, means2d, conics, radii,
                              depths, colors, compensations, (hipStream_t)stream);
}

int gsr_intersect_count(const gsr_params *p, int C, int N, const int32_t *W, const int32_t *H,
                        const float *means2d, const int32_t *radii, int32_t *tiles_per_gauss,
                        int64_t *offsets, int64_t *total_dev, int64_t *total_host,
                        void *ws, size_t ws_bytes, gsr_stream_t stream) {
    static const char *fn = "gsr_intersect_count";
    int rc = check_params(p);
    CamTable cams;
    if (rc == GSR_OK) rc = make_cams(C, N, W, H, cams);
    if (rc != GSR_OK) return rc;
    GSR_NEED(total_dev);
    const int64_t n = (int64_t)C * N;
    if (n > 0) {
        GSR_NEED(means2d); GSR_NEED(radii); GSR_NEED(tiles_per_gauss); GSR_NEED(offsets);
        const size_t need = count_workspace_bytes(n);
        if (!ws || ws_bytes < need)
            return fail(GSR_EWORKSPACE, "%s: workspace of %zu bytes needed, %zu given", fn, need, ws ? ws_bytes : 0);
    }
    hipStream_t s = (hipStream_t)stream;
    rc = launch_intersect_count(*p, cams, N, means2d, radii, tiles_per_gauss, offsets, total_dev, ws, s);
    if (rc != GSR_OK || !total_host) return rc;
    rc = hip_check(hipMemcpyAsync(total_host, total_dev, sizeof(int64_t), hipMemcpyDeviceToHost, s), fn);
    if (rc == GSR_OK) rc = hip_check(hipStreamSynchronize(s), fn);
    if (rc == GSR_OK && *total_host >= (int64_t)INT32_MAX)
        return fail(GSR_EOVERFLOW, "%s: %lld intersections exceed the int32 index range", fn, (long long)*total_host);
    return rc;
}

int gsr_intersect_emit(const gsr_params *p, int C, int N, const int32_t *W, const int32_t *H,
                       const float *means2d, const int32_t *radii, const float *depths,
                       const int64_t *offsets, int64_t M_capacity, uint64_t *keys, int32_t *ids,
                       gsr_stream_t stream) {
    static const char *fn = "gsr_intersect_emit";
    int rc = check_params(p);
    CamTable cams;
    if (rc == GSR_OK) rc = make_cams(C, N, W, H, cams);
    if (rc != GSR_OK) return rc;
    if (M_capacity < 0 || M_capacity >= (int64_t)INT32_MAX) return fail(GSR_EINVAL, "%s: bad M_capacity", fn);
    if ((int64_t)C * N == 0 || M_capacity == 0) return GSR_OK;
    GSR_NEED(means2d); GSR_NEED(radii); GSR_NEED(depths); GSR_NEED(offsets); GSR_NEED(keys); GSR_NEED(ids);
    return launch_intersect_emit(*p, cams, N, means2d, radii, depths, offsets, M_capacity, keys, ids,
                                 (hipStream_t)stream);
}

int gsr_sort_pairs(int64_t M, int key_bits, uint64_t *keys, int32_t *ids, uint64_t *keys_alt,
                   int32_t *ids_alt, void *ws, size_t ws_bytes, gsr_stream_t stream) {
    static const char *fn = "gsr_sort_pairs";
    if (M < 0 || M >= (int64_t)INT32_MAX) return fail(GSR_EINVAL, "%s: M out of range", fn);
    if (key_bits < 1 || key_bits > 64) return fail(GSR_EINVAL, "%s: key_bits must be in 1..64", fn);
    if (M <= 1) return GSR_OK;
    GSR_NEED(keys); GSR_NEED(ids); GSR_NEED(keys_alt); GSR_NEED(ids_alt);
    const size_t need = sort_workspace_bytes(M);
    if (!ws || ws_bytes < need)
        return fail(GSR_EWORKSPACE, "%s: workspace of %zu bytes needed, %zu given", fn, need, ws ? ws_bytes : 0);
    return launch_sort_pairs(M, key_bits, keys, ids, keys_alt, ids_alt, ws, (hipStream_t)stream);
}

int gsr_tile_ranges(int64_t M, const uint64_t *keys, int32_t total_tiles, int32_t *ranges, gsr_stream_t stream) {
    static const char *fn = "gsr_tile_ranges";
    if (M < 0 || M >= (int64_t)INT32_MAX || total_tiles < 0) return fail(GSR_EINVAL, "%s: bad sizes", fn);
    if (total_tiles == 0) return GSR_OK;
    GSR_NEED(ranges);
    if (M > 0) GSR_NEED(keys);
    return launch_tile_ranges(M, keys, total_tiles, ranges, (hipStream_t)stream);
}

int gsr_tile_order(int32_t total_tiles, const int32_t *ranges, int32_t *order, void *ws, size_t ws_bytes,
                   gsr_stream_t stream) {
    static const char *fn = "gsr_tile_order";
    if (total_tiles < 0) return fail(GSR_EINVAL, "%s: total_tiles < 0", fn);
    if (total_tiles == 0) return GSR_OK;
    GSR_NEED(ranges); GSR_NEED(order);
    if (!ws || ws_bytes < tile_order_bytes())
        return fail(GSR_EWORKSPACE, "%s: workspace of %zu bytes needed", fn, tile_order_bytes());
    return launch_tile_order(total_tiles, ranges, order, ws, (hipStream_t)stream);
}

int gsr_bin_prepare(const gsr_params *p, int C, int N, const int32_t *W, const int32_t *H,
                    const float *means2d, const int32_t *radii, const float *depths, const float *conics,
                    const float *opacities, const float *compensations, int64_t *total_dev, int64_t *total_host, void *ws_prep, size_t ws_prep_bytes,
                    gsr_stream_t stream) {
    static const char *fn = "gsr_bin_prepare";
    int rc = check_params(p);
    CamTable cams;
    if (rc == GSR_OK) rc = make_cams(C, N, W, H, cams);
    if (rc != GSR_OK) return rc;
    const int64_t n = (int64_t)C * N;
    if (n > 0) { GSR_NEED(means2d); GSR_NEED(radii); GSR_NEED(depths); }
    if (n > 0 && p->tile_cull) { GSR_NEED(conics); GSR_NEED(opacities); if (p->antialiased) GSR_NEED(compensations); }
    const size_t need = bin_prepare_bytes(n);
    if (!ws_prep || ws_prep_bytes < need)
        return fail(GSR_EWORKSPACE, "%s: workspace of %zu bytes needed, %zu given", fn, need, ws_prep ? ws_prep_bytes : 0);
    hipStream_t s = (hipStream_t)stream;
    rc = launch_bin_prepare(*p, cams, N, means2d, radii, depths, conics, opacities, compensations, ws_prep, total_dev,
                            s);
    if (rc != GSR_OK || !total_host) return rc;
    rc = hip_check(hipMemcpyAsync(total_host, bin_total_ptr(ws_prep, n), sizeof(int64_t), hipMemcpyDeviceToHost, s),
                   fn);
    if (rc == GSR_OK) rc = hip_check(hipStreamSynchronize(s), fn);
    if (rc == GSR_OK && *total_host >= (int64_t)INT32_MAX)
        return fail(GSR_EOVERFLOW, "%s: %lld intersections exceed the int32 index range", fn, (long long)*total_host);
    return rc;
}

int gsr_bin_finish(const gsr_params *p, int C, int N, const int32_t *W, const int32_t *H,
                   const float *means2d, const int32_t *radii, const float *depths, const float *conics,
                   const float *opacities, const float *compensations, int64_t M,
                   int32_t *ids, int32_t *ranges, uint64_t *keys, void *ws_prep, size_t ws_prep_bytes,
                   void *ws_fin, size_t ws_fin_bytes, gsr_stream_t stream) {
    static const char *fn = "gsr_bin_finish";
    int rc = check_params(p);
    CamTable cams;
    if (rc == GSR_OK) rc = make_cams(C, N, W, H, cams);
    if (rc != GSR_OK) return rc;
    if (M < 0 || M >= (int64_t)INT32_MAX) return fail(GSR_EINVAL, "%s: M out of range", fn);
    const int64_t n = (int64_t)C * N;
    if (cams.total_tiles > 0) GSR_NEED(ranges);
    if (M > 0) { GSR_NEED(means2d); GSR_NEED(radii); GSR_NEED(depths); GSR_NEED(ids); }
    if (M > 0 && p->tile_cull) { GSR_NEED(conics); GSR_NEED(opacities); if (p->antialiased) GSR_NEED(compensations); }
    const size_t need_p = bin_prepare_bytes(n), need_f = bin_finish_bytes(M);
    if (!ws_prep || ws_prep_bytes < need_p)
        return fail(GSR_EWORKSPACE, "%s: prepare workspace of %zu bytes needed", fn, need_p);
    if (!ws_fin || ws_fin_bytes < need_f)
        return fail(GSR_EWORKSPACE, "%s: finish workspace of %zu bytes needed, %zu given", fn, need_f,
                    ws_fin ? ws_fin_bytes : 0);
    if (cams.total_tiles == 0) return GSR_OK;
    return launch_bin_finish(*p, cams, N, means2d, radii, depths, conics, opacities, compensations, M, ws_prep,
                             ws_fin, ids, ranges, keys, (hipStream_t)stream);
}

// The channel count: D features (0 .. 32) plus the depth channel, 1 .. 32 in all.
static int check_channels(const char *fn, const gsr_params *p, int D) {
    const int Dt = D + (p->render_depth != GSR_DEPTH_NONE ? 1 : 0);
    if (D < 0 || Dt < 1 || Dt > kMaxChannels)
        return fail(GSR_EINVAL, "%s: D = %d features%s: 1 .. %d channels supported", fn, D,
                    p->render_depth != GSR_DEPTH_NONE ? " plus depth" : "", kMaxChannels);
    return GSR_OK;
}

int gsr_rasterize_fwd(const gsr_params *p, int C, int N, int D, const int32_t *W, const int32_t *H,
                      const float *means2d, const float *conics, const float *colors, const float *depths,
                      const float *opacities, const float *compensations, const float *background,
                      const int32_t *ranges, const int32_t *ids, const int32_t *tile_order, float *image,
                      float *alpha, float *final_T, int32_t *last_ids, int32_t *n_eval, void *ws,
                      size_t ws_bytes, gsr_stream_t stream) {
    static const char *fn = "gsr_rasterize_fwd";
    int rc = check_params(p);
    if (rc == GSR_OK) rc = check_channels(fn, p, D);
    CamTable cams;
    if (rc == GSR_OK) rc = make_cams(C, N, W, H, cams);
    if (rc != GSR_OK) return rc;
    if (cams.total_pix == 0) return GSR_OK;
    GSR_NEED(ranges); GSR_NEED(image); GSR_NEED(alpha); GSR_NEED(final_T); GSR_NEED(last_ids);
    if (N > 0) { GSR_NEED(means2d); GSR_NEED(conics); GSR_NEED(opacities); GSR_NEED(ids); }
    if (N > 0 && D > 0) GSR_NEED(colors);
    if (N > 0 && p->render_depth != GSR_DEPTH_NONE) GSR_NEED(depths);
    if (p->antialiased && N > 0) GSR_NEED(compensations);
    if (N > 0) {
        const size_t need = pack_workspace_bytes((int64_t)C * N);
        if (!ws || ws_bytes < need)
            return fail(GSR_EWORKSPACE, "%s: workspace of %zu bytes needed, %zu given", fn, need, ws ? ws_bytes : 0);
    }
    return launch_rasterize_fwd(*p, cams, N, D, means2d, conics, colors, depths, opacities, compensations, background,
                                ranges, ids, tile_order, image, alpha, final_T, last_ids, n_eval, ws,
                                (hipStream_t)stream);
}

int gsr_rasterize_bwd(const gsr_params *p, int C, int N, int D, const int32_t *W, const int32_t *H,
                      const float *means2d, const float *conics, const float *colors, const float *depths,
                      const float *opacities, const float *compensations, const float *background,
                      const int32_t *ranges, const int32_t *ids, const int32_t *tile_order,
                      const float *image, const float *final_T, const int32_t *last_ids,
                      const float *v_image, const float *v_alpha,
                      float *v_means2d, float *v_conics, float *v_colors, float *v_depths, float *v_opacities,
                      float *v_means2d_abs, void *ws, size_t ws_bytes, int flags, gsr_stream_t stream) {
    static const char *fn = "gsr_rasterize_bwd";
    if (flags & ~(GSR_BWD_ACCUMULATE | GSR_BWD_PACKED)) return fail(GSR_EINVAL, "%s: unknown flags 0x%x", fn, flags);
    int rc = check_params(p);
    if (rc == GSR_OK) rc = check_channels(fn, p, D);
    CamTable cams;
    if (rc == GSR_OK) rc = make_cams(C, N, W, H, cams);
    if (rc != GSR_OK) return rc;
    if ((int64_t)C * N == 0) return GSR_OK;
    GSR_NEED(means2d); GSR_NEED(conics); GSR_NEED(opacities); GSR_NEED(ranges); GSR_NEED(ids);
    GSR_NEED(final_T); GSR_NEED(last_ids); GSR_NEED(v_image);
    GSR_NEED(v_means2d); GSR_NEED(v_conics); GSR_NEED(v_opacities);
    if (D > 0) { GSR_NEED(colors); GSR_NEED(v_colors); }
    if (p->render_depth != GSR_DEPTH_NONE) { GSR_NEED(depths); GSR_NEED(v_depths); }
    if (p->render_depth == GSR_DEPTH_EXPECTED) GSR_NEED(image);
    if (p->antialiased) GSR_NEED(compensations);
    const size_t need = pack_workspace_bytes((int64_t)C * N);
    if (!ws || ws_bytes < need)
        return fail(GSR_EWORKSPACE, "%s: workspace of %zu bytes needed, %zu given", fn, need, ws ? ws_bytes : 0);
    return launch_rasterize_bwd(*p, cams, N, D, means2d, conics, colors, depths, opacities, compensations,
                                background, ranges, ids, tile_order, image, final_T, last_ids, v_image, v_alpha,
                                v_means2d, v_conics, v_colors, v_depths, v_opacities, v_means2d_abs, ws, flags,
                                (hipStream_t)stream);
}

int gsr_project_bwd(const gsr_params *p, int C, int N, const int32_t *W, const int32_t *H,
                    const float *means, const float *quats, const float *scales, const float *opacities,
                    const float *sh_or_colors, const float *viewmats, const float *Ks,
                    const int32_t *radii, const float *compensations,
                    const float *v_means2d, const float *v_conics, const float *v_colors,
                    const float *v_opacities_cn, const float *v_depths,
                    float *v_means, float *v_quats, float *v_scales, float *v_opacities,
                    float *v_sh_or_colors, float *v_viewmats, void *ws, size_t ws_bytes, gsr_stream_t stream) {
    static const char *fn = "gsr_project_bwd";
    int rc = check_params(p);
    CamTable cams;
    if (rc == GSR_OK) rc = make_cams(C, N, W, H, cams);
    if (rc != GSR_OK) return rc;
    if (N == 0)   // no Gaussians: the pose gradient is zero
        return (v_viewmats && C > 0) ? launch_fill_zero(v_viewmats, (size_t)C * 16 * sizeof(float),
                                                        (hipStream_t)stream) : GSR_OK;
    GSR_NEED(means); GSR_NEED(quats); GSR_NEED(scales); GSR_NEED(opacities);
    GSR_NEED(v_means); GSR_NEED(v_quats); GSR_NEED(v_scales); GSR_NEED(v_opacities);
    const bool colour_grad = p->sh_degree >= 0 || v_colors;   // direct colours may be left out
    if (colour_grad) { GSR_NEED(sh_or_colors); GSR_NEED(v_sh_or_colors); }
    if (C > 0) {
        GSR_NEED(viewmats); GSR_NEED(Ks); GSR_NEED(radii);
        GSR_NEED(v_means2d); GSR_NEED(v_conics); GSR_NEED(v_opacities_cn);
        if (colour_grad) GSR_NEED(v_colors);
        if (p->antialiased) GSR_NEED(compensations);
    }
    if (v_viewmats && C > 0 && N > 0) {
        const size_t need = pose_workspace_bytes(C, N);
        if (!ws || ws_bytes < need)
            return fail(GSR_EWORKSPACE, "%s: workspace of %zu bytes needed for v_viewmats, %zu given", fn, need,
                        ws ? ws_bytes : 0);
    }
    return launch_project_bwd(*p, cams, N, means, quats, scales, opacities, sh_or_colors, viewmats, Ks, radii,
                              compensations, v_means2d, v_conics, v_colors, v_opacities_cn, v_depths, v_means,
                              v_quats, v_scales, v_opacities, v_sh_or_colors, v_viewmats, ws, (hipStream_t)stream);
}

}  // extern "C"
