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
    if (p->grad_records != 0 && p->grad_records != 1) return fail(GSR_EINVAL, "grad_records must be 0 or 1");
    return GSR_OK;
}

// The grad_records layout holds plain RGB only: three colour channels per (camera, Gaussian).
int check_grad_records(const char *fn, const gsr_params *p, int D) {
    if (!p->grad_records) return GSR_OK;
    if (D != 3 || p->render_depth != GSR_DEPTH_NONE || p->colors_shared)
        return fail(GSR_EINVAL, "%s: grad_records needs D = 3, no depth channel and colours per camera", fn);
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
    p->grad_records = 0;
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
        case GSR_OP_L1_LOSS: return (size_t)kL1Blocks * sizeof(double);
        case GSR_OP_DENSIFY_PLAN: return densify_plan_bytes(N > 0 ? N : 0);
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

int gsr_sort_pairs_noalloc(int64_t M, int key_bits, uint64_t *keys, int32_t *ids, uint64_t *keys_alt,
                           int32_t *ids_alt, gsr_stream_t stream) {
    static const char *fn = "gsr_sort_pairs_noalloc";
    if (M < 0 || M > sort_static_max_pairs())
        return fail(GSR_EINVAL, "%s: M must be in 0..%lld (got %lld)", fn, (long long)sort_static_max_pairs(),
                    (long long)M);
    if (key_bits < 1 || key_bits > 64) return fail(GSR_EINVAL, "%s: key_bits must be in 1..64", fn);
    if (M <= 1) return GSR_OK;
    GSR_NEED(keys); GSR_NEED(ids); GSR_NEED(keys_alt); GSR_NEED(ids_alt);
    return launch_sort_pairs_static(M, key_bits, keys, ids, keys_alt, ids_alt, (hipStream_t)stream);
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

int gsr_fill_zero(void *ptr, size_t bytes, gsr_stream_t stream) {
    static const char *fn = "gsr_fill_zero";
    if (bytes == 0) return GSR_OK;
    GSR_NEED(ptr);
    if (bytes % 4 != 0 || ((uintptr_t)ptr & 3u) != 0)
        return fail(GSR_EINVAL, "%s: ptr must be 4-byte aligned and bytes a multiple of 4", fn);
    return launch_fill_zero(ptr, bytes, (hipStream_t)stream);
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
    GSR_NEED(v_means2d);
    if (p->grad_records) {
        rc = check_grad_records(fn, p, D);
        if (rc != GSR_OK) return rc;
        if (v_conics || v_colors || v_opacities)
            return fail(GSR_EINVAL, "%s: with grad_records v_conics, v_colors and v_opacities must be NULL", fn);
        GSR_NEED(colors);
    } else {
        GSR_NEED(v_conics); GSR_NEED(v_opacities);
        if (D > 0) { GSR_NEED(colors); GSR_NEED(v_colors); }
    }
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
    if (p->grad_records) {
        rc = check_grad_records(fn, p, 3);
        if (rc != GSR_OK) return rc;
        if (v_conics || v_colors || v_opacities_cn)
            return fail(GSR_EINVAL, "%s: with grad_records v_conics, v_colors and v_opacities_cn must be NULL", fn);
    }
    // direct colours may be left out (records always carry a colour gradient: read when sh_or_colors is given)
    const bool colour_grad = p->sh_degree >= 0 || (p->grad_records ? v_sh_or_colors != nullptr : v_colors != nullptr);
    if (colour_grad) { GSR_NEED(sh_or_colors); GSR_NEED(v_sh_or_colors); }
    if (C > 0) {
        GSR_NEED(viewmats); GSR_NEED(Ks); GSR_NEED(radii);
        GSR_NEED(v_means2d);
        if (!p->grad_records) {
            GSR_NEED(v_conics); GSR_NEED(v_opacities_cn);
            if (colour_grad) GSR_NEED(v_colors);
        }
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

// ---- training-loop steps ----------------------------------------------------------------
int gsr_l1_loss(int64_t n, const float *image, const float *target, float scale, float *v_image, float *loss,
                void *ws, size_t ws_bytes, gsr_stream_t stream) {
    static const char *fn = "gsr_l1_loss";
    if (n < 0) return fail(GSR_EINVAL, "%s: n < 0", fn);
    GSR_NEED(loss);
    if (n == 0) return launch_fill_zero(loss, sizeof(float), (hipStream_t)stream);
    GSR_NEED(image); GSR_NEED(target); GSR_NEED(v_image);
    if (v_image == image || v_image == target) return fail(GSR_EINVAL, "%s: v_image aliases an input", fn);
    const size_t need = (size_t)kL1Blocks * sizeof(double);
    if (!ws || ws_bytes < need) return fail(GSR_EWORKSPACE, "%s: workspace of %zu bytes needed", fn, need);
    return launch_l1_loss(n, image, target, scale, v_image, loss, ws, (hipStream_t)stream);
}

int gsr_activate(int64_t n, const float *raw, int32_t activation, float *out, gsr_stream_t stream) {
    static const char *fn = "gsr_activate";
    if (n < 0 || n > ((int64_t)INT32_MAX << 8)) return fail(GSR_EINVAL, "%s: n out of range", fn);
    if (activation < GSR_ACT_NONE || activation > GSR_ACT_SIGMOID)
        return fail(GSR_EINVAL, "%s: unknown activation %d", fn, activation);
    if (n == 0) return GSR_OK;
    GSR_NEED(raw); GSR_NEED(out);
    return launch_activate(n, raw, activation, out, (hipStream_t)stream);
}

int gsr_adam_step(int n_groups, const gsr_adam_group *groups, int32_t step, float beta1, float beta2, float eps,
                  gsr_stream_t stream) {
    static const char *fn = "gsr_adam_step";
    if (n_groups < 0 || n_groups > GSR_ADAM_MAX_GROUPS)
        return fail(GSR_EINVAL, "%s: n_groups must be in 0..%d", fn, GSR_ADAM_MAX_GROUPS);
    if (n_groups > 0 && !groups) return fail(GSR_EINVAL, "%s: groups is NULL", fn);
    if (step < 1) return fail(GSR_EINVAL, "%s: step must be >= 1", fn);
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f))
        return fail(GSR_EINVAL, "%s: betas must be in [0, 1)", fn);
    if (!(eps >= 0.0f)) return fail(GSR_EINVAL, "%s: eps must be >= 0", fn);
    AdamLaunch a;
    memset(&a, 0, sizeof(a));
    for (int i = 0; i < n_groups; i++) {
        const gsr_adam_group &g = groups[i];
        if (g.n < 0) return fail(GSR_EINVAL, "%s: group %d: n < 0", fn, i);
        if (g.activation < GSR_ACT_NONE || g.activation > GSR_ACT_SIGMOID)
            return fail(GSR_EINVAL, "%s: group %d: unknown activation %d", fn, i, g.activation);
        if (g.activation == GSR_ACT_NONE && g.reg != 0.0f)
            return fail(GSR_EINVAL, "%s: group %d: reg needs an activation", fn, i);
        if (g.row < 0 || g.row_first < 0) return fail(GSR_EINVAL, "%s: group %d: row < 0", fn, i);
        if (g.n > 0 && (!g.param || !g.grad || !g.exp_avg || !g.exp_avg_sq))
            return fail(GSR_EINVAL, "%s: group %d: NULL tensor", fn, i);
        a.g[i] = g;
    }
    a.n_groups = n_groups;
    a.c = adam_consts(beta1, beta2, eps, step);
    return launch_adam(a, (hipStream_t)stream);
}

int gsr_densify_stats(int C, int N, const int32_t *W, const int32_t *H, const int32_t *radii,
                      const float *v_means2d, float scale, float *grad_accum, int32_t *count, gsr_stream_t stream) {
    static const char *fn = "gsr_densify_stats";
    CamTable cams;
    int rc = make_cams(C, N, W, H, cams);
    if (rc != GSR_OK) return rc;
    if ((int64_t)C * N == 0) return GSR_OK;
    GSR_NEED(radii); GSR_NEED(v_means2d); GSR_NEED(grad_accum); GSR_NEED(count);
    return launch_densify_stats(cams, N, radii, v_means2d, scale, grad_accum, count, (hipStream_t)stream);
}

int gsr_densify_plan(int N, const float *grad_accum, const int32_t *count, const float *scales,
                     const float *opacities, float grad_threshold, float scale_threshold, float prune_opacity,
                     int32_t *action, int64_t *offsets, int64_t *total_host, void *ws, size_t ws_bytes,
                     gsr_stream_t stream) {
    static const char *fn = "gsr_densify_plan";
    if (N < 0 || N > INT32_MAX / 2) return fail(GSR_EINVAL, "%s: N must be in 0..2^30", fn);
    GSR_NEED(offsets);
    if (N > 0) { GSR_NEED(grad_accum); GSR_NEED(count); GSR_NEED(scales); GSR_NEED(opacities); GSR_NEED(action); }
    if (grad_threshold != grad_threshold || scale_threshold != scale_threshold || prune_opacity != prune_opacity)
        return fail(GSR_EINVAL, "%s: NaN threshold", fn);
    const size_t need = densify_plan_bytes(N);
    if (!ws || ws_bytes < need) return fail(GSR_EWORKSPACE, "%s: workspace of %zu bytes needed", fn, need);
    hipStream_t s = (hipStream_t)stream;
    int rc = launch_densify_plan(N, grad_accum, count, scales, opacities, grad_threshold, scale_threshold,
                                 prune_opacity, action, offsets, ws, s);
    if (rc != GSR_OK || !total_host) return rc;
    rc = hip_check(hipMemcpyAsync(total_host, offsets + N, sizeof(int64_t), hipMemcpyDeviceToHost, s), fn);
    if (rc == GSR_OK) rc = hip_check(hipStreamSynchronize(s), fn);
    return rc;
}

int gsr_densify_apply(int N, const int32_t *action, const int64_t *offsets, const float *quats,
                      const float *log_scales, const float *split_normals, float split_shrink, int n_columns,
                      const gsr_densify_column *columns, gsr_stream_t stream) {
    static const char *fn = "gsr_densify_apply";
    if (N < 0 || N > INT32_MAX / 2) return fail(GSR_EINVAL, "%s: N must be in 0..2^30", fn);
    if (n_columns < 0 || n_columns > GSR_DENSIFY_MAX_COLUMNS)
        return fail(GSR_EINVAL, "%s: n_columns must be in 0..%d", fn, GSR_DENSIFY_MAX_COLUMNS);
    if (n_columns > 0 && !columns) return fail(GSR_EINVAL, "%s: columns is NULL", fn);
    bool means = false, logs = false;
    for (int i = 0; i < n_columns; i++) {
        const gsr_densify_column &c = columns[i];
        if (c.kind < GSR_COLUMN_COPY || c.kind > GSR_COLUMN_STATE)
            return fail(GSR_EINVAL, "%s: column %d: unknown kind %d", fn, i, c.kind);
        if (c.width < 1 || c.width > 4096) return fail(GSR_EINVAL, "%s: column %d: width must be in 1..4096", fn, i);
        if ((c.kind == GSR_COLUMN_MEANS || c.kind == GSR_COLUMN_LOG_SCALES) && c.width != 3)
            return fail(GSR_EINVAL, "%s: column %d: means and log-scales have width 3", fn, i);
        if (N > 0 && (!c.src || !c.dst)) return fail(GSR_EINVAL, "%s: column %d: NULL array", fn, i);
        if (N > 0 && c.src == c.dst) return fail(GSR_EINVAL, "%s: column %d: dst must not be src", fn, i);
        means |= c.kind == GSR_COLUMN_MEANS;
        logs |= c.kind == GSR_COLUMN_LOG_SCALES;
    }
    if (N == 0 || n_columns == 0) return GSR_OK;
    GSR_NEED(action); GSR_NEED(offsets);
    if (means) { GSR_NEED(quats); GSR_NEED(log_scales); GSR_NEED(split_normals); }
    if (logs && !(split_shrink > 0.0f && split_shrink < 3.0e38f))
        return fail(GSR_EINVAL, "%s: split_shrink must be positive and finite", fn);
    const float log_shrink = logs ? (float)log((double)split_shrink) : 0.0f;
    return launch_densify_apply(N, action, offsets, quats, log_scales, split_normals, log_shrink, n_columns, columns,
                                (hipStream_t)stream);
}

int gsr_opacity_reset(int N, float *logits, float *exp_avg, float *exp_avg_sq, float *opacities,
                      float max_opacity, gsr_stream_t stream) {
    static const char *fn = "gsr_opacity_reset";
    if (N < 0) return fail(GSR_EINVAL, "%s: N < 0", fn);
    if (!(max_opacity > 0.0f && max_opacity < 1.0f)) return fail(GSR_EINVAL, "%s: need 0 < max_opacity < 1", fn);
    if (N == 0) return GSR_OK;
    GSR_NEED(logits); GSR_NEED(exp_avg); GSR_NEED(exp_avg_sq);
    const double v = max_opacity;
    return launch_opacity_reset(N, logits, exp_avg, exp_avg_sq, opacities, (float)log(v / (1.0 - v)),
                                (hipStream_t)stream);
}

int gsr_mcmc_noise(int N, float *means, const float *quats, const float *scales, const float *opacities,
                   const float *normals, float coeff, float k, float t, gsr_stream_t stream) {
    static const char *fn = "gsr_mcmc_noise";
    if (N < 0) return fail(GSR_EINVAL, "%s: N < 0", fn);
    if (!(fabsf(coeff) < 3.0e38f) || !(fabsf(k) < 3.0e38f) || !(fabsf(t) < 3.0e38f))
        return fail(GSR_EINVAL, "%s: coeff, k and t must be finite", fn);
    if (N == 0) return GSR_OK;
    GSR_NEED(means); GSR_NEED(quats); GSR_NEED(scales); GSR_NEED(opacities); GSR_NEED(normals);
    return launch_mcmc_noise(N, means, quats, scales, opacities, normals, coeff, k, t, (hipStream_t)stream);
}
