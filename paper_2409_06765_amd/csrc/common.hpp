// Internal declarations shared by the HIP translation units of libgsraster.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "gsraster.h"

namespace gsr {

constexpr int kTile = 16;
constexpr int kWave = 64;

// Per-camera layout, passed to kernels by value (GSR_MAX_CAMERAS entries fit
// well inside the kernel-argument limit).
struct CamInfo {
    int32_t W, H, TX, TY;
    int64_t pix_off;     // first pixel of this camera in the packed images
    int32_t tile_base;   // first global tile id of this camera
    int32_t pad;
};

struct CamTable {
    int32_t C;
    int32_t total_tiles;
    int64_t total_pix;
    CamInfo cam[GSR_MAX_CAMERAS];
};

// Adam constants of one step: betas, 1 - betas, reciprocal bias corrections.
struct AdamConsts {
    float beta1, beta2, omb1, omb2, inv_bc1, inv_bc2, eps;
};

// One Adam element: the chain
// rule through the activation, with the L1 penalty reg on the activated value,
// then the moments and the update; a = act(p) afterwards.  Contraction is off
// here, so the rounding does not depend on the translation unit's flags.
__device__ __forceinline__ void adam_update(const AdamConsts &c, int kind, float reg, float lr, float &p, float g,
                                            float &m, float &v, float &a) {
#pragma clang fp contract(off)
    if (kind == GSR_ACT_EXP) {
        g = (g + reg) * expf(p);
    } else if (kind == GSR_ACT_SIGMOID) {
        const float o = 1.0f / (1.0f + expf(-p));
        g = (g + reg) * (o * (1.0f - o));
    }
    m = c.beta1 * m + c.omb1 * g;
    v = c.beta2 * v + c.omb2 * (g * g);
    const float mh = m * c.inv_bc1;
    const float vh = v * c.inv_bc2;
    p = p - lr * mh / (sqrtf(vh) + c.eps);
    a = kind == GSR_ACT_EXP ? expf(p) : (kind == GSR_ACT_SIGMOID ? 1.0f / (1.0f + expf(-p)) : p);
}
// Status handling (abi.hip): records a message for gsr_last_error().
int fail(int code, const char *fmt, ...);
int hip_check(hipError_t e, const char *what);
int launch_check(const char *what);

// ---- launchers (one per translation unit) ----------------------------------
int launch_project_fwd(const gsr_params &p, const CamTable &cams, int N, const float *means,
                       const float *quats, const float *scales, const float *sh, const float *viewmats,
                       const float *Ks, float *means2d, float *conics, int32_t *radii, float *depths,
                       float *colors, float *comps, hipStream_t s);

int launch_project_bwd(const gsr_params &p, const CamTable &cams, int N, const float *means,
                       const float *quats, const float *scales, const float *opacities, const float *sh,
                       const float *viewmats, const float *Ks, const int32_t *radii, const float *comps,
                       const float *v_means2d, const float *v_conics, const float *v_colors,
                       const float *v_opac_cn, const float *v_depths, float *v_means, float *v_quats,
                       float *v_scales, float *v_opac, float *v_sh, float *v_viewmats, void *ws, hipStream_t s);
size_t pose_workspace_bytes(int C, int N);

size_t count_workspace_bytes(int64_t n);
int launch_intersect_count(const gsr_params &p, const CamTable &cams, int N, const float *means2d,
                           const int32_t *radii, int32_t *counts, int64_t *offsets, int64_t *total_dev,
                           void *ws, hipStream_t s);
int launch_intersect_emit(const gsr_params &p, const CamTable &cams, int N, const float *means2d,
                          const int32_t *radii, const float *depths, const int64_t *offsets, int64_t cap,
                          uint64_t *keys, int32_t *ids, hipStream_t s);

size_t sort_workspace_bytes(int64_t M);
int64_t sort_static_max_pairs();
int launch_sort_pairs_static(int64_t M, int key_bits, uint64_t *keys, int32_t *ids, uint64_t *keys_alt,
                             int32_t *ids_alt, hipStream_t s);
int launch_sort_pairs(int64_t M, int key_bits, uint64_t *keys, int32_t *ids, uint64_t *keys_alt,
                      int32_t *ids_alt, void *ws, hipStream_t s);
int launch_tile_ranges(int64_t M, const uint64_t *keys, int32_t total_tiles, int32_t *ranges, hipStream_t s);

size_t tile_order_bytes();
int launch_tile_order(int32_t T, const int32_t *ranges, int32_t *order, void *ws, hipStream_t s);

size_t bin_prepare_bytes(int64_t n);
size_t bin_finish_bytes(int64_t M);
const int64_t *bin_total_ptr(void *ws_prep, int64_t n);
int launch_bin_prepare(const gsr_params &p, const CamTable &cams, int N, const float *means2d,
                       const int32_t *radii, const float *depths, const float *conics, const float *opacities,
                       const float *comps, void *ws_prep, int64_t *total_dev, hipStream_t s);
int launch_bin_finish(const gsr_params &p, const CamTable &cams, int N, const float *means2d,
                      const int32_t *radii, const float *depths, const float *conics, const float *opacities,
                      const float *comps, int64_t M, void *ws_prep, void *ws_fin, int32_t *ids, int32_t *ranges,
                      uint64_t *keys64, hipStream_t s);

int launch_rasterize_fwd(const gsr_params &p, const CamTable &cams, int N, int D, const float *means2d,
                         const float *conics, const float *colors, const float *depths, const float *opacities,
                         const float *comps, const float *background, const int32_t *ranges,
                         const int32_t *ids, const int32_t *tile_order, float *image, float *alpha, float *final_T,
                         int32_t *last_ids,
                         int32_t *n_eval, void *ws, hipStream_t s);

int launch_rasterize_bwd(const gsr_params &p, const CamTable &cams, int N, int D, const float *means2d,
                         const float *conics, const float *colors, const float *depths, const float *opacities,
                         const float *comps, const float *background, const int32_t *ranges,
                         const int32_t *ids, const int32_t *tile_order, const float *image, const float *final_T,
                         const int32_t *last_ids,
                         const float *v_image, const float *v_alpha, float *v_means2d, float *v_conics,
                         float *v_colors, float *v_depths, float *v_opac, float *v_means2d_abs, void *ws, int flags,
                         hipStream_t s);

int launch_fill_zero(void *ptr, size_t bytes, hipStream_t s);
// Zeroes up to 8 buffers in one launch (NULL or empty entries are skipped).
int launch_fill_zero_multi(int n, void *const *ptrs, const size_t *bytes, hipStream_t s);

// Exclusive prefix sums of int32 counts into int64 offsets, total to *total
// (device); ws of scan_workspace_bytes(n).
size_t scan_workspace_bytes(int64_t n);
int launch_scan_i32(int64_t n, const int32_t *counts, int64_t *offsets, int64_t *total, void *ws, hipStream_t s);

AdamConsts adam_consts(float beta1, float beta2, float eps, int32_t step);

// Training-loop steps (train.hip).
constexpr int kL1Blocks = 1024;
int launch_l1_loss(int64_t n, const float *image, const float *target, float scale, float *v_image, float *loss,
                   void *ws, hipStream_t s);
struct AdamLaunch {
    gsr_adam_group g[GSR_ADAM_MAX_GROUPS];
    int n_groups;
    AdamConsts c;
};
int launch_adam(const AdamLaunch &a, hipStream_t s);
int launch_activate(int64_t n, const float *raw, int kind, float *out, hipStream_t s);
int launch_densify_stats(const CamTable &cams, int N, const int32_t *radii, const float *v_means2d, float scale,
                         float *accum, int32_t *count, hipStream_t s);
size_t densify_plan_bytes(int N);
int launch_densify_plan(int N, const float *accum, const int32_t *count, const float *scales, const float *opacities,
                        float grad_threshold, float scale_threshold, float prune_opacity, int32_t *action,
                        int64_t *offsets, void *ws, hipStream_t s);
int launch_densify_apply(int N, const int32_t *action, const int64_t *offsets, const float *quats,
                         const float *log_scales, const float *normals, float log_shrink, int n_columns,
                         const gsr_densify_column *columns, hipStream_t s);
int launch_opacity_reset(int N, float *logits, float *exp_avg, float *exp_avg_sq, float *opacities, float cap,
                         hipStream_t s);
int launch_mcmc_noise(int N, float *means, const float *quats, const float *scales, const float *opacities,
                      const float *normals, float coeff, float k, float t, hipStream_t s);

// ---- device helpers ----------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// The tile a compositing block works on: blockIdx.x through the dispatch
// order when one is given; -1 (the block does nothing) for an index outside
// the tile range.
__device__ __forceinline__ int block_tile(const int32_t *order, int total_tiles) {
    const int t = order ? order[blockIdx.x] : (int)blockIdx.x;
    return (unsigned)t < (unsigned)total_tiles ? t : -1;
}

// Camera of a global tile id (linear scan; C is small and the value uniform).
__device__ __forceinline__ int camera_of_tile(const CamTable &cams, int tile) {
    int c = 0;
    while (c + 1 < cams.C && tile >= cams.cam[c + 1].tile_base) c++;
    return c;
}

// Tile rectangle of a projected Gaussian (square box of half-width r around
// the 2D mean, clipped to the camera's tile grid).  Evaluated in float32 in
// this exact order: it fixes tile counts and keys bit for bit.
__device__ __forceinline__ void tile_rect(float mx, float my, int r, int TX, int TY,
                                          int &x0, int &x1, int &y0, int &y1) {
#pragma clang fp contract(off)
    const float rf = (float)r;
    const float tl = (float)kTile;
    const float fx0 = floorf((mx - rf) / tl), fx1 = floorf((mx + rf) / tl) + 1.0f;
    const float fy0 = floorf((my - rf) / tl), fy1 = floorf((my + rf) / tl) + 1.0f;
    x0 = (int)fminf(fmaxf(fx0, 0.0f), (float)TX);
    x1 = (int)fminf(fmaxf(fx1, 0.0f), (float)TX);
    y0 = (int)fminf(fmaxf(fy0, 0.0f), (float)TY);
    y1 = (int)fminf(fmaxf(fy1, 0.0f), (float)TY);
}

// Half-extents of the bounding box of a projected Gaussian's alpha >=
// alpha_min support.  alpha = o exp(-sigma) reaches alpha_min only where
// sigma <= L = ln(o / alpha_min), an ellipse with half-widths
// sqrt(2 L Sigma'_xx), sqrt(2 L Sigma'_yy), Sigma' being the inverse conic.  L
// is inflated by a margin larger than the float32 rounding of sigma at any
// pixel (the absolute terms of sigma sum to at most 3 kappa sigma, kappa the
// conic's condition number, so its relative error stays below about
// 1e-6 kappa): a pixel outside the box takes the alpha < alpha_min skip in
// the per-pixel test too.  Returns (-1e30, -1e30) when alpha never reaches
// alpha_min and (1e30, 1e30) (no culling) for ill-conditioned conics.
__device__ __forceinline__ float2 support_extent(float ca, float cb, float cc, float o, float alpha_min) {
    if (!(o >= alpha_min)) return make_float2(-1e30f, -1e30f);   // o exp(-sigma) <= o < alpha_min
    const float det = ca * cc - cb * cb;
    if (!(det > 0.0f)) return make_float2(1e30f, 1e30f);
    const float half_tr = 0.5f * (ca + cc);
    const float lmax = half_tr + sqrtf(fmaxf(half_tr * half_tr - det, 0.0f));
    const float kappa = lmax * lmax / det;
    if (!(kappa < 1e5f)) return make_float2(1e30f, 1e30f);
    const float L = logf(o / alpha_min);
    const float grow = 1.0f + 4e-6f * kappa + 1e-4f;
    const float Lp = L * grow + 1e-4f;
    return make_float2(sqrtf(2.0f * Lp * cc / det) * grow + 1e-3f, sqrtf(2.0f * Lp * ca / det) * grow + 1e-3f);
}

// Which of the four 8x8 pixel quads of a tile (origin tile_x0, tile_y0) meet
// the support box; bit q is quad (q & 1, q >> 1).
__device__ __forceinline__ uint32_t quad_mask(float mx, float my, float hx, float hy, float tile_x0, float tile_y0) {
    uint32_t m = 0u;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const float x0 = tile_x0 + (float)((q & 1) * 8) + 0.5f, x1 = x0 + 7.0f;
        const float y0 = tile_y0 + (float)((q >> 1) * 8) + 0.5f, y1 = y0 + 7.0f;
        if (mx + hx >= x0 && mx - hx <= x1 && my + hy >= y0 && my - hy <= y1) m |= 1u << q;
    }
    return m;
}

// Per projected Gaussian record read by the compositing kernels:
// {mean x, mean y, opacity (times compensation), support half-width x},
// {A, r, Q, support half-width y}, {colour r, g, b, log2(opacity / alpha_min)},
// where, with (a, b, c) the conic, sigma = 1/2 (a dx^2 + c dy^2) + b dx dy is
// held as the completed square
//     log2(e) sigma = A (dx + r dy)^2 + Q dy^2,
//     A = log2(e) a / 2,  r = b / a,  Q = log2(e) (a c - b^2) / (2 a)
// (a > 0 for every projected Gaussian: Sigma' is positive definite).  Both
// terms are non-negative, so unlike the three-term sum it does not cancel
// for needle-like Gaussians: its float32 value is within a few ulps of the
// definition's (plus one ulp of r carried through dy), which is what keeps
// the skip/stop decisions the same as an exact evaluation's everywhere but
// on a hair's breadth of the thresholds.  The scaling gives log2(e) sigma
// directly (scaled_sigma), the argument of the hardware base-2 exponential;
// alpha >= alpha_min exactly where log2(e) sigma <= log2(opacity / alpha_min).
constexpr float kLog2e = 1.4426950408889634f;

// The default skip, clamp and stop thresholds (gsr_default_params); kernels
// specialised for them take the values as constants.
constexpr float kStdAlphaMin = 1.0f / 255.0f, kStdAlphaMax = 0.99f, kStdTMin = 1e-4f;
inline bool standard_thresholds(const gsr_params &p) {
    return p.alpha_min == kStdAlphaMin && p.alpha_max == kStdAlphaMax && p.T_min == kStdTMin;
}
constexpr double kLog2eD = 1.4426950408889634074;

// min(alpha, alpha_max) for a non-NaN alpha in one instruction: the median of
// (alpha, -inf, alpha_max).
__device__ __forceinline__ float min_alpha(float alpha, float alpha_max) {
    return __builtin_amdgcn_fmed3f(alpha, -__builtin_inff(), alpha_max);
}

__device__ __forceinline__ float scaled_sigma(float4 con, float dx, float dy) {
    const float u = fmaf(con.y, dy, dx);               // dx + (b / a) dy
    return fmaf(con.x * u, u, con.z * dy * dy);        // A u^2 + Q dy^2
}

// The scaled conic (A', B', C') = log2(e) (a/2, b, c/2) of a record's
// completed square: B' = 2 A r, C' = Q + A r^2.
__device__ __forceinline__ float3 scaled_conic(float4 con) {
    const float ar = con.x * con.y;
    return make_float3(con.x, 2.0f * ar, fmaf(ar, con.y, con.z));
}

// The quadratic q(u, v) = A u^2 + B u v + C v^2 (A, C > 0, 4AC > B^2) on the
// segment u = u0, v in [v0, v1]: its minimum, at v = clamp(-B u0 / (2C)).
__device__ __forceinline__ float edge_min(float A, float B, float C, float r, float u0, float v0, float v1) {
    const float v = fminf(fmaxf(r * u0, v0), v1);
    return fmaf(u0, fmaf(A, u0, B * v), C * v * v);
}

// Refines a quad mask with the exact support: quad q stays only if the
// scaled sigma's minimum over the quad's rectangle of pixel centres reaches
// the threshold Lq = log2(opacity / alpha_min) (plus a margin far above the
// float32 error of this test and of the per-pixel evaluation); a bounding
// box keeps many quads that an elongated, tilted ellipse misses.  In terms
// of d = mean - pixel the rectangle is [u0, u1] x [v0, v1]; the minimum of
// the convex quadratic is 0 if the rectangle holds d = 0, else on an edge.
__device__ __forceinline__ uint32_t refine_quad_mask(uint32_t m, float4 xyoh, float4 conh, float Lq,
                                                    float tile_x0, float tile_y0) {
    const float3 k = scaled_conic(conh);
    const float A = k.x, B = k.y, C = k.z;
    if (m == 0u || !(A > 0.0f) || !(C > 0.0f) || !(4.0f * A * C > B * B)) return m;
    const float ru = -B / (2.0f * C), rv = -B / (2.0f * A);
#pragma unroll
    for (int q = 0; q < 4; q++) {
        if (!((m >> q) & 1u)) continue;
        const float x0 = tile_x0 + (float)((q & 1) * 8) + 0.5f, y0 = tile_y0 + (float)((q >> 1) * 8) + 0.5f;
        const float u0 = xyoh.x - (x0 + 7.0f), u1 = xyoh.x - x0;
        const float v0 = xyoh.y - (y0 + 7.0f), v1 = xyoh.y - y0;
        if (u0 <= 0.0f && u1 >= 0.0f && v0 <= 0.0f && v1 >= 0.0f) continue;
        float smin = fminf(edge_min(A, B, C, ru, u0, v0, v1), edge_min(A, B, C, ru, u1, v0, v1));
        smin = fminf(smin, fminf(edge_min(C, B, A, rv, v0, u0, u1), edge_min(C, B, A, rv, v1, u0, u1)));
        const float U = fmaxf(fabsf(u0), fabsf(u1)), V = fmaxf(fabsf(v0), fabsf(v1));
        const float smag = fmaf(A, U * U, fmaf(fabsf(B), U * V, C * V * V));
        if (smin > Lq + 1e-5f * smag + 1e-4f * fabsf(Lq) + 1e-4f) m &= ~(1u << q);
    }
    return m;
}

// Tile culling of the binning (params tile_cull): per row of tiles, the
// columns whose rectangle of pixel centres the scaled quadratic reaches at
// or below a threshold L.  For a fixed v = mean_y - y the quadratic
// A u^2 + B u v + C v^2 <= L holds for u between the roots
// (-B v -+ sqrt(4 A L - (4 A C - B^2) v^2)) / (2 A); over a strip of v the
// largest u is at the v of the ellipse's rightmost point clamped to the
// strip (the upper root is concave in v), the smallest at the mirror image.
// Pixel centres x = mean_x - u in that range give a contiguous run of tile
// columns.  L is built so that the run holds every tile in which
// refine_quad_mask can keep a quad: the quad test's threshold Lq + 1e-5
// smag + 1e-4 |Lq| + 1e-4, with 2e-5 times a bound on smag (every quad of
// the 3-sigma square lies within radius + 16 px of the mean in x and y) for
// the float error of that test, then 1e-4 relative and absolute on top.
// The arithmetic is float with the hardware's approximate reciprocal, square
// root and log2 (a few ulp): 4AC - B^2 keeps its digits (B^2 is split into a
// rounded product and its exact error), and the strip and the run are
// widened by 2e-3 of the ellipse's extent plus 1e-2 px, far above the
// rounding error of the rest.  Without a positive-definite conic (the quad
// test keeps every box quad then) the whole rectangle is kept; below
// alpha_min opacity nothing is.
struct TileCull {
    int mode;          // 0: cull, 1: whole rectangle, 2: no tile
    float mx, my, B, det, L4A, vmax, vr, inv2A, su;
};

__device__ __forceinline__ TileCull tile_cull_setup(float mx, float my, float ca, float cb, float cc, float o,
                                                    float alpha_min, int radius) {
    TileCull t;
    t.mode = 0;
    t.mx = mx;
    t.my = my;
    if (!(o >= alpha_min)) { t.mode = 2; return t; }
    const float A = 0.5f * kLog2e * ca, B = kLog2e * cb, C = 0.5f * kLog2e * cc;
    if (!(A > 0.0f) || !(C > 0.0f) || !(4.0f * A * C > B * B)) { t.mode = 1; return t; }
    const float bb = B * B, bbe = fmaf(B, B, -bb);
    const float det = fmaf(4.0f * A, C, -bb) - bbe;
    const float Lq = __builtin_amdgcn_logf(o * __builtin_amdgcn_rcpf(alpha_min));   // log2, within 1e-6
    const float ub = (float)radius + 16.0f;
    const float smag = (A + fabsf(B) + C) * ub * ub;
    const float L = (Lq + 1e-4f * fabsf(Lq) + 1e-4f + 2e-5f * smag) * (1.0f + 1e-4f) + 1e-4f;
    const float idet = __builtin_amdgcn_rcpf(det);
    const float umax = __builtin_amdgcn_sqrtf(4.0f * C * L * idet), vmax = __builtin_amdgcn_sqrtf(4.0f * A * L * idet);
    if (!(det > 0.0f) || !(L > 0.0f) || !(umax < 1e7f) || !(vmax < 1e7f)) { t.mode = 1; return t; }
    t.B = B;
    t.det = det;
    t.L4A = 4.0f * A * L;
    t.inv2A = 0.5f * __builtin_amdgcn_rcpf(A);
    t.vr = -B * umax * (0.5f * __builtin_amdgcn_rcpf(C));     // v of the rightmost point
    t.vmax = vmax;
    t.su = 2e-3f * (umax + vmax) + 1e-2f;
    return t;
}

// Columns [xa, xb) of tile row ty, within the rectangle [x0, x1).
__device__ __forceinline__ void tile_cull_row(const TileCull &t, int ty, int x0, int x1, int &xa, int &xb) {
    xa = x0;
    xb = t.mode == 1 ? x1 : x0;
    if (t.mode != 0) return;
    const float y0 = (float)(kTile * ty) + 0.5f, y1 = y0 + (float)(kTile - 1);
    const float v0 = t.my - y1 - t.su, v1 = t.my - y0 + t.su;
    if (v1 < -t.vmax || v0 > t.vmax) return;
    const float va = fmaxf(v0, -t.vmax), vb = fminf(v1, t.vmax);
    const float vr = fminf(fmaxf(t.vr, va), vb), vl = fminf(fmaxf(-t.vr, va), vb);
    const float ur = (-t.B * vr + __builtin_amdgcn_sqrtf(fmaxf(t.L4A - t.det * vr * vr, 0.0f))) * t.inv2A;
    const float ul = (-t.B * vl - __builtin_amdgcn_sqrtf(fmaxf(t.L4A - t.det * vl * vl, 0.0f))) * t.inv2A;
    const float xl = t.mx - ur - t.su, xr = t.mx - ul + t.su;     // pixel centres x = mean_x - u
    const float a = ceilf((xl - (float)(kTile - 1) - 0.5f) * (1.0f / kTile));
    const float b = floorf((xr - 0.5f) * (1.0f / kTile)) + 1.0f;
    xa = (int)fminf(fmaxf(a, (float)x0), (float)x1);
    xb = (int)fminf(fmaxf(b, (float)xa), (float)x1);
}

struct PackedGauss {
    float4 xyoh;
    float4 conh;
    float4 col;
};

size_t pack_workspace_bytes(int64_t cn);
int launch_pack(const gsr_params &p, int CN, int N, int D, const float *means2d, const float *conics,
                const float *colors, const float *opacities, const float *comps, PackedGauss *out, hipStream_t s);
// Channel capacity of the compositing kernels for D channels: 3 (RGB in the
// packed records), 4, 8, 16 or 32 (channels staged in LDS).
// Channels composited (D features plus the depth channel when rendered) and
// the capacity of the kernel instance that composites them: 3 for plain RGB
// (colours ride in the packed records), else the next of 4, 8, 16, 32.
int composited_channels(const gsr_params &p, int D);
int channel_capacity(const gsr_params &p, int D);
constexpr int kMaxChannels = 32;

// Stages the a.Dt channels of list entry g (a Gaussian of camera c) into
// column t of s_feat, laid out [DM][B] (conflict-free stores, broadcast
// reads): features from a.feat ([C,N,D], or [N,D] when colors_shared), then
// the camera-space depth as channel a.D when depth is rendered, zeros up to DM.
template <int DM, int B, typename Args>
__device__ __forceinline__ void stage_features(const Args &a, int c, int g, int t, float *s_feat) {
    int n = g - c * a.N;
    if ((unsigned)n >= (unsigned)a.N) n = 0;      // only a bad id can leave the tile's camera
    const float *f = a.feat + (size_t)(a.p.colors_shared ? n : g) * a.D;
#pragma unroll
    for (int d = 0; d < DM; d++)
        s_feat[d * B + t] = d < a.D ? f[d] : (d < a.Dt ? a.depths[g] : 0.0f);
}

// Per-quad lists of a staged batch.  Thread t holds batch entry t with quad
// mask m (0 when the entry is past the list end); afterwards list[q][0 ..
// count[q]) holds, in increasing order, the entries whose mask has bit q.
// Must be called by all kThreadsPerTile threads; ends with a barrier.
constexpr int kThreadsPerTile = 256;
// L = uint8_t stores the slot t, L = uint16_t its byte offset in a float4 array (16 t).
template <typename L>
__device__ __forceinline__ void compact_quads(uint32_t m, L (*list)[kThreadsPerTile], int32_t (*wcnt)[4],
                                              int32_t *count) {
    const int t = threadIdx.x, lane = t % kWave, w = t / kWave;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    int32_t pre[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const uint64_t bal = __ballot((m >> q) & 1u);
        pre[q] = (int32_t)__popcll(bal & lt);
        if (lane == 0) wcnt[q][w] = (int32_t)__popcll(bal);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; q++) {
        int32_t base = 0;
        for (int v = 0; v < w; v++) base += wcnt[q][v];
        if ((m >> q) & 1u) list[q][base + pre[q]] = sizeof(L) == 1 ? (L)t : (L)(16 * t);
    }
    if (t < 4) count[t] = wcnt[t][0] + wcnt[t][1] + wcnt[t][2] + wcnt[t][3];
    __syncthreads();
}

}  // namespace gsr
