// Internal declarations shared by the HIP translation units of libgsraster.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
                       float *v_scales, float *v_opac, float *v_sh, hipStream_t s);

size_t count_workspace_bytes(int64_t n);
int launch_intersect_count(const gsr_params &p, const CamTable &cams, int N, const float *means2d,
                           const int32_t *radii, int32_t *counts, int64_t *offsets, int64_t *total_dev,
                           void *ws, hipStream_t s);
int launch_intersect_emit(const gsr_params &p, const CamTable &cams, int N, const float *means2d,
                          const int32_t *radii, const float *depths, const int64_t *offsets, int64_t cap,
                          uint64_t *keys, int32_t *ids, hipStream_t s);

size_t sort_workspace_bytes(int64_t M);
int launch_sort_pairs(int64_t M, int key_bits, uint64_t *keys, int32_t *ids, uint64_t *keys_alt,
                      int32_t *ids_alt, void *ws, hipStream_t s);
int launch_tile_ranges(int64_t M, const uint64_t *keys, int32_t total_tiles, int32_t *ranges, hipStream_t s);

int launch_rasterize_fwd(const gsr_params &p, const CamTable &cams, int N, const float *means2d,
                         const float *conics, const float *colors, const float *opacities,
                         const float *comps, const float *background, const int32_t *ranges,
                         const int32_t *ids, float *image, float *alpha, float *final_T, int32_t *last_ids,
                         int32_t *n_eval, hipStream_t s);

int launch_rasterize_bwd(const gsr_params &p, const CamTable &cams, int N, const float *means2d,
                         const float *conics, const float *colors, const float *opacities,
                         const float *comps, const float *background, const int32_t *ranges,
                         const int32_t *ids, const float *final_T, const int32_t *last_ids,
                         const float *v_image, const float *v_alpha, float *v_means2d, float *v_conics,
                         float *v_colors, float *v_opac, float *v_means2d_abs, hipStream_t s);

int launch_fill_zero(void *ptr, size_t bytes, hipStream_t s);

// ---- device helpers ----------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

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

}  // namespace gsr
