/*
 * gsraster.h -- C ABI of the MI355X (gfx950) differentiable tile rasterizer
 * for 3D Gaussian Splatting, following the forward and backward passes of
 * gsplat (arXiv 2409.06765, appendices "Forward Pass", "Backward Pass",
 * "Data Conventions", "Anti-aliasing").
 *
 * Conventions shared by every call
 * --------------------------------
 * Pointers.  Every tensor pointer is a DEVICE pointer (for instance a torch
 *   HIP tensor's data_ptr()), contiguous, row-major.  The only host pointers
 *   are the gsr_params struct, the per-camera image sizes W[C] and H[C], and
 *   the optional total_host output of gsr_intersect_count.
 * Types.  Floating point is float32; per-Gaussian indices and counts are
 *   int32; prefix offsets are int64; sort keys are uint64.
 * Layout.  C cameras (views), N Gaussians.  Per-view projected arrays are
 *   [C, N, ...]; a projected Gaussian is addressed by its flat id c*N + n
 *   (C*N must be below 2^31).  Images are packed per camera: pixel (c, y, x)
 *   is element pix_off[c] + y*W[c] + x with pix_off[c] = sum_{c'<c} W[c']H[c'];
 *   for equal sizes that is [C, H, W, ...].  Tiles are 16x16 pixels, numbered
 *   row-major inside a camera and offset by tile_base[c] = sum_{c'<c}
 *   ceil(W/16) ceil(H/16), so global tile ids of all cameras are disjoint.
 * Ownership.  The caller allocates and owns every buffer; the library keeps
 *   no pointer after a call returns and allocates no device memory.  Scratch
 *   space is passed in as a workspace sized by gsr_workspace_bytes().
 * Streams.  Every call takes a hipStream_t (passed as void*, NULL = the null
 *   stream), enqueues its kernels and returns without waiting, except
 *   gsr_intersect_count with a non-NULL total_host, which waits for the
 *   8-byte intersection count.
 * Errors.  Every call returns GSR_OK (0) or an error code; arguments are
 *   checked before anything is enqueued, so an error leaves outputs
 *   untouched.  gsr_last_error() returns a message for the calling thread.
 *   No C++ exception crosses this boundary.
 * Limits.  At most GSR_MAX_CAMERAS cameras per call; 1 <= W, H <= 16384;
 *   tile must be 16; sh_degree in -1..3; C*N < 2^31; intersections M < 2^31.
 */
#ifndef GSRASTER_H
#define GSRASTER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSR_ABI_VERSION 9
#define GSR_MAX_CAMERAS 64
#define GSR_GRAD_RECORD 9   /* floats per (camera, Gaussian) in the grad_records layout */

enum gsr_status {
    GSR_OK = 0,
    GSR_EINVAL = 1,      /* an argument is out of range or a required pointer is NULL */
    GSR_EOVERFLOW = 2,   /* intersections exceed the capacity passed in               */
    GSR_EWORKSPACE = 3,  /* workspace smaller than gsr_workspace_bytes()              */
    GSR_EHIP = 4         /* a HIP launch or runtime call failed                       */
};

/* Rasterizer constants.  Defaults (gsr_default_params): near 0.01, far +inf,
 * eps2d 0.3, jac_clamp 1.3, alpha_min 1/255, alpha_max 0.99, T_min 1e-4,
 * tile 16, sh_degree -1, antialiased 0, render_depth none, colors_shared 0,
 * tile_cull 1, grad_records 0. */
typedef struct gsr_params {
    float near_plane;   /* cull when the camera-space depth t_z < near_plane          */
    float far_plane;    /* cull when t_z > far_plane                                   */
    float eps2d;        /* low-pass dilation s added to the diagonal of Sigma'         */
    float jac_clamp;    /* > 0: t_x/t_z, t_y/t_z clamped to +-jac_clamp*(W/2)/f in J   */
    float alpha_min;    /* a Gaussian is skipped at a pixel when alpha < alpha_min      */
    float alpha_max;    /* alpha = min(alpha_max, o exp(-sigma))                        */
    float T_min;        /* a pixel stops before the Gaussian that would take T below it */
    int32_t tile;       /* tile edge in pixels; must be 16                              */
    int32_t sh_degree;  /* -1: direct colours [N,3]; 0..3: SH coefficients [N,(d+1)^2,3] */
    int32_t antialiased;/* 1: opacity times sqrt(|Sigma'| / |Sigma' + eps2d I|)         */
    int32_t render_depth;  /* gsr_depth_mode: composite the depth t_z as a last channel */
    int32_t colors_shared; /* rasterizer colours [N,D] shared by all cameras, not [C,N,D] */
    int32_t tile_cull;     /* gsr_bin_*: 1 drops the tiles of a Gaussian's 3-sigma square
                              that no pixel centre can see at alpha >= alpha_min; 0 keeps
                              the whole square, as the paper bins                       */
    int32_t grad_records;  /* gsr_rasterize_bwd, gsr_project_bwd: 1 keeps the 2D gradients
                              of each (camera, Gaussian) together in one record of
                              GSR_GRAD_RECORD floats at v_means2d; 0: four arrays  */
} gsr_params;

/* Depth rendering (Depth rendering appendix): the camera-space depth t_z of
 * every Gaussian composited as one more channel after the D features, with
 * no background; EXPECTED divides it by the sum of alpha T at the pixel
 * (0 where that sum is 0). */
enum gsr_depth_mode {
    GSR_DEPTH_NONE = 0,
    GSR_DEPTH_ACCUMULATED = 1,
    GSR_DEPTH_EXPECTED = 2
};

typedef void *gsr_stream_t;   /* a hipStream_t */

enum gsr_op {
    GSR_OP_INTERSECT_COUNT = 1,   /* workspace of gsr_intersect_count for C*N entries */
    GSR_OP_SORT = 2,              /* workspace of gsr_sort_pairs for M pairs          */
    GSR_OP_RASTERIZE = 3,         /* workspace of gsr_rasterize_fwd / _bwd, C*N       */
    GSR_OP_BIN_PREPARE = 4,       /* workspace kept from gsr_bin_prepare to _finish   */
    GSR_OP_BIN_FINISH = 5,        /* workspace of gsr_bin_finish for M intersections  */
    GSR_OP_PROJECT_BWD = 6,       /* workspace of gsr_project_bwd with v_viewmats     */
    GSR_OP_TILE_ORDER = 7,        /* workspace of gsr_tile_order                      */
    GSR_OP_L1_LOSS = 8,           /* workspace of gsr_l1_loss (any size)              */
    GSR_OP_DENSIFY_PLAN = 9       /* workspace of gsr_densify_plan for N Gaussians    */
};

/* Flags of gsr_rasterize_bwd. */
enum gsr_bwd_flags {
    GSR_BWD_ACCUMULATE = 1,
    GSR_BWD_PACKED = 2
};

int gsr_abi_version(void);
const char *gsr_last_error(void);
void gsr_default_params(gsr_params *p);

/* Bytes of workspace the operation needs (0 if none); C, N, M as in the call. */
size_t gsr_workspace_bytes(int op, int C, int N, int64_t M);

/* Projection of Gaussians (Forward Pass, Projection; Data Conventions;
 * Anti-aliasing).  For every camera c and Gaussian n:
 *   t = R_cw mu + t_cw (viewmats [C,4,4] world->camera, OpenCV axes),
 *   culled when t_z < near or t_z > far;
 *   Sigma = R(q/|q|) diag(s)^2 R(q/|q|)^T (quats [N,4] as w,x,y,z, scales [N,3]
 *   already activated);  T = J R_cw with J the pinhole Jacobian at t (its
 *   t_x/t_z, t_y/t_z clamped by jac_clamp);  Sigma' = T Sigma T^T + eps2d I;
 *   conic = entries (a, b, c) of Sigma'^-1;  radius = ceil(3 sqrt(lambda_max));
 *   means2d = (fx t_x/t_z + cx, fy t_y/t_z + cy) with fx = K[0][0],
 *   fy = K[1][1], cx = K[0][2], cy = K[1][2] (Ks [C,3,3]);  depth = t_z;
 *   colour = max(SH(dir) + 0.5, 0) with dir the unit vector from the camera
 *   centre to mu, or the direct colour when sh_degree = -1.
 * A Gaussian is culled (radius 0, all outputs 0) also when Sigma' is not
 * positive definite or its tile rectangle misses the image.
 * Outputs: means2d [C,N,2], conics [C,N,3], radii [C,N] int32, depths [C,N],
 * colors [C,N,3], compensations [C,N] (nullable; 1 unless antialiased).
 * With sh_degree = -1, colors may be NULL (and sh_or_colors then too): no
 * colour is written, for callers that hand the rasterizer features of their
 * own.  opacities [N] is not read (kept for a uniform argument list). */
int gsr_project_fwd(const gsr_params *p, int C, int N, const int32_t *W, const int32_t *H,
                    const float *means, const float *quats, const float *scales, const float *opacities,
                    const float *sh_or_colors, const float *viewmats, const float *Ks,
                    float *means2d, float *conics, int32_t *radii, float *depths, float *colors,
                    float *compensations, gsr_stream_t stream);

/* Tile binning (Rasterization of Gaussians, first step): the 16x16 tiles
 * met by the square box [mu' - r, mu' + r] of each projected Gaussian, as the
 * rectangle x0 = clamp(floor((mu'_x - r)/16), 0, TX), x1 = clamp(floor((mu'_x
 * + r)/16) + 1, 0, TX) (same in y).  Writes tiles_per_gauss [C,N] int32
 * (0 when radius is 0), their exclusive prefix sum offsets [C,N] int64, and
 * the total M into total_dev (device int64[1]).  When total_host is not NULL
 * the call also copies M to *total_host and waits for the stream.
 * ws: workspace of gsr_workspace_bytes(GSR_OP_INTERSECT_COUNT, C, N, 0). */
int gsr_intersect_count(const gsr_params *p, int C, int N, const int32_t *W, const int32_t *H,
                        const float *means2d, const int32_t *radii, int32_t *tiles_per_gauss,
                        int64_t *offsets, int64_t *total_dev, int64_t *total_host,
                        void *ws, size_t ws_bytes, gsr_stream_t stream);

/* One (key, id) per (Gaussian, tile): for the j-th tile of Gaussian g's
 * rectangle in row-major order, keys[offsets[g] + j] = (global tile id << 32)
 * | float bits of depth[g], ids[offsets[g] + j] = g (= c*N + n).  Depths are
 * positive, so the bit order is the numeric order.  M_capacity is the length
 * of keys/ids: pass the M of gsr_intersect_count; entries at or beyond it are
 * never written. */
int gsr_intersect_emit(const gsr_params *p, int C, int N, const int32_t *W, const int32_t *H,
                       const float *means2d, const int32_t *radii, const float *depths,
                       const int64_t *offsets, int64_t M_capacity, uint64_t *keys, int32_t *ids,
                       gsr_stream_t stream);

/* Stable LSD radix sort of M (key, id) pairs by the low key_bits bits of the
 * keys (key_bits in 1..64; 32 + ceil(log2(total tiles)) suffices).  Ties keep
 * their input order, so the emitted lists end up ordered by (tile, depth, id)
 * (per-tile depth sort of Rasterization of Gaussians).  The sorted result is
 * in keys/ids; keys_alt/ids_alt [M] are scratch.
 * ws: workspace of gsr_workspace_bytes(GSR_OP_SORT, 0, 0, M). */
int gsr_sort_pairs(int64_t M, int key_bits, uint64_t *keys, int32_t *ids, uint64_t *keys_alt,
                   int32_t *ids_alt, void *ws, size_t ws_bytes, gsr_stream_t stream);

/* gsr_sort_pairs without the workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): the same kernels and the same result,
 * bit for bit, with the digit histograms in a static device array of the
 * library (16 MiB + 1 KiB per GPU it runs on, held until the process ends).
 * M must be at most GSR_SORT_NOALLOC_MAX_PAIRS (2^25); larger M is rejected
 * with GSR_EINVAL before anything is enqueued.  keys_alt/ids_alt [M] are
 * still the caller's.  Runs on the current device (the stream must belong to
 * it); the first call on a device looks up that device's copy of the array.
 * Every call on one GPU uses the same array: calls that overlap in time on
 * one GPU (different streams, or host threads) race and must be serialised
 * by the caller; calls on one stream are. */
#define GSR_SORT_NOALLOC_MAX_PAIRS ((int64_t)1 << 25)
int gsr_sort_pairs_noalloc(int64_t M, int key_bits, uint64_t *keys, int32_t *ids, uint64_t *keys_alt,
                           int32_t *ids_alt, gsr_stream_t stream);

/* ranges [total_tiles, 2] int32: [start, end) of each tile's run in the
 * sorted keys; (0, 0) for an empty tile.  Keys must be sorted. */
int gsr_tile_ranges(int64_t M, const uint64_t *keys, int32_t total_tiles, int32_t *ranges,
                    gsr_stream_t stream);

/* Tile binning and per-tile depth order in two calls, giving the same ids
 * and ranges, bit for bit, as gsr_intersect_count + gsr_intersect_emit +
 * gsr_sort_pairs(key_bits = 32 + tile bits) + gsr_tile_ranges, with far less
 * sorting: the projected Gaussians are stably ordered by the bits of their
 * depth, their tiles are emitted in that order with 32-bit tile keys, and a
 * stable sort on the tile bits alone leaves every tile's run in (depth, id)
 * order (per-tile depth sort of Rasterization of Gaussians).
 * With p->tile_cull the lists leave out the tiles that no pixel centre of
 * theirs sees at alpha >= alpha_min: per tile row, the run of columns whose
 * pixel centres the ellipse sigma <= ln(o / alpha_min) reaches, with margins
 * that keep every tile in which the compositing kernels' own per-quad test
 * keeps a quad.  Every entry a pixel composites, and the order of those
 * entries, is then the same as with whole squares, so images and gradients
 * are too (bit for bit in the forward); only the lists are shorter and the
 * positions in them (last_ids) differ.  conics [C,N,3], opacities [N] and
 * compensations [C,N] (nullable unless antialiased) are read only then.
 * gsr_bin_prepare: counts and depth order; writes M to total_dev (device,
 * nullable) and, when total_host is not NULL, to *total_host after waiting
 * for the stream.  ws_prep: gsr_workspace_bytes(GSR_OP_BIN_PREPARE, C, N, 0),
 * which must be passed unchanged to gsr_bin_finish.
 * gsr_bin_finish: ids [M] int32 and ranges [total_tiles, 2] int32 as above;
 * keys [M] uint64 (nullable) receives the 64-bit keys of the sorted lists.
 * M is a capacity: the kernels read the true count from ws_prep on the
 * device, so the host need not wait for gsr_bin_prepare.  When the true
 * count exceeds M nothing is written past M and the lists are incomplete:
 * the caller compares the count (total_dev of gsr_bin_prepare) with M after
 * the fact and calls again with a larger M.  Unused capacity costs sort
 * launches over empty blocks.
 * ws_fin: gsr_workspace_bytes(GSR_OP_BIN_FINISH, C, N, M). */
int gsr_bin_prepare(const gsr_params *p, int C, int N, const int32_t *W, const int32_t *H,
                    const float *means2d, const int32_t *radii, const float *depths, const float *conics,
                    const float *opacities, const float *compensations, int64_t *total_dev, int64_t *total_host, void *ws_prep, size_t ws_prep_bytes,
                    gsr_stream_t stream);
int gsr_bin_finish(const gsr_params *p, int C, int N, const int32_t *W, const int32_t *H,
                   const float *means2d, const int32_t *radii, const float *depths, const float *conics,
                   const float *opacities, const float *compensations, int64_t M,
                   int32_t *ids, int32_t *ranges, uint64_t *keys, void *ws_prep, size_t ws_prep_bytes,
                   void *ws_fin, size_t ws_fin_bytes, gsr_stream_t stream);

/* Dispatch order for the compositing entry points: the tiles' indices
 * sorted by the length of their lists (ranges [T,2] from gsr_tile_ranges or
 * gsr_bin_finish), longest first, lengths grouped in buckets of an eighth of
 * an octave (the order within a bucket is not fixed).  Launching the longest
 * lists first keeps the GPU full until the end of a compositing pass; the
 * images and gradients do not depend on the order.  order [T] int32 (output),
 * ws of gsr_workspace_bytes(GSR_OP_TILE_ORDER, 0, 0, 0) bytes. */
int gsr_tile_order(int32_t total_tiles, const int32_t *ranges, int32_t *order, void *ws, size_t ws_bytes,
                   gsr_stream_t stream);

/* Zeroes bytes (a multiple of 4) of device memory at ptr (4-byte aligned)
 * with a kernel on the stream: a captured graph replays it like any other
 * launch, where a memset node may not be. */
int gsr_fill_zero(void *ptr, size_t bytes, gsr_stream_t stream);

/* Front-to-back compositing (Rasterization of Gaussians).  For every pixel
 * with centre p = (x + 0.5, y + 0.5), over its tile's sorted list:
 *   Delta = mu' - p;  sigma = 0.5 (a Dx^2 + c Dy^2) + b Dx Dy (skipped if < 0);
 *   alpha = min(alpha_max, o exp(-sigma)) with o = opacities[n] (times
 *   compensations[c*N+n] when antialiased); skipped if alpha < alpha_min;
 *   T' = T (1 - alpha); if T' < T_min the pixel stops here, without this one;
 *   otherwise C += f alpha T, T = T'.
 * Finally C += T background[c] on the feature channels (background [C,D],
 * NULL = zero).
 * Channels: D (0 .. 32) features f from colors, [C,N,D] ([N,D] shared by
 * all cameras when p->colors_shared; NULL when D = 0), then, when
 * p->render_depth is set, the depth t_z from depths [C,N] as channel D (Depth
 * rendering appendix; GSR_DEPTH_EXPECTED divides it by the sum of alpha T, 0
 * where nothing was composited).  Dt = D (+1 with depth) is 1 .. 32.  Every
 * channel takes the same alpha and T, so channels are independent.  Plain RGB
 * (D = 3, no depth) is the fastest case: the colours travel in the
 * per-Gaussian record; other channel sets are staged in LDS per batch.
 * tile_order [T] (nullable): the order in which the tiles' blocks are
 * launched, a permutation of 0 .. T-1 such as gsr_tile_order writes (NULL:
 * tile index order; an index out of range skips that block).
 * Outputs: image [P,Dt], alpha [P] = 1 - T, final_T [P] = T, last_ids [P] int32
 * (position in the sorted list of the last composited entry, -1 if none),
 * n_eval [P,5] int32 (nullable; work counters, slower): per pixel, (0) the
 * entries of its tile's list up to and including the one that stopped it (the
 * whole list if none did), (1) the entries composited, (2) the entries of the
 * pixel's 8x8 quad list (the tile-list entries whose alpha >= alpha_min
 * support reaches the quad) that it evaluated while not yet stopped, (3) the
 * entries of that quad list up to its last composited one, (4) the quad-list
 * entries its wave stepped through, stopped lanes included.
 * ws: workspace of gsr_workspace_bytes(GSR_OP_RASTERIZE, C, N, 0). */
int gsr_rasterize_fwd(const gsr_params *p, int C, int N, int D, const int32_t *W, const int32_t *H,
                      const float *means2d, const float *conics, const float *colors, const float *depths,
                      const float *opacities, const float *compensations, const float *background,
                      const int32_t *ranges, const int32_t *ids, const int32_t *tile_order, float *image,
                      float *alpha, float *final_T, int32_t *last_ids, int32_t *n_eval, void *ws,
                      size_t ws_bytes, gsr_stream_t stream);

/* Depth Compositing Gradients.  Per pixel, from last_ids back to its tile's
 * start, recomputes alpha, restores T_k = T_{k+1} / (1 - alpha_k) from final_T,
 * keeps S = sum of f alpha T behind entry k plus final_T background, and
 * accumulates
 *   dL/df += alpha T v_C;
 *   dL/dalpha = sum_ch (f T - S/(1 - alpha)) v_C + v_alpha final_T/(1 - alpha);
 *   unless alpha was clamped at alpha_max:
 *     dL/do += exp(-sigma) dL/dalpha,  dL/dsigma = -o exp(-sigma) dL/dalpha,
 *     dL/dmu' += dL/dsigma Sigma'^-1 Delta,
 *     dL/d(a, b, c) += dL/dsigma (Dx^2/2, Dx Dy, Dy^2/2).
 * Expected depth E = A / W (A the composited depth, W = sum alpha T = 1 -
 * final_T) passes v_E / W on to A and -v_E E / W to the alpha output; image
 * (the forward's output, [P,Dt]) supplies E and is read only in that mode.
 * Channels, p, D, colors, depths and tile_order as in gsr_rasterize_fwd.  v_image
 * [P,Dt], v_alpha [P] (nullable).  Outputs, overwritten: v_means2d [C,N,2],
 * v_conics [C,N,3], v_colors (shape of colors; NULL when D = 0), v_depths
 * [C,N] (depth channel; NULL unless depth is rendered), v_opacities [C,N]
 * (gradient with respect to the opacity the rasterizer used, o times
 * compensation), v_means2d_abs [C,N,2] (nullable: per-pixel absolute values
 * of the mu' gradient summed, the absgrad statistic).  Sums use float
 * atomics, so their rounding order is not fixed.
 * ws: workspace of gsr_workspace_bytes(GSR_OP_RASTERIZE, C, N, 0).
 * flags (bitwise or; 0 = overwrite the outputs and pack the records anew):
 *   GSR_BWD_ACCUMULATE  add into the outputs instead of overwriting them
 *                       (the caller zeroes them, or sums several calls);
 *   GSR_BWD_PACKED      ws still holds the per-Gaussian records that
 *                       gsr_rasterize_fwd wrote into it for these same
 *                       means2d, conics, colors, opacities, compensations and
 *                       params (not rewritten since), so they are not packed
 *                       again; with other contents the gradients are wrong. */
int gsr_rasterize_bwd(const gsr_params *p, int C, int N, int D, const int32_t *W, const int32_t *H,
                      const float *means2d, const float *conics, const float *colors, const float *depths,
                      const float *opacities, const float *compensations, const float *background,
                      const int32_t *ranges, const int32_t *ids, const int32_t *tile_order,
                      const float *image, const float *final_T, const int32_t *last_ids,
                      const float *v_image, const float *v_alpha,
                      float *v_means2d, float *v_conics, float *v_colors, float *v_depths, float *v_opacities,
                      float *v_means2d_abs, void *ws, size_t ws_bytes, int flags, gsr_stream_t stream);

/* The grad_records layout (params.grad_records = 1), a layout of the same
 * sums: v_means2d points to [C,N,GSR_GRAD_RECORD] floats, each record
 * {dL/dmu' x, y, dL/d(a, b, c) of the conic, dL/dcolour r, g, b, dL/dopacity};
 * v_conics, v_colors and v_opacities (gsr_project_bwd: v_opacities_cn) are
 * NULL.  Only for plain RGB: D = 3, no depth channel, colours not shared
 * (GSR_EINVAL otherwise).  The compositing backward adds the nine sums of a
 * (tile, Gaussian) with one atomic instruction whose lanes then fall in one
 * or two cache lines instead of four arrays; gsr_project_bwd reads the same
 * records.  v_means2d_abs and v_depths stay separate arrays. */

/* Projection Gradients, Scale and rotation gradients, SH backward.  Per
 * Gaussian, summed over the C cameras (no atomics: one thread per Gaussian):
 *   dL/dSigma' = -Y G Y with Y = Sigma'^-1, G = [[g_a, g_b/2], [g_b/2, g_c]];
 *   dL/dSigma = T^T dL/dSigma' T;  dL/dT = 2 dL/dSigma' T Sigma;  dL/dJ =
 *   dL/dT R_cw^T;  dL/dt from mu', from J (clamped coordinates follow t_z) and
 *   from v_depths;  dL/dmu = R_cw^T dL/dt plus the SH direction term;
 *   dL/dM = 2 dL/dSigma M;  dL/dR = dL/dM S^T;  dL/ds_j = (R^T dL/dM)_jj;
 *   dL/dq through dR/dq and the normalisation q/|q|;  dL/dSH_k = Y_k(dir)
 *   dL/dcolour (zero where the colour clamp at 0 is active).
 * Inputs: the gsr_project_fwd inputs, its radii and compensations
 * (nullable unless antialiased), and the per-camera gradients v_means2d,
 * v_conics, v_colors, v_opacities_cn [C,N] (from gsr_rasterize_bwd),
 * v_depths [C,N] (nullable).  Outputs, overwritten: v_means [N,3],
 * v_quats [N,4], v_scales [N,3], v_opacities [N], v_sh_or_colors (shape of
 * sh_or_colors).  With sh_degree = -1, v_colors may be NULL (and
 * sh_or_colors, v_sh_or_colors then too): the colours are not differentiated.
 * v_viewmats [C,4,4] (nullable; pose gradient, the paper's view-matrix
 * gradient read for world-to-camera matrices): with V = [R | t],
 * t_cam = R mu + t, T = J R and camera centre -R^T t, per camera the sum
 * over Gaussians of dL/dR = dL/dt_cam mu^T + J^T dL/dT + t g_dir^T and
 * dL/dt = dL/dt_cam + R g_dir, g_dir being the mean gradient through the SH
 * view direction; R is treated as a plain matrix; the last row is 0.  It
 * needs ws of gsr_workspace_bytes(GSR_OP_PROJECT_BWD, C, N, 0) bytes
 * (NULL and 0 when v_viewmats is NULL); its sums are deterministic. */
int gsr_project_bwd(const gsr_params *p, int C, int N, const int32_t *W, const int32_t *H,
                    const float *means, const float *quats, const float *scales, const float *opacities,
                    const float *sh_or_colors, const float *viewmats, const float *Ks,
                    const int32_t *radii, const float *compensations,
                    const float *v_means2d, const float *v_conics, const float *v_colors,
                    const float *v_opacities_cn, const float *v_depths,
                    float *v_means, float *v_quats, float *v_scales, float *v_opacities,
                    float *v_sh_or_colors, float *v_viewmats, void *ws, size_t ws_bytes,
                    gsr_stream_t stream);

/* ==== Training-loop steps (Densification Strategies appendix) ================
 * One optimisation step of a fit around the rasterizer: photometric loss,
 * Adam on the raw parameters (scales = exp(raw), opacities = sigmoid(raw)),
 * the ADC densification statistics, plan and apply, the opacity reset, and
 * the MCMC strategy's noise on the centres.  Same conventions as above
 * (device pointers, caller-owned buffers, status codes, asynchronous on the
 * stream unless a host output is asked for). */

#define GSR_ADAM_MAX_GROUPS 8
#define GSR_DENSIFY_MAX_COLUMNS 16

enum gsr_activation {
    GSR_ACT_NONE = 0,     /* the rasterizer takes the raw value               */
    GSR_ACT_EXP = 1,      /* it takes exp(raw) (scales)                       */
    GSR_ACT_SIGMOID = 2   /* it takes 1 / (1 + exp(-raw)) (opacities)         */
};

/* One parameter tensor of gsr_adam_step. */
typedef struct gsr_adam_group {
    float *param;          /* [n] raw values, updated in place                                 */
    const float *grad;     /* [n] gradient with respect to the ACTIVATED value                  */
    float *exp_avg;        /* [n] first moment, updated in place (zero before the first step)   */
    float *exp_avg_sq;     /* [n] second moment, updated in place                                */
    float *activated;      /* [n] nullable: receives act(param) after the update                 */
    int64_t n;             /* elements (0 allowed)                                               */
    float lr;              /* learning rate                                                      */
    float lr_rest;         /* learning rate of elements i with row > 0 and i % row >= row_first  */
    int32_t row;           /* 0: lr for every element; else the row length of the split          */
    int32_t row_first;     /* elements of a row that take lr (SH: the 3 degree-0 coefficients)  */
    int32_t activation;    /* gsr_activation                                                     */
    float reg;             /* L1 penalty weight per element on the activated value (> 0 values):
                              added to the activated gradient; must be 0 with GSR_ACT_NONE      */
} gsr_adam_group;

/* out_i = act(raw_i) for n values (the activated scales or opacities the
 * rasterizer takes; the same arithmetic as gsr_adam_step's activated output).
 * out may be raw (in place). */
int gsr_activate(int64_t n, const float *raw, int32_t activation, float *out, gsr_stream_t stream);

/* L1 photometric loss over n values (the paper leaves the loss open; this is
 * the mean absolute error when scale = 1/n):
 *   loss[0] = scale * sum_i |image_i - target_i|  (device float; block
 *             partial sums in float, combined in double in a fixed order, so
 *             the value depends on n and the data only),
 *   v_image_i = scale * sign(image_i - target_i), sign(0) = 0.
 * v_image may alias neither input.  ws: gsr_workspace_bytes(GSR_OP_L1_LOSS,
 * 0, 0, n) bytes.  n = 0 writes loss = 0. */
int gsr_l1_loss(int64_t n, const float *image, const float *target, float scale, float *v_image, float *loss,
                void *ws, size_t ws_bytes, gsr_stream_t stream);

/* Adam (Kingma and Ba, with bias correction) on up to GSR_ADAM_MAX_GROUPS
 * tensors in one launch, at step t >= 1:
 *   g = grad                                  (GSR_ACT_NONE)
 *   g = (grad + reg) * exp(param)             (GSR_ACT_EXP)
 *   g = (grad + reg) * o (1 - o), o = sigmoid(param)   (GSR_ACT_SIGMOID)
 *   m = beta1 m + (1 - beta1) g;  v = beta2 v + (1 - beta2) g^2
 *   param -= lr_i * (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps)
 *   activated = act(param).
 * Groups must not overlap.  Errors: n_groups outside 0..GSR_ADAM_MAX_GROUPS,
 * t < 1, betas outside [0, 1), eps < 0, a NULL required pointer, reg != 0
 * without an activation. */
int gsr_adam_step(int n_groups, const gsr_adam_group *groups, int32_t step, float beta1, float beta2, float eps,
                  gsr_stream_t stream);

/* ADC statistics (ADC and Absgrad): for every Gaussian n, over the cameras c
 * with radii[c,n] > 0,
 *   grad_accum[n] += sum_c scale * |(v_x W[c] / 2, v_y H[c] / 2)|,
 *   count[n]      += number of such cameras,
 * with (v_x, v_y) = v_means2d[c,n] (pass the absolute sums of
 * gsr_rasterize_bwd's v_means2d_abs for Absgrad).  The factors W/2, H/2 turn
 * pixel gradients into gradients with respect to normalised device
 * coordinates, the units of the paper's threshold 0.0002; scale is the number
 * of views a loss averaged over, so the statistic is that of a per-view loss.
 * Cameras are summed in order per Gaussian (deterministic). */
int gsr_densify_stats(int C, int N, const int32_t *W, const int32_t *H, const int32_t *radii,
                      const float *v_means2d, float scale, float *grad_accum, int32_t *count, gsr_stream_t stream);

enum gsr_densify_action {
    GSR_PRUNE = 0,   /* removed                                           */
    GSR_KEEP = 1,    /* one output slot, copied                           */
    GSR_CLONE = 2,   /* two slots: the original and a copy                */
    GSR_SPLIT = 3    /* two slots: children sampled from N(mu, Sigma)      */
};

/* ADC plan: per Gaussian (float32 comparisons),
 *   PRUNE if opacities[n] < prune_opacity; else
 *   SPLIT if count[n] > 0 and grad_accum[n] > grad_threshold * count[n] and
 *         max(scales[n]) > scale_threshold;
 *   CLONE under the same gradient test otherwise; else KEEP.
 * scales [N,3] and opacities [N] are the activated values.  Writes action
 * [N] and offsets [N+1] (int64, exclusive prefix sums of the slots 0/1/2/2;
 * offsets[N] is the new count).  total_host (nullable): the new count is also
 * copied to the host, and the call then waits for the stream.  Pass
 * grad_threshold = +inf for pruning alone, prune_opacity = 0 for none.
 * ws: gsr_workspace_bytes(GSR_OP_DENSIFY_PLAN, 0, N, 0) bytes. */
int gsr_densify_plan(int N, const float *grad_accum, const int32_t *count, const float *scales,
                     const float *opacities, float grad_threshold, float scale_threshold, float prune_opacity,
                     int32_t *action, int64_t *offsets, int64_t *total_host, void *ws, size_t ws_bytes,
                     gsr_stream_t stream);

enum gsr_column_kind {
    GSR_COLUMN_COPY = 0,        /* every output slot copies the row                        */
    GSR_COLUMN_MEANS = 1,       /* width 3; split children: mu + R(q) diag(exp(ls)) eta_k  */
    GSR_COLUMN_LOG_SCALES = 2,  /* width 3; split children: ls - log(split_shrink)         */
    GSR_COLUMN_STATE = 3        /* optimiser state: copied for KEEP and a clone's original,
                                   zero for a clone's copy and both split children         */
};

/* One per-Gaussian array of gsr_densify_apply: src [N,width] -> dst
 * [offsets[N],width] (dst must not overlap src). */
typedef struct gsr_densify_column {
    const float *src;
    float *dst;
    int32_t width;   /* floats per Gaussian, 1..4096 */
    int32_t kind;    /* gsr_column_kind */
} gsr_densify_column;

/* ADC apply (the paper's split and clone): Gaussian n with action and
 * offsets from gsr_densify_plan writes its slots offsets[n] .. offsets[n+1]-1
 * of every column, in input order.  quats [N,4] (w,x,y,z, normalised here)
 * and log_scales [N,3] are the raw parameters the split children are drawn
 * with; split_normals [N,2,3] are standard normal draws eta_k (an input: the
 * library draws no random numbers).  Required when a MEANS column is given;
 * log(split_shrink) is subtracted from a split child's log-scales (3D
 * Gaussian Splatting divides the scale by 1.6). */
int gsr_densify_apply(int N, const int32_t *action, const int64_t *offsets, const float *quats,
                      const float *log_scales, const float *split_normals, float split_shrink, int n_columns,
                      const gsr_densify_column *columns, gsr_stream_t stream);

/* ADC opacity reset: logits[n] = min(logits[n], logit(max_opacity)), so the
 * opacity becomes min(o, max_opacity); the Adam moments of the logits are
 * cleared; opacities (nullable) receives sigmoid(logits). 0 < max_opacity < 1. */
int gsr_opacity_reset(int N, float *logits, float *exp_avg, float *exp_avg_sq, float *opacities,
                      float max_opacity, gsr_stream_t stream);

/* MCMC noise on the centres (the MCMC strategy's SGLD update):
 *   means[n] += coeff * sigmoid(-k (o_n - t)) * Sigma_n eta_n,
 *   Sigma_n = R(q_n) diag(s_n)^2 R(q_n)^T,
 * with quats [N,4] (normalised here), scales [N,3] and opacities [N]
 * activated, normals [N,3] standard normal draws (an input), and coeff =
 * lambda_noise * lr of the means.  The cited MCMC work uses k = 100 and
 * t = 0.005. */
int gsr_mcmc_noise(int N, float *means, const float *quats, const float *scales, const float *opacities,
                   const float *normals, float coeff, float k, float t, gsr_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* GSRASTER_H */
