// Training-loop steps around the rasterizer (Densification Strategies
// appendix): L1 loss, Adam over several raw-parameter tensors with the
// activation chain fused in, ADC statistics / plan / apply, the opacity reset
// and the MCMC noise on the centres.
//
// All of these are streaming passes over per-pixel or per-Gaussian arrays,
// so they are HBM-bound: every kernel reads and writes each element once,
// coalesced, and the element-wise ones move 16 bytes per lane where the
// pointers allow it.
#include <math.h>
#include <string.h>

#include "common.hpp"

namespace gsr {
namespace {

constexpr int kThreads = 256;

// Sum over a 256-thread block in double; every thread gets the total.
__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

__device__ __forceinline__ float l1_term(float a, float b, float scale, float &acc) {
    const float d = a - b;
    acc += fabsf(d);
    return d > 0.0f ? scale : (d < 0.0f ? -scale : 0.0f);
}

// ---- L1 loss ---------------------------------------------------------------------
// Grid-stride over the values; each block leaves one double partial.  The
// grid depends on n alone, so the summation order does too.
template <bool kVec>
__global__ void __launch_bounds__(kThreads) l1_kernel(int64_t n, const float *__restrict__ img,
                                                      const float *__restrict__ tgt, float scale,
                                                      float *__restrict__ v, double *__restrict__ partial) {
    __shared__ double red[kThreads / kWave];
    float acc = 0.0f;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    if (kVec) {
        const int64_t n4 = n >> 2;
        const float4 *a4 = reinterpret_cast<const float4 *>(img);
        const float4 *b4 = reinterpret_cast<const float4 *>(tgt);
        float4 *v4 = reinterpret_cast<float4 *>(v);
        for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < n4; q += stride) {
            const float4 a = a4[q], b = b4[q];
            float4 g;
            g.x = l1_term(a.x, b.x, scale, acc);
            g.y = l1_term(a.y, b.y, scale, acc);
            g.z = l1_term(a.z, b.z, scale, acc);
            g.w = l1_term(a.w, b.w, scale, acc);
            v4[q] = g;
        }
        if (blockIdx.x == 0)
            for (int64_t i = (n4 << 2) + threadIdx.x; i < n; i += kThreads) v[i] = l1_term(img[i], tgt[i], scale, acc);
    } else {
        for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride)
            v[i] = l1_term(img[i], tgt[i], scale, acc);
    }
    const double s = block_sum((double)acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kThreads) l1_final_kernel(int nb, const double *__restrict__ partial, double scale,
                                                            float *__restrict__ loss) {
    __shared__ double red[kThreads / kWave];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += kThreads) s += partial[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) loss[0] = (float)(s * scale);
}

// ---- Adam ----------------------------------------------------------------------------
constexpr int kAdamItems = 4;
constexpr int kAdamPerBlock = kThreads * kAdamItems;

struct AdamGroupK {
    float *p;
    const float *g;
    float *m;
    float *v;
    float *act;
    int64_t n;
    float lr, lr_rest, reg;
    int32_t row, row_first, kind, vec;
};

struct AdamTable {
    AdamGroupK g[GSR_ADAM_MAX_GROUPS];
    int64_t first_block[GSR_ADAM_MAX_GROUPS + 1];
    int32_t n_groups;
    AdamConsts c;
};

__device__ __forceinline__ float activate(float x, int kind) {
    if (kind == GSR_ACT_EXP) return expf(x);
    if (kind == GSR_ACT_SIGMOID) return 1.0f / (1.0f + expf(-x));
    return x;
}

__device__ __forceinline__ void adam_one(const AdamTable &t, const AdamGroupK &G, float lr, float &p, float g,
                                         float &m, float &v, float &a) {
    adam_update(t.c, G.kind, G.reg, lr, p, g, m, v, a);
}

__global__ void __launch_bounds__(kThreads) adam_kernel(AdamTable t) {
    int gi = 0;
#pragma unroll
    for (int k = 1; k < GSR_ADAM_MAX_GROUPS; k++)
        if (k < t.n_groups && (int64_t)blockIdx.x >= t.first_block[k]) gi = k;
    const AdamGroupK G = t.g[gi];
    const int64_t base = ((int64_t)blockIdx.x - t.first_block[gi]) * kAdamPerBlock + (int64_t)threadIdx.x * kAdamItems;
    if (base >= G.n) return;
    float lr[kAdamItems];
    {
        int r = G.row > 0 ? (int)(base % G.row) : 0;
#pragma unroll
        for (int i = 0; i < kAdamItems; i++) {
            lr[i] = (G.row > 0 && r >= G.row_first) ? G.lr_rest : G.lr;
            if (G.row > 0 && ++r == G.row) r = 0;
        }
    }
    if (G.vec && base + kAdamItems <= G.n) {
        float4 p = *reinterpret_cast<const float4 *>(G.p + base);
        const float4 g = *reinterpret_cast<const float4 *>(G.g + base);
        float4 m = *reinterpret_cast<const float4 *>(G.m + base);
        float4 v = *reinterpret_cast<const float4 *>(G.v + base);
        float4 a;
        adam_one(t, G, lr[0], p.x, g.x, m.x, v.x, a.x);
        adam_one(t, G, lr[1], p.y, g.y, m.y, v.y, a.y);
        adam_one(t, G, lr[2], p.z, g.z, m.z, v.z, a.z);
        adam_one(t, G, lr[3], p.w, g.w, m.w, v.w, a.w);
        *reinterpret_cast<float4 *>(G.p + base) = p;
        *reinterpret_cast<float4 *>(G.m + base) = m;
        *reinterpret_cast<float4 *>(G.v + base) = v;
        if (G.act) *reinterpret_cast<float4 *>(G.act + base) = a;
        return;
    }
#pragma unroll
    for (int i = 0; i < kAdamItems; i++) {
        const int64_t e = base + i;
        if (e < G.n) {
            float p = G.p[e], m = G.m[e], v = G.v[e], a;
            adam_one(t, G, lr[i], p, G.g[e], m, v, a);
            G.p[e] = p;
            G.m[e] = m;
            G.v[e] = v;
            if (G.act) G.act[e] = a;
        }
    }
}

__global__ void __launch_bounds__(kThreads) activate_kernel(int64_t n, const float *raw, int kind, float *out) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) out[i] = activate(raw[i], kind);
}

// ---- ADC statistics --------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) densify_stats_kernel(CamTable cams, int N,
        const int32_t *__restrict__ radii, const float2 *__restrict__ v, float scale, float *__restrict__ accum,
        int32_t *__restrict__ count) {
    const int n = blockIdx.x * kThreads + threadIdx.x;
    if (n >= N) return;
    float s = 0.0f;
    int k = 0;
    for (int c = 0; c < cams.C; c++) {
        const int64_t i = (int64_t)c * N + n;
        if (radii[i] > 0) {
            const float2 g = v[i];
            const float gx = g.x * (0.5f * (float)cams.cam[c].W) * scale;
            const float gy = g.y * (0.5f * (float)cams.cam[c].H) * scale;
            s += sqrtf(gx * gx + gy * gy);
            k++;
        }
    }
    if (k > 0) {
        accum[n] += s;
        count[n] += k;
    }
}

// ---- ADC plan --------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) densify_plan_kernel(int N, const float *__restrict__ accum,
        const int32_t *__restrict__ count, const float *__restrict__ scales, const float *__restrict__ opac,
        float gthr, float sthr, float othr, int32_t *__restrict__ action, int32_t *__restrict__ slots) {
    const int n = blockIdx.x * kThreads + threadIdx.x;
    if (n >= N) return;
    const int k = count[n];
    const float smax = fmaxf(fmaxf(scales[3 * n], scales[3 * n + 1]), scales[3 * n + 2]);
    int a = GSR_KEEP;
    if (k > 0 && accum[n] > gthr * (float)k) a = smax > sthr ? GSR_SPLIT : GSR_CLONE;
    if (opac[n] < othr) a = GSR_PRUNE;
    action[n] = a;
    slots[n] = a == GSR_PRUNE ? 0 : (a == GSR_KEEP ? 1 : 2);
}

// ---- ADC apply -------------------------------------------------------------------------
// One thread per (Gaussian, float) of each column, the columns concatenated
// block-wise (first_block), so reads are coalesced for every width and the
// writes of a kept Gaussian land next to its neighbours'.
constexpr int kApplyItems = 4;
constexpr int kApplyPerBlock = kThreads * kApplyItems;

struct ColumnTable {
    const float *src[GSR_DENSIFY_MAX_COLUMNS];
    float *dst[GSR_DENSIFY_MAX_COLUMNS];
    int32_t width[GSR_DENSIFY_MAX_COLUMNS];
    int32_t kind[GSR_DENSIFY_MAX_COLUMNS];
    int64_t first_block[GSR_DENSIFY_MAX_COLUMNS + 1];
    int32_t n;
};

// Rotation of a quaternion (w, x, y, z), normalised here; row-major R.
__device__ __forceinline__ void quat_rot(const float *q4, float R[9]) {
    const float inv = 1.0f / sqrtf(q4[0] * q4[0] + q4[1] * q4[1] + q4[2] * q4[2] + q4[3] * q4[3]);
    const float w = q4[0] * inv, x = q4[1] * inv, y = q4[2] * inv, z = q4[3] * inv;
    R[0] = 1.0f - 2.0f * (y * y + z * z);
    R[1] = 2.0f * (x * y - w * z);
    R[2] = 2.0f * (x * z + w * y);
    R[3] = 2.0f * (x * y + w * z);
    R[4] = 1.0f - 2.0f * (x * x + z * z);
    R[5] = 2.0f * (y * z - w * x);
    R[6] = 2.0f * (x * z - w * y);
    R[7] = 2.0f * (y * z + w * x);
    R[8] = 1.0f - 2.0f * (x * x + y * y);
}

// Component j of split child k: mu_j + (R diag(exp(ls)) eta_k)_j.
__device__ __forceinline__ float split_mean(float mu, int n, int j, int k, const float *quats, const float *log_scales,
                                            const float *normals) {
    float R[9];
    quat_rot(quats + 4 * (int64_t)n, R);
    const float *ls = log_scales + 3 * (int64_t)n;
    const float *eta = normals + 6 * (int64_t)n + 3 * k;
    return mu + (R[3 * j] * (expf(ls[0]) * eta[0]) + R[3 * j + 1] * (expf(ls[1]) * eta[1]) +
                 R[3 * j + 2] * (expf(ls[2]) * eta[2]));
}

template <bool kWide>
__global__ void __launch_bounds__(kThreads) densify_apply_kernel(int N, const int32_t *__restrict__ action,
        const int64_t *__restrict__ offsets, const float *__restrict__ quats, const float *__restrict__ log_scales,
        const float *__restrict__ normals, float log_shrink, ColumnTable t) {
    int col = 0;
#pragma unroll
    for (int k = 1; k < GSR_DENSIFY_MAX_COLUMNS; k++)
        if (k < t.n && (int64_t)blockIdx.x >= t.first_block[k]) col = k;
    const int w = t.width[col];
    const int kind = t.kind[col];
    const float *src = t.src[col];
    float *dst = t.dst[col];
    const int64_t total = (int64_t)N * w;
    const int64_t base = ((int64_t)blockIdx.x - t.first_block[col]) * kApplyPerBlock + threadIdx.x;
#pragma unroll
    for (int i = 0; i < kApplyItems; i++) {
        const int64_t e = base + (int64_t)i * kThreads;
        if (e >= total) break;
        int n, j;
        if (kWide) {
            n = (int)(e / w);
            j = (int)(e - (int64_t)n * w);
        } else {
            n = (int)((uint32_t)e / (uint32_t)w);
            j = (int)((uint32_t)e - (uint32_t)n * (uint32_t)w);
        }
        const int a = action[n];
        if (a == GSR_PRUNE) continue;
        const float x = src[e];
        float *d = dst + offsets[n] * w + j;
        if (a == GSR_KEEP) {
            d[0] = x;
        } else if (a == GSR_CLONE) {
            d[0] = x;
            d[w] = kind == GSR_COLUMN_STATE ? 0.0f : x;
        } else if (kind == GSR_COLUMN_MEANS) {
            d[0] = split_mean(x, n, j, 0, quats, log_scales, normals);
            d[w] = split_mean(x, n, j, 1, quats, log_scales, normals);
        } else {
            const float y = kind == GSR_COLUMN_STATE ? 0.0f : (kind == GSR_COLUMN_LOG_SCALES ? x - log_shrink : x);
            d[0] = y;
            d[w] = y;
        }
    }
}

// ---- opacity reset -----------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) opacity_reset_kernel(int N, float *__restrict__ logits,
        float *__restrict__ m, float *__restrict__ v, float *__restrict__ opac, float cap) {
    const int n = blockIdx.x * kThreads + threadIdx.x;
    if (n >= N) return;
    const float l = fminf(logits[n], cap);
    logits[n] = l;
    m[n] = 0.0f;
    v[n] = 0.0f;
    if (opac) opac[n] = 1.0f / (1.0f + expf(-l));
}

// ---- MCMC noise ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) mcmc_noise_kernel(int N, float *__restrict__ means,
        const float *__restrict__ quats, const float *__restrict__ scales, const float *__restrict__ opac,
        const float *__restrict__ normals, float coeff, float k, float t) {
    const int n = blockIdx.x * kThreads + threadIdx.x;
    if (n >= N) return;
    float R[9];
    quat_rot(quats + 4 * (int64_t)n, R);
    const float *eta = normals + 3 * (int64_t)n;
    const float *s = scales + 3 * (int64_t)n;
    // Sigma eta = R S^2 R^T eta
    float u[3];
#pragma unroll
    for (int j = 0; j < 3; j++) u[j] = (R[j] * eta[0] + R[3 + j] * eta[1] + R[6 + j] * eta[2]) * (s[j] * s[j]);
    const float gate = 1.0f / (1.0f + expf(k * (opac[n] - t)));
    const float c = coeff * gate;
#pragma unroll
    for (int j = 0; j < 3; j++) means[3 * (int64_t)n + j] += c * (R[3 * j] * u[0] + R[3 * j + 1] * u[1] + R[3 * j + 2] * u[2]);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }
inline bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace

int launch_l1_loss(int64_t n, const float *image, const float *target, float scale, float *v_image, float *loss,
                   void *ws, hipStream_t s) {
    double *partial = (double *)ws;
    const bool vec = aligned16(image) && aligned16(target) && aligned16(v_image);
    const int64_t work = vec ? (n >> 2) : n;
    int nb = (int)((work + kThreads - 1) / kThreads);
    nb = nb < 1 ? 1 : (nb > kL1Blocks ? kL1Blocks : nb);
    if (vec)
        l1_kernel<true><<<nb, kThreads, 0, s>>>(n, image, target, scale, v_image, partial);
    else
        l1_kernel<false><<<nb, kThreads, 0, s>>>(n, image, target, scale, v_image, partial);
    l1_final_kernel<<<1, kThreads, 0, s>>>(nb, partial, (double)scale, loss);
    return launch_check("l1_loss");
}

AdamConsts adam_consts(float beta1, float beta2, float eps, int32_t step) {
    AdamConsts c;
    c.beta1 = beta1;
    c.beta2 = beta2;
    c.omb1 = (float)(1.0 - (double)beta1);
    c.omb2 = (float)(1.0 - (double)beta2);
    c.inv_bc1 = (float)(1.0 / (1.0 - pow((double)beta1, (double)step)));
    c.inv_bc2 = (float)(1.0 / (1.0 - pow((double)beta2, (double)step)));
    c.eps = eps;
    return c;
}

int launch_adam(const AdamLaunch &a, hipStream_t s) {
    AdamTable t;
    memset(&t, 0, sizeof(t));
    int64_t blocks = 0;
    int ng = 0;
    for (int i = 0; i < a.n_groups; i++) {
        const gsr_adam_group &g = a.g[i];
        if (g.n == 0) continue;
        AdamGroupK &k = t.g[ng];
        k.p = g.param;
        k.g = g.grad;
        k.m = g.exp_avg;
        k.v = g.exp_avg_sq;
        k.act = g.activated;
        k.n = g.n;
        k.lr = g.lr;
        k.lr_rest = g.lr_rest;
        k.reg = g.reg;
        k.row = g.row;
        k.row_first = g.row_first;
        k.kind = g.activation;
        k.vec = aligned16(g.param) && aligned16(g.grad) && aligned16(g.exp_avg) && aligned16(g.exp_avg_sq) &&
                (!g.activated || aligned16(g.activated));
        t.first_block[ng] = blocks;
        blocks += (g.n + kAdamPerBlock - 1) / kAdamPerBlock;
        ng++;
    }
    for (int i = ng; i <= GSR_ADAM_MAX_GROUPS; i++) t.first_block[i] = blocks;
    if (ng == 0) return GSR_OK;
    if (blocks > INT32_MAX) return fail(GSR_EINVAL, "gsr_adam_step: too many elements");
    t.n_groups = ng;
    t.c = a.c;
    adam_kernel<<<(unsigned)blocks, kThreads, 0, s>>>(t);
    return launch_check("adam_step");
}

int launch_activate(int64_t n, const float *raw, int kind, float *out, hipStream_t s) {
    if (n == 0) return GSR_OK;
    activate_kernel<<<blocks_for(n), kThreads, 0, s>>>(n, raw, kind, out);
    return launch_check("activate");
}

int launch_densify_stats(const CamTable &cams, int N, const int32_t *radii, const float *v_means2d, float scale,
                         float *accum, int32_t *count, hipStream_t s) {
    if (N == 0 || cams.C == 0) return GSR_OK;
    densify_stats_kernel<<<blocks_for(N), kThreads, 0, s>>>(cams, N, radii, reinterpret_cast<const float2 *>(v_means2d),
                                                            scale, accum, count);
    return launch_check("densify_stats");
}

size_t densify_plan_bytes(int N) {
    const size_t slots = ((size_t)(N > 0 ? N : 0) * sizeof(int32_t) + 255) & ~(size_t)255;
    return slots + scan_workspace_bytes(N > 0 ? N : 0);
}

int launch_densify_plan(int N, const float *accum, const int32_t *count, const float *scales, const float *opacities,
                        float grad_threshold, float scale_threshold, float prune_opacity, int32_t *action,
                        int64_t *offsets, void *ws, hipStream_t s) {
    int32_t *slots = (int32_t *)ws;
    void *scan_ws = (char *)ws + (((size_t)N * sizeof(int32_t) + 255) & ~(size_t)255);
    if (N > 0)
        densify_plan_kernel<<<blocks_for(N), kThreads, 0, s>>>(N, accum, count, scales, opacities, grad_threshold,
                                                               scale_threshold, prune_opacity, action, slots);
    int rc = launch_check("densify_plan");
    if (rc != GSR_OK) return rc;
    return launch_scan_i32(N, slots, offsets, offsets + N, scan_ws, s);
}

int launch_densify_apply(int N, const int32_t *action, const int64_t *offsets, const float *quats,
                         const float *log_scales, const float *normals, float log_shrink, int n_columns,
                         const gsr_densify_column *columns, hipStream_t s) {
    if (N == 0 || n_columns == 0) return GSR_OK;
    ColumnTable t;
    memset(&t, 0, sizeof(t));
    int64_t blocks = 0, widest = 0;
    for (int i = 0; i < n_columns; i++) {
        t.src[i] = columns[i].src;
        t.dst[i] = columns[i].dst;
        t.width[i] = columns[i].width;
        t.kind[i] = columns[i].kind;
        t.first_block[i] = blocks;
        const int64_t total = (int64_t)N * columns[i].width;
        blocks += (total + kApplyPerBlock - 1) / kApplyPerBlock;
        widest = total > widest ? total : widest;
    }
    for (int i = n_columns; i <= GSR_DENSIFY_MAX_COLUMNS; i++) t.first_block[i] = blocks;
    t.n = n_columns;
    if (blocks > INT32_MAX) return fail(GSR_EINVAL, "gsr_densify_apply: too many elements");
    if (widest > INT32_MAX)
        densify_apply_kernel<true><<<(unsigned)blocks, kThreads, 0, s>>>(N, action, offsets, quats, log_scales,
                                                                         normals, log_shrink, t);
    else
        densify_apply_kernel<false><<<(unsigned)blocks, kThreads, 0, s>>>(N, action, offsets, quats, log_scales,
                                                                          normals, log_shrink, t);
    return launch_check("densify_apply");
}

int launch_opacity_reset(int N, float *logits, float *exp_avg, float *exp_avg_sq, float *opacities, float cap,
                         hipStream_t s) {
    if (N == 0) return GSR_OK;
    opacity_reset_kernel<<<blocks_for(N), kThreads, 0, s>>>(N, logits, exp_avg, exp_avg_sq, opacities, cap);
    return launch_check("opacity_reset");
}

int launch_mcmc_noise(int N, float *means, const float *quats, const float *scales, const float *opacities,
                      const float *normals, float coeff, float k, float t, hipStream_t s) {
    if (N == 0) return GSR_OK;
    mcmc_noise_kernel<<<blocks_for(N), kThreads, 0, s>>>(N, means, quats, scales, opacities, normals, coeff, k, t);
    return launch_check("mcmc_noise");
}

}  // namespace gsr
