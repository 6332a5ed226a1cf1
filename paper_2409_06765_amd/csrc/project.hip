// Projection of 3D Gaussians to 2D conics (Forward Pass, Projection of
// Gaussians; Data Conventions; Anti-aliasing) and its gradients (Projection
// Gradients; Scale and rotation gradients; SH colour backward).
//
// One thread per Gaussian, looping over the cameras so that the Gaussian's
// parameters (up to 236 bytes with degree-3 SH) are read once per launch.
// Every expression that feeds a discrete output (radius, tile rectangle,
// depth key bits) is evaluated in float32 with IEEE-rounded + - * / sqrt in
// a fixed order; this file is built with -ffp-contract=off.
#include "common.hpp"

#pragma clang fp contract(off)

namespace gsr {
namespace {

// Real spherical-harmonic normalisations up to degree 3 (Condon-Shortley
// phase), sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) times sqrt(2) for m != 0,
// folded into the Cartesian polynomial of each basis function.
constexpr float kSH0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
constexpr float kSH1 = 0.48860251190291992f;   // sqrt(3/(4 pi))
constexpr float kSH2a = 1.0925484305920792f;   // sqrt(15/pi)/2     (xy, yz, xz)
constexpr float kSH2b = 0.31539156525252005f;  // sqrt(5/pi)/4      (2z^2 - x^2 - y^2)
constexpr float kSH2c = 0.54627421529603959f;  // sqrt(15/pi)/4     (x^2 - y^2)
constexpr float kSH3a = 0.59004358992664352f;  // sqrt(35/(2 pi))/4 (m = +-3)
constexpr float kSH3b = 2.8906114426405538f;   // sqrt(105/pi)/2    (xyz)
constexpr float kSH3c = 0.45704579946446572f;  // sqrt(21/(2 pi))/4 (m = +-1)
constexpr float kSH3d = 0.3731763325901154f;   // sqrt(7/pi)/4      (m = 0)
constexpr float kSH3e = 1.4453057213202769f;   // sqrt(105/pi)/4    (m = 2)

template <int NK>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float *Y) {
    Y[0] = kSH0;
    if (NK > 1) {
        Y[1] = -kSH1 * y;
        Y[2] = kSH1 * z;
        Y[3] = -kSH1 * x;
    }
    if (NK > 4) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = kSH2a * (x * y);
        Y[5] = -kSH2a * (y * z);
        Y[6] = kSH2b * (2.0f * zz - xx - yy);
        Y[7] = -kSH2a * (x * z);
        Y[8] = kSH2c * (xx - yy);
        if (NK > 9) {
            Y[9] = -kSH3a * y * (3.0f * xx - yy);
            Y[10] = kSH3b * (x * y) * z;
            Y[11] = -kSH3c * y * (4.0f * zz - xx - yy);
            Y[12] = kSH3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
            Y[13] = -kSH3c * x * (4.0f * zz - xx - yy);
            Y[14] = kSH3e * z * (xx - yy);
            Y[15] = -kSH3a * x * (xx - 3.0f * yy);
        }
    }
}

// d/d(x, y, z) of sum_k w_k Y_k, accumulated into g.
template <int NK>
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, const float *w, float g[3]) {
    if (NK > 1) {
        g[1] += -kSH1 * w[1];
        g[2] += kSH1 * w[2];
        g[0] += -kSH1 * w[3];
    }
    if (NK > 4) {
        const float xx = x * x, yy = y * y, zz = z * z;
        g[0] += kSH2a * y * w[4];            g[1] += kSH2a * x * w[4];
        g[1] += -kSH2a * z * w[5];           g[2] += -kSH2a * y * w[5];
        g[0] += -2.0f * kSH2b * x * w[6];    g[1] += -2.0f * kSH2b * y * w[6];  g[2] += 4.0f * kSH2b * z * w[6];
        g[0] += -kSH2a * z * w[7];           g[2] += -kSH2a * x * w[7];
        g[0] += 2.0f * kSH2c * x * w[8];     g[1] += -2.0f * kSH2c * y * w[8];
        if (NK > 9) {
            g[0] += -6.0f * kSH3a * x * y * w[9];
            g[1] += -kSH3a * (3.0f * xx - 3.0f * yy) * w[9];
            g[0] += kSH3b * y * z * w[10];  g[1] += kSH3b * x * z * w[10];  g[2] += kSH3b * x * y * w[10];
            g[0] += 2.0f * kSH3c * x * y * w[11];
            g[1] += -kSH3c * (4.0f * zz - xx - 3.0f * yy) * w[11];
            g[2] += -8.0f * kSH3c * y * z * w[11];
            g[0] += -6.0f * kSH3d * x * z * w[12];
            g[1] += -6.0f * kSH3d * y * z * w[12];
            g[2] += kSH3d * (6.0f * zz - 3.0f * xx - 3.0f * yy) * w[12];
            g[0] += -kSH3c * (4.0f * zz - 3.0f * xx - yy) * w[13];
            g[1] += 2.0f * kSH3c * x * y * w[13];
            g[2] += -8.0f * kSH3c * x * z * w[13];
            g[0] += 2.0f * kSH3e * x * z * w[14];  g[1] += -2.0f * kSH3e * y * z * w[14];
            g[2] += kSH3e * (xx - yy) * w[14];
            g[0] += -kSH3a * (3.0f * xx - 3.0f * yy) * w[15];
            g[1] += 6.0f * kSH3a * x * y * w[15];
        }
    }
}

// Everything the forward computes for one (camera, Gaussian), kept for the
// backward, which recomputes it instead of storing it.
struct Proj {
    bool valid;
    float t[3];
    float qn[4], qnorm;
    float R[3][3], M[3][3], Sig[3][3];
    float J00, J02, J11, J12;
    int clx, cly;
    float limx, limy;
    float T[2][3];
    float cov[3];        // Sigma' before dilation: 00, 01, 11
    float a, b, c, det;  // dilated
    float mx, my;
    int radius;
};

// The canonical float32 evaluation order of the projection; identical
// expression trees give identical bits on any IEEE-conforming machine.
__device__ __forceinline__ void project_core(const gsr_params &p, int W, int H, int TX, int TY,
                                             const float mu[3], const float q[4], const float s[3],
                                             const float *__restrict__ V, const float *__restrict__ Kc, Proj &o) {
    o.valid = false;
    o.radius = 0;
    const float fx = Kc[0], fy = Kc[4], cx = Kc[2], cy = Kc[5];
    for (int i = 0; i < 3; i++)
        o.t[i] = ((V[4 * i + 0] * mu[0] + V[4 * i + 1] * mu[1]) + V[4 * i + 2] * mu[2]) + V[4 * i + 3];
    const float tx = o.t[0], ty = o.t[1], tz = o.t[2];
    if (tz < p.near_plane || tz > p.far_plane) return;

    const float n2 = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
    const float nrm = sqrtf(n2);
    if (!(nrm > 0.0f)) return;
    o.qnorm = nrm;
    o.qn[0] = q[0] / nrm; o.qn[1] = q[1] / nrm; o.qn[2] = q[2] / nrm; o.qn[3] = q[3] / nrm;
    const float w = o.qn[0], x = o.qn[1], y = o.qn[2], z = o.qn[3];
    o.R[0][0] = 1.0f - 2.0f * (y * y + z * z);
    o.R[0][1] = 2.0f * (x * y - w * z);
    o.R[0][2] = 2.0f * (x * z + w * y);
    o.R[1][0] = 2.0f * (x * y + w * z);
    o.R[1][1] = 1.0f - 2.0f * (x * x + z * z);
    o.R[1][2] = 2.0f * (y * z - w * x);
    o.R[2][0] = 2.0f * (x * z - w * y);
    o.R[2][1] = 2.0f * (y * z + w * x);
    o.R[2][2] = 1.0f - 2.0f * (x * x + y * y);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) o.M[i][j] = o.R[i][j] * s[j];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            o.Sig[i][j] = (o.M[i][0] * o.M[j][0] + o.M[i][1] * o.M[j][1]) + o.M[i][2] * o.M[j][2];

    float txc = tx, tyc = ty;
    o.clx = o.cly = 0;
    o.limx = o.limy = 0.0f;
    if (p.jac_clamp > 0.0f) {
        o.limx = p.jac_clamp * ((0.5f * (float)W) / fx);
        o.limy = p.jac_clamp * ((0.5f * (float)H) / fy);
        const float ux = tx / tz, uy = ty / tz;
        if (ux > o.limx) { txc = o.limx * tz; o.clx = 1; }
        else if (ux < -o.limx) { txc = (-o.limx) * tz; o.clx = -1; }
        if (uy > o.limy) { tyc = o.limy * tz; o.cly = 1; }
        else if (uy < -o.limy) { tyc = (-o.limy) * tz; o.cly = -1; }
    }
    const float tz2 = tz * tz;
    o.J00 = fx / tz;
    o.J02 = -(fx * txc) / tz2;
    o.J11 = fy / tz;
    o.J12 = -(fy * tyc) / tz2;
    for (int j = 0; j < 3; j++) {
        o.T[0][j] = o.J00 * V[j] + o.J02 * V[8 + j];
        o.T[1][j] = o.J11 * V[4 + j] + o.J12 * V[8 + j];
    }
    float B[2][3];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 3; j++)
            B[i][j] = (o.T[i][0] * o.Sig[0][j] + o.T[i][1] * o.Sig[1][j]) + o.T[i][2] * o.Sig[2][j];
    o.cov[0] = (B[0][0] * o.T[0][0] + B[0][1] * o.T[0][1]) + B[0][2] * o.T[0][2];
    o.cov[1] = (B[0][0] * o.T[1][0] + B[0][1] * o.T[1][1]) + B[0][2] * o.T[1][2];
    o.cov[2] = (B[1][0] * o.T[1][0] + B[1][1] * o.T[1][1]) + B[1][2] * o.T[1][2];
    o.a = o.cov[0] + p.eps2d;
    o.b = o.cov[1];
    o.c = o.cov[2] + p.eps2d;
    o.det = o.a * o.c - o.b * o.b;
    if (!(o.det > 0.0f)) return;

    const float mid = 0.5f * (o.a + o.c);
    const float h = 0.5f * (o.a - o.c);
    const float lam = mid + sqrtf(h * h + o.b * o.b);
    float rf = ceilf(3.0f * sqrtf(lam));
    if (rf > 1073741824.0f) rf = 1073741824.0f;
    o.mx = (fx * tx) / tz + cx;
    o.my = (fy * ty) / tz + cy;
    int x0, x1, y0, y1;
    tile_rect(o.mx, o.my, (int)rf, TX, TY, x0, x1, y0, y1);
    if (x0 >= x1 || y0 >= y1) return;
    o.radius = (int)rf;
    o.valid = true;
}

template <int NK>
__device__ __forceinline__ void load_colour_coeffs(const float *__restrict__ shc, int n, float *out) {
    constexpr int L = NK > 0 ? 3 * NK : 3;
    const float *src = shc + (size_t)n * L;
    if constexpr (L % 4 == 0) {
        const float4 *s4 = reinterpret_cast<const float4 *>(src);
#pragma unroll
        for (int i = 0; i < L / 4; i++) {
            float4 v = s4[i];
            out[4 * i] = v.x; out[4 * i + 1] = v.y; out[4 * i + 2] = v.z; out[4 * i + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < L; i++) out[i] = src[i];
    }
}

// NK = number of SH coefficients per channel, 0 for direct colours.
template <int NK>
__global__ void __launch_bounds__(256) project_fwd_kernel(gsr_params p, CamTable cams, int N,
        const float *__restrict__ means, const float *__restrict__ quats, const float *__restrict__ scales,
        const float *__restrict__ shc, const float *__restrict__ viewmats, const float *__restrict__ Ks,
        float *__restrict__ means2d, float *__restrict__ conics, int32_t *__restrict__ radii,
        float *__restrict__ depths, float *__restrict__ colors, float *__restrict__ comps) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const float mu[3] = {means[3 * n], means[3 * n + 1], means[3 * n + 2]};
    const float4 q4 = reinterpret_cast<const float4 *>(quats)[n];
    const float q[4] = {q4.x, q4.y, q4.z, q4.w};
    const float s[3] = {scales[3 * n], scales[3 * n + 1], scales[3 * n + 2]};
    constexpr int L = NK > 0 ? 3 * NK : 3;
    float coef[L];
    bool have_coef = false;
    for (int c = 0; c < cams.C; c++) {
        const CamInfo ci = cams.cam[c];
        const float *V = viewmats + 16 * c;
        const float *Kc = Ks + 9 * c;
        Proj o;
        project_core(p, ci.W, ci.H, ci.TX, ci.TY, mu, q, s, V, Kc, o);
        const size_t g = (size_t)c * N + n;
        if (!o.valid) {
            means2d[2 * g] = 0.0f; means2d[2 * g + 1] = 0.0f;
            conics[3 * g] = 0.0f; conics[3 * g + 1] = 0.0f; conics[3 * g + 2] = 0.0f;
            if (colors) { colors[3 * g] = 0.0f; colors[3 * g + 1] = 0.0f; colors[3 * g + 2] = 0.0f; }
            radii[g] = 0;
            depths[g] = 0.0f;
            if (comps) comps[g] = 0.0f;
            continue;
        }
        if (colors && !have_coef) {   // culled Gaussians never read their colour coefficients
            load_colour_coeffs<NK>(shc, n, coef);
            have_coef = true;
        }
        means2d[2 * g] = o.mx; means2d[2 * g + 1] = o.my;
        conics[3 * g] = o.c / o.det;
        conics[3 * g + 1] = -o.b / o.det;
        conics[3 * g + 2] = o.a / o.det;
        radii[g] = o.radius;
        depths[g] = o.t[2];
        if (comps) {
            float cv = 1.0f;
            if (p.antialiased) {
                const float det0 = o.cov[0] * o.cov[2] - o.cov[1] * o.cov[1];
                cv = sqrtf(fmaxf(det0 / o.det, 0.0f));
            }
            comps[g] = cv;
        }
        if constexpr (NK > 0) {
            // view direction from the camera centre -R^T t to the mean
            float cp[3], d[3];
            for (int j = 0; j < 3; j++) cp[j] = -((V[j] * V[3] + V[4 + j] * V[7]) + V[8 + j] * V[11]);
            for (int j = 0; j < 3; j++) d[j] = mu[j] - cp[j];
            const float dn = sqrtf((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
            float Y[NK];
            sh_basis<NK>(d[0] / dn, d[1] / dn, d[2] / dn, Y);
            for (int ch = 0; ch < 3; ch++) {
                float acc = 0.0f;
#pragma unroll
                for (int k = 0; k < NK; k++) acc += Y[k] * coef[3 * k + ch];
                colors[3 * g + ch] = fmaxf(acc + 0.5f, 0.0f);
            }
        } else if (colors) {   // direct colours; none when the rasterizer takes features of its own
            colors[3 * g] = coef[0]; colors[3 * g + 1] = coef[1]; colors[3 * g + 2] = coef[2];
        }
    }
}

// kPose: also the gradient with respect to the world-to-camera matrices.  Per camera, each
// (camera, Gaussian) contributes to the 12 entries of [R | t] (t_cam = R mu + t: vt mu^T and vt;
// T = J R: J^T dL/dT; camera centre -R^T t of the SH direction: t gdir^T and R gdir, gdir being the
// mean gradient through the direction); the sums over the block go to pose_part[block][c][12].
template <int NK, bool kPose>
__global__ void __launch_bounds__(256) project_bwd_kernel(gsr_params p, CamTable cams, int N,
        const float *__restrict__ means, const float *__restrict__ quats, const float *__restrict__ scales,
        const float *__restrict__ opacities, const float *__restrict__ shc, const float *__restrict__ viewmats,
        const float *__restrict__ Ks, const int32_t *__restrict__ radii, const float *__restrict__ comps,
        const float *__restrict__ v_means2d, const float *__restrict__ v_conics,
        const float *__restrict__ v_colors, const float *__restrict__ v_opac_cn,
        const float *__restrict__ v_depths, float *__restrict__ v_means, float *__restrict__ v_quats,
        float *__restrict__ v_scales, float *__restrict__ v_opac, float *__restrict__ v_sh,
        float *__restrict__ pose_part) {
    __shared__ float s_pose[kPose ? GSR_MAX_CAMERAS * 12 : 1];
    const int n_raw = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = n_raw < N;
    if (!kPose && !in) return;
    const int n = in ? n_raw : 0;   // lanes past the end stay for the block's pose sums and add zero
    if (kPose) {
        for (int i = threadIdx.x; i < cams.C * 12; i += blockDim.x) s_pose[i] = 0.0f;
        __syncthreads();
    }
    const float mu[3] = {means[3 * n], means[3 * n + 1], means[3 * n + 2]};
    const float4 q4 = reinterpret_cast<const float4 *>(quats)[n];
    const float q[4] = {q4.x, q4.y, q4.z, q4.w};
    const float s[3] = {scales[3 * n], scales[3 * n + 1], scales[3 * n + 2]};
    constexpr int L = NK > 0 ? 3 * NK : 3;
    float coef[L];
    float acc_sh[L];
    for (int i = 0; i < L; i++) acc_sh[i] = 0.0f;
    float acc_mu[3] = {0.0f, 0.0f, 0.0f}, acc_q[4] = {0.0f, 0.0f, 0.0f, 0.0f}, acc_s[3] = {0.0f, 0.0f, 0.0f};
    float acc_o = 0.0f;
    bool have_coef = false;
    for (int c = 0; c < cams.C; c++) {
        float pv[kPose ? 12 : 1];   // this Gaussian's share of dL/d[R | t] for camera c
        if (kPose)
            for (int k = 0; k < 12; k++) pv[k] = 0.0f;
        do {
        if (!in) break;
        const size_t g = (size_t)c * N + n;
        // the 2D gradients of (c, n): four arrays, or one record per (camera, Gaussian); loaded with the
        // radius, before the projection is recomputed, so that their latency overlaps it
        const bool rec = p.grad_records != 0;
        const float *gm = rec ? v_means2d + g * GSR_GRAD_RECORD : v_means2d + 2 * g;
        const float *gc = rec ? gm + 2 : v_conics + 3 * g;
        const float *gcol = rec ? gm + 5 : (v_colors ? v_colors + 3 * g : nullptr);
        const int rad = radii[g];
        const float vmx = gm[0], vmy = gm[1];
        const float ga = gc[0], gb = 0.5f * gc[1], gcc = gc[2];
        float vc[3] = {0.0f, 0.0f, 0.0f};   // no v_colors: direct colours are not differentiated here
        if (gcol) { vc[0] = gcol[0]; vc[1] = gcol[1]; vc[2] = gcol[2]; }
        const float vo = rec ? gm[8] : v_opac_cn[g];
        const float vdep = v_depths ? v_depths[g] : 0.0f;
        const float comp = (p.antialiased && comps) ? comps[g] : 1.0f;
        if (rad <= 0) break;
        const CamInfo ci = cams.cam[c];
        const float *V = viewmats + 16 * c;
        const float *Kc = Ks + 9 * c;
        Proj o;
        project_core(p, ci.W, ci.H, ci.TX, ci.TY, mu, q, s, V, Kc, o);
        if (!o.valid) break;
        if (NK > 0 && !have_coef) {
            load_colour_coeffs<NK>(shc, n, coef);
            have_coef = true;
        }
        const float fx = Kc[0], fy = Kc[4];
        const float tx = o.t[0], ty = o.t[1], tz = o.t[2];
        float vt[3] = {0.0f, 0.0f, 0.0f};

        // opacity (the rasterizer's opacity is o times the compensation)
        acc_o += vo * comp;

        // 2D mean
        vt[0] += vmx * fx / tz;
        vt[1] += vmy * fy / tz;
        vt[2] += -(vmx * fx * tx + vmy * fy * ty) / (tz * tz);
        if (v_depths) vt[2] += vdep;

        // conic -> Sigma':  dL/dSigma' = -Y G Y,  G = [[ga, gb/2], [gb/2, gc]].  The product is
        // formed in full (S10 apart from S01, each row from the same row of Y G): for needle-like
        // Gaussians Y is nearly singular and the later products with T and Sigma cancel, which
        // amplifies errors that differ between rows; rows built consistently keep them small.
        const float ya = o.c / o.det, yb = -o.b / o.det, yc = o.a / o.det;
        const float YG00 = ya * ga + yb * gb, YG01 = ya * gb + yb * gcc;
        const float YG10 = yb * ga + yc * gb, YG11 = yb * gb + yc * gcc;
        float S00 = -(YG00 * ya + YG01 * yb);
        float S01 = -(YG00 * yb + YG01 * yc);
        float S10 = -(YG10 * ya + YG11 * yb);
        float S11 = -(YG10 * yb + YG11 * yc);
        if (p.antialiased) {
            const float det0 = o.cov[0] * o.cov[2] - o.cov[1] * o.cov[1];
            const float vcomp = vo * opacities[n];
            if (comp > 0.0f && det0 > 0.0f && vcomp != 0.0f) {
                // comp = sqrt(det0/det): d comp = comp/2 (d det0/det0 - d det/det)
                const float k0 = 0.5f * comp * vcomp;
                S00 += k0 * (o.cov[2] / det0 - o.c / o.det);
                S01 += k0 * (-o.cov[1] / det0 + o.b / o.det);
                S10 += k0 * (-o.cov[1] / det0 + o.b / o.det);
                S11 += k0 * (o.cov[0] / det0 - o.a / o.det);
            }
        }
        // Sigma' = T Sigma T^T:  U = dL/dSigma' T (2x3)
        float U[2][3];
        for (int j = 0; j < 3; j++) {
            U[0][j] = S00 * o.T[0][j] + S01 * o.T[1][j];
            U[1][j] = S10 * o.T[0][j] + S11 * o.T[1][j];
        }
        // dL/dSigma = T^T U ;  dL/dT = 2 U Sigma
        float vSig[3][3];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) vSig[i][j] = o.T[0][i] * U[0][j] + o.T[1][i] * U[1][j];
        float vT[2][3];
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 3; j++)
                vT[i][j] = 2.0f * ((U[i][0] * o.Sig[0][j] + U[i][1] * o.Sig[1][j]) + U[i][2] * o.Sig[2][j]);
        // T = J R_cw: dL/dJ = dL/dT R_cw^T (only the four non-zero entries of J)
        const float vJ00 = (vT[0][0] * V[0] + vT[0][1] * V[1]) + vT[0][2] * V[2];
        const float vJ02 = (vT[0][0] * V[8] + vT[0][1] * V[9]) + vT[0][2] * V[10];
        const float vJ11 = (vT[1][0] * V[4] + vT[1][1] * V[5]) + vT[1][2] * V[6];
        const float vJ12 = (vT[1][0] * V[8] + vT[1][1] * V[9]) + vT[1][2] * V[10];
        const float txc = o.clx ? (float)o.clx * o.limx * tz : tx;
        const float tyc = o.cly ? (float)o.cly * o.limy * tz : ty;
        const float tz2 = tz * tz, tz3 = tz2 * tz;
        const float vtxc = vJ02 * (-fx / tz2);
        const float vtyc = vJ12 * (-fy / tz2);
        vt[2] += vJ00 * (-fx / tz2) + vJ02 * (2.0f * fx * txc / tz3) + vJ11 * (-fy / tz2) +
                 vJ12 * (2.0f * fy * tyc / tz3);
        if (o.clx) vt[2] += vtxc * ((float)o.clx * o.limx); else vt[0] += vtxc;
        if (o.cly) vt[2] += vtyc * ((float)o.cly * o.limy); else vt[1] += vtyc;

        // t = R_cw mu + t_cw
        float vmu[3];
        for (int j = 0; j < 3; j++) vmu[j] = (V[j] * vt[0] + V[4 + j] * vt[1]) + V[8 + j] * vt[2];

        // Sigma = M M^T, M = R S
        float vM[3][3];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++)
                vM[i][j] = 2.0f * ((vSig[i][0] * o.M[0][j] + vSig[i][1] * o.M[1][j]) + vSig[i][2] * o.M[2][j]);
        float vR[3][3];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) vR[i][j] = vM[i][j] * s[j];
        for (int j = 0; j < 3; j++) acc_s[j] += (o.R[0][j] * vM[0][j] + o.R[1][j] * vM[1][j]) + o.R[2][j] * vM[2][j];
        // dR/d(w, x, y, z) at the unit quaternion
        const float w = o.qn[0], x = o.qn[1], y = o.qn[2], z = o.qn[3];
        const float gw = 2.0f * (-z * vR[0][1] + y * vR[0][2] + z * vR[1][0] - x * vR[1][2] - y * vR[2][0] + x * vR[2][1]);
        const float gx = 2.0f * (y * vR[0][1] + z * vR[0][2] + y * vR[1][0] - 2.0f * x * vR[1][1] - w * vR[1][2] +
                                 z * vR[2][0] + w * vR[2][1] - 2.0f * x * vR[2][2]);
        const float gy = 2.0f * (-2.0f * y * vR[0][0] + x * vR[0][1] + w * vR[0][2] + x * vR[1][0] + z * vR[1][2] -
                                 w * vR[2][0] + z * vR[2][1] - 2.0f * y * vR[2][2]);
        const float gz = 2.0f * (-2.0f * z * vR[0][0] - w * vR[0][1] + x * vR[0][2] + w * vR[1][0] - 2.0f * z * vR[1][1] +
                                 y * vR[1][2] + x * vR[2][0] + y * vR[2][1]);
        const float dq = ((w * gw + x * gx) + y * gy) + z * gz;
        acc_q[0] += (gw - w * dq) / o.qnorm;
        acc_q[1] += (gx - x * dq) / o.qnorm;
        acc_q[2] += (gy - y * dq) / o.qnorm;
        acc_q[3] += (gz - z * dq) / o.qnorm;

        // colour
        float gdir[3] = {0.0f, 0.0f, 0.0f};   // mean gradient through the SH view direction
        if constexpr (NK > 0) {
            float cp[3], d[3];
            for (int j = 0; j < 3; j++) cp[j] = -((V[j] * V[3] + V[4 + j] * V[7]) + V[8 + j] * V[11]);
            for (int j = 0; j < 3; j++) d[j] = mu[j] - cp[j];
            const float dn = sqrtf((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
            const float dir[3] = {d[0] / dn, d[1] / dn, d[2] / dn};
            float Y[NK];
            sh_basis<NK>(dir[0], dir[1], dir[2], Y);
            float vraw[3];
            for (int ch = 0; ch < 3; ch++) {
                float raw = 0.0f;
#pragma unroll
                for (int k = 0; k < NK; k++) raw += Y[k] * coef[3 * k + ch];
                vraw[ch] = (raw + 0.5f < 0.0f) ? 0.0f : vc[ch];
            }
            float wk[NK];
#pragma unroll
            for (int k = 0; k < NK; k++) {
                acc_sh[3 * k] += Y[k] * vraw[0];
                acc_sh[3 * k + 1] += Y[k] * vraw[1];
                acc_sh[3 * k + 2] += Y[k] * vraw[2];
                wk[k] = (coef[3 * k] * vraw[0] + coef[3 * k + 1] * vraw[1]) + coef[3 * k + 2] * vraw[2];
            }
            float vdir[3] = {0.0f, 0.0f, 0.0f};
            sh_basis_grad<NK>(dir[0], dir[1], dir[2], wk, vdir);
            const float dd = (dir[0] * vdir[0] + dir[1] * vdir[1]) + dir[2] * vdir[2];
            for (int j = 0; j < 3; j++) {
                gdir[j] = (vdir[j] - dir[j] * dd) / dn;
                vmu[j] += gdir[j];
            }
        } else {
            acc_sh[0] += vc[0]; acc_sh[1] += vc[1]; acc_sh[2] += vc[2];
        }
        for (int j = 0; j < 3; j++) acc_mu[j] += vmu[j];
        if (kPose) {
            for (int i = 0; i < 3; i++) {
                for (int j = 0; j < 3; j++) {
                    const float jt = i == 0 ? o.J00 * vT[0][j]
                                   : i == 1 ? o.J11 * vT[1][j] : o.J02 * vT[0][j] + o.J12 * vT[1][j];
                    pv[4 * i + j] = (vt[i] * mu[j] + jt) + V[4 * i + 3] * gdir[j];
                }
                pv[4 * i + 3] = vt[i] + ((V[4 * i] * gdir[0] + V[4 * i + 1] * gdir[1]) + V[4 * i + 2] * gdir[2]);
            }
        }
        } while (0);
        if (kPose) {
            // wave sums with every lane active, then one LDS add per value and wave
#pragma unroll
            for (int k = 0; k < 12; k++) {
                float v = pv[k];
#pragma unroll
                for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
                pv[k] = v;
            }
            if (__lane_id() == 0)
                for (int k = 0; k < 12; k++) atomicAdd(&s_pose[c * 12 + k], pv[k]);
        }
    }
    if (in) {
        for (int j = 0; j < 3; j++) { v_means[3 * n + j] = acc_mu[j]; v_scales[3 * n + j] = acc_s[j]; }
        reinterpret_cast<float4 *>(v_quats)[n] = make_float4(acc_q[0], acc_q[1], acc_q[2], acc_q[3]);
        v_opac[n] = acc_o;
        if (v_sh) {
            float *dst = v_sh + (size_t)n * L;
#pragma unroll
            for (int i = 0; i < L; i++) dst[i] = acc_sh[i];
        }
    }
    if (kPose) {
        __syncthreads();
        for (int i = threadIdx.x; i < cams.C * 12; i += blockDim.x)
            pose_part[(size_t)blockIdx.x * cams.C * 12 + i] = s_pose[i];
    }
}

// dL/dviewmats [C,4,4]: one block per (camera, entry of [R | t]) sums the per-block parts; the
// last row is zero.
__global__ void __launch_bounds__(256) pose_reduce_kernel(int nblocks, int C, const float *__restrict__ part,
                                                         float *__restrict__ v_viewmats) {
    __shared__ float red[256];
    const int c = blockIdx.x / 12, k = blockIdx.x % 12;
    float acc = 0.0f;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) acc += part[((size_t)b * C + c) * 12 + k];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        v_viewmats[16 * c + k] = red[0];
        if (k < 4) v_viewmats[16 * c + 12 + k] = 0.0f;
    }
}

int num_coeffs(int sh_degree) { return sh_degree < 0 ? 0 : (sh_degree + 1) * (sh_degree + 1); }

}  // namespace

int launch_project_fwd(const gsr_params &p, const CamTable &cams, int N, const float *means,
                       const float *quats, const float *scales, const float *sh, const float *viewmats,
                       const float *Ks, float *means2d, float *conics, int32_t *radii, float *depths,
                       float *colors, float *comps, hipStream_t s) {
    if (N == 0 || cams.C == 0) return GSR_OK;
    dim3 block(256), grid((N + 255) / 256);
#define GSR_PF(NK) project_fwd_kernel<NK><<<grid, block, 0, s>>>(p, cams, N, means, quats, scales, sh, \
        viewmats, Ks, means2d, conics, radii, depths, colors, comps)
    switch (num_coeffs(p.sh_degree)) {
        case 0: GSR_PF(0); break;
        case 1: GSR_PF(1); break;
        case 4: GSR_PF(4); break;
        case 9: GSR_PF(9); break;
        default: GSR_PF(16); break;
    }
#undef GSR_PF
    return launch_check("project_fwd");
}

int launch_project_bwd(const gsr_params &p, const CamTable &cams, int N, const float *means,
                       const float *quats, const float *scales, const float *opacities, const float *sh,
                       const float *viewmats, const float *Ks, const int32_t *radii, const float *comps,
                       const float *v_means2d, const float *v_conics, const float *v_colors,
                       const float *v_opac_cn, const float *v_depths, float *v_means, float *v_quats,
                       float *v_scales, float *v_opac, float *v_sh, float *v_viewmats, void *ws, hipStream_t s) {
    const int nb = (N + 255) / 256;
    if (N == 0) return GSR_OK;
    dim3 block(256), grid((unsigned)nb);
    float *part = (float *)ws;
#define GSR_PB(NK, POSE) project_bwd_kernel<NK, POSE><<<grid, block, 0, s>>>(p, cams, N, means, quats, scales, \
        opacities, sh, viewmats, Ks, radii, comps, v_means2d, v_conics, v_colors, v_opac_cn, v_depths, v_means, \
        v_quats, v_scales, v_opac, v_sh, part)
#define GSR_PB2(NK) if (v_viewmats) GSR_PB(NK, true); else GSR_PB(NK, false)
    switch (num_coeffs(p.sh_degree)) {
        case 0: GSR_PB2(0); break;
        case 1: GSR_PB2(1); break;
        case 4: GSR_PB2(4); break;
        case 9: GSR_PB2(9); break;
        default: GSR_PB2(16); break;
    }
#undef GSR_PB2
#undef GSR_PB
    if (v_viewmats && cams.C > 0)
        pose_reduce_kernel<<<dim3((unsigned)(cams.C * 12)), dim3(256), 0, s>>>(nb, cams.C, part, v_viewmats);
    return launch_check("project_bwd");
}

size_t pose_workspace_bytes(int C, int N) {
    return (size_t)((N + 255) / 256) * (size_t)(C > 0 ? C : 1) * 12 * sizeof(float);
}

}  // namespace gsr
