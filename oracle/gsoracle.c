/*
 * gsoracle.c -- plain, slow CPU oracle for the differentiable tile rasterizer
 * of gsplat (arXiv 2409.06765).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or constant table with the HIP
 * library.
 *
 * One source, two builds: -DREAL=float (the kernels' precision, used wherever
 * floating point decides an integer: radii, tile rectangles, depth key bits,
 * skip/stop decisions) and -DREAL=double (pins, invariants, finite
 * differences).  Build with  gcc -O2 -ffp-contract=off -fno-fast-math  so
 * that every expression below is evaluated exactly in the order written, with
 * IEEE correctly-rounded + - * / sqrt.
 *
 * Section references are to the paper's appendices:
 *   "Forward Pass / Projection of Gaussians", "Rasterization of Gaussians",
 *   "Backward Pass / Depth Compositing Gradients", "Projection Gradients",
 *   "Scale and rotation gradients", "Data Conventions", "Anti-aliasing".
 * Where the paper is silent or garbled the reading used is the one listed in
 * the design notes (camera convention world->camera, strict near cull,
 * 0.3 dilation, square 3-sigma box, alpha clamp 0.99, skip alpha < 1/255,
 * stop when T would drop below 1e-4, SH with +0.5 offset and clamp at 0).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef REAL
#define REAL double
#endif

#define K(x) ((REAL)(x))

static REAL r_sqrt(REAL x) { return (sizeof(REAL) == 4) ? (REAL)sqrtf((float)x) : (REAL)sqrt((double)x); }
static REAL r_exp(REAL x) { return (sizeof(REAL) == 4) ? (REAL)expf((float)x) : (REAL)exp((double)x); }
static REAL r_floor(REAL x) { return (sizeof(REAL) == 4) ? (REAL)floorf((float)x) : (REAL)floor((double)x); }
static REAL r_ceil(REAL x) { return (sizeof(REAL) == 4) ? (REAL)ceilf((float)x) : (REAL)ceil((double)x); }
static REAL r_min(REAL a, REAL b) { return a < b ? a : b; }
static REAL r_max(REAL a, REAL b) { return a > b ? a : b; }

typedef struct {
    double near_plane;   /* cull when t_z < near (strict)                     */
    double far_plane;    /* cull when t_z > far                               */
    double eps2d;        /* low-pass dilation s added to the 2D covariance    */
    double jac_clamp;    /* >0: clamp t_x/t_z, t_y/t_z for J only; 0: literal */
    double alpha_min;    /* skip when alpha < alpha_min                       */
    double alpha_max;    /* alpha = min(alpha_max, o exp(-sigma))             */
    double T_min;        /* stop when T (1 - alpha) < T_min                   */
    int tile;            /* tile edge in pixels (16)                          */
    int sh_degree;       /* -1: direct colours [N,3]; 0..3: SH [N,(d+1)^2,3]  */
    int antialiased;     /* 1: multiply opacity by sqrt(|S'|/|S'+sI|)         */
} orc_params;

/* ------------------------------------------------------------------------ */
/* Data Conventions: rotation matrix of a unit quaternion (w,x,y,z), Hamilton */
/* ------------------------------------------------------------------------ */
static int normalize_quat(const REAL *q, REAL qn[4], REAL *norm_out)
{
    REAL n2 = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
    REAL nrm = r_sqrt(n2);
    if (!(nrm > K(0))) return 0;
    qn[0] = q[0] / nrm; qn[1] = q[1] / nrm; qn[2] = q[2] / nrm; qn[3] = q[3] / nrm;
    if (norm_out) *norm_out = nrm;
    return 1;
}

static void quat_to_R(const REAL qn[4], REAL R[3][3])
{
    REAL w = qn[0], x = qn[1], y = qn[2], z = qn[3];
    R[0][0] = K(1) - K(2) * (y * y + z * z);
    R[0][1] = K(2) * (x * y - w * z);
    R[0][2] = K(2) * (x * z + w * y);
    R[1][0] = K(2) * (x * y + w * z);
    R[1][1] = K(1) - K(2) * (x * x + z * z);
    R[1][2] = K(2) * (y * z - w * x);
    R[2][0] = K(2) * (x * z - w * y);
    R[2][1] = K(2) * (y * z + w * x);
    R[2][2] = K(1) - K(2) * (x * x + y * y);
}

/* 3D covariance Sigma = M M^T with M = R S (Scale and rotation gradients). */
static void covariance3d(const REAL R[3][3], const REAL s[3], REAL M[3][3], REAL Sig[3][3])
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) M[i][j] = R[i][j] * s[j];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            Sig[i][j] = (M[i][0] * M[j][0] + M[i][1] * M[j][1]) + M[i][2] * M[j][2];
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics up to degree 3, ordered k = l*l + l + m.        */
/* Each basis function is a homogeneous polynomial in the unit direction,    */
/* stored as a monomial table (coefficient, powers of x, y, z).  The         */
/* coefficients are the normalisation sqrt((2l+1)/(4pi) (l-|m|)!/(l+|m|)!),  */
/* times sqrt(2) for m != 0, with the Condon-Shortley phase; the tests pin   */
/* the table against scipy's complex spherical harmonics.                    */
/* ------------------------------------------------------------------------ */
typedef struct { int k; double c; int px, py, pz; } sh_mono;

#define PI_D 3.14159265358979323846
static sh_mono SH_TABLE[40];
static int SH_TABLE_N = 0;

static void sh_add(int k, double c, int px, int py, int pz)
{
    SH_TABLE[SH_TABLE_N].k = k; SH_TABLE[SH_TABLE_N].c = c;
    SH_TABLE[SH_TABLE_N].px = px; SH_TABLE[SH_TABLE_N].py = py; SH_TABLE[SH_TABLE_N].pz = pz;
    SH_TABLE_N++;
}

static void sh_init(void)
{
    if (SH_TABLE_N) return;
    double c0 = 0.5 * sqrt(1.0 / PI_D);
    double c1 = sqrt(3.0 / (4.0 * PI_D));
    double c2a = 0.5 * sqrt(15.0 / PI_D);           /* l=2, |m|=1,2 (xy, yz, xz) */
    double c2b = 0.25 * sqrt(5.0 / PI_D);           /* l=2, m=0                  */
    double c2c = 0.25 * sqrt(15.0 / PI_D);          /* l=2, |m|=2 (x^2-y^2)      */
    double c3a = 0.25 * sqrt(35.0 / (2.0 * PI_D));  /* l=3, |m|=3                */
    double c3b = 0.5 * sqrt(105.0 / PI_D);          /* l=3, m=-2                 */
    double c3c = 0.25 * sqrt(21.0 / (2.0 * PI_D));  /* l=3, |m|=1                */
    double c3d = 0.25 * sqrt(7.0 / PI_D);           /* l=3, m=0                  */
    double c3e = 0.25 * sqrt(105.0 / PI_D);         /* l=3, m=2                  */
    sh_add(0, c0, 0, 0, 0);
    sh_add(1, -c1, 0, 1, 0);
    sh_add(2, c1, 0, 0, 1);
    sh_add(3, -c1, 1, 0, 0);
    sh_add(4, c2a, 1, 1, 0);
    sh_add(5, -c2a, 0, 1, 1);
    sh_add(6, 2.0 * c2b, 0, 0, 2); sh_add(6, -c2b, 2, 0, 0); sh_add(6, -c2b, 0, 2, 0);
    sh_add(7, -c2a, 1, 0, 1);
    sh_add(8, c2c, 2, 0, 0); sh_add(8, -c2c, 0, 2, 0);
    sh_add(9, -3.0 * c3a, 2, 1, 0); sh_add(9, c3a, 0, 3, 0);
    sh_add(10, c3b, 1, 1, 1);
    sh_add(11, -4.0 * c3c, 0, 1, 2); sh_add(11, c3c, 2, 1, 0); sh_add(11, c3c, 0, 3, 0);
    sh_add(12, 2.0 * c3d, 0, 0, 3); sh_add(12, -3.0 * c3d, 2, 0, 1); sh_add(12, -3.0 * c3d, 0, 2, 1);
    sh_add(13, -4.0 * c3c, 1, 0, 2); sh_add(13, c3c, 3, 0, 0); sh_add(13, c3c, 1, 2, 0);
    sh_add(14, c3e, 2, 0, 1); sh_add(14, -c3e, 0, 2, 1);
    sh_add(15, -c3a, 3, 0, 0); sh_add(15, 3.0 * c3a, 1, 2, 0);
}

static REAL ipow(REAL x, int p)
{
    REAL r = K(1);
    for (int i = 0; i < p; i++) r = r * x;
    return r;
}

/* Y[k] for k < nk, and optionally dY[k][3] = gradient w.r.t. (x, y, z). */
static void sh_eval(int nk, const REAL d[3], REAL *Y, REAL (*dY)[3])
{
    sh_init();
    for (int k = 0; k < nk; k++) {
        Y[k] = K(0);
        if (dY) dY[k][0] = dY[k][1] = dY[k][2] = K(0);
    }
    for (int t = 0; t < SH_TABLE_N; t++) {
        const sh_mono *m = &SH_TABLE[t];
        if (m->k >= nk) continue;
        REAL c = (REAL)m->c;
        Y[m->k] += c * ipow(d[0], m->px) * ipow(d[1], m->py) * ipow(d[2], m->pz);
        if (dY) {
            if (m->px) dY[m->k][0] += c * (REAL)m->px * ipow(d[0], m->px - 1) * ipow(d[1], m->py) * ipow(d[2], m->pz);
            if (m->py) dY[m->k][1] += c * (REAL)m->py * ipow(d[0], m->px) * ipow(d[1], m->py - 1) * ipow(d[2], m->pz);
            if (m->pz) dY[m->k][2] += c * (REAL)m->pz * ipow(d[0], m->px) * ipow(d[1], m->py) * ipow(d[2], m->pz - 1);
        }
    }
}

/* Exposed for the SH pins: Y[k] (and gradient) at one direction, in double. */
void orc_sh_basis(int nk, const double *dir, double *Y, double *dY)
{
    REAL d[3] = {(REAL)dir[0], (REAL)dir[1], (REAL)dir[2]};
    REAL y[16], dy[16][3];
    if (nk > 16) nk = 16;
    sh_eval(nk, d, y, dy);
    for (int k = 0; k < nk; k++) {
        Y[k] = (double)y[k];
        if (dY) { dY[3 * k] = (double)dy[k][0]; dY[3 * k + 1] = (double)dy[k][1]; dY[3 * k + 2] = (double)dy[k][2]; }
    }
}

/* Exposed for the covariance pin: Sigma = R(q/|q|) diag(s)^2 R^T. */
void orc_cov3d(const REAL *q, const REAL *s, REAL *Sig_out, REAL *R_out)
{
    REAL qn[4], R[3][3], M[3][3], Sig[3][3];
    if (!normalize_quat(q, qn, NULL)) { memset(Sig_out, 0, 9 * sizeof(REAL)); return; }
    quat_to_R(qn, R);
    covariance3d(R, s, M, Sig);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) { Sig_out[3 * i + j] = Sig[i][j]; if (R_out) R_out[3 * i + j] = R[i][j]; }
}

/* ------------------------------------------------------------------------ */
/* Projection of Gaussians (Forward Pass) for one (camera, Gaussian).        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int valid;            /* survived the near/far and determinant culls      */
    REAL t[3];            /* camera-space mean t = R_cw mu + t_cw              */
    REAL qn[4], qnorm;    /* normalised quaternion and |q|                     */
    REAL R[3][3], M[3][3], Sig[3][3];
    REAL J00, J02, J11, J12;
    int clx, cly;         /* jac clamp state: 0 free, +1/-1 clamped high/low   */
    REAL limx, limy;
    REAL T[2][3];         /* T = J R_cw                                        */
    REAL cov2d[3];        /* Sigma' before dilation (00, 01, 11)               */
    REAL a, b, c;         /* dilated Sigma'                                    */
    REAL det, det0;
    REAL conic[3];
    REAL comp;            /* anti-aliasing compensation (1 when off)           */
    REAL mx, my;
    int radius;
    int x0, x1, y0, y1;   /* tile rectangle [x0,x1) x [y0,y1)                  */
    REAL dir[3], dnorm;   /* SH view direction and |mu - campos|               */
    REAL raw[3];          /* SH sum + 0.5 before the clamp                     */
    REAL color[3];
} proj_t;

static void project_one(const orc_params *P, int W, int H, const REAL *mu, const REAL *q, const REAL *s,
                        const REAL *sh, int nk, const REAL *V, const REAL *Kc, proj_t *o)
{
    memset(o, 0, sizeof(*o));
    o->comp = K(1);
    REAL fx = Kc[0], fy = Kc[4], cx = Kc[2], cy = Kc[5];

    /* t = R_cw mu + t_cw  (world -> camera) */
    for (int i = 0; i < 3; i++)
        o->t[i] = ((V[4 * i + 0] * mu[0] + V[4 * i + 1] * mu[1]) + V[4 * i + 2] * mu[2]) + V[4 * i + 3];
    REAL tx = o->t[0], ty = o->t[1], tz = o->t[2];
    if (tz < (REAL)P->near_plane || tz > (REAL)P->far_plane) return;

    if (!normalize_quat(q, o->qn, &o->qnorm)) return;
    quat_to_R(o->qn, o->R);
    covariance3d(o->R, s, o->M, o->Sig);

    /* Pinhole Jacobian of (fx tx/tz + cx, fy ty/tz + cy), evaluated at the
     * (optionally clamped) camera-space mean. */
    REAL txc = tx, tyc = ty;
    if (P->jac_clamp > 0) {
        o->limx = (REAL)P->jac_clamp * ((K(0.5) * (REAL)W) / fx);
        o->limy = (REAL)P->jac_clamp * ((K(0.5) * (REAL)H) / fy);
        REAL ux = tx / tz, uy = ty / tz;
        if (ux > o->limx) { txc = o->limx * tz; o->clx = 1; }
        else if (ux < -o->limx) { txc = (-o->limx) * tz; o->clx = -1; }
        if (uy > o->limy) { tyc = o->limy * tz; o->cly = 1; }
        else if (uy < -o->limy) { tyc = (-o->limy) * tz; o->cly = -1; }
    }
    REAL tz2 = tz * tz;
    o->J00 = fx / tz;
    o->J02 = -(fx * txc) / tz2;
    o->J11 = fy / tz;
    o->J12 = -(fy * tyc) / tz2;

    /* T = J R_cw;  Sigma' = T Sigma T^T */
    for (int j = 0; j < 3; j++) {
        o->T[0][j] = o->J00 * V[0 + j] + o->J02 * V[8 + j];
        o->T[1][j] = o->J11 * V[4 + j] + o->J12 * V[8 + j];
    }
    REAL B[2][3];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 3; j++)
            B[i][j] = (o->T[i][0] * o->Sig[0][j] + o->T[i][1] * o->Sig[1][j]) + o->T[i][2] * o->Sig[2][j];
    o->cov2d[0] = (B[0][0] * o->T[0][0] + B[0][1] * o->T[0][1]) + B[0][2] * o->T[0][2];
    o->cov2d[1] = (B[0][0] * o->T[1][0] + B[0][1] * o->T[1][1]) + B[0][2] * o->T[1][2];
    o->cov2d[2] = (B[1][0] * o->T[1][0] + B[1][1] * o->T[1][1]) + B[1][2] * o->T[1][2];

    /* low-pass dilation (Anti-aliasing: classic mode) */
    o->a = o->cov2d[0] + (REAL)P->eps2d;
    o->b = o->cov2d[1];
    o->c = o->cov2d[2] + (REAL)P->eps2d;
    o->det = o->a * o->c - o->b * o->b;
    if (!(o->det > K(0))) return;
    o->conic[0] = o->c / o->det;
    o->conic[1] = -o->b / o->det;
    o->conic[2] = o->a / o->det;
    if (P->antialiased) {
        o->det0 = o->cov2d[0] * o->cov2d[2] - o->cov2d[1] * o->cov2d[1];
        o->comp = r_sqrt(r_max(o->det0 / o->det, K(0)));
    }

    /* square box around the 3-sigma ellipse: largest eigenvalue of Sigma' */
    REAL mid = K(0.5) * (o->a + o->c);
    REAL h = K(0.5) * (o->a - o->c);
    REAL lam = mid + r_sqrt(h * h + o->b * o->b);
    REAL rf = r_ceil(K(3) * r_sqrt(lam));
    if (rf > K(1073741824)) rf = K(1073741824);

    /* Data Conventions: pixel coordinates */
    o->mx = (fx * tx) / tz + cx;
    o->my = (fy * ty) / tz + cy;

    int TX = (W + P->tile - 1) / P->tile, TY = (H + P->tile - 1) / P->tile;
    REAL tl = (REAL)P->tile;
    REAL fx0 = r_floor((o->mx - rf) / tl), fx1 = r_floor((o->mx + rf) / tl) + K(1);
    REAL fy0 = r_floor((o->my - rf) / tl), fy1 = r_floor((o->my + rf) / tl) + K(1);
    o->x0 = (int)r_min(r_max(fx0, K(0)), (REAL)TX);
    o->x1 = (int)r_min(r_max(fx1, K(0)), (REAL)TX);
    o->y0 = (int)r_min(r_max(fy0, K(0)), (REAL)TY);
    o->y1 = (int)r_min(r_max(fy1, K(0)), (REAL)TY);
    if (o->x0 >= o->x1 || o->y0 >= o->y1) return;

    /* view-dependent colour: SH of the unit direction from the camera centre */
    if (nk > 0) {
        REAL cp[3];
        for (int j = 0; j < 3; j++)
            cp[j] = -((V[0 + j] * V[3] + V[4 + j] * V[7]) + V[8 + j] * V[11]);
        REAL d[3] = {mu[0] - cp[0], mu[1] - cp[1], mu[2] - cp[2]};
        o->dnorm = r_sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
        o->dir[0] = d[0] / o->dnorm; o->dir[1] = d[1] / o->dnorm; o->dir[2] = d[2] / o->dnorm;
        REAL Y[16];
        sh_eval(nk, o->dir, Y, NULL);
        for (int ch = 0; ch < 3; ch++) {
            REAL acc = K(0);
            for (int k = 0; k < nk; k++) acc += Y[k] * sh[3 * k + ch];
            o->raw[ch] = acc + K(0.5);
            o->color[ch] = r_max(o->raw[ch], K(0));
        }
    } else {
        for (int ch = 0; ch < 3; ch++) o->color[ch] = o->raw[ch] = sh[ch];
    }
    o->radius = (int)rf;
    o->valid = 1;
}

static int num_sh(const orc_params *P) { return P->sh_degree < 0 ? 0 : (P->sh_degree + 1) * (P->sh_degree + 1); }

/* project_fwd: (means, quats, scales, opacities, SH or colours, viewmats, Ks)
 * -> (means2d [C,N,2], conics [C,N,3], radii [C,N], depths [C,N], colors [C,N,3],
 *     compensations [C,N] nullable).  Culled entries are all zero. */
int orc_project(const orc_params *P, int C, int N, const int *W, const int *H,
                const REAL *means, const REAL *quats, const REAL *scales, const REAL *opacities,
                const REAL *sh_or_colors, const REAL *viewmats, const REAL *Ks,
                REAL *means2d, REAL *conics, int32_t *radii, REAL *depths, REAL *colors, REAL *comps)
{
    (void)opacities;
    int nk = num_sh(P);
    int stride = nk > 0 ? 3 * nk : 3;
    for (int c = 0; c < C; c++)
        for (int n = 0; n < N; n++) {
            proj_t o;
            project_one(P, W[c], H[c], means + 3 * (size_t)n, quats + 4 * (size_t)n, scales + 3 * (size_t)n,
                        sh_or_colors + (size_t)stride * n, nk, viewmats + 16 * c, Ks + 9 * c, &o);
            size_t g = (size_t)c * N + n;
            if (!o.valid) {
                means2d[2 * g] = means2d[2 * g + 1] = K(0);
                conics[3 * g] = conics[3 * g + 1] = conics[3 * g + 2] = K(0);
                colors[3 * g] = colors[3 * g + 1] = colors[3 * g + 2] = K(0);
                radii[g] = 0; depths[g] = K(0);
                if (comps) comps[g] = K(0);
                continue;
            }
            means2d[2 * g] = o.mx; means2d[2 * g + 1] = o.my;
            conics[3 * g] = o.conic[0]; conics[3 * g + 1] = o.conic[1]; conics[3 * g + 2] = o.conic[2];
            colors[3 * g] = o.color[0]; colors[3 * g + 1] = o.color[1]; colors[3 * g + 2] = o.color[2];
            radii[g] = o.radius; depths[g] = o.t[2];
            if (comps) comps[g] = o.comp;
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Rasterization of Gaussians: tile binning and per-tile depth sort.        */
/* ------------------------------------------------------------------------ */
static void tile_rect(const orc_params *P, int W, int H, REAL mx, REAL my, int r, int *x0, int *x1, int *y0, int *y1)
{
    int TX = (W + P->tile - 1) / P->tile, TY = (H + P->tile - 1) / P->tile;
    REAL tl = (REAL)P->tile, rf = (REAL)r;
    REAL fx0 = r_floor((mx - rf) / tl), fx1 = r_floor((mx + rf) / tl) + K(1);
    REAL fy0 = r_floor((my - rf) / tl), fy1 = r_floor((my + rf) / tl) + K(1);
    *x0 = (int)r_min(r_max(fx0, K(0)), (REAL)TX);
    *x1 = (int)r_min(r_max(fx1, K(0)), (REAL)TX);
    *y0 = (int)r_min(r_max(fy0, K(0)), (REAL)TY);
    *y1 = (int)r_min(r_max(fy1, K(0)), (REAL)TY);
}

/* tiles touched per (camera, Gaussian), their exclusive prefix sum, total M */
int64_t orc_intersect_count(const orc_params *P, int C, int N, const int *W, const int *H,
                            const REAL *means2d, const int32_t *radii, int32_t *counts, int64_t *offsets)
{
    int64_t acc = 0;
    for (int c = 0; c < C; c++)
        for (int n = 0; n < N; n++) {
            size_t g = (size_t)c * N + n;
            int cnt = 0;
            if (radii[g] > 0) {
                int x0, x1, y0, y1;
                tile_rect(P, W[c], H[c], means2d[2 * g], means2d[2 * g + 1], radii[g], &x0, &x1, &y0, &y1);
                if (x1 > x0 && y1 > y0) cnt = (x1 - x0) * (y1 - y0);
            }
            counts[g] = cnt;
            offsets[g] = acc;
            acc += cnt;
        }
    return acc;
}

static uint32_t float_bits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }

/* one (key, id) per (Gaussian, tile): key = global_tile << 32 | bits(depth) */
int orc_intersect_emit(const orc_params *P, int C, int N, const int *W, const int *H,
                       const REAL *means2d, const int32_t *radii, const REAL *depths,
                       const int64_t *offsets, uint64_t *keys, int32_t *ids)
{
    int64_t tile_base = 0;
    for (int c = 0; c < C; c++) {
        int TX = (W[c] + P->tile - 1) / P->tile, TY = (H[c] + P->tile - 1) / P->tile;
        for (int n = 0; n < N; n++) {
            size_t g = (size_t)c * N + n;
            if (radii[g] <= 0) continue;
            int x0, x1, y0, y1;
            tile_rect(P, W[c], H[c], means2d[2 * g], means2d[2 * g + 1], radii[g], &x0, &x1, &y0, &y1);
            int64_t j = offsets[g];
            uint64_t dbits = float_bits((float)depths[g]);
            for (int ty = y0; ty < y1; ty++)
                for (int tx = x0; tx < x1; tx++) {
                    uint64_t tid = (uint64_t)(tile_base + (int64_t)ty * TX + tx);
                    keys[j] = (tid << 32) | dbits;
                    ids[j] = (int32_t)g;
                    j++;
                }
        }
        tile_base += (int64_t)TX * TY;
    }
    return 0;
}

typedef struct { uint64_t key; int32_t id; } kv_t;
static int kv_cmp(const void *pa, const void *pb)
{
    const kv_t *a = (const kv_t *)pa, *b = (const kv_t *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return (a->id > b->id) - (a->id < b->id);
}

/* stable sort by key: ties keep emission order, i.e. ascending id */
int orc_sort_pairs(int64_t M, uint64_t *keys, int32_t *ids)
{
    kv_t *buf = (kv_t *)malloc((size_t)(M > 0 ? M : 1) * sizeof(kv_t));
    if (!buf) return -1;
    for (int64_t i = 0; i < M; i++) { buf[i].key = keys[i]; buf[i].id = ids[i]; }
    qsort(buf, (size_t)M, sizeof(kv_t), kv_cmp);
    for (int64_t i = 0; i < M; i++) { keys[i] = buf[i].key; ids[i] = buf[i].id; }
    free(buf);
    return 0;
}

/* [start, end) of each tile's run in the sorted list; empty tiles (0, 0) */
int orc_tile_ranges(int64_t M, const uint64_t *keys, int32_t total_tiles, int32_t *ranges)
{
    for (int32_t t = 0; t < total_tiles; t++) ranges[2 * t] = ranges[2 * t + 1] = 0;
    for (int64_t i = 0; i < M; i++) {
        int32_t t = (int32_t)(keys[i] >> 32);
        if (i == 0 || (int32_t)(keys[i - 1] >> 32) != t) ranges[2 * t] = (int32_t)i;
        ranges[2 * t + 1] = (int32_t)(i + 1);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Front-to-back compositing of one pixel over a depth-ordered list.        */
/* ------------------------------------------------------------------------ */
/* colors [C,N,D]: D feature channels per projected Gaussian (N-dimensional
 * rasterization; RGB is D = 3, RGB plus depth D = 4), at most ORC_MAX_D. */
#define ORC_MAX_D 64
typedef struct {
    const orc_params *P;
    int N;
    const REAL *means2d, *conics, *colors, *opacities, *comps;
    int D;
} scene2d_t;

/* Per-pixel decision flags (reading R24 of the design notes: several
 * results are correct).  A pixel is flagged when one of its decisions -- the
 * sign test on sigma, the alpha < alpha_min skip, the alpha_max clamp, the
 * T < T_min stop -- lies within the error bound of an accurate float32
 * implementation of the compositing, so that such an implementation may
 * decide it the other way; everything downstream of that decision may then
 * differ.  One bit per kind of decision. */
#define FLAG_SIGN  1u
#define FLAG_SKIP  2u
#define FLAG_CLAMP 4u
#define FLAG_STOP  8u

typedef struct {
    REAL color[ORC_MAX_D], T;
    int last;            /* list position of the last composited entry, -1 if none */
    int n_eval;          /* entries evaluated, including the one that stopped it   */
    int n_comp;          /* entries composited                                     */
    uint32_t trace;      /* hash of the composited positions and their clamp states */
    uint32_t flags;
    double margin;       /* smallest |ln(value / threshold)| over the skip, clamp and
                            stop decisions (the double-precision values)            */
} pix_out_t;

static REAL gauss_opacity(const scene2d_t *S, int g)
{
    REAL o = S->opacities[g % S->N];
    if (S->comps) o = o * S->comps[g];
    return o;
}

/* v lies within a factor exp(+-tol) of thr. */
static int within_factor(double v, double thr, double tol)
{
    return v >= thr * exp(-tol) && v <= thr * exp(tol);
}

/* sigma = 1/2 (a dx^2 + c dy^2) + b dx dy (Rasterization of Gaussians) of the
 * offsets dx, dy as REAL values, evaluated in double precision: for float32
 * inputs the products a dx, b dx, c dy are exact and the result is within a
 * few double ulps of the magnitude of its terms, so even where the terms
 * cancel (a needle-like Gaussian seen along its long axis) the value is the
 * definition's to far better than float32 resolution.  The REAL result is
 * that value rounded once.  *smag: the sum of the terms' magnitudes. */
static double sigma_of(double a, double b, double c, double dx, double dy, double *smag)
{
    *smag = 0.5 * (fabs(a * dx * dx) + fabs(c * dy * dy)) + fabs(b * dx * dy);
    return 0.5 * ((a * dx) * dx + (c * dy) * dy) + (b * dx) * dy;
}

/* The accuracy bound the flags assume of the implementation being compared:
 * its sigma is within
 *     es = u (8 S + |b u_c dy|)
 * of the definition, u the unit roundoff, S = 1/2 (a u_c^2 + |c - b^2/a| dy^2)
 * with u_c = dx + (b/a) dy: a few ulps of sigma written as a sum of two
 * squares (which does not cancel) plus one ulp of b/a carried through dy.
 * That is what evaluating the completed square achieves; the naive sum of
 * the three terms does not meet it where they cancel, and its decisions are
 * then genuinely open (an error of many ulps of the largest term).  Its
 * alpha = o exp(-sigma) is then within a factor exp(+-(es + 4u)), which also
 * covers the rounding of the exponential and of the product with o. */
static double sigma_budget(double a, double b, double c, double dx, double dy, double u)
{
    if (!(a > 0.0)) return u * 16.0 * (0.5 * (fabs(a * dx * dx) + fabs(c * dy * dy)) + fabs(b * dx * dy));
    const double uc = dx + (b / a) * dy;
    const double q = (a * c - b * b) / a;
    const double S = 0.5 * (a * uc * uc + fabs(q) * dy * dy);
    return u * (8.0 * S + fabs(b * uc * dy));
}

static void composite_pixel(const scene2d_t *S, const int32_t *list, int len, REAL px, REAL py,
                            const REAL *bg, pix_out_t *out)
{
    const orc_params *P = S->P;
    const int D = S->D;
    REAL T = K(1), Cacc[ORC_MAX_D];
    for (int ch = 0; ch < D; ch++) Cacc[ch] = K(0);
    int last = -1, n_eval = 0, n_comp = 0;
    uint32_t trace = 0, flags = 0;
    /* Tt: the transmittance from the double-precision alphas of the entries
     * composited so far; eT: a bound on |ln T - ln Tt| for an implementation
     * within the budget above (each factor 1 - alpha is known to alpha /
     * (1 - alpha) times alpha's relative error, plus the two roundings of
     * 1 - alpha and of the product). */
    double Tt = 1.0, eT = 0.0, margin = INFINITY;
    const double u = (sizeof(REAL) == 4) ? 0x1p-24 : 0x1p-53;
    const double amin = (double)(REAL)P->alpha_min, amax = (double)(REAL)P->alpha_max, tmin = (double)(REAL)P->T_min;
    for (int k = 0; k < len; k++) {
        int g = list[k];
        n_eval++;
        REAL dx = S->means2d[2 * g] - px, dy = S->means2d[2 * g + 1] - py;
        double a = S->conics[3 * g], b = S->conics[3 * g + 1], c = S->conics[3 * g + 2];
        double smag;
        double sd = sigma_of(a, b, c, dx, dy, &smag);
        REAL sigma = (REAL)sd;
        /* the double evaluation's own error (a few double ulps of smag) joins the budget */
        double es = sigma_budget(a, b, c, dx, dy, u) + 4.0 * 0x1p-53 * smag;
        if (fabs(sd) < es) flags |= FLAG_SIGN;
        if (sigma < K(0)) continue;
        REAL o = gauss_opacity(S, g);
        REAL araw = o * r_exp(-sigma);
        REAL alpha = r_min((REAL)P->alpha_max, araw);
        double at = (double)o * exp(-sd);    /* alpha from the double sigma, before the clamp */
        double ea = es + 4.0 * u;            /* its relative error bound in an implementation */
        if (within_factor(at, amin, ea)) flags |= FLAG_SKIP;
        if (within_factor(at, amax, ea)) flags |= FLAG_CLAMP;
        if (at > 0.0) margin = fmin(margin, fmin(fabs(log(at / amin)), fabs(log(at / amax))));
        if (alpha < (REAL)P->alpha_min) continue;
        double alt = at < amax ? at : amax;
        double Ttn = Tt * (1.0 - alt);
        double eTn = eT + (at < amax ? ea * alt / (1.0 - alt) : 0.0) + 2.0 * u;
        if (within_factor(Ttn, tmin, eTn)) flags |= FLAG_STOP;
        margin = fmin(margin, fabs(log(Ttn / tmin)));
        REAL Tn = T * (K(1) - alpha);
        if (Tn < (REAL)P->T_min) break;
        REAL w = alpha * T;
        const REAL *col = S->colors + (size_t)D * g;
        for (int ch = 0; ch < D; ch++) Cacc[ch] += col[ch] * w;
        T = Tn;
        Tt = Ttn;
        eT = eTn;
        last = k;
        n_comp++;
        trace = trace * 2654435761u + (uint32_t)(2 * (k + 1) + (araw > (REAL)P->alpha_max));
    }
    for (int ch = 0; ch < D; ch++) out->color[ch] = Cacc[ch] + T * (bg ? bg[ch] : K(0));
    out->T = T; out->last = last; out->n_eval = n_eval; out->n_comp = n_comp;
    out->trace = trace; out->flags = flags; out->margin = margin;
}

/* Reverse recursion (Depth Compositing Gradients) for one pixel.  Gradient
 * sums go to double accumulators indexed by the Gaussian's [C,N] id. */
/* abs (nullable): per id 6 + D sums of the magnitudes of the terms that make
 * up each gradient element (mean x, y; conic a, b, c; opacity; channels),
 * each term's magnitude taken over its parts before they cancel (for the
 * alpha gradient: sum over channels of |colour T_k| + |S / (1 - alpha)|
 * times |v_C|, plus |v_alpha final_T / (1 - alpha)|): the scale of the
 * rounding error any float32 evaluation and summation of the terms makes. */
typedef struct { double *v_means2d, *v_conics, *v_colors, *v_opac, *abs, *v_means2d_abs; int D, nslot; } grad2d_t;

static void add_term(grad2d_t *G, double *dst, size_t g, int slot, double x, double mag)
{
    *dst += x;
    if (G->abs) G->abs[(size_t)G->nslot * g + (size_t)slot] += mag;
}

static void grad2d_alloc(grad2d_t *G, size_t CN, int D, int want_abs, int want_absgrad)
{
    G->D = D;
    G->nslot = 6 + D;
    G->v_means2d_abs = want_absgrad ? (double *)calloc(2 * CN + 1, sizeof(double)) : NULL;
    G->v_means2d = (double *)calloc(2 * CN + 1, sizeof(double));
    G->v_conics = (double *)calloc(3 * CN + 1, sizeof(double));
    G->v_colors = (double *)calloc((size_t)D * CN + 1, sizeof(double));
    G->v_opac = (double *)calloc(CN + 1, sizeof(double));
    G->abs = want_abs ? (double *)calloc((size_t)(6 + D) * CN + 1, sizeof(double)) : NULL;
}

static void grad2d_store(grad2d_t *G, size_t CN, REAL *v_means2d, REAL *v_conics, REAL *v_colors,
                         REAL *v_opacities, REAL *abs_sums, REAL *v_means2d_abs)
{
    if (v_means2d_abs && G->v_means2d_abs)
        for (size_t i = 0; i < 2 * CN; i++) v_means2d_abs[i] = (REAL)G->v_means2d_abs[i];
    free(G->v_means2d_abs);
    for (size_t i = 0; i < 2 * CN; i++) v_means2d[i] = (REAL)G->v_means2d[i];
    for (size_t i = 0; i < 3 * CN; i++) v_conics[i] = (REAL)G->v_conics[i];
    for (size_t i = 0; i < (size_t)G->D * CN; i++) v_colors[i] = (REAL)G->v_colors[i];
    for (size_t i = 0; i < CN; i++) v_opacities[i] = (REAL)G->v_opac[i];
    if (abs_sums && G->abs)
        for (size_t i = 0; i < (size_t)(6 + G->D) * CN; i++) abs_sums[i] = (REAL)G->abs[i];
    free(G->v_means2d); free(G->v_conics); free(G->v_colors); free(G->v_opac); free(G->abs);
}

static void composite_pixel_bwd(const scene2d_t *S, const int32_t *list, int last, REAL px, REAL py,
                                const REAL *bg, REAL T_final, const REAL *vC, REAL vA, grad2d_t *G)
{
    const orc_params *P = S->P;
    const int D = S->D;
    REAL T = T_final;
    REAL Sacc[ORC_MAX_D];
    for (int ch = 0; ch < D; ch++) Sacc[ch] = T_final * (bg ? bg[ch] : K(0));
    for (int k = last; k >= 0; k--) {
        int g = list[k];
        REAL dx = S->means2d[2 * g] - px, dy = S->means2d[2 * g + 1] - py;
        REAL a = S->conics[3 * g], b = S->conics[3 * g + 1], c = S->conics[3 * g + 2];
        double smag;
        REAL sigma = (REAL)sigma_of(a, b, c, dx, dy, &smag);    /* as in the forward */
        if (sigma < K(0)) continue;
        REAL o = gauss_opacity(S, g);
        REAL e = r_exp(-sigma);
        REAL araw = o * e;
        REAL alpha = r_min((REAL)P->alpha_max, araw);
        if (alpha < (REAL)P->alpha_min) continue;
        REAL one_m = K(1) - alpha;
        REAL Tk = T / one_m;                 /* transmittance in front of entry k */
        const REAL *col = S->colors + (size_t)D * g;
        REAL v_alpha = K(0);
        double m_alpha = 0.0;                /* magnitude of v_alpha's parts */
        for (int ch = 0; ch < D; ch++) {
            double t = (double)(alpha * Tk * vC[ch]);
            add_term(G, &G->v_colors[(size_t)D * g + ch], (size_t)g, 6 + ch, t, fabs(t));
            v_alpha += (col[ch] * Tk - Sacc[ch] / one_m) * vC[ch];
            m_alpha += (fabs((double)(col[ch] * Tk)) + fabs((double)(Sacc[ch] / one_m))) * fabs((double)vC[ch]);
        }
        v_alpha += vA * (T_final / one_m);
        m_alpha += fabs((double)(vA * (T_final / one_m)));
        for (int ch = 0; ch < D; ch++) Sacc[ch] += col[ch] * alpha * Tk;
        T = Tk;
        if (araw > (REAL)P->alpha_max) continue;    /* clamped: no gradient to o or sigma */
        /* d alpha / d o = exp(-sigma), o being the opacity the rasterizer
         * used (times the anti-aliasing compensation when that is on) */
        add_term(G, &G->v_opac[g], (size_t)g, 5, (double)(e * v_alpha), (double)e * m_alpha);
        REAL v_sigma = -araw * v_alpha;
        double m_sigma = (double)araw * m_alpha;
        /* d sigma / d mu' = Y Delta with Delta = mu' - p; d sigma / d(a,b,c) */
        REAL gx = v_sigma * (a * dx + b * dy), gy = v_sigma * (b * dx + c * dy);
        add_term(G, &G->v_means2d[2 * (size_t)g], (size_t)g, 0, (double)gx,
                 m_sigma * (fabs((double)(a * dx)) + fabs((double)(b * dy))));
        add_term(G, &G->v_means2d[2 * (size_t)g + 1], (size_t)g, 1, (double)gy,
                 m_sigma * (fabs((double)(b * dx)) + fabs((double)(c * dy))));
        /* absgrad (Absgrad): this pixel's contribution to the mean gradient, in absolute value */
        if (G->v_means2d_abs) {
            G->v_means2d_abs[2 * (size_t)g] += fabs((double)gx);
            G->v_means2d_abs[2 * (size_t)g + 1] += fabs((double)gy);
        }
        add_term(G, &G->v_conics[3 * (size_t)g], (size_t)g, 2, (double)(v_sigma * (K(0.5) * dx * dx)),
                 m_sigma * 0.5 * (double)(dx * dx));
        add_term(G, &G->v_conics[3 * (size_t)g + 1], (size_t)g, 3, (double)(v_sigma * (dx * dy)),
                 m_sigma * fabs((double)(dx * dy)));
        add_term(G, &G->v_conics[3 * (size_t)g + 2], (size_t)g, 4, (double)(v_sigma * (K(0.5) * dy * dy)),
                 m_sigma * 0.5 * (double)(dy * dy));
    }
}

static void camera_offsets(const orc_params *P, int C, const int *W, const int *H, int64_t *pix_off, int64_t *tile_off)
{
    int64_t po = 0, to = 0;
    for (int c = 0; c < C; c++) {
        pix_off[c] = po; tile_off[c] = to;
        po += (int64_t)W[c] * H[c];
        to += (int64_t)((W[c] + P->tile - 1) / P->tile) * ((H[c] + P->tile - 1) / P->tile);
    }
    pix_off[C] = po; tile_off[C] = to;
}

/* Threads of the loops over tiles (OpenMP; 1 by default).  Used only to time
 * the oracle on every host core and to run whole frames in the tests: the
 * tiles are independent, so the forward results do not depend on it; the
 * backward's per-thread double sums are added in thread order at the end. */
static int g_threads = 1;
void orc_set_threads(int n) { g_threads = n > 0 ? n : 1; }
int orc_get_threads(void) { return g_threads; }

/* (camera, tile x, tile y) of global tile t */
static void tile_coords(const orc_params *P, int C, const int *W, const int64_t *tile_off, int64_t t,
                        int *c, int *tx, int *ty)
{
    int cc = 0;
    while (cc + 1 < C && t >= tile_off[cc + 1]) cc++;
    int TX = (W[cc] + P->tile - 1) / P->tile;
    int64_t lt = t - tile_off[cc];
    *c = cc; *ty = (int)(lt / TX); *tx = (int)(lt % TX);
}

static void store_pixel(const pix_out_t *po, int D, int64_t p, REAL *image, REAL *alpha, REAL *final_T,
                        int32_t *n_eval, int32_t *n_comp, uint8_t *flags, uint32_t *trace, double *margin)
{
    for (int ch = 0; ch < D; ch++) image[(size_t)D * p + ch] = po->color[ch];
    alpha[p] = K(1) - po->T;
    final_T[p] = po->T;
    if (n_eval) n_eval[p] = po->n_eval;
    if (n_comp) n_comp[p] = po->n_comp;
    if (flags) flags[p] = (uint8_t)po->flags;
    if (trace) trace[p] = po->trace;
    if (margin) margin[p] = po->margin;
}

/* Render every pixel of every (selected) tile from the sorted list.
 * Images are packed per camera: pixel (c, y, x) at pix_off[c] + y W_c + x.
 * last_ids holds the global position in the sorted list (-1: none).
 * margin (nullable): per pixel the smallest |ln(value / threshold)| over its
 * skip, clamp and stop decisions. */
int orc_rasterize_fwd(const orc_params *P, int C, int N, int D, const int *W, const int *H,
                      const REAL *means2d, const REAL *conics, const REAL *colors, const REAL *opacities,
                      const REAL *comps, const REAL *background, const int32_t *ranges, const int32_t *ids,
                      const uint8_t *tile_mask, REAL *image, REAL *alpha, REAL *final_T, int32_t *last_ids,
                      int32_t *n_eval, int32_t *n_comp, uint8_t *flags, uint32_t *trace, double *margin)
{
    if (D < 1 || D > ORC_MAX_D) return -1;
    int64_t *pix_off = (int64_t *)malloc(sizeof(int64_t) * (C + 1));
    int64_t *tile_off = (int64_t *)malloc(sizeof(int64_t) * (C + 1));
    camera_offsets(P, C, W, H, pix_off, tile_off);
    scene2d_t S = {P, N, means2d, conics, colors, opacities, comps, D};
    const int ts = P->tile;
    const int64_t nt = tile_off[C];
#pragma omp parallel for schedule(dynamic, 1) num_threads(g_threads)
    for (int64_t t = 0; t < nt; t++) {
        if (tile_mask && !tile_mask[t]) continue;
        int c, tx, ty;
        tile_coords(P, C, W, tile_off, t, &c, &tx, &ty);
        const REAL *bg = background ? background + (size_t)D * c : NULL;
        int start = ranges[2 * t], end = ranges[2 * t + 1];
        for (int y = ty * ts; y < (ty + 1) * ts && y < H[c]; y++)
            for (int x = tx * ts; x < (tx + 1) * ts && x < W[c]; x++) {
                pix_out_t po;
                composite_pixel(&S, ids + start, end - start, (REAL)x + K(0.5), (REAL)y + K(0.5), bg, &po);
                int64_t p = pix_off[c] + (int64_t)y * W[c] + x;
                store_pixel(&po, D, p, image, alpha, final_T, n_eval, n_comp, flags, trace, margin);
                last_ids[p] = po.last >= 0 ? start + po.last : -1;
            }
    }
    free(pix_off); free(tile_off);
    return 0;
}

/* One gradient accumulator per thread, added into the first in thread order. */
static grad2d_t *grads_per_thread(size_t CN, int D, int want_abs, int want_absgrad, int n)
{
    grad2d_t *G = (grad2d_t *)malloc(sizeof(grad2d_t) * (size_t)n);
    for (int i = 0; i < n; i++) grad2d_alloc(&G[i], CN, D, want_abs, want_absgrad);
    return G;
}

static void grads_merge(grad2d_t *G, int n, size_t CN)
{
    for (int i = 1; i < n; i++) {
        const int D = G[0].D;
        for (size_t j = 0; j < 2 * CN; j++) G[0].v_means2d[j] += G[i].v_means2d[j];
        for (size_t j = 0; j < 3 * CN; j++) G[0].v_conics[j] += G[i].v_conics[j];
        for (size_t j = 0; j < (size_t)D * CN; j++) G[0].v_colors[j] += G[i].v_colors[j];
        for (size_t j = 0; j < CN; j++) G[0].v_opac[j] += G[i].v_opac[j];
        if (G[0].abs)
            for (size_t j = 0; j < (size_t)G[0].nslot * CN; j++) G[0].abs[j] += G[i].abs[j];
        if (G[0].v_means2d_abs)
            for (size_t j = 0; j < 2 * CN; j++) G[0].v_means2d_abs[j] += G[i].v_means2d_abs[j];
        free(G[i].v_means2d); free(G[i].v_conics); free(G[i].v_colors); free(G[i].v_opac); free(G[i].abs);
        free(G[i].v_means2d_abs);
    }
}

int orc_rasterize_bwd(const orc_params *P, int C, int N, int D, const int *W, const int *H,
                      const REAL *means2d, const REAL *conics, const REAL *colors, const REAL *opacities,
                      const REAL *comps, const REAL *background, const int32_t *ranges, const int32_t *ids,
                      const uint8_t *tile_mask, const REAL *final_T, const int32_t *last_ids,
                      const REAL *v_image, const REAL *v_alpha,
                      REAL *v_means2d, REAL *v_conics, REAL *v_colors, REAL *v_opacities, REAL *abs_sums,
                      REAL *v_means2d_abs)
{
    if (D < 1 || D > ORC_MAX_D) return -1;
    int64_t *pix_off = (int64_t *)malloc(sizeof(int64_t) * (C + 1));
    int64_t *tile_off = (int64_t *)malloc(sizeof(int64_t) * (C + 1));
    camera_offsets(P, C, W, H, pix_off, tile_off);
    size_t CN = (size_t)C * N;
    const int nth = g_threads;
    grad2d_t *G = grads_per_thread(CN, D, abs_sums != NULL, v_means2d_abs != NULL, nth);
    scene2d_t S = {P, N, means2d, conics, colors, opacities, comps, D};
    const int ts = P->tile;
    const int64_t nt = tile_off[C];
#pragma omp parallel num_threads(nth)
    {
#ifdef _OPENMP
        grad2d_t *Gt = &G[omp_get_thread_num()];
#else
        grad2d_t *Gt = &G[0];
#endif
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < nt; t++) {
            if (tile_mask && !tile_mask[t]) continue;
            int c, tx, ty;
            tile_coords(P, C, W, tile_off, t, &c, &tx, &ty);
            const REAL *bg = background ? background + (size_t)D * c : NULL;
            int start = ranges[2 * t];
            for (int y = ty * ts; y < (ty + 1) * ts && y < H[c]; y++)
                for (int x = tx * ts; x < (tx + 1) * ts && x < W[c]; x++) {
                    int64_t p = pix_off[c] + (int64_t)y * W[c] + x;
                    if (last_ids[p] < 0) continue;
                    composite_pixel_bwd(&S, ids + start, last_ids[p] - start, (REAL)x + K(0.5), (REAL)y + K(0.5),
                                        bg, final_T[p], v_image + (size_t)D * p, v_alpha ? v_alpha[p] : K(0), Gt);
                }
        }
    }
    grads_merge(G, nth, CN);
    grad2d_store(&G[0], CN, v_means2d, v_conics, v_colors, v_opacities, abs_sums, v_means2d_abs);
    free(G); free(pix_off); free(tile_off);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The plain definition, tile by tile: the list of a tile is every projected */
/* Gaussian whose rectangle contains the tile (untiled mode: every projected */
/* Gaussian), ordered by (depth bits, id).  No keys, no radix sort.          */
/* ------------------------------------------------------------------------ */
typedef struct { uint32_t dbits; int32_t id; } did_t;
static int did_cmp(const void *pa, const void *pb)
{
    const did_t *a = (const did_t *)pa, *b = (const did_t *)pb;
    if (a->dbits != b->dbits) return a->dbits < b->dbits ? -1 : 1;
    return (a->id > b->id) - (a->id < b->id);
}

static int build_tile_list(const orc_params *P, int N, int c, int W, int H, int tx, int ty,
                           const REAL *means2d, const int32_t *radii, const REAL *depths, int untiled, int32_t *list, did_t *tmp)
{
    int len = 0;
    for (int n = 0; n < N; n++) {
        size_t g = (size_t)c * N + n;
        if (radii[g] <= 0) continue;
        if (!untiled) {
            int x0, x1, y0, y1;
            tile_rect(P, W, H, means2d[2 * g], means2d[2 * g + 1], radii[g], &x0, &x1, &y0, &y1);
            if (tx < x0 || tx >= x1 || ty < y0 || ty >= y1) continue;
        }
        tmp[len].dbits = float_bits((float)depths[g]);
        tmp[len].id = (int32_t)g;
        len++;
    }
    qsort(tmp, (size_t)len, sizeof(did_t), did_cmp);
    for (int i = 0; i < len; i++) list[i] = tmp[i].id;
    return len;
}

/* The definition's list of one tile: ids c*N+n of the projected Gaussians
 * whose rectangle holds tile (tx, ty) of camera c, in (depth bits, id) order.
 * Returns its length; list must hold N entries. */
int orc_tile_list(const orc_params *P, int C, int N, const int *W, const int *H, const REAL *means2d,
                  const int32_t *radii, const REAL *depths, int c, int tx, int ty, int32_t *list)
{
    (void)C;
    did_t *tmp = (did_t *)malloc(sizeof(did_t) * (N > 0 ? N : 1));
    int len = build_tile_list(P, N, c, W[c], H[c], tx, ty, means2d, radii, depths, 0, list, tmp);
    free(tmp);
    return len;
}

/* tiles[3*i] = camera, tiles[3*i+1] = tile x, tiles[3*i+2] = tile y.
 * Outputs are written into full packed images (only listed tiles touched).
 * last_gid: [C,N] id of the last composited Gaussian (-1); last_pos: its
 * position in the tile's list (-1). */
int orc_render_tiles_fwd(const orc_params *P, int C, int N, int D, const int *W, const int *H,
                         const REAL *means2d, const REAL *conics, const REAL *colors, const REAL *opacities,
                         const REAL *comps, const int32_t *radii, const REAL *depths, const REAL *background,
                         int ntiles, const int32_t *tiles, int untiled,
                         REAL *image, REAL *alpha, REAL *final_T, int32_t *last_gid, int32_t *last_pos,
                         int32_t *n_eval, int32_t *n_comp, uint8_t *flags, uint32_t *trace, int32_t *list_len,
                         double *margin)
{
    if (D < 1 || D > ORC_MAX_D) return -1;
    int64_t *pix_off = (int64_t *)malloc(sizeof(int64_t) * (C + 1));
    int64_t *tile_off = (int64_t *)malloc(sizeof(int64_t) * (C + 1));
    camera_offsets(P, C, W, H, pix_off, tile_off);
    scene2d_t S = {P, N, means2d, conics, colors, opacities, comps, D};
    const int ts = P->tile;
#pragma omp parallel num_threads(g_threads)
    {
        int32_t *list = (int32_t *)malloc(sizeof(int32_t) * (N > 0 ? N : 1));
        did_t *tmp = (did_t *)malloc(sizeof(did_t) * (N > 0 ? N : 1));
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < ntiles; i++) {
            int c = tiles[3 * i], tx = tiles[3 * i + 1], ty = tiles[3 * i + 2];
            const REAL *bg = background ? background + (size_t)D * c : NULL;
            int len = build_tile_list(P, N, c, W[c], H[c], tx, ty, means2d, radii, depths, untiled, list, tmp);
            if (list_len) list_len[i] = len;
            for (int y = ty * ts; y < (ty + 1) * ts && y < H[c]; y++)
                for (int x = tx * ts; x < (tx + 1) * ts && x < W[c]; x++) {
                    pix_out_t po;
                    composite_pixel(&S, list, len, (REAL)x + K(0.5), (REAL)y + K(0.5), bg, &po);
                    int64_t p = pix_off[c] + (int64_t)y * W[c] + x;
                    store_pixel(&po, D, p, image, alpha, final_T, n_eval, n_comp, flags, trace, margin);
                    if (last_gid) last_gid[p] = po.last >= 0 ? list[po.last] : -1;
                    if (last_pos) last_pos[p] = po.last;
                }
        }
        free(list); free(tmp);
    }
    free(pix_off); free(tile_off);
    return 0;
}

/* Gradients of sum(v_image * image) + sum(v_alpha * alpha) over the listed
 * tiles only, by the definition lists.  Outputs are [C,N]-indexed sums. */
int orc_render_tiles_bwd(const orc_params *P, int C, int N, int D, const int *W, const int *H,
                         const REAL *means2d, const REAL *conics, const REAL *colors, const REAL *opacities,
                         const REAL *comps, const int32_t *radii, const REAL *depths, const REAL *background,
                         int ntiles, const int32_t *tiles, const REAL *v_image, const REAL *v_alpha,
                         REAL *v_means2d, REAL *v_conics, REAL *v_colors, REAL *v_opacities, REAL *abs_sums,
                         REAL *v_means2d_abs)
{
    if (D < 1 || D > ORC_MAX_D) return -1;
    int64_t *pix_off = (int64_t *)malloc(sizeof(int64_t) * (C + 1));
    int64_t *tile_off = (int64_t *)malloc(sizeof(int64_t) * (C + 1));
    camera_offsets(P, C, W, H, pix_off, tile_off);
    size_t CN = (size_t)C * N;
    const int nth = g_threads;
    grad2d_t *G = grads_per_thread(CN, D, abs_sums != NULL, v_means2d_abs != NULL, nth);
    scene2d_t S = {P, N, means2d, conics, colors, opacities, comps, D};
    const int ts = P->tile;
#pragma omp parallel num_threads(nth)
    {
#ifdef _OPENMP
        grad2d_t *Gt = &G[omp_get_thread_num()];
#else
        grad2d_t *Gt = &G[0];
#endif
        int32_t *list = (int32_t *)malloc(sizeof(int32_t) * (N > 0 ? N : 1));
        did_t *tmp = (did_t *)malloc(sizeof(did_t) * (N > 0 ? N : 1));
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < ntiles; i++) {
            int c = tiles[3 * i], tx = tiles[3 * i + 1], ty = tiles[3 * i + 2];
            const REAL *bg = background ? background + (size_t)D * c : NULL;
            int len = build_tile_list(P, N, c, W[c], H[c], tx, ty, means2d, radii, depths, 0, list, tmp);
            for (int y = ty * ts; y < (ty + 1) * ts && y < H[c]; y++)
                for (int x = tx * ts; x < (tx + 1) * ts && x < W[c]; x++) {
                    pix_out_t po;
                    REAL px = (REAL)x + K(0.5), py = (REAL)y + K(0.5);
                    composite_pixel(&S, list, len, px, py, bg, &po);
                    if (po.last < 0) continue;
                    int64_t p = pix_off[c] + (int64_t)y * W[c] + x;
                    composite_pixel_bwd(&S, list, po.last, px, py, bg, po.T, v_image + (size_t)D * p,
                                        v_alpha ? v_alpha[p] : K(0), Gt);
                }
        }
        free(list); free(tmp);
    }
    grads_merge(G, nth, CN);
    grad2d_store(&G[0], CN, v_means2d, v_conics, v_colors, v_opacities, abs_sums, v_means2d_abs);
    free(G); free(pix_off); free(tile_off);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Projection Gradients + Scale and rotation gradients + SH backward.       */
/* ------------------------------------------------------------------------ */
static void matmul(int n, int k, int m, const REAL *A, const REAL *B, REAL *Cm)
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < m; j++) {
            REAL acc = K(0);
            for (int l = 0; l < k; l++) acc += A[i * k + l] * B[l * m + j];
            Cm[i * m + j] = acc;
        }
}

/* Inputs: the forward inputs, the per-(camera, Gaussian) gradients of the
 * projected quantities, and v_opacities_cn [C,N] from the rasterizer.
 * Outputs (summed over cameras): v_means [N,3], v_quats [N,4],
 * v_scales [N,3], v_opacities [N], v_sh_or_colors [N,K,3] or [N,3]. */
int orc_project_bwd(const orc_params *P, int C, int N, const int *W, const int *H,
                    const REAL *means, const REAL *quats, const REAL *scales, const REAL *opacities,
                    const REAL *sh_or_colors, const REAL *viewmats, const REAL *Ks,
                    const REAL *v_means2d, const REAL *v_conics, const REAL *v_colors,
                    const REAL *v_opacities_cn, const REAL *v_depths,
                    REAL *v_means, REAL *v_quats, REAL *v_scales, REAL *v_opacities, REAL *v_sh_or_colors,
                    REAL *v_viewmats)
{
    int nk = num_sh(P);
    int stride = nk > 0 ? 3 * nk : 3;
    /* pose gradient: per camera, d L / d (R | t) of the world-to-camera matrix, summed over Gaussians */
    double *vV = v_viewmats ? (double *)calloc((size_t)12 * (C > 0 ? C : 1), sizeof(double)) : NULL;
    for (int n = 0; n < N; n++) {
        double am[3] = {0, 0, 0}, aq[4] = {0, 0, 0, 0}, as[3] = {0, 0, 0}, ao = 0;
        double ash[48];
        memset(ash, 0, sizeof(ash));
        const REAL *mu = means + 3 * (size_t)n, *q = quats + 4 * (size_t)n, *s = scales + 3 * (size_t)n;
        const REAL *sh = sh_or_colors + (size_t)stride * n;
        for (int c = 0; c < C; c++) {
            size_t g = (size_t)c * N + n;
            const REAL *V = viewmats + 16 * c, *Kc = Ks + 9 * c;
            proj_t o;
            project_one(P, W[c], H[c], mu, q, s, sh, nk, V, Kc, &o);
            if (!o.valid) continue;
            REAL fx = Kc[0], fy = Kc[4];
            REAL tx = o.t[0], ty = o.t[1], tz = o.t[2];
            REAL vt[3] = {K(0), K(0), K(0)};

            /* opacity: rasterizer gradient w.r.t. the (compensated) opacity */
            REAL vo_cn = v_opacities_cn[g];
            ao += (double)(vo_cn * o.comp);
            REAL v_comp = vo_cn * opacities[n];

            /* 2D mean: mu' = (fx tx / tz + cx, fy ty / tz + cy) */
            REAL vmx = v_means2d[2 * g], vmy = v_means2d[2 * g + 1];
            vt[0] += vmx * fx / tz;
            vt[1] += vmy * fy / tz;
            vt[2] += -(vmx * fx * tx + vmy * fy * ty) / (tz * tz);
            if (v_depths) vt[2] += v_depths[g];

            /* conic (a, b, c) of Y = Sigma'^-1: G = [[ga, gb/2], [gb/2, gc]],
             * dL/dSigma' = -Y G Y (symmetric). */
            REAL Y[4] = {o.conic[0], o.conic[1], o.conic[1], o.conic[2]};
            REAL Gm[4] = {v_conics[3 * g], K(0.5) * v_conics[3 * g + 1], K(0.5) * v_conics[3 * g + 1], v_conics[3 * g + 2]};
            REAL YG[4], vS2[4];
            matmul(2, 2, 2, Y, Gm, YG);
            matmul(2, 2, 2, YG, Y, vS2);
            for (int i = 0; i < 4; i++) vS2[i] = -vS2[i];
            if (P->antialiased && v_comp != K(0)) {
                /* comp = sqrt(det0 / det): d comp = comp/2 (d det0/det0 - d det/det),
                 * d det0/d Sigma' = adj(Sigma' undilated), d det/d Sigma' = adj(Sigma' dilated) */
                if (o.comp > K(0) && o.det0 > K(0)) {
                    REAL k0 = K(0.5) * o.comp * v_comp;
                    REAL adj0[4] = {o.cov2d[2], -o.cov2d[1], -o.cov2d[1], o.cov2d[0]};
                    REAL adj1[4] = {o.c, -o.b, -o.b, o.a};
                    for (int i = 0; i < 4; i++) vS2[i] += k0 * (adj0[i] / o.det0 - adj1[i] / o.det);
                }
            }
            /* Sigma' = T Sigma T^T:  dL/dSigma = T^T G T,  dL/dT = 2 G T Sigma */
            REAL Tm[6], TtG[6], vSig[9], GT[6], vT[6];
            for (int i = 0; i < 2; i++) for (int j = 0; j < 3; j++) Tm[3 * i + j] = o.T[i][j];
            REAL Tt[6];
            for (int i = 0; i < 3; i++) for (int j = 0; j < 2; j++) Tt[2 * i + j] = Tm[3 * j + i];
            matmul(3, 2, 2, Tt, vS2, TtG);
            matmul(3, 2, 3, TtG, Tm, vSig);
            REAL Sg[9];
            for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) Sg[3 * i + j] = o.Sig[i][j];
            matmul(2, 2, 3, vS2, Tm, GT);
            matmul(2, 3, 3, GT, Sg, vT);
            for (int i = 0; i < 6; i++) vT[i] = K(2) * vT[i];
            /* T = J R_cw: dL/dJ = dL/dT R_cw^T */
            REAL Rcw[9], RcwT[9], vJ[6];
            for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) { Rcw[3 * i + j] = V[4 * i + j]; RcwT[3 * j + i] = V[4 * i + j]; }
            matmul(2, 3, 3, vT, RcwT, vJ);
            /* J = [[fx/tz, 0, -fx txc/tz^2], [0, fy/tz, -fy tyc/tz^2]] */
            REAL txc = o.clx ? (REAL)o.clx * o.limx * tz : tx;
            REAL tyc = o.cly ? (REAL)o.cly * o.limy * tz : ty;
            REAL tz2 = tz * tz, tz3 = tz2 * tz;
            REAL vtxc = vJ[2] * (-fx / tz2);
            REAL vtyc = vJ[5] * (-fy / tz2);
            vt[2] += vJ[0] * (-fx / tz2) + vJ[2] * (K(2) * fx * txc / tz3)
                   + vJ[4] * (-fy / tz2) + vJ[5] * (K(2) * fy * tyc / tz3);
            if (o.clx) vt[2] += vtxc * ((REAL)o.clx * o.limx); else vt[0] += vtxc;
            if (o.cly) vt[2] += vtyc * ((REAL)o.cly * o.limy); else vt[1] += vtyc;

            /* t = R_cw mu + t_cw: dL/dmu = R_cw^T dL/dt */
            REAL vmu[3];
            matmul(3, 3, 1, RcwT, vt, vmu);
            (void)Rcw;
            REAL gdir[3] = {K(0), K(0), K(0)};   /* dL/dmu through the SH view direction */

            /* Sigma = M M^T: dL/dM = 2 dL/dSigma M;  M = R S:
             * dL/dR = dL/dM S^T,  dL/ds_j = (R^T dL/dM)_jj */
            REAL Mm[9], vM[9];
            for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) Mm[3 * i + j] = o.M[i][j];
            matmul(3, 3, 3, vSig, Mm, vM);
            for (int i = 0; i < 9; i++) vM[i] = K(2) * vM[i];
            REAL vR[9];
            for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) vR[3 * i + j] = vM[3 * i + j] * s[j];
            for (int j = 0; j < 3; j++) {
                REAL acc = K(0);
                for (int i = 0; i < 3; i++) acc += o.R[i][j] * vM[3 * i + j];
                as[j] += (double)acc;
            }
            /* dR/d(w,x,y,z) at the normalised quaternion (Scale and rotation gradients) */
            REAL w = o.qn[0], x = o.qn[1], y = o.qn[2], z = o.qn[3];
            REAL dRw[9] = {0, -z, y, z, 0, -x, -y, x, 0};
            REAL dRx[9] = {0, y, z, y, -2 * x, -w, z, w, -2 * x};
            REAL dRy[9] = {-2 * y, x, w, x, 0, z, -w, z, -2 * y};
            REAL dRz[9] = {-2 * z, -w, x, w, -2 * z, y, x, y, 0};
            REAL vqn[4] = {K(0), K(0), K(0), K(0)};
            for (int i = 0; i < 9; i++) {
                vqn[0] += K(2) * dRw[i] * vR[i];
                vqn[1] += K(2) * dRx[i] * vR[i];
                vqn[2] += K(2) * dRy[i] * vR[i];
                vqn[3] += K(2) * dRz[i] * vR[i];
            }
            /* q_hat = q / |q|:  dL/dq = (dL/dq_hat - q_hat (q_hat . dL/dq_hat)) / |q| */
            REAL dotq = ((o.qn[0] * vqn[0] + o.qn[1] * vqn[1]) + o.qn[2] * vqn[2]) + o.qn[3] * vqn[3];
            for (int i = 0; i < 4; i++) aq[i] += (double)((vqn[i] - o.qn[i] * dotq) / o.qnorm);

            /* colour */
            const REAL *vc = v_colors + 3 * g;
            if (nk > 0) {
                REAL Yb[16], dY[16][3];
                sh_eval(nk, o.dir, Yb, dY);
                REAL vraw[3];
                for (int ch = 0; ch < 3; ch++) vraw[ch] = (o.raw[ch] < K(0)) ? K(0) : vc[ch];
                REAL vdir[3] = {K(0), K(0), K(0)};
                for (int k = 0; k < nk; k++)
                    for (int ch = 0; ch < 3; ch++) {
                        ash[3 * k + ch] += (double)(Yb[k] * vraw[ch]);
                        for (int j = 0; j < 3; j++) vdir[j] += dY[k][j] * sh[3 * k + ch] * vraw[ch];
                    }
                /* dir = d / |d|, d = mu - campos */
                REAL dd = (o.dir[0] * vdir[0] + o.dir[1] * vdir[1]) + o.dir[2] * vdir[2];
                for (int j = 0; j < 3; j++) {
                    gdir[j] = (vdir[j] - o.dir[j] * dd) / o.dnorm;
                    vmu[j] += gdir[j];
                }
            } else {
                for (int ch = 0; ch < 3; ch++) ash[ch] += (double)vc[ch];
            }
            for (int j = 0; j < 3; j++) am[j] += (double)vmu[j];
            if (vV) {
                /* t_cam = R mu + t:   dL/dR += vt mu^T,  dL/dt += vt;
                 * T = J R:            dL/dR += J^T dL/dT;
                 * centre = -R^T t (SH direction; dL/dcentre = -gdir):
                 *                     dL/dR += t gdir^T,  dL/dt += R gdir. */
                const REAL *mu = means + 3 * (size_t)n;
                double *d = vV + 12 * (size_t)c;
                for (int i = 0; i < 3; i++) {
                    for (int j = 0; j < 3; j++) {
                        double jt = 0.0;
                        if (i == 0) jt = (double)o.J00 * vT[j];
                        else if (i == 1) jt = (double)o.J11 * vT[3 + j];
                        else jt = (double)o.J02 * vT[j] + (double)o.J12 * vT[3 + j];
                        d[4 * i + j] += (double)vt[i] * mu[j] + jt + (double)V[4 * i + 3] * gdir[j];
                    }
                    d[4 * i + 3] += (double)vt[i] + ((double)V[4 * i] * gdir[0] + (double)V[4 * i + 1] * gdir[1]
                                                     + (double)V[4 * i + 2] * gdir[2]);
                }
            }
        }
        for (int j = 0; j < 3; j++) { v_means[3 * (size_t)n + j] = (REAL)am[j]; v_scales[3 * (size_t)n + j] = (REAL)as[j]; }
        for (int j = 0; j < 4; j++) v_quats[4 * (size_t)n + j] = (REAL)aq[j];
        v_opacities[n] = (REAL)ao;
        for (int j = 0; j < stride; j++) v_sh_or_colors[(size_t)stride * n + j] = (REAL)ash[j];
    }
    if (vV) {
        for (int c = 0; c < C; c++)
            for (int e = 0; e < 16; e++) v_viewmats[16 * c + e] = e < 12 ? (REAL)vV[12 * c + e] : K(0);
        free(vV);
    }
    return 0;
}

int orc_real_size(void) { return (int)sizeof(REAL); }
