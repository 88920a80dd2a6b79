/*
 * FP64 CPU oracle for the photorealistic-mapping optimisation of Photo-SLAM
 * (Huang et al., CVPR 2024, arXiv 2311.16728).
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU
 * baseline leg of the benchmark are the only callers.  This file shares no
 * code, header, constant or table with the GPU library; the two meet only at
 * the seeded inputs.
 *
 * It is deliberately plain: every pixel gathers the Gaussians whose opacity
 * reaches the cutoff at that pixel, sorts them by depth, composites them, and
 * (for the gradient) walks the same stored list backwards.  No tiles, no
 * recompute, no fused steps.  The only speed-up is a candidate pre-filter with
 * a provably conservative bounding box of the cutoff ellipse; a brute-force
 * switch turns it off and the tests check both give identical bits.
 *
 * What each part follows:
 *   - primitive parameters (position, rotation, scaling, density, SH):
 *     Section 3.1 (Hyper Primitives Map);
 *   - rendering C(R,t) = sum_i c_i a_i prod_{j<i} (1 - a_j), with
 *     a_i = sigma_i * G(R, t, P_i, r_i, s_i) and G the 3D Gaussian splat:
 *     Section 3.3, Eq. 3 (the product index printed there is read as j);
 *   - photometric loss (1 - lambda) |I_r - I_gt|_1 + lambda (1 - SSIM):
 *     Section 3.3, Eq. 4, with lambda = 0.2 from Section 4.1;
 *   - Gaussian pyramid by repeated smoothing and downsampling and level-wise
 *     supervision: Section 3.4, Eq. 5;
 *   - gradient-based optimisation with a fixed learning rate: Section 4.1
 *     (Adam update with torch's bias-corrected formula).
 * Details the paper leaves to the splatting method it builds on (projection
 * Jacobian, dilation, cutoffs, SH basis, window sizes) follow the readings
 * listed in the design notes; each is named where it is used.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NROWS 59
#define ROW_MU 0
#define ROW_LOGS 3
#define ROW_QUAT 6
#define ROW_OPAC 10
#define ROW_SH 11

/* Per-Gaussian record exported by orc_preprocess (doubles). */
enum {
    R_VALID = 0, R_MX, R_MY, R_Z, R_CA, R_CB, R_CC, R_OPA, R_RGB0, R_RGB1, R_RGB2,
    R_CLAMP0, R_CLAMP1, R_CLAMP2, R_S00, R_S01, R_S11, R_EXTX, R_EXTY, R_COND, REC
};

typedef struct {
    double R[9], t[3], fx, fy, cx, cy;
    int W, H;
    double bg[3];
    double limx, limy;   /* FOV clamp of the Jacobian, |x/z| <= limx, |y/z| <= limy */
} cam_t;

typedef struct {
    double alpha_min, alpha_max, t_min, znear, dilation, fov_clamp;
    int sh_degree;
} set_t;

static cam_t read_cam(const double *c) {
    cam_t k;
    memcpy(k.R, c, 9 * sizeof(double));
    memcpy(k.t, c + 9, 3 * sizeof(double));
    k.fx = c[12]; k.fy = c[13]; k.cx = c[14]; k.cy = c[15];
    k.W = (int)c[16]; k.H = (int)c[17];
    k.bg[0] = c[18]; k.bg[1] = c[19]; k.bg[2] = c[20];
    /* c[21], c[22]: half field of view tan used by the clamp (a pyramid level
     * keeps its keyframe's full-resolution field of view); 0 = from W, H */
    k.limx = c[21] > 0 ? c[21] : 0.5 * k.W / k.fx;
    k.limy = c[22] > 0 ? c[22] : 0.5 * k.H / k.fy;
    return k;
}

static set_t read_set(const double *s) {
    set_t k;
    k.alpha_min = s[0]; k.alpha_max = s[1]; k.t_min = s[2]; k.znear = s[3];
    k.dilation = s[4]; k.fov_clamp = s[5]; k.sh_degree = (int)s[6];
    return k;
}

/* ---------------------------------------------------------------------------
 * Real spherical harmonics up to degree 3 (the primitive's colour is "converted
 * from SH", Section 3.1 and Eq. 3).  Index k = l*l + l + m.  Constants are the
 * textbook normalisations of the real orthonormal basis; Y[] are the values at
 * the unit direction d, dY[k][i] the partial derivative of the polynomial with
 * respect to d_i (the caller projects onto the sphere's tangent plane).
 * ------------------------------------------------------------------------- */
static void sh_basis(int deg, const double d[3], double Y[16], double dY[16][3]) {
    const double PI = 3.14159265358979323846;
    const double x = d[0], y = d[1], z = d[2];
    const double k0 = 0.5 * sqrt(1.0 / PI);
    const double k1 = sqrt(3.0 / (4.0 * PI));
    const double k2a = 0.5 * sqrt(15.0 / PI);   /* xy, yz, xz terms */
    const double k2b = 0.25 * sqrt(5.0 / PI);   /* 2z^2 - x^2 - y^2 */
    const double k2c = 0.25 * sqrt(15.0 / PI);  /* x^2 - y^2 */
    const double k3a = 0.25 * sqrt(35.0 / (2.0 * PI));
    const double k3b = 0.5 * sqrt(105.0 / PI);
    const double k3c = 0.25 * sqrt(21.0 / (2.0 * PI));
    const double k3d = 0.25 * sqrt(7.0 / PI);
    const double k3e = 0.25 * sqrt(105.0 / PI);
    memset(Y, 0, 16 * sizeof(double));
    memset(dY, 0, 16 * 3 * sizeof(double));
    Y[0] = k0;
    if (deg < 1) return;
    Y[1] = -k1 * y; dY[1][1] = -k1;
    Y[2] = k1 * z;  dY[2][2] = k1;
    Y[3] = -k1 * x; dY[3][0] = -k1;
    if (deg < 2) return;
    Y[4] = k2a * x * y;  dY[4][0] = k2a * y; dY[4][1] = k2a * x;
    Y[5] = -k2a * y * z; dY[5][1] = -k2a * z; dY[5][2] = -k2a * y;
    Y[6] = k2b * (2 * z * z - x * x - y * y);
    dY[6][0] = -2 * k2b * x; dY[6][1] = -2 * k2b * y; dY[6][2] = 4 * k2b * z;
    Y[7] = -k2a * x * z; dY[7][0] = -k2a * z; dY[7][2] = -k2a * x;
    Y[8] = k2c * (x * x - y * y); dY[8][0] = 2 * k2c * x; dY[8][1] = -2 * k2c * y;
    if (deg < 3) return;
    Y[9] = -k3a * y * (3 * x * x - y * y);
    dY[9][0] = -6 * k3a * x * y; dY[9][1] = -k3a * (3 * x * x - 3 * y * y);
    Y[10] = k3b * x * y * z;
    dY[10][0] = k3b * y * z; dY[10][1] = k3b * x * z; dY[10][2] = k3b * x * y;
    Y[11] = -k3c * y * (4 * z * z - x * x - y * y);
    dY[11][0] = 2 * k3c * x * y; dY[11][1] = -k3c * (4 * z * z - x * x - 3 * y * y);
    dY[11][2] = -8 * k3c * y * z;
    Y[12] = k3d * z * (2 * z * z - 3 * x * x - 3 * y * y);
    dY[12][0] = -6 * k3d * x * z; dY[12][1] = -6 * k3d * y * z;
    dY[12][2] = k3d * (6 * z * z - 3 * x * x - 3 * y * y);
    Y[13] = -k3c * x * (4 * z * z - x * x - y * y);
    dY[13][0] = -k3c * (4 * z * z - 3 * x * x - y * y); dY[13][1] = 2 * k3c * x * y;
    dY[13][2] = -8 * k3c * x * z;
    Y[14] = k3e * z * (x * x - y * y);
    dY[14][0] = 2 * k3e * x * z; dY[14][1] = -2 * k3e * y * z; dY[14][2] = k3e * (x * x - y * y);
    Y[15] = -k3a * x * (x * x - 3 * y * y);
    dY[15][0] = -k3a * (3 * x * x - 3 * y * y); dY[15][1] = 6 * k3a * x * y;
}

void orc_sh_basis(int deg, const double *d, double *Y, double *dY) {
    double dd[16][3];
    sh_basis(deg, d, Y, dd);
    if (dY) memcpy(dY, dd, sizeof dd);
}

/* Rotation matrix of the unit quaternion (w, x, y, z), row-major. */
static void quat_to_rot(const double q[4], double R[9]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* Everything the forward computes for one Gaussian and one camera. */
typedef struct {
    int valid;
    double mu[3], s[3], qn[4], qlen, o, sh[16][3];
    double Rq[9], M[9], Sig[9];   /* rotation, R*S, 3D covariance */
    double xc[3];                 /* camera-frame mean */
    double u, v, ubar, vbar;      /* normalised image coords, clamped copies */
    int clampx, clampy;           /* 1 when the FOV clamp is active */
    double J[6];                  /* 2x3 projection Jacobian */
    double V[9];                  /* W Sigma W^T */
    double S2[3];                 /* 2D covariance incl. dilation: s00, s01, s11 */
    double det, conic[3];         /* a, b, c */
    double m[2];                  /* 2D mean (pixels) */
    double dir[3], dist;          /* unit view direction and distance */
    double Y[16], dY[16][3];
    double raw[3], rgb[3];
    int clampc[3];
    double extx, exty, cond;
    double em[2], errS[3];         /* FP32 rounding bounds, see power_err32 */
} gauss_t;

static void gauss_forward(const double *P, int64_t ncap, int64_t g, const cam_t *cam,
                          const set_t *st, gauss_t *G) {
    memset(G, 0, sizeof *G);
    for (int i = 0; i < 3; ++i) G->mu[i] = P[(ROW_MU + i) * ncap + g];
    for (int i = 0; i < 3; ++i) G->s[i] = exp(P[(ROW_LOGS + i) * ncap + g]);
    double q[4], qq = 0;
    for (int i = 0; i < 4; ++i) { q[i] = P[(ROW_QUAT + i) * ncap + g]; qq += q[i] * q[i]; }
    G->qlen = sqrt(qq);
    for (int i = 0; i < 4; ++i) G->qn[i] = q[i] / G->qlen;
    G->o = 1.0 / (1.0 + exp(-P[ROW_OPAC * ncap + g]));
    for (int k = 0; k < 16; ++k)
        for (int c = 0; c < 3; ++c) G->sh[k][c] = P[(ROW_SH + 3 * k + c) * ncap + g];

    /* camera frame */
    for (int i = 0; i < 3; ++i)
        G->xc[i] = cam->R[3 * i] * G->mu[0] + cam->R[3 * i + 1] * G->mu[1] +
                   cam->R[3 * i + 2] * G->mu[2] + cam->t[i];
    const double z = G->xc[2];
    if (!(z > st->znear)) return;

    /* Sigma = (Rq S)(Rq S)^T */
    quat_to_rot(G->qn, G->Rq);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) G->M[3 * i + j] = G->Rq[3 * i + j] * G->s[j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += G->M[3 * i + k] * G->M[3 * j + k];
            G->Sig[3 * i + j] = acc;
        }

    /* first-order (EWA) projection with the field-of-view clamp of the Jacobian */
    G->u = G->xc[0] / z;
    G->v = G->xc[1] / z;
    const double limx = st->fov_clamp * cam->limx;
    const double limy = st->fov_clamp * cam->limy;
    G->ubar = G->u; G->vbar = G->v;
    if (G->u < -limx) { G->ubar = -limx; G->clampx = 1; }
    if (G->u > limx) { G->ubar = limx; G->clampx = 1; }
    if (G->v < -limy) { G->vbar = -limy; G->clampy = 1; }
    if (G->v > limy) { G->vbar = limy; G->clampy = 1; }
    G->J[0] = cam->fx / z; G->J[1] = 0; G->J[2] = -cam->fx * G->ubar / z;
    G->J[3] = 0; G->J[4] = cam->fy / z; G->J[5] = -cam->fy * G->vbar / z;

    /* V = W Sigma W^T, Sigma2D = J V J^T + dilation I */
    double WS[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += cam->R[3 * i + k] * G->Sig[3 * k + j];
            WS[3 * i + j] = acc;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += WS[3 * i + k] * cam->R[3 * j + k];
            G->V[3 * i + j] = acc;
        }
    double JV[6];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += G->J[3 * i + k] * G->V[3 * k + j];
            JV[3 * i + j] = acc;
        }
    double C2[4];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += JV[3 * i + k] * G->J[3 * j + k];
            C2[2 * i + j] = acc;
        }
    G->S2[0] = C2[0] + st->dilation;
    G->S2[1] = 0.5 * (C2[1] + C2[2]);
    G->S2[2] = C2[3] + st->dilation;
    G->det = G->S2[0] * G->S2[2] - G->S2[1] * G->S2[1];
    if (!(G->det > 0)) return;
    G->conic[0] = G->S2[2] / G->det;
    G->conic[1] = -G->S2[1] / G->det;
    G->conic[2] = G->S2[0] / G->det;
    G->m[0] = cam->fx * G->u + cam->cx;
    G->m[1] = cam->fy * G->v + cam->cy;

    /* view-dependent colour from the camera centre C = -R^T t */
    double Cw[3];
    for (int i = 0; i < 3; ++i)
        Cw[i] = -(cam->R[i] * cam->t[0] + cam->R[3 + i] * cam->t[1] + cam->R[6 + i] * cam->t[2]);
    double dv[3], dn = 0;
    for (int i = 0; i < 3; ++i) { dv[i] = G->mu[i] - Cw[i]; dn += dv[i] * dv[i]; }
    G->dist = sqrt(dn);
    for (int i = 0; i < 3; ++i) G->dir[i] = dv[i] / G->dist;
    sh_basis(st->sh_degree, G->dir, G->Y, G->dY);
    const int nk = (st->sh_degree + 1) * (st->sh_degree + 1);
    for (int c = 0; c < 3; ++c) {
        double acc = 0.5;
        for (int k = 0; k < nk; ++k) acc += G->Y[k] * G->sh[k][c];
        G->raw[c] = acc;
        G->clampc[c] = acc < 0;
        G->rgb[c] = acc < 0 ? 0.0 : acc;
    }

    /* bounding box of the cutoff ellipse {d : d^T conic d <= 2 ln(o / alpha_min)} */
    if (G->o >= st->alpha_min) {
        const double tq = 2.0 * log(G->o / st->alpha_min);
        G->extx = sqrt(tq * G->S2[0]);
        G->exty = sqrt(tq * G->S2[2]);
    } else {
        G->extx = G->exty = -1.0;   /* can never reach the cutoff */
    }
    {
        const double eps = 5.960464477539063e-08;
        double an = 0, tn = 0;
        for (int i = 0; i < 3; ++i) { an += fabs(G->mu[i]); tn += fabs(cam->t[i]); }
        const double exc = 4.0 * eps * (an + tn);
        G->em[0] = cam->fx * exc * (1.0 + fabs(G->u)) / z + 4.0 * eps * fabs(G->m[0]);
        G->em[1] = cam->fy * exc * (1.0 + fabs(G->v)) / z + 4.0 * eps * fabs(G->m[1]);
        double A[9], B[9], Jw[6], E[4];
        for (int i = 0; i < 9; ++i) A[i] = fabs(G->M[i]);
        for (int i = 0; i < 3; ++i)   /* |W| |M| */
            for (int j = 0; j < 3; ++j) {
                double acc = 0;
                for (int k = 0; k < 3; ++k) acc += fabs(cam->R[3 * i + k]) * A[3 * k + j];
                B[3 * i + j] = acc;
            }
        for (int i = 0; i < 2; ++i)   /* |J| |W| |M| */
            for (int j = 0; j < 3; ++j) {
                double acc = 0;
                for (int k = 0; k < 3; ++k) acc += fabs(G->J[3 * i + k]) * B[3 * k + j];
                Jw[3 * i + j] = acc;
            }
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                double acc = 0;
                for (int k = 0; k < 3; ++k) acc += Jw[3 * i + k] * Jw[3 * j + k];
                E[2 * i + j] = acc;
            }
        G->errS[0] = 32.0 * eps * (E[0] + st->dilation);
        G->errS[1] = 32.0 * eps * E[1];
        G->errS[2] = 32.0 * eps * (E[3] + st->dilation);
    }
    const double tr = 0.5 * (G->S2[0] + G->S2[2]);
    const double disc = sqrt(fmax(tr * tr - G->det, 0.0));
    G->cond = (tr + disc) / fmax(tr - disc, 1e-300);
    G->valid = 1;
}

static void fill_record(const gauss_t *G, double *r) {
    memset(r, 0, REC * sizeof(double));
    r[R_VALID] = G->valid;
    if (!G->valid) return;
    r[R_MX] = G->m[0]; r[R_MY] = G->m[1]; r[R_Z] = G->xc[2];
    r[R_CA] = G->conic[0]; r[R_CB] = G->conic[1]; r[R_CC] = G->conic[2];
    r[R_OPA] = G->o;
    for (int c = 0; c < 3; ++c) { r[R_RGB0 + c] = G->rgb[c]; r[R_CLAMP0 + c] = G->clampc[c]; }
    r[R_S00] = G->S2[0]; r[R_S01] = G->S2[1]; r[R_S11] = G->S2[2];
    r[R_EXTX] = G->extx; r[R_EXTY] = G->exty; r[R_COND] = G->cond;
}

/* Projection of every Gaussian; rec is [n][REC]. */
void orc_preprocess(const double *P, int64_t n, int64_t ncap, const double *camv,
                    const double *setv, double *rec) {
    const cam_t cam = read_cam(camv);
    const set_t st = read_set(setv);
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
        gauss_t G;
        gauss_forward(P, ncap, g, &cam, &st, &G);
        fill_record(&G, rec + g * REC);
    }
}

/* ---------------------------------------------------------------------------
 * Per-pixel compositing (Eq. 3).
 * ------------------------------------------------------------------------- */
typedef struct {
    int64_t g;
    double z, atil, power, dx, dy;
    int contributes;   /* alpha_tilde >= alpha_min */
    int near_cut;      /* FP32 could take the other side of the cutoff */
} cand_t;

typedef struct {
    cand_t *c;
    size_t n, cap;
    double *T, *rejT;
    size_t tcap;
} scratch_t;

static void push(scratch_t *s, const cand_t *c) {
    if (s->n == s->cap) {
        s->cap = s->cap ? 2 * s->cap : 256;
        s->c = (cand_t *)realloc(s->c, s->cap * sizeof(cand_t));
    }
    s->c[s->n++] = *c;
}

static int cmp_cand(const void *a, const void *b) {
    const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
    if (x->z < y->z) return -1;
    if (x->z > y->z) return 1;
    return (x->g > y->g) - (x->g < y->g);
}

/* Conservative FP32 error bound on the exponent of one (pixel, Gaussian) pair.
 * It models rounding of the camera-frame mean and the 2D mean (em, pixels)
 * and of the 2D covariance entries (G->errS, an entrywise bound built from
 * |J| |W| |M| |M|^T |W|^T |J|^T).  Used only to mark pixels whose result FP32
 * arithmetic may legitimately decide the other way. */
static double power_err32(const gauss_t *G, double dx, double dy, double power) {
    const double eps = 5.960464477539063e-08;   /* 2^-24 */
    const double gx = G->conic[0] * dx + G->conic[1] * dy;   /* K (m - p) */
    const double gy = G->conic[1] * dx + G->conic[2] * dy;
    const double e_mean = fabs(gx) * G->em[0] + fabs(gy) * G->em[1];
    const double e_cov = 0.5 * (gx * gx * G->errS[0] + 2 * fabs(gx * gy) * G->errS[1] +
                                gy * gy * G->errS[2]);
    return 4.0 * (e_mean + e_cov + 8.0 * eps * (fabs(power) + 1.0)) + 1e-6;
}

typedef struct {
    const gauss_t *gs;
    int64_t n;
    const cam_t *cam;
    const set_t *st;
    /* candidate pre-filter: bins of BIN x BIN pixels listing Gaussians whose
     * cutoff box touches the bin (NULL = brute force over all Gaussians) */
    int bin, nbx, nby;
    int64_t *bin_start;
    int64_t *bin_list;
    /* >= 0: this Gaussian is skipped in the bin lists and tested at every pixel
     * (its record may have moved, as in a finite-difference perturbation) */
    int64_t extra;
} scene_t;

#define AMB_IMAGE 1   /* the flips FP32 may take change the pixel by > AMB_EFFECT */
#define AMB_COUNT 2   /* a flip FP32 may take changes n_contrib / T_final */
#define AMB_EFFECT 2e-5

/* The candidate record of Gaussian g at pixel (px, py); returns 0 when it
 * neither reaches the cutoff nor lies within FP32 reach of it. */
static int make_cand(const scene_t *S, int64_t g, int px, int py, cand_t *c) {
    const gauss_t *G = &S->gs[g];
    if (!G->valid) return 0;
    const double dx = G->m[0] - px, dy = G->m[1] - py;
    const double power = -0.5 * (G->conic[0] * dx * dx + G->conic[2] * dy * dy) -
                         G->conic[1] * dx * dy;
    const double atil = G->o * exp(power);
    const int contributes = atil >= S->st->alpha_min;
    /* |ln(alpha_tilde / alpha_min)| */
    const double margin = fabs(log(G->o / S->st->alpha_min) + power);
    const int near = margin < power_err32(G, dx, dy, power);
    if (!contributes && !near) return 0;
    cand_t cc = {g, G->xc[2], atil, power, dx, dy, contributes, near};
    *c = cc;
    return 1;
}

/* Builds the candidate list of one pixel, sorted by (z, id). */
static void gather(const scene_t *S, int px, int py, scratch_t *s, int64_t *evaluated) {
    s->n = 0;
    int64_t lo = 0, hi = S->n;
    const int64_t *list = NULL;
    if (S->bin_start) {
        const int b = (py / S->bin) * S->nbx + (px / S->bin);
        lo = S->bin_start[b];
        hi = S->bin_start[b + 1];
        list = S->bin_list;
    }
    for (int64_t i = lo; i <= hi; ++i) {
        int64_t g;
        if (i == hi) {   /* the explicitly tested Gaussian, if any */
            if (S->extra < 0) break;
            g = S->extra;
        } else {
            g = list ? list[i] : i;
            if (g == S->extra) continue;
        }
        if (!S->gs[g].valid) continue;
        ++*evaluated;
        cand_t c;
        if (make_cand(S, g, px, py, &c)) push(s, &c);
    }
    qsort(s->c, s->n, sizeof(cand_t), cmp_cand);
}

/* Two candidates whose FP32 depths may order them differently from FP64: the
 * depths within 4 float32 ulp, unless the two means are bitwise equal (then
 * every precision computes the same depth and both keep index order). */
static int depth_near_tie(const scene_t *S, const cand_t *a, const cand_t *b) {
    if (!(fabs(b->z - a->z) <= 4.8e-7 * (fabs(b->z) + 1.0))) return 0;
    const gauss_t *Ga = &S->gs[a->g], *Gb = &S->gs[b->g];
    if (Ga->mu[0] == Gb->mu[0] && Ga->mu[1] == Gb->mu[1] && Ga->mu[2] == Gb->mu[2]) return 0;
    return 1;
}

typedef struct {
    double C[3], Tfin;
    int ncontrib;
    int amb;
    int64_t contrib_pairs;   /* candidates with alpha >= cutoff, all depths */
} pix_out_t;

/* Composites the sorted candidates of one pixel.  Composited entries are
 * compacted to s->c[0..K) (order kept), with their transmittance in s->T. */
static void composite(const scene_t *S, scratch_t *s, pix_out_t *o) {
    const set_t *st = S->st;
    if (s->tcap < s->n + 1) {
        s->tcap = s->n + 1;
        s->T = (double *)realloc(s->T, s->tcap * sizeof(double));
        s->rejT = (double *)realloc(s->rejT, s->tcap * sizeof(double));
    }
    double T = 1.0;
    double C[3] = {0, 0, 0};
    int K = 0, amb = 0;
    int64_t ncontrib_all = 0;
    for (size_t i = 0; i < s->n; ++i) ncontrib_all += s->c[i].contributes;
    /* Walk the sorted candidates.  Composited entries are compacted to the
     * front of s->c (K <= i, order kept).  Near-cutoff candidates that stay
     * out are recorded with the transmittance at which they would enter. */
    size_t nrej = 0;
    int stopped = 0;
    size_t stop_i = 0;
    double stop_T = 0, stop_alpha = 0, stop_rmax = 0;
    /* relative change of the transmittance that near-cutoff flips ahead of the
     * stop could cause (each flip scales T by 1 - alpha_min or its inverse) */
    double cut_rel = 0;
    /* sum over every decision FP32 may take the other way of its effect on the
     * pixel's colour or final transmittance: they may all flip together */
    double eff = 0;
    const double flip_rel = 1.01 * st->alpha_min / (1.0 - st->alpha_min);
    for (size_t i = 0; i < s->n; ++i) {
        const cand_t c = s->c[i];
        const gauss_t *G = &S->gs[c.g];
        const double rmax = fmax(fmax(G->rgb[0], G->rgb[1]), G->rgb[2]);
        if (!c.contributes) {
            /* effect on the pixel had it been included: ~alpha_min * T * |rgb - behind|,
             * and alpha_min * T_final on the final transmittance (T_final <= T) */
            amb |= AMB_COUNT;
            eff += st->alpha_min * T * (rmax + 1.0);
            s->rejT[nrej++] = T;
            cut_rel += flip_rel;
            continue;
        }
        const double alpha = fmin(st->alpha_max, c.atil);
        const double Tn = T * (1.0 - alpha);
        if (Tn < st->t_min) {   /* early stop: this entry is not added */
            stopped = 1;
            stop_i = i;
            stop_T = T; stop_alpha = alpha; stop_rmax = rmax;
            break;
        }
        if (c.near_cut) cut_rel += flip_rel;
        for (int ch = 0; ch < 3; ++ch) C[ch] += alpha * T * G->rgb[ch];
        s->T[K] = T;
        s->c[K] = c;
        ++K;
        T = Tn;
    }
    /* Depth near-ties: FP32 depths of two primitives within a few ulp may
     * order them the other way.  Primitives with bitwise-equal means have the
     * same depth in any precision and keep index order in both, so they are
     * not a flip.  Swapping neighbours k-1, k changes the pixel by
     * T a_{k-1} a_k |rgb_{k-1} - rgb_k| and leaves the final transmittance
     * alone; a run of near-tied entries is bounded by the sum over its pairs. */
    {
        int k = 1;
        while (k < K) {
            if (!depth_near_tie(S, &s->c[k - 1], &s->c[k])) { ++k; continue; }
            int k1 = k;
            while (k1 + 1 < K && depth_near_tie(S, &s->c[k1], &s->c[k1 + 1])) ++k1;
            /* entries k-1 .. k1 form a run */
            amb |= AMB_COUNT;
            double run = 0;
            for (int i = k - 1; i <= k1; ++i)
                for (int j = i + 1; j <= k1; ++j) {
                    const gauss_t *Gi = &S->gs[s->c[i].g], *Gj = &S->gs[s->c[j].g];
                    double d = 0;
                    for (int ch = 0; ch < 3; ++ch) d = fmax(d, fabs(Gi->rgb[ch] - Gj->rgb[ch]));
                    run += fmin(st->alpha_max, s->c[i].atil) * fmin(st->alpha_max, s->c[j].atil) * d;
                }
            eff += s->T[k - 1] * run;
            k = k1 + 1;
        }
    }
    /* the entry that stopped compositing, near-tied with the last composited
     * one: swapped, it may be composited in its place */
    if (stopped && K > 0 && depth_near_tie(S, &s->c[K - 1], &s->c[stop_i])) {
        const gauss_t *G = &S->gs[s->c[K - 1].g];
        const double rmax = fmax(fmax(G->rgb[0], G->rgb[1]), G->rgb[2]);
        const double aK = fmin(st->alpha_max, s->c[K - 1].atil);
        amb |= AMB_COUNT;
        eff += s->T[K - 1] * (aK * (rmax + 1.0) + stop_alpha * (stop_rmax + 1.0));
    }
    /* composited near-cutoff entries: removing entry k changes the pixel by
     * alpha_k T_k (rgb_k - colour behind k) and the final transmittance by at
     * most alpha_k T_k */
    {
        double B[3] = {S->cam->bg[0], S->cam->bg[1], S->cam->bg[2]};
        for (int k = K - 1; k >= 0; --k) {
            const gauss_t *G = &S->gs[s->c[k].g];
            const double alpha = fmin(st->alpha_max, s->c[k].atil);
            if (s->c[k].near_cut) {
                double diff = 1.0;
                for (int ch = 0; ch < 3; ++ch) diff = fmax(diff, fabs(G->rgb[ch] - B[ch]));
                amb |= AMB_COUNT;
                eff += alpha * s->T[k] * diff;
            }
            for (int ch = 0; ch < 3; ++ch) B[ch] = alpha * G->rgb[ch] + (1 - alpha) * B[ch];
        }
    }
    /* early stop within FP32 reach of t_min, either way; near-cutoff flips
     * ahead of it move the transmittance by cut_rel more */
    const double stop_tol = 2e-3 + cut_rel;
    if (stopped && fabs(stop_T * (1.0 - stop_alpha) / st->t_min - 1.0) < stop_tol) {
        amb |= AMB_COUNT;
        eff += stop_alpha * stop_T * (stop_rmax + 1.0);
    }
    if (K > 0) {
        const double aK = fmin(st->alpha_max, s->c[K - 1].atil);
        if (fabs(s->T[K - 1] * (1.0 - aK) / st->t_min - 1.0) < stop_tol) {
            const gauss_t *G = &S->gs[s->c[K - 1].g];
            const double rmax = fmax(fmax(G->rgb[0], G->rgb[1]), G->rgb[2]);
            amb |= AMB_COUNT;
            eff += aK * s->T[K - 1] * (rmax + 1.0);
        }
    }
    if (eff > AMB_EFFECT) amb |= AMB_IMAGE;
    s->n = (size_t)K;
    s->T[K] = T;
    for (int ch = 0; ch < 3; ++ch) o->C[ch] = C[ch] + T * S->cam->bg[ch];
    o->Tfin = T;
    o->ncontrib = K;
    o->amb = amb;
    o->contrib_pairs = ncontrib_all;
}

static void build_scene(scene_t *S, gauss_t *gs, int64_t n, const cam_t *cam, const set_t *st,
                        int prune) {
    memset(S, 0, sizeof *S);
    S->gs = gs; S->n = n; S->cam = cam; S->st = st;
    S->extra = -1;
    if (!prune) return;
    S->bin = 16;
    S->nbx = (cam->W + S->bin - 1) / S->bin;
    S->nby = (cam->H + S->bin - 1) / S->bin;
    const int nb = S->nbx * S->nby;
    S->bin_start = (int64_t *)calloc((size_t)nb + 1, sizeof(int64_t));
    /* pass 1: count, pass 2: fill, in Gaussian order */
    for (int pass = 0; pass < 2; ++pass) {
        int64_t *cursor = NULL;
        if (pass == 1) {
            for (int b = 0; b < nb; ++b) S->bin_start[b + 1] += S->bin_start[b];
            S->bin_list = (int64_t *)malloc((size_t)(S->bin_start[nb] + 1) * sizeof(int64_t));
            cursor = (int64_t *)malloc((size_t)nb * sizeof(int64_t));
            memcpy(cursor, S->bin_start, (size_t)nb * sizeof(int64_t));
        }
        for (int64_t g = 0; g < n; ++g) {
            const gauss_t *G = &gs[g];
            if (!G->valid || G->extx < 0) continue;
            /* one extra pixel of margin keeps the box conservative under rounding */
            const double x0 = G->m[0] - G->extx - 1.0, x1 = G->m[0] + G->extx + 1.0;
            const double y0 = G->m[1] - G->exty - 1.0, y1 = G->m[1] + G->exty + 1.0;
            if (x1 < 0 || y1 < 0 || x0 > cam->W - 1 || y0 > cam->H - 1) continue;
            const int bx0 = (int)fmax(0.0, floor(x0)) / S->bin;
            const int bx1 = (int)fmin(cam->W - 1.0, ceil(x1)) / S->bin;
            const int by0 = (int)fmax(0.0, floor(y0)) / S->bin;
            const int by1 = (int)fmin(cam->H - 1.0, ceil(y1)) / S->bin;
            for (int by = by0; by <= by1; ++by)
                for (int bx = bx0; bx <= bx1; ++bx) {
                    const int b = by * S->nbx + bx;
                    if (pass == 0) S->bin_start[b + 1]++;
                    else S->bin_list[cursor[b]++] = g;
                }
        }
        free(cursor);
    }
}

static void free_scene(scene_t *S) {
    free(S->bin_start);
    free(S->bin_list);
}

static gauss_t *forward_all(const double *P, int64_t n, int64_t ncap, const cam_t *cam,
                            const set_t *st) {
    gauss_t *gs = (gauss_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(gauss_t));
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) gauss_forward(P, ncap, g, cam, st, &gs[g]);
    return gs;
}

/*
 * Renders the image of Eq. 3.  Outputs (all [H][W] planes; img is [3][H][W]):
 * img, T_final, n_contrib, amb (AMB_* bits).  mask (optional, [H][W] bytes)
 * restricts the pixels computed; others are left untouched.
 * counts[0] = (pixel, Gaussian) pairs evaluated, counts[1] = pairs with
 * alpha >= cutoff at any depth, counts[2] = composited pairs,
 * counts[3] = pixels with AMB_IMAGE, counts[4] = pixels with AMB_COUNT.
 */
void orc_render(const double *P, int64_t n, int64_t ncap, const double *camv, const double *setv,
                int prune, const uint8_t *mask, double *img, double *Tfin, int32_t *ncontrib,
                uint8_t *amb, int64_t *counts) {
    const cam_t cam = read_cam(camv);
    const set_t st = read_set(setv);
    gauss_t *gs = forward_all(P, n, ncap, &cam, &st);
    scene_t S;
    build_scene(&S, gs, n, &cam, &st, prune);
    const int64_t HW = (int64_t)cam.W * cam.H;
    int64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0;
#pragma omp parallel reduction(+ : c0, c1, c2, c3, c4)
    {
        scratch_t s;
        memset(&s, 0, sizeof s);
#pragma omp for schedule(dynamic, 4)
        for (int py = 0; py < cam.H; ++py)
            for (int px = 0; px < cam.W; ++px) {
                const int64_t pix = (int64_t)py * cam.W + px;
                if (mask && !mask[pix]) continue;
                int64_t ev = 0;
                gather(&S, px, py, &s, &ev);
                pix_out_t o;
                composite(&S, &s, &o);
                for (int ch = 0; ch < 3; ++ch) img[ch * HW + pix] = o.C[ch];
                Tfin[pix] = o.Tfin;
                ncontrib[pix] = o.ncontrib;
                amb[pix] = (uint8_t)o.amb;
                c0 += ev; c1 += o.contrib_pairs; c2 += o.ncontrib;
                c3 += (o.amb & AMB_IMAGE) != 0;
                c4 += (o.amb & AMB_COUNT) != 0;
            }
        free(s.c); free(s.T); free(s.rejT);
    }
    if (counts) { counts[0] = c0; counts[1] = c1; counts[2] = c2; counts[3] = c3; counts[4] = c4; }
    free_scene(&S);
    free(gs);
}

/* The sorted list of Gaussians composited at one pixel (ids in order). */
int orc_pixel_list(const double *P, int64_t n, int64_t ncap, const double *camv, const double *setv,
                   int px, int py, int64_t *ids, int cap) {
    const cam_t cam = read_cam(camv);
    const set_t st = read_set(setv);
    gauss_t *gs = forward_all(P, n, ncap, &cam, &st);
    scene_t S;
    build_scene(&S, gs, n, &cam, &st, 0);
    scratch_t s;
    memset(&s, 0, sizeof s);
    int64_t ev = 0;
    gather(&S, px, py, &s, &ev);
    pix_out_t o;
    composite(&S, &s, &o);
    int K = o.ncontrib < cap ? o.ncontrib : cap;
    for (int k = 0; k < K; ++k) ids[k] = s.c[k].g;
    free(s.c); free(s.T); free(s.rejT);
    free_scene(&S);
    free(gs);
    return o.ncontrib;
}

/* ---------------------------------------------------------------------------
 * Reverse mode of Eq. 3 through the projection to the raw parameters.
 * ------------------------------------------------------------------------- */
static inline void atomic_add(double *p, double v) {
#pragma omp atomic
    *p += v;
}

/* Per-Gaussian chain rule from 2D gradients to the raw-parameter gradient.
 * g2 = {dL/dmx, dL/dmy, dL/da, dL/db, dL/dc, dL/do, dL/dr, dL/dg, dL/db}. */
static void gauss_backward(const gauss_t *G, const cam_t *cam, const set_t *st,
                           const double g2[9], double out[NROWS]) {
    memset(out, 0, NROWS * sizeof(double));
    if (!G->valid) return;
    const double z = G->xc[2];
    double dxc[3] = {0, 0, 0};
    double dmu[3] = {0, 0, 0};

    /* colour: rgb = max(raw, 0), raw = 0.5 + sum_k Y_k(d) sh_k */
    double draw[3];
    for (int c = 0; c < 3; ++c) draw[c] = G->clampc[c] ? 0.0 : g2[6 + c];
    const int nk = (st->sh_degree + 1) * (st->sh_degree + 1);
    double ddir[3] = {0, 0, 0};
    for (int k = 0; k < nk; ++k)
        for (int c = 0; c < 3; ++c) {
            out[ROW_SH + 3 * k + c] = G->Y[k] * draw[c];
            for (int i = 0; i < 3; ++i) ddir[i] += draw[c] * G->sh[k][c] * G->dY[k][i];
        }
    /* d = (mu - C)/|mu - C|: dd/dmu = (I - d d^T)/|mu - C| */
    {
        double dot = 0;
        for (int i = 0; i < 3; ++i) dot += G->dir[i] * ddir[i];
        for (int i = 0; i < 3; ++i) dmu[i] += (ddir[i] - G->dir[i] * dot) / G->dist;
    }

    /* 2D mean m = (fx x/z + cx, fy y/z + cy) */
    dxc[0] += g2[0] * cam->fx / z;
    dxc[1] += g2[1] * cam->fy / z;
    dxc[2] += -g2[0] * cam->fx * G->xc[0] / (z * z) - g2[1] * cam->fy * G->xc[1] / (z * z);

    /* conic K = S2^-1: dL/dS2 = -K G_K K, G_K = [[da, db/2], [db/2, dc]] */
    const double a = G->conic[0], b = G->conic[1], c = G->conic[2];
    const double Gk[4] = {g2[2], 0.5 * g2[3], 0.5 * g2[3], g2[4]};
    const double K[4] = {a, b, b, c};
    double KG[4], GS[4];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) KG[2 * i + j] = K[2 * i] * Gk[j] + K[2 * i + 1] * Gk[2 + j];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) GS[2 * i + j] = -(KG[2 * i] * K[j] + KG[2 * i + 1] * K[2 + j]);
    /* S2 = J V J^T + dil I: dL/dV = J^T GS J, dL/dJ = 2 GS J V */
    double dV[9], dJ[6];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int p = 0; p < 2; ++p)
                for (int q = 0; q < 2; ++q) acc += G->J[3 * p + i] * GS[2 * p + q] * G->J[3 * q + j];
            dV[3 * i + j] = acc;
        }
    for (int p = 0; p < 2; ++p)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int q = 0; q < 2; ++q)
                for (int k = 0; k < 3; ++k) acc += GS[2 * p + q] * G->J[3 * q + k] * G->V[3 * k + j];
            dJ[3 * p + j] = 2.0 * acc;
        }
    /* J entries as functions of x_c (FOV clamp freezes the clamped coordinate) */
    const double fx = cam->fx, fy = cam->fy;
    dxc[2] += dJ[0] * (-fx / (z * z)) + dJ[4] * (-fy / (z * z));
    /* J02 = -fx ubar / z */
    dxc[2] += dJ[2] * (fx * G->ubar / (z * z));
    if (!G->clampx) {
        dxc[0] += dJ[2] * (-fx / (z * z));
        dxc[2] += dJ[2] * (fx * G->xc[0] / (z * z * z));
    }
    dxc[2] += dJ[5] * (fy * G->vbar / (z * z));
    if (!G->clampy) {
        dxc[1] += dJ[5] * (-fy / (z * z));
        dxc[2] += dJ[5] * (fy * G->xc[1] / (z * z * z));
    }
    /* x_c = W mu + t */
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) dmu[i] += cam->R[3 * k + i] * dxc[k];

    /* V = W Sigma W^T: dL/dSigma = W^T dV W */
    double dS[9], tmp[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += cam->R[3 * k + i] * dV[3 * k + j];
            tmp[3 * i + j] = acc;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += tmp[3 * i + k] * cam->R[3 * k + j];
            dS[3 * i + j] = acc;
        }
    /* Sigma = M M^T (dS symmetric): dL/dM = 2 dS M; M = Rq diag(s) */
    double dM[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += dS[3 * i + k] * G->M[3 * k + j];
            dM[3 * i + j] = 2.0 * acc;
        }
    double dR[9];
    for (int j = 0; j < 3; ++j) {
        double ds = 0;
        for (int i = 0; i < 3; ++i) {
            ds += dM[3 * i + j] * G->Rq[3 * i + j];
            dR[3 * i + j] = dM[3 * i + j] * G->s[j];
        }
        out[ROW_LOGS + j] = ds * G->s[j];
    }
    /* rotation polynomial of the unit quaternion */
    const double w = G->qn[0], x = G->qn[1], y = G->qn[2], zq = G->qn[3];
    double dq[4];
    dq[0] = 2 * (-zq * dR[1] + y * dR[2] + zq * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2 * (y * dR[1] + zq * dR[2] + y * dR[3] - 2 * x * dR[4] - w * dR[5] + zq * dR[6] +
                 w * dR[7] - 2 * x * dR[8]);
    dq[2] = 2 * (-2 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + zq * dR[5] - w * dR[6] +
                 zq * dR[7] - 2 * y * dR[8]);
    dq[3] = 2 * (-2 * zq * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2 * zq * dR[4] + y * dR[5] +
                 x * dR[6] + y * dR[7]);
    /* normalisation q_hat = q/|q| */
    double dot = 0;
    for (int i = 0; i < 4; ++i) dot += G->qn[i] * dq[i];
    for (int i = 0; i < 4; ++i) out[ROW_QUAT + i] = (dq[i] - G->qn[i] * dot) / G->qlen;

    out[ROW_OPAC] = g2[5] * G->o * (1.0 - G->o);
    for (int i = 0; i < 3; ++i) out[ROW_MU + i] = dmu[i];
}

/*
 * Gradient of sum(dL_dimg * img) with respect to the raw parameters.
 * grad ([59][ncap]) is accumulated (+=).  g2d (optional, [n][9]) receives the
 * per-Gaussian 2D gradients (mean, conic, opacity, rgb), also accumulated.
 * mask restricts the pixels that contribute.
 */
void orc_render_backward(const double *P, int64_t n, int64_t ncap, const double *camv,
                         const double *setv, const uint8_t *mask, const double *dL_dimg,
                         double *grad, double *g2d) {
    const cam_t cam = read_cam(camv);
    const set_t st = read_set(setv);
    gauss_t *gs = forward_all(P, n, ncap, &cam, &st);
    scene_t S;
    build_scene(&S, gs, n, &cam, &st, 1);
    const int64_t HW = (int64_t)cam.W * cam.H;
    double *acc = (double *)calloc((size_t)(n > 0 ? n : 1) * 9, sizeof(double));
#pragma omp parallel
    {
        scratch_t s;
        memset(&s, 0, sizeof s);
#pragma omp for schedule(dynamic, 4)
        for (int py = 0; py < cam.H; ++py)
            for (int px = 0; px < cam.W; ++px) {
                const int64_t pix = (int64_t)py * cam.W + px;
                if (mask && !mask[pix]) continue;
                const double gC[3] = {dL_dimg[pix], dL_dimg[HW + pix], dL_dimg[2 * HW + pix]};
                if (gC[0] == 0 && gC[1] == 0 && gC[2] == 0) continue;
                int64_t ev = 0;
                gather(&S, px, py, &s, &ev);
                pix_out_t o;
                composite(&S, &s, &o);
                const int K = o.ncontrib;
                double B[3] = {cam.bg[0], cam.bg[1], cam.bg[2]};   /* colour behind entry k */
                for (int k = K - 1; k >= 0; --k) {
                    const cand_t *c = &s.c[k];
                    const gauss_t *G = &gs[c->g];
                    const double T = s.T[k];
                    const double alpha = fmin(st.alpha_max, c->atil);
                    double dalpha = 0;
                    for (int ch = 0; ch < 3; ++ch) dalpha += T * (G->rgb[ch] - B[ch]) * gC[ch];
                    double *A = acc + c->g * 9;
                    for (int ch = 0; ch < 3; ++ch) atomic_add(&A[6 + ch], alpha * T * gC[ch]);
                    const double datil = c->atil < st.alpha_max ? dalpha : 0.0;
                    atomic_add(&A[5], exp(c->power) * datil);
                    const double dpow = c->atil * datil;
                    const double dx = c->dx, dy = c->dy;   /* m - p */
                    atomic_add(&A[0], dpow * -(G->conic[0] * dx + G->conic[1] * dy));
                    atomic_add(&A[1], dpow * -(G->conic[1] * dx + G->conic[2] * dy));
                    atomic_add(&A[2], dpow * -0.5 * dx * dx);
                    atomic_add(&A[3], dpow * -dx * dy);
                    atomic_add(&A[4], dpow * -0.5 * dy * dy);
                    for (int ch = 0; ch < 3; ++ch) B[ch] = alpha * G->rgb[ch] + (1 - alpha) * B[ch];
                }
            }
        free(s.c); free(s.T); free(s.rejT);
    }
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
        double out[NROWS];
        gauss_backward(&gs[g], &cam, &st, acc + g * 9, out);
        for (int r = 0; r < NROWS; ++r) grad[r * ncap + g] += out[r];
        if (g2d)
            for (int i = 0; i < 9; ++i) g2d[g * 9 + i] += acc[g * 9 + i];
    }
    free(acc);
    free_scene(&S);
    free(gs);
}

/* Chain rule of one Gaussian from given 2D gradients (for unit tests). */
void orc_gauss_backward(const double *P, int64_t ncap, int64_t g, const double *camv,
                        const double *setv, const double *g2, double *out) {
    const cam_t cam = read_cam(camv);
    const set_t st = read_set(setv);
    gauss_t G;
    gauss_forward(P, ncap, g, &cam, &st, &G);
    gauss_backward(&G, &cam, &st, g2, out);
}

/*
 * Central finite differences of L = <W, I> with respect to raw parameters of
 * Gaussians gids[0..ngids) (output [ngids][nrows]): for each Gaussian and row,
 * the parameter is moved by +-h and that Gaussian alone is re-projected; only
 * pixels inside the union of its cutoff boxes can change, and there each
 * pixel's sorted list of the other Gaussians is computed once and the moved
 * Gaussian is merged into it for every evaluation.  fd receives
 * (L+ - L-) / (2h); changed is 1 when the set of composited Gaussians or of
 * cutoff-passing pairs differs between +h and -h at any of those pixels (a
 * discrete event the derivative does not see).
 */
void orc_fd_gauss(const double *P, int64_t n, int64_t ncap, const double *camv,
                  const double *setv, const double *W, const int64_t *gids, int ngids,
                  const int32_t *rows, int nrows, double h, double *fd_all, int32_t *changed_all) {
    const cam_t cam = read_cam(camv);
    const set_t st = read_set(setv);
    gauss_t *gs = forward_all(P, n, ncap, &cam, &st);
    scene_t S;
    build_scene(&S, gs, n, &cam, &st, 1);
    const int64_t HW = (int64_t)cam.W * cam.H;
    for (int gi = 0; gi < ngids; ++gi) {
        const int64_t gid = gids[gi];
        double *fd = fd_all + (size_t)gi * nrows;
        int32_t *changed = changed_all + (size_t)gi * nrows;
        const gauss_t G0 = gs[gid];
        double col[NROWS];
        for (int r = 0; r < NROWS; ++r) col[r] = P[r * ncap + gid];
        gauss_t *Gp = (gauss_t *)malloc(sizeof(gauss_t) * 2 * (size_t)nrows);
        double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
        for (int k = 0; k < 2 * nrows + 1; ++k) {
            const gauss_t *G = &G0;
            if (k < 2 * nrows) {
                double c2[NROWS];
                memcpy(c2, col, sizeof col);
                c2[rows[k / 2]] += (k & 1) ? -h : h;
                gauss_forward(c2, 1, 0, &cam, &st, &Gp[k]);
                G = &Gp[k];
            }
            if (!G->valid || G->extx < 0) continue;
            x0 = fmin(x0, G->m[0] - G->extx - 2); x1 = fmax(x1, G->m[0] + G->extx + 2);
            y0 = fmin(y0, G->m[1] - G->exty - 2); y1 = fmax(y1, G->m[1] + G->exty + 2);
        }
        const int px0 = (int)fmax(0.0, floor(x0)), px1 = (int)fmin(cam.W - 1.0, ceil(x1));
        const int py0 = (int)fmax(0.0, floor(y0)), py1 = (int)fmin(cam.H - 1.0, ceil(y1));
        if (!(px0 <= px1 && py0 <= py1)) {
            for (int k = 0; k < nrows; ++k) { fd[k] = 0; changed[k] = 0; }
            free(Gp);
            continue;
        }
        const int bw = px1 - px0 + 1, bh = py1 - py0 + 1;
        const size_t npx = (size_t)bw * bh;
        /* sorted candidate lists of the other Gaussians at every box pixel */
        cand_t **lists = (cand_t **)calloc(npx, sizeof(cand_t *));
        size_t *lens = (size_t *)calloc(npx, sizeof(size_t));
        gs[gid].valid = 0;
        S.extra = gid;
#pragma omp parallel
        {
            scratch_t sc;
            memset(&sc, 0, sizeof sc);
#pragma omp for schedule(dynamic, 2)
            for (int py = py0; py <= py1; ++py)
                for (int px = px0; px <= px1; ++px) {
                    int64_t ev = 0;
                    gather(&S, px, py, &sc, &ev);
                    const size_t q = (size_t)(py - py0) * bw + (px - px0);
                    lens[q] = sc.n;
                    lists[q] = (cand_t *)malloc(sizeof(cand_t) * (sc.n + 1));
                    memcpy(lists[q], sc.c, sizeof(cand_t) * sc.n);
                }
            free(sc.c); free(sc.T); free(sc.rejT);
        }
        int *ncs = (int *)malloc(sizeof(int) * 2 * npx);
        int64_t *ccs = (int64_t *)malloc(sizeof(int64_t) * 2 * npx);
        /* per-pixel values of <W, C> at +h and -h; the difference is taken per
         * pixel and summed in pixel order, so the result does not depend on
         * the thread count and no two image-wide sums cancel */
        double *Lpix = (double *)malloc(sizeof(double) * 2 * npx);
        for (int k = 0; k < nrows; ++k) {
            for (int sgn = 0; sgn < 2; ++sgn) {
                gs[gid] = Gp[2 * k + sgn];
#pragma omp parallel
                {
                    scratch_t sc;
                    memset(&sc, 0, sizeof sc);
#pragma omp for schedule(dynamic, 4)
                    for (int py = py0; py <= py1; ++py)
                        for (int px = px0; px <= px1; ++px) {
                            const size_t q = (size_t)(py - py0) * bw + (px - px0);
                            sc.n = 0;
                            if (sc.cap < lens[q] + 1) {
                                sc.cap = lens[q] + 1;
                                sc.c = (cand_t *)realloc(sc.c, sc.cap * sizeof(cand_t));
                            }
                            cand_t c;
                            const int have = make_cand(&S, gid, px, py, &c);
                            size_t w = 0;
                            int pending = have;   /* merge the moved Gaussian once */
                            for (size_t i2 = 0; i2 < lens[q]; ++i2) {
                                if (pending && cmp_cand(&c, &lists[q][i2]) < 0) {
                                    sc.c[w++] = c;
                                    pending = 0;
                                }
                                sc.c[w++] = lists[q][i2];
                            }
                            if (pending) sc.c[w++] = c;
                            sc.n = w;
                            pix_out_t o;
                            composite(&S, &sc, &o);
                            const int64_t pix = (int64_t)py * cam.W + px;
                            double acc = 0;
                            for (int ch = 0; ch < 3; ++ch) acc += W[ch * HW + pix] * o.C[ch];
                            Lpix[sgn * npx + q] = acc;
                            ncs[sgn * npx + q] = o.ncontrib;
                            ccs[sgn * npx + q] = o.contrib_pairs;
                        }
                    free(sc.c); free(sc.T); free(sc.rejT);
                }
            }
            int chg = 0;
            double dsum = 0;
            for (size_t q = 0; q < npx; ++q) {
                if (ncs[q] != ncs[q + npx] || ccs[q] != ccs[q + npx]) chg = 1;
                dsum += Lpix[q] - Lpix[q + npx];
            }
            fd[k] = dsum / (2 * h);
            changed[k] = chg;
        }
        free(Lpix);
        gs[gid] = G0;
        S.extra = -1;
        for (size_t q = 0; q < npx; ++q) free(lists[q]);
        free(lists); free(lens); free(ncs); free(ccs); free(Gp);
    }
    free_scene(&S);
    free(gs);
}

/* ---------------------------------------------------------------------------
 * Gaussian pyramid (Section 3.4): smooth with the 5x5 binomial kernel
 * (1 4 6 4 1)^T (1 4 6 4 1) / 256, borders reflected without repeating the
 * edge sample, keep even rows and columns.  in [C][H][W] ->
 * out [C][ceil(H/2)][ceil(W/2)].
 * ------------------------------------------------------------------------- */
static int reflect101(int i, int n) {
    if (n == 1) return 0;
    while (i < 0 || i >= n) {
        if (i < 0) i = -i;
        if (i >= n) i = 2 * (n - 1) - i;
    }
    return i;
}

void orc_pyr_down(const double *in, int C, int H, int W, double *out) {
    const double k[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};
    const int Ho = (H + 1) / 2, Wo = (W + 1) / 2;
    for (int c = 0; c < C; ++c)
#pragma omp parallel for schedule(static)
        for (int i = 0; i < Ho; ++i)
            for (int j = 0; j < Wo; ++j) {
                double acc = 0;
                for (int a = -2; a <= 2; ++a)
                    for (int b = -2; b <= 2; ++b)
                        acc += k[a + 2] * k[b + 2] *
                               in[((int64_t)c * H + reflect101(2 * i + a, H)) * W +
                                  reflect101(2 * j + b, W)];
                out[((int64_t)c * Ho + i) * Wo + j] = acc;
            }
}

/* ---------------------------------------------------------------------------
 * Photometric loss of Eq. 4 for one image pair, [C][H][W] each:
 *   L = (1 - lambda) * mean|x - y| + lambda * (1 - mean SSIM(x, y)),
 * SSIM with an 11x11 Gaussian window (sigma 1.5), zero padding outside the
 * image, C1 = 0.01^2, C2 = 0.03^2, per channel, mean over all pixels and
 * channels.  dx (optional) receives dL/dx.  parts[0] = mean L1,
 * parts[1] = mean SSIM.
 * ------------------------------------------------------------------------- */
#define SSIM_R 5

static void ssim_window(double w[2 * SSIM_R + 1]) {
    double s = 0;
    for (int i = -SSIM_R; i <= SSIM_R; ++i) {
        w[i + SSIM_R] = exp(-(double)(i * i) / (2.0 * 1.5 * 1.5));
        s += w[i + SSIM_R];
    }
    for (int i = 0; i < 2 * SSIM_R + 1; ++i) w[i] /= s;
}

/* out(p) = sum_{u,v} w(u) w(v) f(p + (u, v)), zero outside; one channel */
static void window_filter(const double *f, int H, int W, double *out) {
    double w[2 * SSIM_R + 1];
    ssim_window(w);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            double acc = 0;
            for (int u = -SSIM_R; u <= SSIM_R; ++u) {
                const int ii = i + u;
                if (ii < 0 || ii >= H) continue;
                for (int v = -SSIM_R; v <= SSIM_R; ++v) {
                    const int jj = j + v;
                    if (jj < 0 || jj >= W) continue;
                    acc += w[u + SSIM_R] * w[v + SSIM_R] * f[(int64_t)ii * W + jj];
                }
            }
            out[(int64_t)i * W + j] = acc;
        }
}

double orc_loss(const double *x, const double *y, int C, int H, int W, double lambda, double *dx,
                double *parts) {
    const double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
    const int64_t HW = (int64_t)H * W;
    const double inv = 1.0 / ((double)C * HW);
    double l1 = 0, ssim = 0;
    double *buf = (double *)malloc((size_t)HW * 13 * sizeof(double));
    double *xx = buf, *yy = buf + HW, *xy = buf + 2 * HW;
    double *mx = buf + 3 * HW, *my = buf + 4 * HW, *exx = buf + 5 * HW, *eyy = buf + 6 * HW,
           *exy = buf + 7 * HW;
    double *dmu = buf + 8 * HW, *dxx = buf + 9 * HW, *dxy = buf + 10 * HW, *f1 = buf + 11 * HW,
           *f2 = buf + 12 * HW;
    for (int c = 0; c < C; ++c) {
        const double *xc = x + c * HW, *yc = y + c * HW;
        for (int64_t p = 0; p < HW; ++p) {
            xx[p] = xc[p] * xc[p];
            yy[p] = yc[p] * yc[p];
            xy[p] = xc[p] * yc[p];
            const double d = xc[p] - yc[p];
            l1 += fabs(d);
        }
        window_filter(xc, H, W, mx);
        window_filter(yc, H, W, my);
        window_filter(xx, H, W, exx);
        window_filter(yy, H, W, eyy);
        window_filter(xy, H, W, exy);
        for (int64_t p = 0; p < HW; ++p) {
            const double sx = exx[p] - mx[p] * mx[p];
            const double sy = eyy[p] - my[p] * my[p];
            const double sxy = exy[p] - mx[p] * my[p];
            const double A1 = 2 * mx[p] * my[p] + C1, A2 = 2 * sxy + C2;
            const double B1 = mx[p] * mx[p] + my[p] * my[p] + C1, B2 = sx + sy + C2;
            const double S = A1 * A2 / (B1 * B2);
            ssim += S;
            /* partials of S with respect to mu_x, E[x^2], E[xy] */
            dmu[p] = 2 * my[p] * (A2 - A1) / (B1 * B2) - 2 * mx[p] * S * (1 / B1 - 1 / B2);
            dxx[p] = -S / B2;
            dxy[p] = 2 * A1 / (B1 * B2);
        }
        if (dx) {
            double *dxc = dx + c * HW;
            /* the adjoint of the zero-padded symmetric window is the same filter */
            window_filter(dmu, H, W, f1);
            window_filter(dxx, H, W, f2);
            window_filter(dxy, H, W, dmu);   /* dmu no longer needed */
            for (int64_t p = 0; p < HW; ++p) {
                const double dssim = inv * (f1[p] + 2 * xc[p] * f2[p] + yc[p] * dmu[p]);
                const double d = xc[p] - yc[p];
                const double sgn = (d > 0) - (d < 0);
                dxc[p] = (1 - lambda) * sgn * inv - lambda * dssim;
            }
        }
    }
    free(buf);
    l1 *= inv;
    ssim *= inv;
    if (parts) { parts[0] = l1; parts[1] = ssim; }
    return (1 - lambda) * l1 + lambda * (1 - ssim);
}

/* ---------------------------------------------------------------------------
 * Optimiser step (Section 4.1 names a fixed-rate gradient method; the update
 * is Adam with torch's bias correction):
 *   m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
 *   p -= lr_row * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * Arrays are [59][ncap]; only columns < n are touched.
 * ------------------------------------------------------------------------- */
void orc_adam(double *p, const double *g, double *m, double *v, int64_t n, int64_t ncap,
              const double *lr_rows, double b1, double b2, double eps, int step) {
    const double bc1 = 1.0 - pow(b1, step), bc2 = 1.0 - pow(b2, step);
    for (int r = 0; r < NROWS; ++r)
        for (int64_t i = 0; i < n; ++i) {
            const int64_t k = r * ncap + i;
            m[k] = b1 * m[k] + (1 - b1) * g[k];
            v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k];
            const double mh = m[k] / bc1, vh = v[k] / bc2;
            p[k] -= lr_rows[r] * mh / (sqrt(vh) + eps);
        }
}

int orc_record_width(void) { return REC; }

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
