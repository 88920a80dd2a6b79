// Projection of the Gaussian map into views, and its reverse mode.
//
// Forward (gs_preprocess): Section 3.3, Eq. 3 -- the splat G of each primitive
// in a keyframe: camera-frame mean, first-order (EWA) projection of the 3D
// covariance through the perspective Jacobian, 2D mean, opacity from the
// density logit, and the colour converted from degree-3 spherical harmonics
// (Section 3.1).  Backward (launched by gs_render_bwd): the chain rule from the
// per-view 2D gradients to the raw parameters (position, log-scale,
// quaternion, opacity logit, SH), summed over views.
//
// One thread per Gaussian; the thread loads the Gaussian's 59 parameters once
// (row-major SoA, so each load instruction is coalesced across the wave) and
// loops over the views.  Both kernels are HBM-bound: 236 B read per Gaussian
// plus 40 B written per (view, Gaussian) forward; 236 B read, 36 B of
// accumulators read per view and 236 B read-modify-written backward.
#include "gs_internal.hpp"

namespace gs {

struct Cam {
    float R[9], t[3], C[3];
    float fx, fy, cx, cy, limx, limy;
};

__device__ __forceinline__ Cam load_cam(const gs_view &v, float fov_clamp) {
    Cam c;
#pragma unroll
    for (int i = 0; i < 9; ++i) c.R[i] = v.R[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) c.t[i] = v.t[i];
    // camera centre -R^T t
#pragma unroll
    for (int i = 0; i < 3; ++i)
        c.C[i] = -(c.R[i] * c.t[0] + c.R[3 + i] * c.t[1] + c.R[6 + i] * c.t[2]);
    c.fx = v.fx; c.fy = v.fy; c.cx = v.cx; c.cy = v.cy;
    c.limx = fov_clamp * 0.5f * static_cast<float>(v.width) / v.fx;
    c.limy = fov_clamp * 0.5f * static_cast<float>(v.height) / v.fy;
    return c;
}

// Real SH normalisation constants (orthonormal real basis, degree <= 3).
struct ShK {
    float k0, k1, k2a, k2b, k2c, k3a, k3b, k3c, k3d, k3e;
};
__device__ __forceinline__ ShK sh_consts() {
    const float pi = 3.14159265358979323846f;
    return ShK{0.5f * sqrtf(1.f / pi),          0.5f * sqrtf(3.f / pi),
               0.5f * sqrtf(15.f / pi),         0.25f * sqrtf(5.f / pi),
               0.25f * sqrtf(15.f / pi),        0.25f * sqrtf(35.f / (2.f * pi)),
               0.5f * sqrtf(105.f / pi),        0.25f * sqrtf(21.f / (2.f * pi)),
               0.25f * sqrtf(7.f / pi),         0.25f * sqrtf(105.f / pi)};
}

// Y_k(d) for k < 16 (index l*l + l + m); entries beyond the degree are zero.
__device__ __forceinline__ void sh_eval(int deg, float x, float y, float z, float Y[16]) {
    const ShK k = sh_consts();
#pragma unroll
    for (int i = 0; i < 16; ++i) Y[i] = 0.f;
    Y[0] = k.k0;
    if (deg < 1) return;
    Y[1] = -k.k1 * y;
    Y[2] = k.k1 * z;
    Y[3] = -k.k1 * x;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = k.k2a * x * y;
    Y[5] = -k.k2a * y * z;
    Y[6] = k.k2b * (2.f * zz - xx - yy);
    Y[7] = -k.k2a * x * z;
    Y[8] = k.k2c * (xx - yy);
    if (deg < 3) return;
    Y[9] = -k.k3a * y * (3.f * xx - yy);
    Y[10] = k.k3b * x * y * z;
    Y[11] = -k.k3c * y * (4.f * zz - xx - yy);
    Y[12] = k.k3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
    Y[13] = -k.k3c * x * (4.f * zz - xx - yy);
    Y[14] = k.k3e * z * (xx - yy);
    Y[15] = -k.k3a * x * (xx - 3.f * yy);
}

// Gradient of sum_k w_k Y_k with respect to the (unnormalised) direction
// components, as polynomials in x, y, z.
__device__ __forceinline__ void sh_grad(int deg, float x, float y, float z, const float w[16],
                                        float g[3]) {
    const ShK k = sh_consts();
    g[0] = g[1] = g[2] = 0.f;
    if (deg < 1) return;
    g[1] += -k.k1 * w[1];
    g[2] += k.k1 * w[2];
    g[0] += -k.k1 * w[3];
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    g[0] += k.k2a * y * w[4];             g[1] += k.k2a * x * w[4];
    g[1] += -k.k2a * z * w[5];            g[2] += -k.k2a * y * w[5];
    g[0] += -2.f * k.k2b * x * w[6];      g[1] += -2.f * k.k2b * y * w[6];
    g[2] += 4.f * k.k2b * z * w[6];
    g[0] += -k.k2a * z * w[7];            g[2] += -k.k2a * x * w[7];
    g[0] += 2.f * k.k2c * x * w[8];       g[1] += -2.f * k.k2c * y * w[8];
    if (deg < 3) return;
    g[0] += -6.f * k.k3a * x * y * w[9];  g[1] += -3.f * k.k3a * (xx - yy) * w[9];
    g[0] += k.k3b * y * z * w[10];        g[1] += k.k3b * x * z * w[10];
    g[2] += k.k3b * x * y * w[10];
    g[0] += 2.f * k.k3c * x * y * w[11];  g[1] += -k.k3c * (4.f * zz - xx - 3.f * yy) * w[11];
    g[2] += -8.f * k.k3c * y * z * w[11];
    g[0] += -6.f * k.k3d * x * z * w[12]; g[1] += -6.f * k.k3d * y * z * w[12];
    g[2] += k.k3d * (6.f * zz - 3.f * xx - 3.f * yy) * w[12];
    g[0] += -k.k3c * (4.f * zz - 3.f * xx - yy) * w[13];
    g[1] += 2.f * k.k3c * x * y * w[13];  g[2] += -8.f * k.k3c * x * z * w[13];
    g[0] += 2.f * k.k3e * x * z * w[14];  g[1] += -2.f * k.k3e * y * z * w[14];
    g[2] += k.k3e * (xx - yy) * w[14];
    g[0] += -3.f * k.k3a * (xx - yy) * w[15];
    g[1] += 6.f * k.k3a * x * y * w[15];
}

// Per-Gaussian quantities independent of the view.
struct Gauss {
    float mu[3], s[3], q[4], qinv, o;
    float Rq[9], M[9], Sig[6];   // Sig: 00 01 02 11 12 22
};

// Activations of the 11 geometric raw parameters (mean, log-scale, quaternion,
// opacity logit) and the derived rotation, M = R S and Sigma = M M^T.
__device__ __forceinline__ void gauss_from_raw(const float (&raw)[11], Gauss &G) {
#pragma unroll
    for (int i = 0; i < 3; ++i) G.mu[i] = raw[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) G.s[i] = __expf(raw[3 + i]);
    float q[4], qq = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) { q[i] = raw[6 + i]; qq += q[i] * q[i]; }
    G.qinv = rsqrtf(qq);
#pragma unroll
    for (int i = 0; i < 4; ++i) G.q[i] = q[i] * G.qinv;
    G.o = 1.f / (1.f + __expf(-raw[10]));
    const float w = G.q[0], x = G.q[1], y = G.q[2], z = G.q[3];
    G.Rq[0] = 1.f - 2.f * (y * y + z * z); G.Rq[1] = 2.f * (x * y - w * z); G.Rq[2] = 2.f * (x * z + w * y);
    G.Rq[3] = 2.f * (x * y + w * z); G.Rq[4] = 1.f - 2.f * (x * x + z * z); G.Rq[5] = 2.f * (y * z - w * x);
    G.Rq[6] = 2.f * (x * z - w * y); G.Rq[7] = 2.f * (y * z + w * x); G.Rq[8] = 1.f - 2.f * (x * x + y * y);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) G.M[3 * i + j] = G.Rq[3 * i + j] * G.s[j];
    auto dot3 = [&](int a, int b) {
        return G.M[3 * a] * G.M[3 * b] + G.M[3 * a + 1] * G.M[3 * b + 1] + G.M[3 * a + 2] * G.M[3 * b + 2];
    };
    G.Sig[0] = dot3(0, 0); G.Sig[1] = dot3(0, 1); G.Sig[2] = dot3(0, 2);
    G.Sig[3] = dot3(1, 1); G.Sig[4] = dot3(1, 2); G.Sig[5] = dot3(2, 2);
}

__device__ __forceinline__ void load_gauss(const float *__restrict__ P, int64_t n_cap, int64_t g,
                                           Gauss &G) {
    float raw[11];
#pragma unroll
    for (int i = 0; i < 11; ++i) raw[i] = P[int64_t(i) * n_cap + g];
    gauss_from_raw(raw, G);
}

// View-dependent projection of one Gaussian.
struct Proj2 {
    float xc[3], ub, vb;
    bool clampx, clampy;
    float T[6];      // J W, 2x3
    float cov[3];    // undilated 2D covariance 00 01 11
    double md[2];    // 2D mean (pixels)
};

__device__ __forceinline__ bool project(const Gauss &G, const Cam &c, float znear, Proj2 &p) {
    // Camera-frame mean and 2D mean in FP64: their rounding would otherwise move
    // every pixel offset of a large image by up to 1e-3 px.
    double xd[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        xd[i] = double(c.R[3 * i]) * G.mu[0] + double(c.R[3 * i + 1]) * G.mu[1] +
                double(c.R[3 * i + 2]) * G.mu[2] + double(c.t[i]);
#pragma unroll
    for (int i = 0; i < 3; ++i) p.xc[i] = float(xd[i]);
    const float z = p.xc[2];
    if (!(z > znear)) return false;
    const double ud = xd[0] / xd[2], vd = xd[1] / xd[2];
    p.md[0] = double(c.fx) * ud + double(c.cx);
    p.md[1] = double(c.fy) * vd + double(c.cy);
    const float iz = 1.f / z;
    const float u = float(ud), v = float(vd);
    p.ub = fminf(fmaxf(u, -c.limx), c.limx);
    p.vb = fminf(fmaxf(v, -c.limy), c.limy);
    p.clampx = (u < -c.limx) || (u > c.limx);
    p.clampy = (v < -c.limy) || (v > c.limy);
    const float J00 = c.fx * iz, J02 = -c.fx * p.ub * iz;
    const float J11 = c.fy * iz, J12 = -c.fy * p.vb * iz;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        p.T[j] = J00 * c.R[j] + J02 * c.R[6 + j];
        p.T[3 + j] = J11 * c.R[3 + j] + J12 * c.R[6 + j];
    }
    // T Sigma T^T
    const float *S = G.Sig;
    float TS[6];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const float a = p.T[3 * r], b = p.T[3 * r + 1], d = p.T[3 * r + 2];
        TS[3 * r + 0] = a * S[0] + b * S[1] + d * S[2];
        TS[3 * r + 1] = a * S[1] + b * S[3] + d * S[4];
        TS[3 * r + 2] = a * S[2] + b * S[4] + d * S[5];
    }
    p.cov[0] = TS[0] * p.T[0] + TS[1] * p.T[1] + TS[2] * p.T[2];
    p.cov[1] = TS[0] * p.T[3] + TS[1] * p.T[4] + TS[2] * p.T[5];
    p.cov[2] = TS[3] * p.T[3] + TS[4] * p.T[4] + TS[5] * p.T[5];
    return true;
}

// Views up to which the optimiser kernel also computes the next records.
constexpr int kFuseProjectionViews = 2;

// Projection records of Gaussian g for every view (see gs_preprocess).
__device__ __forceinline__ void preprocess_one(const gs_settings &s, const float *P, int64_t n_cap,
                                               int64_t g, const gs_view *__restrict__ views,
                                               int32_t n_views, const Proj &out) {
    Gauss G;
    load_gauss(P, n_cap, g, G);
    float sh[16][3];
    const int nk = (s.sh_degree + 1) * (s.sh_degree + 1);
#pragma unroll
    for (int k = 0; k < 16; ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) sh[k][ch] = (k < nk) ? P[(11 + 3 * k + ch) * n_cap + g] : 0.f;
    for (int v = 0; v < n_views; ++v) {
        const int64_t r = int64_t(v) * n_cap + g;
        const Cam c = load_cam(views[v], s.fov_clamp);
        Proj2 p;
        if (!project(G, c, s.znear, p)) {
            out.mean[r] = make_double2(0.0, 0.0);
            out.cov_o[r] = make_float4(0.f, 0.f, 0.f, 0.f);
            out.rgb_z[r] = make_float4(0.f, 0.f, 0.f, 0.f);
            continue;
        }
        float d[3] = {G.mu[0] - c.C[0], G.mu[1] - c.C[1], G.mu[2] - c.C[2]};
        const float dinv = rsqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        float Y[16];
        sh_eval(s.sh_degree, d[0] * dinv, d[1] * dinv, d[2] * dinv, Y);
        float rgb[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float acc = 0.5f;
#pragma unroll
            for (int k = 0; k < 16; ++k) acc += Y[k] * sh[k][ch];
            rgb[ch] = fmaxf(acc, 0.f);
        }
        out.mean[r] = make_double2(p.md[0], p.md[1]);
        out.cov_o[r] = make_float4(p.cov[0], p.cov[1], p.cov[2], G.o);
        out.rgb_z[r] = make_float4(rgb[0], rgb[1], rgb[2], p.xc[2]);
    }
}

// Records of Gaussian g (activated geometry G) for every view, one colour
// channel's coefficients live at a time: channels are read from P, except
// channel 2 when keep2 is given (keep2[k * kTilePix], coefficient k).  Same
// arithmetic in the same order as preprocess_one, so the records are
// identical.
__device__ __forceinline__ void project_records(const gs_settings &s, const float *P, int64_t n_cap,
                                                int64_t g, const Gauss &G, const float *keep2,
                                                const gs_view *__restrict__ views, int32_t n_views,
                                                const Proj &out) {
    const int nk = (s.sh_degree + 1) * (s.sh_degree + 1);
    for (int v = 0; v < n_views; ++v) {
        const int64_t r = int64_t(v) * n_cap + g;
        const Cam c = load_cam(views[v], s.fov_clamp);
        Proj2 p;
        if (!project(G, c, s.znear, p)) {
            out.mean[r] = make_double2(0.0, 0.0);
            out.cov_o[r] = make_float4(0.f, 0.f, 0.f, 0.f);
            out.rgb_z[r] = make_float4(0.f, 0.f, 0.f, 0.f);
            continue;
        }
        float d[3] = {G.mu[0] - c.C[0], G.mu[1] - c.C[1], G.mu[2] - c.C[2]};
        const float dinv = rsqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        float Y[16];
        sh_eval(s.sh_degree, d[0] * dinv, d[1] * dinv, d[2] * dinv, Y);
        float rgb[3];
#pragma unroll 1
        for (int ch = 0; ch < 3; ++ch) {
            float acc = 0.5f;
            if (keep2 && ch == 2) {
#pragma unroll
                for (int k = 0; k < 16; ++k) acc += Y[k] * ((k < nk) ? keep2[k * kTilePix] : 0.f);
            } else {
#pragma unroll
                for (int k = 0; k < 16; ++k) acc += Y[k] * ((k < nk) ? P[(11 + 3 * k + ch) * n_cap + g] : 0.f);
            }
            rgb[ch] = fmaxf(acc, 0.f);
        }
        out.mean[r] = make_double2(p.md[0], p.md[1]);
        out.cov_o[r] = make_float4(p.cov[0], p.cov[1], p.cov[2], G.o);
        out.rgb_z[r] = make_float4(rgb[0], rgb[1], rgb[2], p.xc[2]);
    }
}

__device__ __forceinline__ void preprocess_one_lean(const gs_settings &s, const float *P, int64_t n_cap,
                                                    int64_t g, const gs_view *__restrict__ views,
                                                    int32_t n_views, const Proj &out) {
    Gauss G;
    load_gauss(P, n_cap, g, G);
    project_records(s, P, n_cap, g, G, nullptr, views, n_views, out);
}

// Checked mode: a column with a non-finite parameter, or whose record holds a
// non-finite value, gets culled records (the record of a Gaussian behind the
// near plane) for every view, and the status word learns of it.
__device__ __forceinline__ void guard_records(const gs_settings &s, const float *P, int64_t n_cap,
                                              int64_t g, int32_t n_views, const Proj &out) {
    bool bad = false;
    for (int r = 0; r < kRows; ++r) bad |= !isfinite(P[int64_t(r) * n_cap + g]);
    for (int v = 0; v < n_views && !bad; ++v) {
        const int64_t r = int64_t(v) * n_cap + g;
        const double2 m = out.mean[r];
        const float4 a = out.cov_o[r], b = out.rgb_z[r];
        bad |= !(isfinite(m.x) && isfinite(m.y) && isfinite(a.x) && isfinite(a.y) && isfinite(a.z) &&
                 isfinite(a.w) && isfinite(b.x) && isfinite(b.y) && isfinite(b.z) && isfinite(b.w));
    }
    if (bad) {
        for (int v = 0; v < n_views; ++v) {
            const int64_t r = int64_t(v) * n_cap + g;
            out.mean[r] = make_double2(0.0, 0.0);
            out.cov_o[r] = make_float4(0.f, 0.f, 0.f, 0.f);
            out.rgb_z[r] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
    report_numeric(s.status, bad);
}

__global__ void __launch_bounds__(256) preprocess_kernel(gs_settings s, const float *__restrict__ P,
                                                         int64_t n, int64_t n_cap,
                                                         const gs_view *__restrict__ views,
                                                         int32_t n_views, Proj out) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= n) return;
    preprocess_one(s, P, n_cap, g, views, n_views, out);
    if (s.checked) guard_records(s, P, n_cap, g, n_views, out);
}

// Gradient sinks of the projection backward: accumulate into a gradient
// buffer, or apply the Adam update to the parameter right away (the gradient
// then never leaves registers).  Both take a group of rows (first, stride,
// count) so every load of the group is issued before the first store.
struct GradSink {
    float *__restrict__ grad;
    uint32_t *status;   // checked mode: non-finite gradients are reported here (else NULL)
    struct Scale {};
    __device__ __forceinline__ Scale prepare() const { return {}; }
    static constexpr int kKeepRows = 1;   // no colour rows kept (see AdamSink)
    template <int N>
    __device__ __forceinline__ void group(int first, int stride, int64_t g, int64_t n_cap,
                                          float (&val)[N], const float (&)[N], Scale) const {
        float cur[N];
#pragma unroll
        for (int j = 0; j < N; ++j) cur[j] = grad[int64_t(first + j * stride) * n_cap + g];
#pragma unroll
        for (int j = 0; j < N; ++j) grad[int64_t(first + j * stride) * n_cap + g] = cur[j] + val[j];
        if (status) {
            bool bad = false;
#pragma unroll
            for (int j = 0; j < N; ++j) bad |= !isfinite(val[j]);
            if (bad) atomicOr(status, GS_STATUS_NUMERIC);
        }
    }
    __device__ __forceinline__ void untouched(int64_t, int64_t, Scale) const {}
    __device__ __forceinline__ void finish(const gs_settings &, int64_t, int64_t, const gs_view *,
                                           int32_t) const {}
    __device__ __forceinline__ void finish_updated(const gs_settings &, int64_t, int64_t,
                                                   const gs_view *, int32_t, const float (&)[11],
                                                   const float *) const {}
};

struct AdamSink {
    float *p;   // the parameter store, also read by the kernel through its P argument
    float *__restrict__ m;
    float *__restrict__ v;
    uint32_t *status;   // checked mode: non-finite gradients or updates are reported here (else NULL)
    LrRows lr;
    float b1, omb1, b2, omb2, eps, ibc1, isqbc2;
    // Device step counter (graph replay): when set, the bias corrections come
    // from *d_step with ln(beta) given; 1 - beta^t = -expm1(t ln beta).
    const int32_t *d_step;
    float lnb1, lnb2;
    // Bias corrections of this step.  Returned rather than stored: the sink
    // stays a read-only kernel argument, so the per-row learning rates are
    // read from the argument segment instead of a private copy in scratch.
    struct Scale {
        float ibc1, isqbc2;
    };
    __device__ __forceinline__ Scale prepare() const {
        if (d_step) {
            const float t = float(*d_step);
            return {1.f / -expm1f(t * lnb1), rsqrtf(-expm1f(t * lnb2))};
        }
        return {ibc1, isqbc2};
    }
    // pcur holds the rows' current values (already loaded by the caller); the
    // updated parameters replace the gradients in gv.
    static constexpr int kKeepRows = 16;   // one colour channel's coefficients kept in LDS
    template <int N>
    __device__ __forceinline__ void group(int first, int stride, int64_t g, int64_t n_cap,
                                          float (&gv)[N], const float (&pcur)[N], Scale sc) const {
        float pp[N], mm[N], vv[N];
        bool bad = false;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const int64_t i = int64_t(first + j * stride) * n_cap + g;
            pp[j] = pcur[j];
            mm[j] = m[i];
            vv[j] = v[i];
            if (status) bad |= !isfinite(gv[j]);
        }
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const int64_t i = int64_t(first + j * stride) * n_cap + g;
            const float mv = b1 * mm[j] + omb1 * gv[j];
            const float vq = b2 * vv[j] + omb2 * gv[j] * gv[j];
            m[i] = mv;
            v[i] = vq;
            // hardware sqrt and reciprocal (1 ulp each) keep the unrolled group short
            const float den = __builtin_amdgcn_sqrtf(vq) * sc.isqbc2 + eps;
            const float np = pp[j] - lr.lr[first + j * stride] * sc.ibc1 * mv * __builtin_amdgcn_rcpf(den);
            p[i] = np;
            gv[j] = np;
            if (status) bad |= !isfinite(np);
        }
        if (bad) atomicOr(status, GS_STATUS_NUMERIC);
    }
    __device__ __forceinline__ void untouched(int64_t g, int64_t n_cap, Scale sc) const {
#pragma unroll 1
        for (int r = 0; r < kRows; ++r) {
            float z[1] = {0.f};
            const float cur[1] = {p[int64_t(r) * n_cap + g]};
            group(r, 1, g, n_cap, z, cur, sc);
        }
    }
    // Optionally the projection records of the updated Gaussian for the same
    // views (the next iteration's preprocess).  The rows are read back through
    // the pointer they were written with, so the reads follow the writes.
    Proj next;
    __device__ __forceinline__ void finish(const gs_settings &s, int64_t g, int64_t n_cap,
                                           const gs_view *views, int32_t n_views) const {
        if (next.mean) preprocess_one_lean(s, p, n_cap, g, views, n_views, next);
    }
    // The same records with the updated geometry taken from registers and the
    // last colour channel's coefficients from LDS (keep2[k * 256]); only the
    // other two channels are read back.
    __device__ __forceinline__ void finish_updated(const gs_settings &s, int64_t g, int64_t n_cap,
                                                   const gs_view *views, int32_t n_views,
                                                   const float (&raw)[11], const float *keep2) const {
        if (!next.mean) return;
        Gauss G;
        gauss_from_raw(raw, G);
        project_records(s, p, n_cap, g, G, keep2, views, n_views, next);
    }
};

// Chain rule from the accumulated 2D gradients of every view to the 59 raw
// parameter gradients (added to grad).  Geometry is handled first, view by
// view; the colour part then runs one channel at a time so that only that
// channel's 16 SH coefficients and their gradients are live.
template <class Sink>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) project_backward_kernel(
    gs_settings s, const float *P, int64_t n, int64_t n_cap,
    const gs_view *__restrict__ views, int32_t n_views, const float *__restrict__ acc,
    int64_t records, Sink sink) {
    __shared__ float keep2[Sink::kKeepRows][256];   // updated coefficients of colour channel 2
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const typename Sink::Scale sc = sink.prepare();
    const int nk = (s.sh_degree + 1) * (s.sh_degree + 1);
    float gmu[3] = {0, 0, 0}, gop = 0.f;
    float dSig[6] = {0, 0, 0, 0, 0, 0};   // summed over views: 00 01 02 11 12 22 (matrix entries)
    float mu[3];
    bool any_view = false;

    {   // 1. geometry, view by view: 2D mean and covariance back to mean and Sigma
        Gauss G;
        load_gauss(P, n_cap, g, G);
        mu[0] = G.mu[0]; mu[1] = G.mu[1]; mu[2] = G.mu[2];
        for (int v = 0; v < n_views; ++v) {
            const int64_t r = int64_t(v) * n_cap + g;
            float a[kAccRows];
#pragma unroll
            for (int i = 0; i < kAccRows; ++i) a[i] = acc[r * kAccRows + i];
            bool any = false;
#pragma unroll
            for (int i = 0; i < kAccRows; ++i) any |= (a[i] != 0.f);
            if (!any) continue;
            any_view = true;
            const Cam c = load_cam(views[v], s.fov_clamp);
            Proj2 p;
            if (!project(G, c, s.znear, p)) continue;
            const float z = p.xc[2], iz = 1.f / z, iz2 = iz * iz;
            const float G00 = a[2], G01 = a[3], G11 = a[4];
            {   // dL/dSigma = T^T G T
                float GT[6];
#pragma unroll
                for (int jj = 0; jj < 3; ++jj) {
                    GT[jj] = G00 * p.T[jj] + G01 * p.T[3 + jj];
                    GT[3 + jj] = G01 * p.T[jj] + G11 * p.T[3 + jj];
                }
                auto e = [&](int ii, int jj) { return p.T[ii] * GT[jj] + p.T[3 + ii] * GT[3 + jj]; };
                dSig[0] += e(0, 0); dSig[1] += e(0, 1); dSig[2] += e(0, 2);
                dSig[3] += e(1, 1); dSig[4] += e(1, 2); dSig[5] += e(2, 2);
            }
            // dL/dT = 2 G T Sigma; dL/dJ = dL/dT W^T
            float TS[6];
            {
                const float *S = G.Sig;
#pragma unroll
                for (int r2 = 0; r2 < 2; ++r2) {
                    const float a0 = p.T[3 * r2], b0 = p.T[3 * r2 + 1], d0 = p.T[3 * r2 + 2];
                    TS[3 * r2 + 0] = a0 * S[0] + b0 * S[1] + d0 * S[2];
                    TS[3 * r2 + 1] = a0 * S[1] + b0 * S[3] + d0 * S[4];
                    TS[3 * r2 + 2] = a0 * S[2] + b0 * S[4] + d0 * S[5];
                }
            }
            float dT[6];
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) {
                dT[jj] = 2.f * (G00 * TS[jj] + G01 * TS[3 + jj]);
                dT[3 + jj] = 2.f * (G01 * TS[jj] + G11 * TS[3 + jj]);
            }
            const float dJ00 = dT[0] * c.R[0] + dT[1] * c.R[1] + dT[2] * c.R[2];
            const float dJ02 = dT[0] * c.R[6] + dT[1] * c.R[7] + dT[2] * c.R[8];
            const float dJ11 = dT[3] * c.R[3] + dT[4] * c.R[4] + dT[5] * c.R[5];
            const float dJ12 = dT[3] * c.R[6] + dT[4] * c.R[7] + dT[5] * c.R[8];
            float gx[3] = {0.f, 0.f, 0.f};
            // J00 = fx/z, J11 = fy/z, J02 = -fx ub/z, J12 = -fy vb/z
            gx[2] += -(dJ00 * c.fx + dJ11 * c.fy) * iz2 + (dJ02 * c.fx * p.ub + dJ12 * c.fy * p.vb) * iz2;
            if (!p.clampx) {
                gx[0] += -dJ02 * c.fx * iz2;
                gx[2] += dJ02 * c.fx * p.xc[0] * iz2 * iz;
            }
            if (!p.clampy) {
                gx[1] += -dJ12 * c.fy * iz2;
                gx[2] += dJ12 * c.fy * p.xc[1] * iz2 * iz;
            }
            // 2D mean (fx x/z + cx, fy y/z + cy)
            gx[0] += a[0] * c.fx * iz;
            gx[1] += a[1] * c.fy * iz;
            gx[2] += -(a[0] * c.fx * p.xc[0] + a[1] * c.fy * p.xc[1]) * iz2;
#pragma unroll
            for (int ii = 0; ii < 3; ++ii)
                gmu[ii] += c.R[ii] * gx[0] + c.R[3 + ii] * gx[1] + c.R[6 + ii] * gx[2];
            gop += a[5];
        }
    }
    if (!any_view) {   // no view touched this Gaussian: zero gradient
        sink.untouched(g, n_cap, sc);
        sink.finish(s, g, n_cap, views, n_views);
        return;
    }

    // 2. colour, one channel at a time: rgb = max(0, raw), raw = 0.5 + sum_k Y_k(d) sh_k
#pragma unroll 1
    for (int ch = 0; ch < 3; ++ch) {
        // the rows' stored values (the optimiser step needs them for every k);
        // the colour uses the first nk
        float shv[16], sh[16], gsh[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            shv[k] = P[(11 + 3 * k + ch) * n_cap + g];
            sh[k] = (k < nk) ? shv[k] : 0.f;
            gsh[k] = 0.f;
        }
        for (int v = 0; v < n_views; ++v) {
            const int64_t r = int64_t(v) * n_cap + g;
            const float drgb = acc[r * kAccRows + 6 + ch];
            if (drgb == 0.f) continue;
            const Cam c = load_cam(views[v], s.fov_clamp);
            float d[3] = {mu[0] - c.C[0], mu[1] - c.C[1], mu[2] - c.C[2]};
            const float dinv = rsqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const float dx = d[0] * dinv, dy = d[1] * dinv, dz = d[2] * dinv;
            float Y[16];
            sh_eval(s.sh_degree, dx, dy, dz, Y);
            float raw = 0.5f;
#pragma unroll
            for (int k = 0; k < 16; ++k) raw += Y[k] * sh[k];
            if (raw < 0.f) continue;   // clamped colour passes no gradient
#pragma unroll
            for (int k = 0; k < 16; ++k) gsh[k] += Y[k] * drgb;
            float wk[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) wk[k] = drgb * sh[k];
            float gd[3];
            sh_grad(s.sh_degree, dx, dy, dz, wk, gd);
            // unit-vector normalisation: (I - d d^T) / |mu - C|
            const float dot = gd[0] * dx + gd[1] * dy + gd[2] * dz;
            gmu[0] += (gd[0] - dx * dot) * dinv;
            gmu[1] += (gd[1] - dy * dot) * dinv;
            gmu[2] += (gd[2] - dz * dot) * dinv;
        }
        // four groups of four rows: enough loads in flight, few registers
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float part[4] = {gsh[4 * q], gsh[4 * q + 1], gsh[4 * q + 2], gsh[4 * q + 3]};
            const float cur[4] = {shv[4 * q], shv[4 * q + 1], shv[4 * q + 2], shv[4 * q + 3]};
            sink.group(11 + ch + 12 * q, 3, g, n_cap, part, cur, sc);
            if (Sink::kKeepRows == 16 && ch == 2) {
#pragma unroll
                for (int j = 0; j < 4; ++j) keep2[(4 * q + j) % Sink::kKeepRows][threadIdx.x] = part[j];
            }
        }
    }

    // 3. Sigma = M M^T, M = Rq diag(s): dM = 2 dSigma M (dSigma symmetric).
    // The 11 geometric parameters are reloaded (SH rows may have been updated
    // in place; these rows have not).
    float raw[11];
#pragma unroll
    for (int i = 0; i < 11; ++i) raw[i] = P[int64_t(i) * n_cap + g];
    Gauss G;
    gauss_from_raw(raw, G);
    const float D[9] = {dSig[0], dSig[1], dSig[2], dSig[1], dSig[3], dSig[4], dSig[2], dSig[4], dSig[5]};
    float dM[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
            dM[3 * i + jj] = 2.f * (D[3 * i] * G.M[jj] + D[3 * i + 1] * G.M[3 + jj] + D[3 * i + 2] * G.M[6 + jj]);
    float dR[9], gls[3];
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
        float acc_s = 0.f;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            acc_s += dM[3 * i + jj] * G.Rq[3 * i + jj];
            dR[3 * i + jj] = dM[3 * i + jj] * G.s[jj];
        }
        gls[jj] = acc_s * G.s[jj];   // d/d log-scale
    }
    float gq[4];
    {
        const float w = G.q[0], x = G.q[1], y = G.q[2], z = G.q[3];
        float dq[4];
        dq[0] = 2.f * (z * (dR[3] - dR[1]) + y * (dR[2] - dR[6]) + x * (dR[7] - dR[5]));
        dq[1] = 2.f * (y * (dR[1] + dR[3]) + z * (dR[2] + dR[6]) + w * (dR[7] - dR[5]) -
                       2.f * x * (dR[4] + dR[8]));
        dq[2] = 2.f * (x * (dR[1] + dR[3]) + w * (dR[2] - dR[6]) + z * (dR[5] + dR[7]) -
                       2.f * y * (dR[0] + dR[8]));
        dq[3] = 2.f * (w * (dR[3] - dR[1]) + x * (dR[2] + dR[6]) + y * (dR[5] + dR[7]) -
                       2.f * z * (dR[0] + dR[4]));
        const float dot = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
#pragma unroll
        for (int i = 0; i < 4; ++i) gq[i] = (dq[i] - G.q[i] * dot) * G.qinv;
    }
    // d o / d logit = o (1 - o); for o > 1/2, 1 - o = e^-logit o avoids the
    // cancellation that leaves saturated opacities few significant bits
    const float one_minus_o = G.o > 0.5f ? __expf(-raw[10]) * G.o : 1.f - G.o;
    float geo[11] = {gmu[0], gmu[1], gmu[2], gls[0], gls[1], gls[2],
                     gq[0], gq[1], gq[2], gq[3], gop * G.o * one_minus_o};
    sink.group(0, 1, g, n_cap, geo, raw, sc);
    sink.finish_updated(s, g, n_cap, views, n_views, geo, &keep2[0][threadIdx.x]);
}

// Element at byte offset `off` of row `row` of a [rows][n_cap] array: the row
// base is uniform and the offset a 32-bit lane value, so a load or store takes
// one offset register instead of a 64-bit address per row.
template <class T>
__device__ __forceinline__ T &at_row(T *base, int64_t row, int64_t n_cap, uint32_t off) {
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return *reinterpret_cast<T *>(reinterpret_cast<B *>(base + row * n_cap) + off);
}

// AdamSink::group with 32-bit offsets (same arithmetic).
template <int N>
__device__ __forceinline__ void adam_rows(const AdamSink &a, int first, int stride, int64_t n_cap,
                                          uint32_t off, float (&gv)[N], const float (&pcur)[N],
                                          AdamSink::Scale sc) {
    float mm[N], vv[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        mm[j] = at_row(a.m, first + j * stride, n_cap, off);
        vv[j] = at_row(a.v, first + j * stride, n_cap, off);
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const int row = first + j * stride;
        const float mv = a.b1 * mm[j] + a.omb1 * gv[j];
        const float vq = a.b2 * vv[j] + a.omb2 * gv[j] * gv[j];
        at_row(a.m, row, n_cap, off) = mv;
        at_row(a.v, row, n_cap, off) = vq;
        const float den = __builtin_amdgcn_sqrtf(vq) * sc.isqbc2 + a.eps;
        const float np = pcur[j] - a.lr.lr[row] * sc.ibc1 * mv * __builtin_amdgcn_rcpf(den);
        at_row(a.p, row, n_cap, off) = np;
        gv[j] = np;
    }
}

// The same chain rule fused with Adam and the next records for one view, with
// every parameter loaded once: the 48 colour coefficients stay in registers
// from their load (the view-direction gradient needs them all) through their
// update to the colour of the next record, and the 11 geometric rows
// likewise.  Same arithmetic as project_backward_kernel<AdamSink> with one
// view followed by preprocess_one, so updates and records equal theirs.
// Compiled for SH degree 3 (kDeg), the degree of the mapping workloads.
template <int kDeg>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) project_adam_one_view_kernel(
    gs_settings s, int64_t n, int64_t n_cap, const gs_view *__restrict__ views,
    const float *__restrict__ acc, AdamSink sink) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= n) return;
    // byte offsets of column g (the launch keeps n_cap below 2^26)
    const uint32_t off = uint32_t(g) * 4u;
    const float *P = sink.p;
    const typename AdamSink::Scale sc = sink.prepare();
    constexpr int nk = (kDeg + 1) * (kDeg + 1);
    const Cam c = load_cam(views[0], s.fov_clamp);
    float raw[11];
#pragma unroll
    for (int i = 0; i < 11; ++i) raw[i] = at_row(P, i, n_cap, off);
    float a[kAccRows];
#pragma unroll
    for (int i = 0; i < kAccRows; ++i) a[i] = at_row(acc, 0, 0, uint32_t(g) * uint32_t(4 * kAccRows) + 4u * i);
    float gmu[3] = {0, 0, 0}, gop = 0.f;
    float dSig[6] = {0, 0, 0, 0, 0, 0};

    // 1. geometry: 2D mean and covariance back to mean and Sigma
    bool any = false;
#pragma unroll
    for (int i = 0; i < 6; ++i) any |= (a[i] != 0.f);
    if (any) {
        Gauss G;
        gauss_from_raw(raw, G);
        Proj2 p;
        if (project(G, c, s.znear, p)) {
            const float z = p.xc[2], iz = 1.f / z, iz2 = iz * iz;
            const float G00 = a[2], G01 = a[3], G11 = a[4];
            {
                float GT[6];
#pragma unroll
                for (int jj = 0; jj < 3; ++jj) {
                    GT[jj] = G00 * p.T[jj] + G01 * p.T[3 + jj];
                    GT[3 + jj] = G01 * p.T[jj] + G11 * p.T[3 + jj];
                }
                auto e = [&](int ii, int jj) { return p.T[ii] * GT[jj] + p.T[3 + ii] * GT[3 + jj]; };
                dSig[0] += e(0, 0); dSig[1] += e(0, 1); dSig[2] += e(0, 2);
                dSig[3] += e(1, 1); dSig[4] += e(1, 2); dSig[5] += e(2, 2);
            }
            float TS[6];
            {
                const float *S = G.Sig;
#pragma unroll
                for (int r2 = 0; r2 < 2; ++r2) {
                    const float a0 = p.T[3 * r2], b0 = p.T[3 * r2 + 1], d0 = p.T[3 * r2 + 2];
                    TS[3 * r2 + 0] = a0 * S[0] + b0 * S[1] + d0 * S[2];
                    TS[3 * r2 + 1] = a0 * S[1] + b0 * S[3] + d0 * S[4];
                    TS[3 * r2 + 2] = a0 * S[2] + b0 * S[4] + d0 * S[5];
                }
            }
            float dT[6];
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) {
                dT[jj] = 2.f * (G00 * TS[jj] + G01 * TS[3 + jj]);
                dT[3 + jj] = 2.f * (G01 * TS[jj] + G11 * TS[3 + jj]);
            }
            const float dJ00 = dT[0] * c.R[0] + dT[1] * c.R[1] + dT[2] * c.R[2];
            const float dJ02 = dT[0] * c.R[6] + dT[1] * c.R[7] + dT[2] * c.R[8];
            const float dJ11 = dT[3] * c.R[3] + dT[4] * c.R[4] + dT[5] * c.R[5];
            const float dJ12 = dT[3] * c.R[6] + dT[4] * c.R[7] + dT[5] * c.R[8];
            float gx[3] = {0.f, 0.f, 0.f};
            gx[2] += -(dJ00 * c.fx + dJ11 * c.fy) * iz2 + (dJ02 * c.fx * p.ub + dJ12 * c.fy * p.vb) * iz2;
            if (!p.clampx) {
                gx[0] += -dJ02 * c.fx * iz2;
                gx[2] += dJ02 * c.fx * p.xc[0] * iz2 * iz;
            }
            if (!p.clampy) {
                gx[1] += -dJ12 * c.fy * iz2;
                gx[2] += dJ12 * c.fy * p.xc[1] * iz2 * iz;
            }
            gx[0] += a[0] * c.fx * iz;
            gx[1] += a[1] * c.fy * iz;
            gx[2] += -(a[0] * c.fx * p.xc[0] + a[1] * c.fy * p.xc[1]) * iz2;
#pragma unroll
            for (int ii = 0; ii < 3; ++ii)
                gmu[ii] += c.R[ii] * gx[0] + c.R[3 + ii] * gx[1] + c.R[6 + ii] * gx[2];
            gop += a[5];
        }
    }

    // 2. colour: rgb = max(0, raw), raw = 0.5 + sum_k Y_k(d) sh_k, per channel;
    // a channel's coefficients are updated in place once its gradient is formed
    float shv[48];   // coefficient k of channel ch at 3k + ch
#pragma unroll
    for (int i = 0; i < 48; ++i) shv[i] = at_row(P, 11 + i, n_cap, off);
    {
        float d[3] = {raw[0] - c.C[0], raw[1] - c.C[1], raw[2] - c.C[2]};
        const float dinv = rsqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const float dx = d[0] * dinv, dy = d[1] * dinv, dz = d[2] * dinv;
        float Y[16];
        sh_eval(kDeg, dx, dy, dz, Y);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float drgb = a[6 + ch];
            if (drgb != 0.f) {
                float rawc = 0.5f;
#pragma unroll
                for (int k = 0; k < 16; ++k) rawc += Y[k] * ((k < nk) ? shv[3 * k + ch] : 0.f);
                if (rawc < 0.f) {
                    drgb = 0.f;   // clamped colour passes no gradient
                } else {
                    float wk[16];
#pragma unroll
                    for (int k = 0; k < 16; ++k) wk[k] = drgb * ((k < nk) ? shv[3 * k + ch] : 0.f);
                    float gd[3];
                    sh_grad(kDeg, dx, dy, dz, wk, gd);
                    const float dot = gd[0] * dx + gd[1] * dy + gd[2] * dz;
                    gmu[0] += (gd[0] - dx * dot) * dinv;
                    gmu[1] += (gd[1] - dy * dot) * dinv;
                    gmu[2] += (gd[2] - dz * dot) * dinv;
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float part[4], cur[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    part[j] = drgb != 0.f ? 0.f + Y[4 * q + j] * drgb : 0.f;
                    cur[j] = shv[3 * (4 * q + j) + ch];
                }
                adam_rows(sink, 11 + ch + 12 * q, 3, n_cap, off, part, cur, sc);
#pragma unroll
                for (int j = 0; j < 4; ++j) shv[3 * (4 * q + j) + ch] = part[j];
            }
        }
    }

    // 3. Sigma = M M^T, M = Rq diag(s)
    float geo[11];
    {
        Gauss G;
        gauss_from_raw(raw, G);
        const float D[9] = {dSig[0], dSig[1], dSig[2], dSig[1], dSig[3], dSig[4], dSig[2], dSig[4], dSig[5]};
        float dM[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int jj = 0; jj < 3; ++jj)
                dM[3 * i + jj] =
                    2.f * (D[3 * i] * G.M[jj] + D[3 * i + 1] * G.M[3 + jj] + D[3 * i + 2] * G.M[6 + jj]);
        float dR[9], gls[3];
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
            float acc_s = 0.f;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                acc_s += dM[3 * i + jj] * G.Rq[3 * i + jj];
                dR[3 * i + jj] = dM[3 * i + jj] * G.s[jj];
            }
            gls[jj] = acc_s * G.s[jj];
        }
        float gq[4];
        {
            const float w = G.q[0], x = G.q[1], y = G.q[2], z = G.q[3];
            float dq[4];
            dq[0] = 2.f * (z * (dR[3] - dR[1]) + y * (dR[2] - dR[6]) + x * (dR[7] - dR[5]));
            dq[1] = 2.f * (y * (dR[1] + dR[3]) + z * (dR[2] + dR[6]) + w * (dR[7] - dR[5]) -
                           2.f * x * (dR[4] + dR[8]));
            dq[2] = 2.f * (x * (dR[1] + dR[3]) + w * (dR[2] - dR[6]) + z * (dR[5] + dR[7]) -
                           2.f * y * (dR[0] + dR[8]));
            dq[3] = 2.f * (w * (dR[3] - dR[1]) + x * (dR[2] + dR[6]) + y * (dR[5] + dR[7]) -
                           2.f * z * (dR[0] + dR[4]));
            const float dot = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
#pragma unroll
            for (int i = 0; i < 4; ++i) gq[i] = (dq[i] - G.q[i] * dot) * G.qinv;
        }
        const float one_minus_o = G.o > 0.5f ? __expf(-raw[10]) * G.o : 1.f - G.o;
        const float gv[11] = {gmu[0], gmu[1], gmu[2], gls[0], gls[1], gls[2],
                              gq[0], gq[1], gq[2], gq[3], gop * G.o * one_minus_o};
#pragma unroll
        for (int i = 0; i < 11; ++i) geo[i] = gv[i];
    }
    adam_rows(sink, 0, 1, n_cap, off, geo, raw, sc);

    // 4. the next record (as preprocess_one) from the updated registers
    if (!sink.next.mean) return;
    Gauss G;
    gauss_from_raw(geo, G);
    Proj2 p;
    const uint32_t off16 = uint32_t(g) * 16u;
    if (!project(G, c, s.znear, p)) {
        at_row(sink.next.mean, 0, 0, off16) = make_double2(0.0, 0.0);
        at_row(sink.next.cov_o, 0, 0, off16) = make_float4(0.f, 0.f, 0.f, 0.f);
        at_row(sink.next.rgb_z, 0, 0, off16) = make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    float d[3] = {G.mu[0] - c.C[0], G.mu[1] - c.C[1], G.mu[2] - c.C[2]};
    const float dinv = rsqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    float Y[16];
    sh_eval(kDeg, d[0] * dinv, d[1] * dinv, d[2] * dinv, Y);
    float rgb[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float acc_c = 0.5f;
#pragma unroll
        for (int k = 0; k < 16; ++k) acc_c += Y[k] * ((k < nk) ? shv[3 * k + ch] : 0.f);
        rgb[ch] = fmaxf(acc_c, 0.f);
    }
    at_row(sink.next.mean, 0, 0, off16) = make_double2(p.md[0], p.md[1]);
    at_row(sink.next.cov_o, 0, 0, off16) = make_float4(p.cov[0], p.cov[1], p.cov[2], G.o);
    at_row(sink.next.rgb_z, 0, 0, off16) = make_float4(rgb[0], rgb[1], rgb[2], p.xc[2]);
}

gs_status launch_project_backward(const gs_settings &s, const float *params, int64_t n,
                                  int64_t n_cap, const gs_view *views, int32_t n_views,
                                  const float *acc, float *grad, hipStream_t st) {
    if (n == 0) return GS_OK;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(project_backward_kernel<GradSink>, dim3(blocks), dim3(256), 0, st, s, params, n,
                       n_cap, views, n_views, acc, int64_t(n_views) * n_cap,
                       GradSink{grad, s.checked ? s.status : nullptr});
    GS_CHECK_LAUNCH();
    return GS_OK;
}

gs_status launch_project_backward_adam(const gs_settings &s, float *params, int64_t n, int64_t n_cap,
                                       const gs_view *views, int32_t n_views, const float *acc,
                                       float *m, float *v, const float *lr_rows, double beta1,
                                       double beta2, double eps, int32_t step, const int32_t *d_step,
                                       void *proj_out, hipStream_t st) {
    if (n == 0) return GS_OK;
    // The next records are computed inside the optimiser kernel for few views;
    // with many views the separate projection kernel (parameters read once,
    // colour coefficients kept in registers across views) is faster.
    const Proj next = proj_out ? proj_at(proj_out, int64_t(n_views) * n_cap) : Proj{nullptr, nullptr, nullptr};
    // (in checked mode the next records come from the guarded projection kernel)
    const bool fuse_next = proj_out && n_views <= kFuseProjectionViews && !s.checked;
    AdamSink a;
    a.next = fuse_next ? next : Proj{nullptr, nullptr, nullptr};
    a.p = params;
    a.m = m;
    a.v = v;
    a.status = s.checked ? s.status : nullptr;
    for (int r = 0; r < kRows; ++r) a.lr.lr[r] = lr_rows[r];
    a.b1 = float(beta1);
    a.omb1 = float(1.0 - beta1);
    a.b2 = float(beta2);
    a.omb2 = float(1.0 - beta2);
    a.eps = float(eps);
    a.d_step = d_step;
    a.lnb1 = float(std::log(beta1));
    a.lnb2 = float(std::log(beta2));
    const int32_t t = step > 0 ? step : 1;
    a.ibc1 = float(1.0 / (1.0 - std::pow(beta1, t)));
    a.isqbc2 = float(1.0 / std::sqrt(1.0 - std::pow(beta2, t)));
    const int64_t blocks = (n + 255) / 256;
    if (n_views == 1 && !s.checked && s.sh_degree == 3 && n_cap <= (int64_t(1) << 26))
        hipLaunchKernelGGL(project_adam_one_view_kernel<3>, dim3(blocks), dim3(256), 0, st, s, n, n_cap, views,
                           acc, a);
    else
        hipLaunchKernelGGL(project_backward_kernel<AdamSink>, dim3(blocks), dim3(256), 0, st, s, params, n,
                           n_cap, views, n_views, acc, int64_t(n_views) * n_cap, a);
    if (proj_out && !fuse_next)
        hipLaunchKernelGGL(preprocess_kernel, dim3(blocks), dim3(256), 0, st, s, params, n, n_cap, views,
                           n_views, next);
    GS_CHECK_LAUNCH();
    return GS_OK;
}

}  // namespace gs

extern "C" gs_status gs_preprocess(const gs_settings *s, const float *params, int64_t n,
                                   int64_t n_cap, const gs_view *views, int32_t n_views,
                                   void *proj_ws, void *stream) {
    if (!gs::valid_settings(s) || !params || !views || !proj_ws || n < 0 || n_cap <= 0 || n > n_cap ||
        n_cap % 64 || n_views <= 0 || int64_t(n_views) * n_cap > gs::kMaxRecords)
        return GS_ERR_INVALID_ARGUMENT;
    if (n == 0) return GS_OK;
    gs::Proj out = gs::proj_at(proj_ws, int64_t(n_views) * n_cap);
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(gs::preprocess_kernel, dim3(blocks), dim3(256), 0,
                       static_cast<hipStream_t>(stream), *s, params, n, n_cap, views, n_views, out);
    GS_CHECK_LAUNCH();
    return GS_OK;
}
