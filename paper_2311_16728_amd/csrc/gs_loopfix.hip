// Loop-closure correction of the primitives (Section 3.5): when a loop is
// closed, keyframes and map points move by similarity corrections and the
// hyper primitives follow.  A similarity x' = s R x + t moves a primitive's
// centre to s R mu + t, turns its frame (q_R * q), scales it (log-scale +
// ln s), keeps its opacity and turns its view-dependent colour: the new
// colour along d is the old one along R^T d, a linear map of each real-SH
// band, c_l' = D_l(R)^T c_l with Y_l(R^T d) = D_l(R) Y_l(d).
//
// D_l(R)^T is obtained by collocation: at 2l+1 fixed directions d_k the
// band's values A_l[k][i] = Y_li(d_k) form an invertible matrix (the set below
// keeps every condition number under 4), and B_l[k][i] = Y_li(R^T d_k) =
// (A_l D_l^T)[k][i], so D_l^T = A_l^-1 B_l.  The inverses are constants
// (computed once on the host in double); a setup kernel builds each
// transform's three matrices (9 + 25 + 49 floats) and the per-primitive pass
// is a small mat-vec per colour channel, bound by HBM (58 of the 59 rows read
// and written).

#include "gs_internal.hpp"

#include <cmath>
#include <mutex>
#include <utility>

namespace gs {
namespace {

constexpr int kSimFloats = 104;   // one transform's table entry
// entry layout
constexpr int kSimR = 0, kSimT = 9, kSimS = 12, kSimLogS = 13, kSimQ = 14, kSimValid = 18;
constexpr int kSimM1 = 19, kSimM2 = 28, kSimM3 = 53;   // 9, 25, 49 floats, row-major D_l^T

// Collocation directions (unnormalised integer vectors).
constexpr int kColloc[7][3] = {{1, 2, -3}, {-2, 1, 2}, {3, 2, 3}, {-3, 0, 0},
                               {3, 2, -1}, {1, 2, 2},  {-1, 3, 1}};

struct Colloc {
    float dir[7][3];   // normalised
    float ainv[83];    // A_1^-1 (9), A_2^-1 (25), A_3^-1 (49), row-major
};

// Orthonormal real SH of bands 0..3 (index l*l + l + m), the renderer's basis.
template <class T>
__host__ __device__ __forceinline__ void sh_orthonormal(T x, T y, T z, T Y[16]) {
    const T pi = T(3.14159265358979323846);
    const T k1 = T(0.5) * sqrt(T(3) / pi);
    const T k2a = T(0.5) * sqrt(T(15) / pi), k2b = T(0.25) * sqrt(T(5) / pi);
    const T k2c = T(0.25) * sqrt(T(15) / pi);
    const T k3a = T(0.25) * sqrt(T(35) / (T(2) * pi)), k3b = T(0.5) * sqrt(T(105) / pi);
    const T k3c = T(0.25) * sqrt(T(21) / (T(2) * pi)), k3d = T(0.25) * sqrt(T(7) / pi);
    const T k3e = T(0.25) * sqrt(T(105) / pi);
    const T xx = x * x, yy = y * y, zz = z * z;
    Y[0] = T(0.5) * sqrt(T(1) / pi);
    Y[1] = -k1 * y;
    Y[2] = k1 * z;
    Y[3] = -k1 * x;
    Y[4] = k2a * x * y;
    Y[5] = -k2a * y * z;
    Y[6] = k2b * (T(2) * zz - xx - yy);
    Y[7] = -k2a * x * z;
    Y[8] = k2c * (xx - yy);
    Y[9] = -k3a * y * (T(3) * xx - yy);
    Y[10] = k3b * x * y * z;
    Y[11] = -k3c * y * (T(4) * zz - xx - yy);
    Y[12] = k3d * z * (T(2) * zz - T(3) * xx - T(3) * yy);
    Y[13] = -k3c * x * (T(4) * zz - xx - yy);
    Y[14] = k3e * z * (xx - yy);
    Y[15] = -k3a * x * (xx - T(3) * yy);
}

// In-place inverse of a small matrix (Gauss-Jordan, partial pivoting).
bool invert(double *a, int m) {
    double inv[49];
    for (int i = 0; i < m * m; ++i) inv[i] = (i / m == i % m) ? 1.0 : 0.0;
    for (int c = 0; c < m; ++c) {
        int p = c;
        for (int r = c + 1; r < m; ++r)
            if (std::fabs(a[r * m + c]) > std::fabs(a[p * m + c])) p = r;
        if (std::fabs(a[p * m + c]) < 1e-12) return false;
        for (int j = 0; j < m; ++j) {
            std::swap(a[c * m + j], a[p * m + j]);
            std::swap(inv[c * m + j], inv[p * m + j]);
        }
        const double d = a[c * m + c];
        for (int j = 0; j < m; ++j) { a[c * m + j] /= d; inv[c * m + j] /= d; }
        for (int r = 0; r < m; ++r) {
            if (r == c) continue;
            const double f = a[r * m + c];
            for (int j = 0; j < m; ++j) { a[r * m + j] -= f * a[c * m + j]; inv[r * m + j] -= f * inv[c * m + j]; }
        }
    }
    for (int i = 0; i < m * m; ++i) a[i] = inv[i];
    return true;
}

const Colloc &colloc() {
    static Colloc C;
    static std::once_flag once;
    std::call_once(once, [] {
        double Y[7][16];
        for (int k = 0; k < 7; ++k) {
            const double n = std::sqrt(double(kColloc[k][0] * kColloc[k][0] + kColloc[k][1] * kColloc[k][1] +
                                              kColloc[k][2] * kColloc[k][2]));
            double d[3];
            for (int i = 0; i < 3; ++i) {
                C.dir[k][i] = float(kColloc[k][i] / n);
                d[i] = double(C.dir[k][i]);   // the values the device uses
            }
            sh_orthonormal<double>(d[0], d[1], d[2], Y[k]);
        }
        int at = 0;
        for (int l = 1; l <= 3; ++l) {
            const int m = 2 * l + 1, k0 = l * l;
            double a[49];
            for (int k = 0; k < m; ++k)
                for (int i = 0; i < m; ++i) a[k * m + i] = Y[k][k0 + i];
            invert(a, m);   // the fixed set is invertible (condition numbers 1.8, 3.0, 3.8)
            for (int i = 0; i < m * m; ++i) C.ainv[at + i] = float(a[i]);
            at += m * m;
        }
    });
    return C;
}

__global__ void sim3_setup_kernel(const gs_sim3 *__restrict__ xf, int32_t n_xf, Colloc C,
                                  float *__restrict__ table) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_xf) return;
    float *o = table + int64_t(k) * kSimFloats;
    const gs_sim3 x = xf[k];
    const float qq = x.q[0] * x.q[0] + x.q[1] * x.q[1] + x.q[2] * x.q[2] + x.q[3] * x.q[3];
    const bool valid = x.s > 0.f && qq > 0.f && isfinite(x.s) && isfinite(qq);
    o[kSimValid] = valid ? 1.f : 0.f;
    if (!valid) return;
    const float inv = 1.f / sqrtf(qq);
    const float w = x.q[0] * inv, a = x.q[1] * inv, b = x.q[2] * inv, c = x.q[3] * inv;
    const float R[9] = {1.f - 2.f * (b * b + c * c), 2.f * (a * b - w * c), 2.f * (a * c + w * b),
                        2.f * (a * b + w * c), 1.f - 2.f * (a * a + c * c), 2.f * (b * c - w * a),
                        2.f * (a * c - w * b), 2.f * (b * c + w * a), 1.f - 2.f * (a * a + b * b)};
    for (int i = 0; i < 9; ++i) o[kSimR + i] = R[i];
    for (int i = 0; i < 3; ++i) o[kSimT + i] = x.t[i];
    o[kSimS] = x.s;
    o[kSimLogS] = logf(x.s);
    o[kSimQ + 0] = w; o[kSimQ + 1] = a; o[kSimQ + 2] = b; o[kSimQ + 3] = c;
    // values at R^T d_k
    float B[7][16];
#pragma unroll
    for (int k2 = 0; k2 < 7; ++k2) {
        const float d0 = C.dir[k2][0], d1 = C.dir[k2][1], d2 = C.dir[k2][2];
        const float rx = R[0] * d0 + R[3] * d1 + R[6] * d2;
        const float ry = R[1] * d0 + R[4] * d1 + R[7] * d2;
        const float rz = R[2] * d0 + R[5] * d1 + R[8] * d2;
        sh_orthonormal<float>(rx, ry, rz, B[k2]);
    }
    int at = 0;
    const int dst[3] = {kSimM1, kSimM2, kSimM3};
#pragma unroll
    for (int l = 1; l <= 3; ++l) {
        const int m = 2 * l + 1, k0 = l * l;
#pragma unroll
        for (int i = 0; i < m; ++i)
#pragma unroll
            for (int j = 0; j < m; ++j) {
                float acc = 0.f;
#pragma unroll
                for (int k2 = 0; k2 < m; ++k2) acc += C.ainv[at + i * m + k2] * B[k2][k0 + j];
                o[dst[l - 1] + i * m + j] = acc;
            }
        at += m * m;
    }
}

template <int M>
__device__ __forceinline__ void band(float *__restrict__ P, int64_t n_cap, int64_t g, int ch, int k0,
                                     const float *__restrict__ Mt) {
    float c[M], o[M];
#pragma unroll
    for (int i = 0; i < M; ++i) c[i] = P[int64_t(11 + 3 * (k0 + i) + ch) * n_cap + g];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < M; ++j) acc += Mt[i * M + j] * c[j];
        o[i] = acc;
    }
#pragma unroll
    for (int i = 0; i < M; ++i) P[int64_t(11 + 3 * (k0 + i) + ch) * n_cap + g] = o[i];
}

__global__ void __launch_bounds__(256) sim3_apply_kernel(float *__restrict__ P, int64_t n, int64_t n_cap,
                                                         const int32_t *__restrict__ assign, int32_t n_xf,
                                                         const float *__restrict__ table) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int k = assign ? assign[g] : 0;
    if (k < 0 || k >= n_xf) return;
    const float *T = table + int64_t(k) * kSimFloats;
    if (T[kSimValid] == 0.f) return;
    {
        float mu[3], ls[3], q[4];
#pragma unroll
        for (int i = 0; i < 3; ++i) mu[i] = P[int64_t(i) * n_cap + g];
#pragma unroll
        for (int i = 0; i < 3; ++i) ls[i] = P[int64_t(3 + i) * n_cap + g];
#pragma unroll
        for (int i = 0; i < 4; ++i) q[i] = P[int64_t(6 + i) * n_cap + g];
        const float *R = T + kSimR;
        const float s = T[kSimS], lg = T[kSimLogS];
#pragma unroll
        for (int i = 0; i < 3; ++i)
            P[int64_t(i) * n_cap + g] = s * (R[3 * i] * mu[0] + R[3 * i + 1] * mu[1] + R[3 * i + 2] * mu[2]) +
                                        T[kSimT + i];
#pragma unroll
        for (int i = 0; i < 3; ++i) P[int64_t(3 + i) * n_cap + g] = ls[i] + lg;
        const float aw = T[kSimQ], ax = T[kSimQ + 1], ay = T[kSimQ + 2], az = T[kSimQ + 3];
        const float bw = q[0], bx = q[1], by = q[2], bz = q[3];
        P[6 * n_cap + g] = aw * bw - ax * bx - ay * by - az * bz;
        P[7 * n_cap + g] = aw * bx + ax * bw + ay * bz - az * by;
        P[8 * n_cap + g] = aw * by - ax * bz + ay * bw + az * bx;
        P[9 * n_cap + g] = aw * bz + ax * by - ay * bx + az * bw;
    }
#pragma unroll 1
    for (int ch = 0; ch < 3; ++ch) {
        band<3>(P, n_cap, g, ch, 1, T + kSimM1);
        band<5>(P, n_cap, g, ch, 4, T + kSimM2);
        band<7>(P, n_cap, g, ch, 9, T + kSimM3);
    }
}

}  // namespace
}  // namespace gs

using namespace gs;

extern "C" size_t gs_sim3_workspace_bytes(int32_t n_transforms) {
    return align_up(sizeof(float) * kSimFloats * size_t(n_transforms > 0 ? n_transforms : 1), 256);
}

extern "C" gs_status gs_sim3_apply(float *params, int64_t n, int64_t n_cap, const gs_sim3 *transforms,
                                   int32_t n_transforms, const int32_t *assign, void *ws, void *stream) {
    if (!params || !transforms || !ws || n < 0 || n > n_cap || n_cap % 64 || n_transforms <= 0)
        return GS_ERR_INVALID_ARGUMENT;
    if (n == 0) return GS_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    float *table = static_cast<float *>(ws);
    hipLaunchKernelGGL(sim3_setup_kernel, dim3((n_transforms + 63) / 64), dim3(64), 0, st, transforms,
                       n_transforms, colloc(), table);
    hipLaunchKernelGGL(sim3_apply_kernel, dim3((n + 255) / 256), dim3(256), 0, st, params, n, n_cap, assign,
                       n_transforms, static_cast<const float *>(table));
    GS_CHECK_LAUNCH();
    return GS_OK;
}
