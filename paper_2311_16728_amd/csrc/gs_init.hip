// Initialisation of newly densified primitives (Section 3.3.1: temporary
// primitives are created at inactive 2D keypoints of a new keyframe, placed in
// 3D with the keypoint's depth).  Kernels:
//   features  - network input per keypoint: 7x7 RGB patch of the keyframe image
//               (edge-clamped), depth, keypoint scale, a one-hot of its
//               octave (8), the heuristic's log-scale and log depth,
//               zero-padded to 160, BF16;
//   heuristic - scale = mean distance to the 3 nearest means (existing and
//               new), isotropic, identity rotation, opacity 0.1, colour from
//               the pixel, higher SH zero;
//   decode    - network outputs (corrections to the heuristic's log-scale and
//               SH DC, a camera-frame quaternion, the opacity logit) to
//               world-frame parameters, falling back to the heuristic when the
//               predicted opacity is below 0.01;
//   append    - copy new columns into the parameter store, Adam moments zeroed.
// Keypoints are float4 (u, v, depth, scale) in pixels / metres; scale is
// 1.2^octave.
#include "gs_internal.hpp"

namespace gs {

constexpr int kFeat = 160, kPatch = 7;

__device__ __forceinline__ uint16_t f2bf_init(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

__global__ void __launch_bounds__(256) features_kernel(const float *__restrict__ img, int H, int W,
                                                       const float4 *__restrict__ kp, int B,
                                                       const float *__restrict__ heur,
                                                       uint16_t *__restrict__ x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    const float4 k = kp[i];
    const int cu = int(rintf(k.x)), cv = int(rintf(k.y));
    uint16_t *row = x + int64_t(i) * kFeat;
    int f = 0;
    for (int c = 0; c < 3; ++c)
        for (int dy = -kPatch / 2; dy <= kPatch / 2; ++dy)
            for (int dx = -kPatch / 2; dx <= kPatch / 2; ++dx) {
                const int yy = min(max(cv + dy, 0), H - 1), xx = min(max(cu + dx, 0), W - 1);
                row[f++] = f2bf_init(img[(int64_t(c) * H + yy) * W + xx]);
            }
    row[f++] = f2bf_init(k.z);                                  // depth
    row[f++] = f2bf_init(k.w);                                  // scale
    const int oct = min(max(int(rintf(__logf(fmaxf(k.w, 1.f)) / __logf(1.2f))), 0), 7);
    for (int o = 0; o < 8; ++o) row[f++] = f2bf_init(o == oct ? 1.f : 0.f);
    row[f++] = f2bf_init(heur ? heur[int64_t(3) * B + i] : 0.f);   // heuristic log-scale (metres)
    row[f++] = f2bf_init(logf(k.z));                                 // log depth
    for (; f < kFeat; ++f) row[f] = 0;
}

// 3 nearest neighbours of every new mean among the n existing means and the
// other new means (brute force, existing means streamed through LDS).
__global__ void __launch_bounds__(256) heuristic_kernel(const float *__restrict__ new_mu, const float *__restrict__ new_rgb,
                                                        int B, const float *__restrict__ P, int64_t n,
                                                        int64_t n_cap, float *__restrict__ out) {
    __shared__ float sx[256], sy[256], sz[256];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < B;
    float px = 0, py = 0, pz = 0;
    if (live) { px = new_mu[i]; py = new_mu[B + i]; pz = new_mu[2 * B + i]; }
    float d0 = 3.4e38f, d1 = 3.4e38f, d2 = 3.4e38f;
    auto consider = [&](float d) {
        if (d < d2) {
            if (d < d1) {
                d2 = d1;
                if (d < d0) { d1 = d0; d0 = d; } else { d1 = d; }
            } else {
                d2 = d;
            }
        }
    };
    const int64_t total = n + B;
    for (int64_t base = 0; base < total; base += 256) {
        __syncthreads();
        const int64_t j = base + threadIdx.x;
        if (j < n) {
            sx[threadIdx.x] = P[j]; sy[threadIdx.x] = P[n_cap + j]; sz[threadIdx.x] = P[2 * n_cap + j];
        } else if (j < total) {
            const int64_t q = j - n;
            sx[threadIdx.x] = new_mu[q]; sy[threadIdx.x] = new_mu[B + q]; sz[threadIdx.x] = new_mu[2 * B + q];
        }
        __syncthreads();
        const int cnt = int(min(int64_t(256), total - base));
        if (live)
            for (int t = 0; t < cnt; ++t) {
                if (base + t == n + i) continue;   // itself
                const float dx = sx[t] - px, dy = sy[t] - py, dz = sz[t] - pz;
                consider(dx * dx + dy * dy + dz * dz);
            }
    }
    if (!live) return;
    const float mean_d = (sqrtf(d0) + sqrtf(d1) + sqrtf(d2)) / 3.f;
    const float ls = logf(fmaxf(mean_d, 1e-7f));
    const float c0 = 0.28209479177387814f;   // degree-0 real SH value
    float col[kRows];
    for (int r = 0; r < kRows; ++r) col[r] = 0.f;
    col[0] = px; col[1] = py; col[2] = pz;
    col[3] = col[4] = col[5] = ls;
    col[6] = 1.f;
    col[10] = logf(0.1f / 0.9f);
    for (int c = 0; c < 3; ++c) col[11 + c] = (new_rgb[c * B + i] - 0.5f) / c0;
    for (int r = 0; r < kRows; ++r) out[int64_t(r) * B + i] = col[r];
}

// Rotation matrix (row-major) to unit quaternion (w, x, y, z).
__device__ __forceinline__ void mat_to_quat(const float R[9], float q[4]) {
    const float tr = R[0] + R[4] + R[8];
    if (tr > 0.f) {
        const float s = sqrtf(tr + 1.f) * 2.f;
        q[0] = 0.25f * s; q[1] = (R[7] - R[5]) / s; q[2] = (R[2] - R[6]) / s; q[3] = (R[3] - R[1]) / s;
    } else if (R[0] > R[4] && R[0] > R[8]) {
        const float s = sqrtf(1.f + R[0] - R[4] - R[8]) * 2.f;
        q[0] = (R[7] - R[5]) / s; q[1] = 0.25f * s; q[2] = (R[1] + R[3]) / s; q[3] = (R[2] + R[6]) / s;
    } else if (R[4] > R[8]) {
        const float s = sqrtf(1.f + R[4] - R[0] - R[8]) * 2.f;
        q[0] = (R[2] - R[6]) / s; q[1] = (R[1] + R[3]) / s; q[2] = 0.25f * s; q[3] = (R[5] + R[7]) / s;
    } else {
        const float s = sqrtf(1.f + R[8] - R[0] - R[4]) * 2.f;
        q[0] = (R[3] - R[1]) / s; q[1] = (R[2] + R[6]) / s; q[2] = (R[5] + R[7]) / s; q[3] = 0.25f * s;
    }
}

__global__ void __launch_bounds__(256) decode_kernel(const float *__restrict__ y, const float4 *__restrict__ kp,
                                                     gs_view view, int B, const float *__restrict__ heur,
                                                     float *__restrict__ out, int32_t *__restrict__ used_fallback) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    const float *yi = y + int64_t(i) * 16;
    const float opac = 1.f / (1.f + __expf(-yi[7]));
    if (opac < 0.01f) {
        for (int r = 0; r < kRows; ++r) out[int64_t(r) * B + i] = heur[int64_t(r) * B + i];
        if (used_fallback) used_fallback[i] = 1;
        return;
    }
    if (used_fallback) used_fallback[i] = 0;
    const float4 k = kp[i];
    // camera frame point, then world: mu = R^T (xc - t)
    const float xc[3] = {k.z * (k.x - view.cx) / view.fx, k.z * (k.y - view.cy) / view.fy, k.z};
    const float *R = view.R;
    float d[3] = {xc[0] - view.t[0], xc[1] - view.t[1], xc[2] - view.t[2]};
    float col[kRows];
    for (int r = 0; r < kRows; ++r) col[r] = 0.f;
    for (int a = 0; a < 3; ++a) col[a] = R[a] * d[0] + R[3 + a] * d[1] + R[6 + a] * d[2];
    // log-scale: the heuristic's plus the predicted correction
    for (int a = 0; a < 3; ++a) col[3 + a] = heur[int64_t(3 + a) * B + i] + yi[a];
    // camera-frame rotation to world: q_w = q(R^T) * q_c
    float Rt[9] = {R[0], R[3], R[6], R[1], R[4], R[7], R[2], R[5], R[8]};
    float qa[4];
    mat_to_quat(Rt, qa);
    const float qb[4] = {yi[3], yi[4], yi[5], yi[6]};
    col[6] = qa[0] * qb[0] - qa[1] * qb[1] - qa[2] * qb[2] - qa[3] * qb[3];
    col[7] = qa[0] * qb[1] + qa[1] * qb[0] + qa[2] * qb[3] - qa[3] * qb[2];
    col[8] = qa[0] * qb[2] - qa[1] * qb[3] + qa[2] * qb[0] + qa[3] * qb[1];
    col[9] = qa[0] * qb[3] + qa[1] * qb[2] - qa[2] * qb[1] + qa[3] * qb[0];
    col[10] = yi[7];
    // SH DC: the heuristic's (pixel colour) plus the predicted correction
    for (int c = 0; c < 3; ++c) col[11 + c] = heur[int64_t(11 + c) * B + i] + yi[8 + c];
    for (int r = 0; r < kRows; ++r) out[int64_t(r) * B + i] = col[r];
}

__global__ void __launch_bounds__(256) append_kernel(float *__restrict__ P, float *__restrict__ m,
                                                     float *__restrict__ v, int64_t n, int64_t n_cap,
                                                     const float *__restrict__ newp, int B) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    for (int r = 0; r < kRows; ++r) {
        const int64_t dst = int64_t(r) * n_cap + n + i;
        P[dst] = newp[int64_t(r) * B + i];
        if (m) m[dst] = 0.f;
        if (v) v[dst] = 0.f;
    }
}

}  // namespace gs

extern "C" gs_status gs_init_features(const float *img, int32_t H, int32_t W, const float *kp,
                                      int32_t B, const float *heuristic, void *x_bf16, void *stream) {
    if (!img || !kp || !x_bf16 || H <= 0 || W <= 0 || B <= 0) return GS_ERR_INVALID_ARGUMENT;
    hipLaunchKernelGGL(gs::features_kernel, dim3((B + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), img, H, W, reinterpret_cast<const float4 *>(kp), B,
                       heuristic, static_cast<uint16_t *>(x_bf16));
    GS_CHECK_LAUNCH();
    return GS_OK;
}

extern "C" gs_status gs_init_heuristic(const float *new_mu, const float *new_rgb, int32_t B,
                                       const float *params, int64_t n, int64_t n_cap, float *out,
                                       void *stream) {
    if (!new_mu || !new_rgb || !out || B <= 0 || n < 0 || (n > 0 && !params) || n > n_cap || n_cap % 64)
        return GS_ERR_INVALID_ARGUMENT;
    hipLaunchKernelGGL(gs::heuristic_kernel, dim3((B + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), new_mu, new_rgb, B, params, n, n_cap, out);
    GS_CHECK_LAUNCH();
    return GS_OK;
}

extern "C" gs_status gs_init_decode(const float *y, const float *kp, const gs_view *view, int32_t B,
                                    const float *heuristic, float *out, int32_t *used_fallback,
                                    void *stream) {
    if (!y || !kp || !view || !heuristic || !out || B <= 0) return GS_ERR_INVALID_ARGUMENT;
    hipLaunchKernelGGL(gs::decode_kernel, dim3((B + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), y, reinterpret_cast<const float4 *>(kp), *view, B,
                       heuristic, out, used_fallback);
    GS_CHECK_LAUNCH();
    return GS_OK;
}

extern "C" gs_status gs_append(float *params, float *m, float *v, int64_t n, int64_t n_cap,
                               const float *new_params, int32_t B, void *stream) {
    if (!params || !new_params || B < 0 || n < 0 || n + B > n_cap || n_cap % 64)
        return GS_ERR_INVALID_ARGUMENT;
    if (B == 0) return GS_OK;
    hipLaunchKernelGGL(gs::append_kernel, dim3((B + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), params, m, v, n, n_cap, new_params, B);
    GS_CHECK_LAUNCH();
    return GS_OK;
}
