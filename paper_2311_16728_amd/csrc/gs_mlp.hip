// Learned initialiser for newly densified primitives: a 3-layer MLP
// 160 (157 used) -> 128 -> 128 -> 16 (11 used), ReLU between layers, BF16
// weights and activations on the matrix cores (v_mfma_f32_16x16x16_bf16) with
// FP32 accumulation.  The paper creates temporary primitives at inactive
// keypoints when a keyframe arrives (Section 3.3.1); this network proposes
// their scale, rotation, opacity and colour.
//
// Weight block (BF16 and FP32 master copies share the layout), row-major
// [out][in]: W1 [128][160] at 0, W2 [128][128] at 20480, W3 [16][128] at 36864;
// 38912 values.  Biases (FP32): b1[128], b2[128], b3[16]; 272 values.
//
// A workgroup of 2 waves owns 32 batch rows (16 per wave).  MFMA operand
// layout (16x16x16): lane l supplies A[row l%16][k 4(l/16)..+3] and
// B[k 4(l/16)..+3][col l%16]; the accumulator holds D[row 4(l/16)+j][col l%16].
#include "gs_internal.hpp"

namespace gs {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 160, kH = 128, kOut = 16;
constexpr int kW1 = 0, kW2 = kH * kIn, kW3 = kW2 + kH * kH, kWCount = kW3 + kOut * kH;
constexpr int kB1 = 0, kB2 = kH, kB3 = 2 * kH, kBCount = 2 * kH + kOut;
constexpr int kRowsPerBlock = 32;
constexpr int kMlpThreads = 128;   // 2 waves, 16 rows each

// float -> bf16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// A fragment from a row-major [rows][ld] BF16 matrix: rows r0.., columns k0..
__device__ __forceinline__ bf16x4 frag_rows(const uint16_t *M, int ld, int r0, int k0) {
    const int l = lane_id();
    const uint16_t *p = M + (r0 + (l & 15)) * ld + k0 + 4 * (l >> 4);
    bf16x4 v;
    v[0] = short(p[0]); v[1] = short(p[1]); v[2] = short(p[2]); v[3] = short(p[3]);
    return v;
}

// A fragment whose rows are the columns of a row-major [K][ld] matrix:
// A[m][k] = M[k0 + k][m0 + m]
__device__ __forceinline__ bf16x4 frag_cols(const uint16_t *M, int ld, int m0, int k0) {
    const int l = lane_id();
    const int m = m0 + (l & 15), k = k0 + 4 * (l >> 4);
    bf16x4 v;
    v[0] = short(M[(k + 0) * ld + m]); v[1] = short(M[(k + 1) * ld + m]);
    v[2] = short(M[(k + 2) * ld + m]); v[3] = short(M[(k + 3) * ld + m]);
    return v;
}

// ---------------------------------------------------------------------------
// Forward: y = W3 relu(W2 relu(W1 x + b1) + b2) + b3; H1, H2 (BF16) kept in act.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kMlpThreads) mlp_fwd_kernel(const uint16_t *__restrict__ w,
                                                      const float *__restrict__ bias,
                                                      const uint16_t *__restrict__ x, int B,
                                                      float *__restrict__ y,
                                                      uint16_t *__restrict__ act) {
    __shared__ uint16_t sW[kWCount];
    __shared__ uint16_t sX[kRowsPerBlock][kIn];
    __shared__ uint16_t sH1[kRowsPerBlock][kH];
    __shared__ uint16_t sH2[kRowsPerBlock][kH];
    const int tid = threadIdx.x, wave = tid / kWave, l = lane_id();
    const int row0 = blockIdx.x * kRowsPerBlock;
    for (int i = tid; i < kWCount; i += kMlpThreads) sW[i] = w[i];
    for (int i = tid; i < kRowsPerBlock * kIn; i += kMlpThreads) {
        const int r = i / kIn, c = i % kIn;
        sX[r][c] = (row0 + r < B) ? x[int64_t(row0 + r) * kIn + c] : uint16_t(0);
    }
    __syncthreads();
    const int r0 = wave * 16;                 // this wave's rows inside the block
    uint16_t *H1g = act, *H2g = act + int64_t(B) * kH;
    // layer 1
    for (int nt = 0; nt < kH / 16; ++nt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int kt = 0; kt < kIn / 16; ++kt)
            acc = mfma16(frag_rows(&sX[0][0], kIn, r0, 16 * kt), frag_rows(sW + kW1, kIn, 16 * nt, 16 * kt), acc);
        const int col = 16 * nt + (l & 15);
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + 4 * (l >> 4) + j;
            const uint16_t h = f2bf(fmaxf(acc[j] + bias[kB1 + col], 0.f));
            sH1[r][col] = h;
            if (row0 + r < B) H1g[int64_t(row0 + r) * kH + col] = h;
        }
    }
    __syncthreads();
    // layer 2
    for (int nt = 0; nt < kH / 16; ++nt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int kt = 0; kt < kH / 16; ++kt)
            acc = mfma16(frag_rows(&sH1[0][0], kH, r0, 16 * kt), frag_rows(sW + kW2, kH, 16 * nt, 16 * kt), acc);
        const int col = 16 * nt + (l & 15);
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + 4 * (l >> 4) + j;
            const uint16_t h = f2bf(fmaxf(acc[j] + bias[kB2 + col], 0.f));
            sH2[r][col] = h;
            if (row0 + r < B) H2g[int64_t(row0 + r) * kH + col] = h;
        }
    }
    __syncthreads();
    // layer 3 (linear)
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < kH / 16; ++kt)
        acc = mfma16(frag_rows(&sH2[0][0], kH, r0, 16 * kt), frag_rows(sW + kW3, kH, 0, 16 * kt), acc);
    const int col = l & 15;
    for (int j = 0; j < 4; ++j) {
        const int r = row0 + r0 + 4 * (l >> 4) + j;
        if (r < B) y[int64_t(r) * kOut + col] = acc[j] + bias[kB3 + col];
    }
}

// ---------------------------------------------------------------------------
// Backward of a sum over rows of <dy, y>: dW (FP32, [out][in]) and db are
// ADDED to.  Products take BF16 operands (dy and the hidden gradients are
// rounded to BF16 where they enter a product), FP32 accumulation; bias
// gradients are summed in FP32.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kMlpThreads) mlp_bwd_kernel(const uint16_t *__restrict__ w,
                                                      const uint16_t *__restrict__ x,
                                                      const uint16_t *__restrict__ act,
                                                      const float *__restrict__ dy, int B,
                                                      float *__restrict__ dw,
                                                      float *__restrict__ db) {
    __shared__ uint16_t sW[kWCount];
    __shared__ uint16_t sX[kRowsPerBlock][kIn];
    __shared__ uint16_t sH1[kRowsPerBlock][kH];
    __shared__ uint16_t sH2[kRowsPerBlock][kH];
    __shared__ uint16_t sD3[kRowsPerBlock][kOut];   // dy (BF16)
    __shared__ uint16_t sD2[kRowsPerBlock][kH];     // dL/d(pre-activation 2) (BF16)
    __shared__ uint16_t sD1[kRowsPerBlock][kH];     // dL/d(pre-activation 1) (BF16)
    __shared__ float sDb[kBCount];
    const int tid = threadIdx.x, wave = tid / kWave, l = lane_id();
    const int row0 = blockIdx.x * kRowsPerBlock;
    const int nrows = min(kRowsPerBlock, B - row0);
    const uint16_t *H1g = act, *H2g = act + int64_t(B) * kH;
    for (int i = tid; i < kWCount; i += kMlpThreads) sW[i] = w[i];
    for (int i = tid; i < kBCount; i += kMlpThreads) sDb[i] = 0.f;
    for (int i = tid; i < kRowsPerBlock * kIn; i += kMlpThreads) {
        const int r = i / kIn, c = i % kIn;
        sX[r][c] = (r < nrows) ? x[int64_t(row0 + r) * kIn + c] : uint16_t(0);
    }
    for (int i = tid; i < kRowsPerBlock * kH; i += kMlpThreads) {
        const int r = i / kH, c = i % kH;
        sH1[r][c] = (r < nrows) ? H1g[int64_t(row0 + r) * kH + c] : uint16_t(0);
        sH2[r][c] = (r < nrows) ? H2g[int64_t(row0 + r) * kH + c] : uint16_t(0);
    }
    __syncthreads();
    for (int i = tid; i < kRowsPerBlock * kOut; i += kMlpThreads) {
        const int r = i / kOut, c = i % kOut;
        const float g = (r < nrows) ? dy[int64_t(row0 + r) * kOut + c] : 0.f;
        sD3[r][c] = f2bf(g);
        atomicAdd(&sDb[kB3 + c], g);
    }
    __syncthreads();
    const int r0 = wave * 16;
    // dpre2 = (dy W3) * [H2 > 0]: A = dy rows (K = 16 outputs), B[k][n] = W3[k][n]
    for (int nt = 0; nt < kH / 16; ++nt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma16(frag_rows(&sD3[0][0], kOut, r0, 0), frag_cols(sW + kW3, kH, 16 * nt, 0), acc);
        const int col = 16 * nt + (l & 15);
        float bsum = 0.f;
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + 4 * (l >> 4) + j;
            const float g = (bf2f(sH2[r][col]) > 0.f) ? acc[j] : 0.f;
            sD2[r][col] = f2bf(g);
            bsum += g;
        }
        atomicAdd(&sDb[kB2 + col], bsum);
    }
    __syncthreads();
    // dpre1 = (dpre2 W2) * [H1 > 0]
    for (int nt = 0; nt < kH / 16; ++nt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int kt = 0; kt < kH / 16; ++kt)
            acc = mfma16(frag_rows(&sD2[0][0], kH, r0, 16 * kt), frag_cols(sW + kW2, kH, 16 * nt, 16 * kt), acc);
        const int col = 16 * nt + (l & 15);
        float bsum = 0.f;
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + 4 * (l >> 4) + j;
            const float g = (bf2f(sH1[r][col]) > 0.f) ? acc[j] : 0.f;
            sD1[r][col] = f2bf(g);
            bsum += g;
        }
        atomicAdd(&sDb[kB1 + col], bsum);
    }
    __syncthreads();
    // weight gradients dW[out][in] = sum_rows dpre[row][out] act[row][in];
    // tile (out block ot, in block it): A[m=out][k=row] = D[row][out] (columns of
    // a row-major [rows][out] matrix), B[k=row][n=in] = act[row][in].
    auto wgrad = [&](const uint16_t *D, int ldD, const uint16_t *Act, int ldA, int nout, int nin,
                     int off) {
        const int tiles = (nout / 16) * (nin / 16);
        for (int t = wave; t < tiles; t += kMlpThreads / kWave) {
            const int ot = t / (nin / 16), it = t % (nin / 16);
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            for (int kt = 0; kt < kRowsPerBlock / 16; ++kt) {
                const bf16x4 a = frag_cols(D, ldD, 16 * ot, 16 * kt);
                // B fragment: lane supplies B[k = 4(l/16)..+3][n = l%16] = Act[row k][in n]
                bf16x4 b;
                const int n = 16 * it + (l & 15), k = 16 * kt + 4 * (l >> 4);
                b[0] = short(Act[(k + 0) * ldA + n]); b[1] = short(Act[(k + 1) * ldA + n]);
                b[2] = short(Act[(k + 2) * ldA + n]); b[3] = short(Act[(k + 3) * ldA + n]);
                acc = mfma16(a, b, acc);
            }
            const int in = 16 * it + (l & 15);
            for (int j = 0; j < 4; ++j) {
                const int out = 16 * ot + 4 * (l >> 4) + j;
                if (acc[j] != 0.f) atomicAdd(&dw[off + out * nin + in], acc[j]);
            }
        }
    };
    wgrad(&sD3[0][0], kOut, &sH2[0][0], kH, kOut, kH, kW3);
    wgrad(&sD2[0][0], kH, &sH1[0][0], kH, kH, kH, kW2);
    wgrad(&sD1[0][0], kH, &sX[0][0], kIn, kH, kIn, kW1);
    __syncthreads();
    for (int i = tid; i < kBCount; i += kMlpThreads)
        if (sDb[i] != 0.f) atomicAdd(&db[i], sDb[i]);
}

// Adam on the FP32 master weights and biases; the BF16 weight copy is
// refreshed (round to nearest even).
__global__ void __launch_bounds__(256) mlp_adam_kernel(float *__restrict__ wm, uint16_t *__restrict__ wb,
                                                       const float *__restrict__ g, float *__restrict__ m,
                                                       float *__restrict__ v, int count, int nbf16,
                                                       float lr, float b1, float omb1, float b2,
                                                       float omb2, float eps, float ibc1, float isqbc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float p = wm[i] - lr * ibc1 * mi / (sqrtf(vi) * isqbc2 + eps);
    wm[i] = p;
    if (i < nbf16) wb[i] = f2bf(p);
}

__global__ void f32_to_bf16_kernel(const float *__restrict__ a, uint16_t *__restrict__ b, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) b[i] = f2bf(a[i]);
}

}  // namespace gs

extern "C" gs_status gs_init_mlp_fwd(const void *w_bf16, const float *bias, const void *x_bf16,
                                     int32_t B, float *y, void *act_ws, void *stream) {
    using namespace gs;
    if (!w_bf16 || !bias || !x_bf16 || !y || !act_ws || B <= 0) return GS_ERR_INVALID_ARGUMENT;
    const int blocks = (B + kRowsPerBlock - 1) / kRowsPerBlock;
    hipLaunchKernelGGL(mlp_fwd_kernel, dim3(blocks), dim3(kMlpThreads), 0, static_cast<hipStream_t>(stream),
                       static_cast<const uint16_t *>(w_bf16), bias, static_cast<const uint16_t *>(x_bf16),
                       B, y, static_cast<uint16_t *>(act_ws));
    GS_CHECK_LAUNCH();
    return GS_OK;
}

extern "C" gs_status gs_init_mlp_bwd(const void *w_bf16, const void *x_bf16, const void *act_ws,
                                     const float *dy, int32_t B, float *dw, float *db, void *stream) {
    using namespace gs;
    if (!w_bf16 || !x_bf16 || !act_ws || !dy || !dw || !db || B <= 0) return GS_ERR_INVALID_ARGUMENT;
    const int blocks = (B + kRowsPerBlock - 1) / kRowsPerBlock;
    hipLaunchKernelGGL(mlp_bwd_kernel, dim3(blocks), dim3(kMlpThreads), 0, static_cast<hipStream_t>(stream),
                       static_cast<const uint16_t *>(w_bf16), static_cast<const uint16_t *>(x_bf16),
                       static_cast<const uint16_t *>(act_ws), dy, B, dw, db);
    GS_CHECK_LAUNCH();
    return GS_OK;
}

extern "C" gs_status gs_init_mlp_adam(float *w_master, float *b_master, void *w_bf16,
                                      const float *dw, const float *db, float *m, float *v,
                                      float lr, double beta1, double beta2, double eps, int32_t step,
                                      void *stream) {
    using namespace gs;
    if (!w_master || !b_master || !w_bf16 || !dw || !db || !m || !v || step < 1)
        return GS_ERR_INVALID_ARGUMENT;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const float ibc1 = float(1.0 / (1.0 - std::pow(beta1, step)));
    const float isqbc2 = float(1.0 / std::sqrt(1.0 - std::pow(beta2, step)));
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kWCount + 255) / 256), dim3(256), 0, st, w_master,
                       static_cast<uint16_t *>(w_bf16), dw, m, v, kWCount, kWCount, lr, float(beta1),
                       float(1.0 - beta1), float(beta2), float(1.0 - beta2), float(eps), ibc1, isqbc2);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kBCount + 255) / 256), dim3(256), 0, st, b_master,
                       static_cast<uint16_t *>(w_bf16), db, m + kWCount, v + kWCount, kBCount, 0, lr,
                       float(beta1), float(1.0 - beta1), float(beta2), float(1.0 - beta2), float(eps), ibc1,
                       isqbc2);
    GS_CHECK_LAUNCH();
    return GS_OK;
}

extern "C" gs_status gs_to_bf16(const float *src, void *dst, int64_t count, void *stream) {
    if (!src || !dst || count < 0) return GS_ERR_INVALID_ARGUMENT;
    if (count == 0) return GS_OK;
    hipLaunchKernelGGL(gs::f32_to_bf16_kernel, dim3((count + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), src, static_cast<uint16_t *>(dst), count);
    GS_CHECK_LAUNCH();
    return GS_OK;
}
