// Optimiser step of the mapper (Section 4.1 uses a fixed learning rate; the
// update is Adam with torch's bias correction and a per-row rate).
//
// Pure streaming: 16 B loads and stores of p, g, m, v (28 B of HBM traffic per
// parameter: 4 reads + 3 writes).  n_cap is a multiple of 64, so a float4
// never straddles two parameter rows.
#include "gs_internal.hpp"

namespace gs {

// grid.y = parameter row, grid.x * 256 threads = float4 columns of that row
__global__ void __launch_bounds__(256) adam_kernel(float4 *__restrict__ p, const float4 *__restrict__ g,
                                                   float4 *__restrict__ m, float4 *__restrict__ v,
                                                   int64_t n, int64_t n_cap, LrRows lr, float b1,
                                                   float omb1, float b2, float omb2, float eps,
                                                   float ibc1, float isqbc2, const int32_t *d_step,
                                                   float lnb1, float lnb2) {
    const int row = blockIdx.y;
    if (d_step) {   // step counter in device memory (graph replay): 1 - b^t = -expm1(t ln b)
        const float t = float(*d_step);
        ibc1 = 1.f / -expm1f(t * lnb1);
        isqbc2 = rsqrtf(-expm1f(t * lnb2));
    }
    const int64_t c4 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;   // float4 column
    const int64_t col = c4 * 4;
    if (col >= n) return;
    const int64_t i = int64_t(row) * (n_cap / 4) + c4;
    const float rate = lr.lr[row] * ibc1;
    float4 pp = p[i], gg = g[i], mm = m[i], vv = v[i];
    auto step = [&](float &pv, float gv, float &mv, float &vvv, int64_t c) {
        if (c >= n) return;
        mv = b1 * mv + omb1 * gv;
        vvv = b2 * vvv + omb2 * gv * gv;
        pv -= rate * mv * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(vvv) * isqbc2 + eps);
    };
    step(pp.x, gg.x, mm.x, vv.x, col);
    step(pp.y, gg.y, mm.y, vv.y, col + 1);
    step(pp.z, gg.z, mm.z, vv.z, col + 2);
    step(pp.w, gg.w, mm.w, vv.w, col + 3);
    p[i] = pp;
    m[i] = mm;
    v[i] = vv;
}

}  // namespace gs

extern "C" gs_status gs_adam_step(float *params, const float *grad, float *m, float *v, int64_t n,
                                  int64_t n_cap, const float *lr_rows, double beta1, double beta2,
                                  double eps, int32_t step, const int32_t *d_step, void *stream) {
    using namespace gs;
    if (!params || !grad || !m || !v || !lr_rows || n < 0 || n_cap <= 0 || n > n_cap ||
        n_cap % 64 || (step < 1 && !d_step) || !(beta1 >= 0.0 && beta1 < 1.0) ||
        !(beta2 >= 0.0 && beta2 < 1.0) ||
        !(eps >= 0.0))
        return GS_ERR_INVALID_ARGUMENT;
    if (n == 0) return GS_OK;
    LrRows lr;
    for (int r = 0; r < kRows; ++r) lr.lr[r] = lr_rows[r];
    // decay factors and their complements are rounded once, from double
    const int32_t t = step > 0 ? step : 1;
    const double bc1 = 1.0 - std::pow(beta1, t);
    const double bc2 = 1.0 - std::pow(beta2, t);
    const int64_t cols4 = (n + 3) / 4;
    const dim3 grid(unsigned((cols4 + 255) / 256), kRows);
    hipLaunchKernelGGL(adam_kernel, grid, dim3(256), 0, static_cast<hipStream_t>(stream),
                       reinterpret_cast<float4 *>(params), reinterpret_cast<const float4 *>(grad),
                       reinterpret_cast<float4 *>(m), reinterpret_cast<float4 *>(v), n, n_cap, lr,
                       float(beta1), float(1.0 - beta1), float(beta2), float(1.0 - beta2), float(eps),
                       float(1.0 / bc1), float(1.0 / std::sqrt(bc2)), step < 1 ? d_step : nullptr,
                       float(std::log(beta1)), float(std::log(beta2)));
    GS_CHECK_LAUNCH();
    return GS_OK;
}
