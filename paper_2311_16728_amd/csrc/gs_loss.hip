// Gaussian pyramid (Section 3.4) and the photometric loss of Eq. 4 with its
// gradient, over every render target at once.
//
// The loss uses the rasteriser's tiling (the target's tile shape, 256 pixels):
// one 256-thread workgroup per tile stages the tile plus a 5-pixel halo of
// render and target
// in LDS, runs the separable 11-tap Gaussian window horizontally then
// vertically for the five SSIM moments, and writes per-pixel partial
// derivatives of the SSIM map (with respect to the window mean, the second
// moment and the cross moment).  A second pass filters those three maps with
// the same (self-adjoint) window and forms dL/dI.  Partial sums are reduced
// per tile and then per target in a fixed order, so the loss is deterministic.
#include "gs_internal.hpp"

namespace gs {

constexpr int kR = 5;                       // SSIM window radius (11 taps)

struct Window {
    float w[2 * kR + 1];
};

static Window ssim_window() {
    Window W;
    double v[2 * kR + 1], s = 0;
    for (int i = -kR; i <= kR; ++i) {
        v[i + kR] = std::exp(-double(i * i) / (2.0 * 1.5 * 1.5));
        s += v[i + kR];
    }
    for (int i = 0; i < 2 * kR + 1; ++i) W.w[i] = float(v[i] / s);
    return W;
}

__device__ __forceinline__ int find_target_loss(const gs_target *__restrict__ targets, int n,
                                                int tile) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (targets[mid].tile_offset <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Tile geometry of the loss kernels: the target's raster tile (TW x TH
// pixels, TW * TH = 256) plus an R-pixel halo, HX x HY.  Each kernel
// dispatches on the target's tile width to a body compiled for that shape;
// LDS is sized for the largest (16 x 16: 48 x 26 halo with its padded rows;
// 32 x 8: 18 x 32 horizontal pass).
// LDS row stride of a halo window: the horizontal passes read 32 / TW rows of
// TW consecutive floats per half wave; row strides that put those rows on
// disjoint banks keep the reads conflict-free (16-wide: 48, two rows 16
// banks apart; 8-wide: 24, four rows at bank offsets 0, 24, 16, 8).
template <int TW>
__host__ __device__ constexpr int halo_stride() {
    return TW == 16 ? 48 : TW == 8 ? 24 : TW + 2 * kR;
}
constexpr int kHaloMax = 48 * (16 + 2 * kR);   // the largest of the three shapes (16 x 16)
static_assert(halo_stride<8>() * (32 + 2 * kR) <= kHaloMax && halo_stride<32>() * (8 + 2 * kR) <= kHaloMax,
              "halo buffers");
constexpr int kHPassMax = 32 * (8 + 2 * kR);

// The HX x HY window of kP channel planes around the tile, zero outside the
// image: fetched into registers (kHaloRounds values per plane and thread,
// every load unconditional at a clamped address, so all are in flight
// together), then put into LDS (row stride halo_stride<TW>()).  Fetching
// the next channel while the current one is filtered hides the loads.
template <int TW>
__host__ __device__ constexpr int halo_rounds() {
    return ((TW + 2 * kR) * (kTilePix / TW + 2 * kR) + kTilePix - 1) / kTilePix;
}
template <int TW, int kP>
struct Halo {
    float v[kP][halo_rounds<TW>()];   // as loaded (clamped address)
    uint32_t in;                      // bit r: round r's pixel lies in the image
};
template <int TW, int kP>
__device__ __forceinline__ void fetch_halo(const float *const (&planes)[kP], int W, int H, int x0, int y0,
                                           Halo<TW, kP> &hv) {
    constexpr int TH = kTilePix / TW, HX = TW + 2 * kR, HY = TH + 2 * kR;
    constexpr int kRounds = halo_rounds<TW>();
    static_assert(kRounds <= 32, "one bit per round");
    hv.in = 0u;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int i = threadIdx.x + r * kTilePix;
        const int yy = i / HX, xx = i % HX;
        const int gx = x0 - kR + xx, gy = y0 - kR + yy;
        const bool in = i < HX * HY && gx >= 0 && gx < W && gy >= 0 && gy < H;
        const int64_t at = int64_t(min(max(gy, 0), H - 1)) * W + min(max(gx, 0), W - 1);
        hv.in |= uint32_t(in) << r;
        // (zeroed when put, so that nothing waits for the loads before then)
#pragma unroll
        for (int p = 0; p < kP; ++p) hv.v[p][r] = planes[p][at];
    }
}
template <int TW, int kP>
__device__ __forceinline__ void put_halo(const Halo<TW, kP> &hv, float *const (&dst)[kP]) {
    constexpr int HX = TW + 2 * kR, HY = kTilePix / TW + 2 * kR, HS = halo_stride<TW>();
#pragma unroll
    for (int r = 0; r < halo_rounds<TW>(); ++r) {
        const int i = threadIdx.x + r * kTilePix;
        if (i < HX * HY) {
            const bool in = (hv.in >> r) & 1u;
#pragma unroll
            for (int p = 0; p < kP; ++p) dst[p][(i / HX) * HS + i % HX] = in ? hv.v[p][r] : 0.f;
        }
    }
}

struct alignas(16) SsimLds {
    float sx[kHaloMax];
    float sy[kHaloMax];
    float h[5][kHPassMax];
    float red[2][kTilePix / kWave];
};

template <int TW>
__device__ __forceinline__ void ssim_fwd_tile(const float *__restrict__ render,
                                              const float *__restrict__ target, const gs_target &t,
                                              int tile, const Window &win, float *__restrict__ maps,
                                              float *__restrict__ partial, SsimLds &L) {
    constexpr int TH = kTilePix / TW, HY = TH + 2 * kR, HS = halo_stride<TW>();
    const float C1 = 0.01f * 0.01f, C2 = 0.03f * 0.03f;
    const int tid = threadIdx.x;
    const int local = tile - t.tile_offset;
    const int x0 = (local % t.tiles_x) * TW, y0 = (local / t.tiles_x) * TH;
    const int lx = tid % TW, ly = tid / TW;
    const int px = x0 + lx, py = y0 + ly;
    const bool inside = px < t.width && py < t.height;
    const int64_t HW = int64_t(t.width) * t.height;
    const int64_t pix = int64_t(py) * t.width + px;
    float l1 = 0.f, ss = 0.f;
    Halo<TW, 2> hv;
    auto fetch = [&](int c) {
        const float *const planes[2] = {render + 3 * t.pix_offset + c * HW, target + 3 * t.pix_offset + c * HW};
        fetch_halo<TW, 2>(planes, t.width, t.height, x0, y0, hv);
    };
    float *const dst[2] = {L.sx, L.sy};
    fetch(0);
    for (int c = 0; c < 3; ++c) {
        __syncthreads();   // the previous channel's reads of the windows are done
        put_halo<TW, 2>(hv, dst);
        __syncthreads();
        if (c + 1 < 3) fetch(c + 1);
        // two horizontally adjacent outputs per thread (one round for 16-
        // and 8-wide tiles): each input and its products are formed once;
        // every output sums its taps in the same order as one alone would
        constexpr int kTaps = 2 * kR + 1;
#pragma unroll
        for (int s2 = tid; s2 < HY * (TW / 2); s2 += kTilePix) {
            const int r = s2 / (TW / 2), cc = 2 * (s2 % (TW / 2));
            const float *rx = L.sx + r * HS + cc, *ry = L.sy + r * HS + cc;
            float m1[2] = {0, 0}, m2[2] = {0, 0}, e11[2] = {0, 0}, e22[2] = {0, 0}, e12[2] = {0, 0};
#pragma unroll
            for (int k = 0; k <= kTaps; ++k) {
                const float a = rx[k], b = ry[k];
                const float aa = a * a, bb = b * b, ab = a * b;
#pragma unroll
                for (int o = 0; o < 2; ++o) {
                    const int t = k - o;   // tap of output o
                    if (t < 0 || t >= kTaps) continue;
                    const float w = win.w[t];
                    m1[o] = fmaf(w, a, m1[o]);
                    m2[o] = fmaf(w, b, m2[o]);
                    e11[o] = fmaf(w, aa, e11[o]);
                    e22[o] = fmaf(w, bb, e22[o]);
                    e12[o] = fmaf(w, ab, e12[o]);
                }
            }
            const int i = r * TW + cc;
            *reinterpret_cast<float2 *>(&L.h[0][i]) = make_float2(m1[0], m1[1]);
            *reinterpret_cast<float2 *>(&L.h[1][i]) = make_float2(m2[0], m2[1]);
            *reinterpret_cast<float2 *>(&L.h[2][i]) = make_float2(e11[0], e11[1]);
            *reinterpret_cast<float2 *>(&L.h[3][i]) = make_float2(e22[0], e22[1]);
            *reinterpret_cast<float2 *>(&L.h[4][i]) = make_float2(e12[0], e12[1]);
        }
        __syncthreads();
        float mx = 0, my = 0, exx = 0, eyy = 0, exy = 0;
#pragma unroll
        for (int k = 0; k < 2 * kR + 1; ++k) {
            const float w = win.w[k];
            const int i = (ly + k) * TW + lx;
            mx = fmaf(w, L.h[0][i], mx);
            my = fmaf(w, L.h[1][i], my);
            exx = fmaf(w, L.h[2][i], exx);
            eyy = fmaf(w, L.h[3][i], eyy);
            exy = fmaf(w, L.h[4][i], exy);
        }
        if (inside) {
            const float vx = exx - mx * mx, vy = eyy - my * my, cxy = exy - mx * my;
            const float A1 = 2.f * mx * my + C1, A2 = 2.f * cxy + C2;
            const float B1 = mx * mx + my * my + C1, B2 = vx + vy + C2;
            // B1 >= C1 and B2 >= C2 (up to rounding of the variances): the
            // hardware reciprocal (1 ulp) instead of four IEEE divisions
            const float iB1 = __builtin_amdgcn_rcpf(B1), iB2 = __builtin_amdgcn_rcpf(B2);
            const float iB1B2 = iB1 * iB2;
            const float S = A1 * A2 * iB1B2;
            ss += S;
            const int ci = (ly + kR) * HS + lx + kR;
            l1 += fabsf(L.sx[ci] - L.sy[ci]);
            float *mp = maps + 9 * t.pix_offset + (3 * c) * HW;
            mp[pix] = 2.f * my * (A2 - A1) * iB1B2 - 2.f * mx * S * (iB1 - iB2);
            mp[HW + pix] = -S * iB2;
            mp[2 * HW + pix] = 2.f * A1 * iB1B2;
        }
    }
    l1 = wave_sum(l1);
    ss = wave_sum(ss);
    if (lane_id() == 0) { L.red[0][tid / kWave] = l1; L.red[1][tid / kWave] = ss; }
    __syncthreads();
    if (tid == 0) {
        float a = 0, b = 0;
        for (int w = 0; w < kTilePix / kWave; ++w) { a += L.red[0][w]; b += L.red[1][w]; }
        partial[2 * int64_t(tile)] = a;
        partial[2 * int64_t(tile) + 1] = b;
    }
}

// (seven workgroups per CU, as many as its LDS allows)
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) ssim_fwd_kernel(const float *__restrict__ render,
                                                       const float *__restrict__ target,
                                                       const gs_target *__restrict__ targets,
                                                       int n_targets, int total_tiles, Window win,
                                                       float *__restrict__ maps,
                                                       float *__restrict__ partial) {
    __shared__ SsimLds L;
    const int tile = int(xcd_tile(blockIdx.x, total_tiles));
    if (tile >= total_tiles) return;
    const gs_target t = targets[find_target_loss(targets, n_targets, tile)];
    switch (tile_shape(t.tile_w).w) {
        case 8: ssim_fwd_tile<8>(render, target, t, tile, win, maps, partial, L); break;
        case 32: ssim_fwd_tile<32>(render, target, t, tile, win, maps, partial, L); break;
        default: ssim_fwd_tile<16>(render, target, t, tile, win, maps, partial, L); break;
    }
}

// One block: per-target means from the tile partials (fixed order), then the
// weighted total.
// Eq. 4 per target (one workgroup each, tile partials summed in double in a
// fixed order), then the weighted sum over targets in target order.
__device__ __forceinline__ void loss_of_target(const gs_target *__restrict__ targets, int ti,
                                               float lambda, const float *__restrict__ partial,
                                               double *__restrict__ tloss, float *__restrict__ d_loss) {
    __shared__ double red[2][kTilePix / kWave];
    const gs_target t = targets[ti];
    const int nt = t.tiles_x * t.tiles_y;
    double a = 0, b = 0;
    // unrolled so that the loads of several tiles are in flight; the sums keep
    // their order
#pragma unroll 8
    for (int i = threadIdx.x; i < nt; i += blockDim.x) {
        a += partial[2 * int64_t(t.tile_offset + i)];
        b += partial[2 * int64_t(t.tile_offset + i) + 1];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane_id() == 0) { red[0][threadIdx.x / kWave] = a; red[1][threadIdx.x / kWave] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0, sb = 0;
        for (int w = 0; w < kTilePix / kWave; ++w) { sa += red[0][w]; sb += red[1][w]; }
        const double n = 3.0 * double(t.width) * double(t.height);
        const double L = (1.0 - lambda) * sa / n + lambda * (1.0 - sb / n);
        tloss[ti] = double(t.weight) * L;
        if (d_loss) d_loss[ti] = float(L);
    }
    __syncthreads();   // red is reused by the next call
}

struct alignas(16) SsimBwdLds {
    float sm[3][kHaloMax];
    float h[3][kHPassMax];
};

template <int TW>
__device__ __forceinline__ void ssim_bwd_tile(const float *__restrict__ render,
                                              const float *__restrict__ target, const gs_target &t,
                                              int tile, const Window &win, float lambda,
                                              const float *__restrict__ maps, float *__restrict__ dL,
                                              SsimBwdLds &L) {
    constexpr int TH = kTilePix / TW, HY = TH + 2 * kR, HS = halo_stride<TW>();
    const int tid = threadIdx.x;
    const int local = tile - t.tile_offset;
    const int x0 = (local % t.tiles_x) * TW, y0 = (local / t.tiles_x) * TH;
    const int lx = tid % TW, ly = tid / TW;
    const int px = x0 + lx, py = y0 + ly;
    const bool inside = px < t.width && py < t.height;
    const int64_t HW = int64_t(t.width) * t.height;
    const int64_t pix = int64_t(py) * t.width + px;
    const float inv = 1.f / (3.f * float(HW));
    Halo<TW, 3> hv;
    auto fetch = [&](int c) {
        const float *mp = maps + 9 * t.pix_offset + (3 * c) * HW;
        const float *const planes[3] = {mp, mp + HW, mp + 2 * HW};
        fetch_halo<TW, 3>(planes, t.width, t.height, x0, y0, hv);
    };
    float *const dst[3] = {L.sm[0], L.sm[1], L.sm[2]};
    fetch(0);
    for (int c = 0; c < 3; ++c) {
        __syncthreads();   // the previous channel's reads of the windows are done
        put_halo<TW, 3>(hv, dst);
        __syncthreads();
        if (c + 1 < 3) fetch(c + 1);
        // two horizontally adjacent outputs per thread, each input read once
        constexpr int kTaps = 2 * kR + 1;
#pragma unroll
        for (int s2 = tid; s2 < HY * (TW / 2); s2 += kTilePix) {
            const int r = s2 / (TW / 2), cc = 2 * (s2 % (TW / 2));
            const int base = r * HS + cc;
            float a0[2] = {0, 0}, a1[2] = {0, 0}, a2[2] = {0, 0};
#pragma unroll
            for (int k = 0; k <= kTaps; ++k) {
                const float x0 = L.sm[0][base + k], x1 = L.sm[1][base + k], x2 = L.sm[2][base + k];
#pragma unroll
                for (int o = 0; o < 2; ++o) {
                    const int t = k - o;
                    if (t < 0 || t >= kTaps) continue;
                    const float w = win.w[t];
                    a0[o] = fmaf(w, x0, a0[o]);
                    a1[o] = fmaf(w, x1, a1[o]);
                    a2[o] = fmaf(w, x2, a2[o]);
                }
            }
            const int i = r * TW + cc;
            *reinterpret_cast<float2 *>(&L.h[0][i]) = make_float2(a0[0], a0[1]);
            *reinterpret_cast<float2 *>(&L.h[1][i]) = make_float2(a1[0], a1[1]);
            *reinterpret_cast<float2 *>(&L.h[2][i]) = make_float2(a2[0], a2[1]);
        }
        __syncthreads();
        float f0 = 0, f1 = 0, f2 = 0;
#pragma unroll
        for (int k = 0; k < 2 * kR + 1; ++k) {
            const float w = win.w[k];
            const int i = (ly + k) * TW + lx;
            f0 = fmaf(w, L.h[0][i], f0);
            f1 = fmaf(w, L.h[1][i], f1);
            f2 = fmaf(w, L.h[2][i], f2);
        }
        if (inside) {
            const float x = render[3 * t.pix_offset + c * HW + pix];
            const float y = target[3 * t.pix_offset + c * HW + pix];
            const float d = x - y;
            const float sgn = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
            const float dssim = f0 + 2.f * x * f1 + y * f2;
            dL[3 * t.pix_offset + c * HW + pix] =
                t.weight * inv * ((1.f - lambda) * sgn - lambda * dssim);
        }
    }
}

// A few targets (kFold): workgroup 0 also forms the per-target losses and the
// total from the forward's tile partials before its tile (the sums and order
// of loss_few_kernel, one launch fewer).
constexpr int kLossOneBlockTargets = 8;
template <bool kFold>
// (62 VGPRs: seven workgroups per CU, as many as its LDS allows; without the
// hint the prefetched windows take it to 95 and five)
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) ssim_bwd_kernel(const float *__restrict__ render,
                                                       const float *__restrict__ target,
                                                       const gs_target *__restrict__ targets,
                                                       int n_targets, int total_tiles, Window win,
                                                       float lambda,
                                                       const float *__restrict__ maps,
                                                       float *__restrict__ dL,
                                                       const float *__restrict__ partial,
                                                       double *__restrict__ tloss,
                                                       float *__restrict__ d_loss,
                                                       float *__restrict__ d_total) {
    __shared__ SsimBwdLds L;
    if (kFold && blockIdx.x == 0) {   // uniform over the workgroup
        for (int ti = 0; ti < n_targets; ++ti) loss_of_target(targets, ti, lambda, partial, tloss, d_loss);
        if (threadIdx.x == 0 && d_total) {
            double total = 0.0;
            for (int ti = 0; ti < n_targets; ++ti) total += tloss[ti];
            *d_total = float(total);
        }
    }
    const int tile = int(xcd_tile(blockIdx.x, total_tiles));
    if (tile >= total_tiles) return;
    const gs_target t = targets[find_target_loss(targets, n_targets, tile)];
    switch (tile_shape(t.tile_w).w) {
        case 8: ssim_bwd_tile<8>(render, target, t, tile, win, lambda, maps, dL, L); break;
        case 32: ssim_bwd_tile<32>(render, target, t, tile, win, lambda, maps, dL, L); break;
        default: ssim_bwd_tile<16>(render, target, t, tile, win, lambda, maps, dL, L); break;
    }
}

__global__ void __launch_bounds__(256) loss_target_kernel(const gs_target *__restrict__ targets,
                                                          float lambda,
                                                          const float *__restrict__ partial,
                                                          double *__restrict__ tloss,
                                                          float *__restrict__ d_loss) {
    loss_of_target(targets, blockIdx.x, lambda, partial, tloss, d_loss);
}

// A few targets: one workgroup takes them in order and forms the total
// (the same sums in the same order as the two kernels above and below).
__global__ void __launch_bounds__(256) loss_few_kernel(const gs_target *__restrict__ targets,
                                                       int n_targets, float lambda,
                                                       const float *__restrict__ partial,
                                                       double *__restrict__ tloss,
                                                       float *__restrict__ d_loss,
                                                       float *__restrict__ d_total) {
    for (int ti = 0; ti < n_targets; ++ti) loss_of_target(targets, ti, lambda, partial, tloss, d_loss);
    if (threadIdx.x == 0 && d_total) {
        double total = 0.0;
        for (int ti = 0; ti < n_targets; ++ti) total += tloss[ti];
        *d_total = float(total);
    }
}

__global__ void __launch_bounds__(64) loss_total_kernel(int n_targets, const double *__restrict__ tloss,
                                                        float *__restrict__ d_total) {
    if (threadIdx.x != 0) return;
    double total = 0.0;
#pragma unroll 8
    for (int ti = 0; ti < n_targets; ++ti) total += tloss[ti];   // in target order
    if (d_total) *d_total = float(total);
}

// One pyramid level down: 5x5 binomial, reflected borders (edge not repeated),
// even rows/columns kept.
__device__ __forceinline__ int refl101(int i, int n) {
    if (n == 1) return 0;
    while (i < 0 || i >= n) {
        if (i < 0) i = -i;
        if (i >= n) i = 2 * (n - 1) - i;
    }
    return i;
}

__global__ void __launch_bounds__(256) pyr_down_kernel(const float *__restrict__ in, int C, int H, int W,
                                                       float *__restrict__ out) {
    const int Ho = (H + 1) / 2, Wo = (W + 1) / 2;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= int64_t(C) * Ho * Wo) return;
    const int c = int(i / (int64_t(Ho) * Wo));
    const int rem = int(i - int64_t(c) * Ho * Wo);
    const int oy = rem / Wo, ox = rem % Wo;
    const float k[5] = {1.f / 16, 4.f / 16, 6.f / 16, 4.f / 16, 1.f / 16};
    const float *src = in + int64_t(c) * H * W;
    float acc = 0.f;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        const int yy = refl101(2 * oy + a - 2, H);
        float row = 0.f;
#pragma unroll
        for (int b = 0; b < 5; ++b) row = fmaf(k[b], src[int64_t(yy) * W + refl101(2 * ox + b - 2, W)], row);
        acc = fmaf(k[a], row, acc);
    }
    out[i] = acc;
}

__global__ void copy_f32_kernel(const float *__restrict__ a, float *__restrict__ b, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

}  // namespace gs

extern "C" gs_status gs_pyramid_build(const float *img, int32_t C, int32_t H, int32_t W,
                                      int32_t levels, float *out, void *stream) {
    using namespace gs;
    if (!img || !out || C <= 0 || H <= 0 || W <= 0 || levels <= 0 || levels > 16)
        return GS_ERR_INVALID_ARGUMENT;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n0 = int64_t(C) * H * W;
    hipLaunchKernelGGL(copy_f32_kernel, dim3((n0 + 255) / 256), dim3(256), 0, st, img, out, n0);
    const float *prev = out;
    float *cur = out + n0;
    int h = H, w = W;
    for (int l = 1; l < levels; ++l) {
        const int ho = (h + 1) / 2, wo = (w + 1) / 2;
        const int64_t no = int64_t(C) * ho * wo;
        hipLaunchKernelGGL(pyr_down_kernel, dim3((no + 255) / 256), dim3(256), 0, st, prev, C, h, w, cur);
        prev = cur;
        cur += no;
        h = ho;
        w = wo;
    }
    GS_CHECK_LAUNCH();
    return GS_OK;
}

extern "C" gs_status gs_pyramid_loss(const float *render, const float *target,
                                     const gs_target *targets, int32_t n_targets,
                                     int32_t total_tiles, int64_t total_pixels, float lambda,
                                     void *loss_ws, float *d_loss, float *d_total,
                                     float *dL_drender, void *stream) {
    using namespace gs;
    if (!render || !target || !targets || !loss_ws || n_targets <= 0 || total_tiles <= 0 || n_targets > total_tiles ||
        total_pixels <= 0 || !(lambda >= 0.f && lambda <= 1.f))
        return GS_ERR_INVALID_ARGUMENT;
    hipStream_t st = static_cast<hipStream_t>(stream);
    LossLayout L = LossLayout::make(total_pixels, total_tiles);
    char *b = static_cast<char *>(loss_ws);
    float *partial = reinterpret_cast<float *>(b + L.partial);
    float *maps = reinterpret_cast<float *>(b + L.maps);
    const Window win = ssim_window();
    const int64_t grid = xcd_grid(total_tiles);
    hipLaunchKernelGGL(ssim_fwd_kernel, dim3(grid), dim3(kTilePix), 0, st, render, target, targets,
                       n_targets, total_tiles, win, maps, partial);
    double *tloss = reinterpret_cast<double *>(b + L.tloss);
    const bool few = n_targets <= kLossOneBlockTargets;
    if (dL_drender && few) {
        hipLaunchKernelGGL(ssim_bwd_kernel<true>, dim3(grid), dim3(kTilePix), 0, st, render, target, targets,
                           n_targets, total_tiles, win, lambda, maps, dL_drender, partial, tloss, d_loss, d_total);
        GS_CHECK_LAUNCH();
        return GS_OK;
    }
    if (dL_drender)
        hipLaunchKernelGGL(ssim_bwd_kernel<false>, dim3(grid), dim3(kTilePix), 0, st, render, target, targets,
                           n_targets, total_tiles, win, lambda, maps, dL_drender, partial, tloss, d_loss, d_total);
    if (few) {
        hipLaunchKernelGGL(loss_few_kernel, dim3(1), dim3(256), 0, st, targets, n_targets, lambda, partial,
                           tloss, d_loss, d_total);
    } else {
        hipLaunchKernelGGL(loss_target_kernel, dim3(n_targets), dim3(256), 0, st, targets, lambda, partial,
                           tloss, d_loss);
        hipLaunchKernelGGL(loss_total_kernel, dim3(1), dim3(64), 0, st, n_targets, tloss, d_total);
    }
    GS_CHECK_LAUNCH();
    return GS_OK;
}
