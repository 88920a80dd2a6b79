// Tile rasteriser: Eq. 3 forward (front-to-back alpha compositing) and its
// reverse mode, recomputed back to front.
//
// One 256-thread workgroup (four waves) per 16x16 tile, one pixel per thread;
// wave w owns pixel rows 4w..4w+3 of the tile.  The tile's sorted list is
// consumed in batches: each thread gathers one Gaussian's record, converts it
// to the target's pyramid level (2D mean scaled by 2^-l, covariance by 4^-l
// plus the dilation, then inverted to the conic) and stages it in LDS; every
// pixel then reads the batch as LDS broadcasts.  The forward keeps, per
// pixel, only the final transmittance and one past the list position of the
// last composited Gaussian; the backward restarts from those, divides the
// transmittance back out Gaussian by Gaussian, and keeps a running colour of
// what lies behind, so no per-pixel list is stored.  Gradients of the nine 2D
// quantities are summed over the wave with cross-lane shuffles and committed
// with one atomic per quantity per wave.
#include "gs_internal.hpp"

namespace gs {

// Finds the target owning global tile `tile` (targets sorted by tile_offset).
__device__ __forceinline__ int find_target(const gs_target *__restrict__ targets, int n_targets,
                                           int tile) {
    int lo = 0, hi = n_targets - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (targets[mid].tile_offset <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The record of source `src` as seen by a target at pyramid level `level`,
// with its 2D mean relative to the tile origin (ox, oy): the FP64 mean is
// reduced before rounding, so offsets inside the tile are accurate to a few
// 1e-7 px.
__device__ __forceinline__ void stage_record(const gs_settings &s, const Proj &proj, int64_t n_cap,
                                             int view, int level, double ox, double oy, uint32_t src,
                                             float4 &A, float4 &B, float &blue, int64_t &rec) {
    const int64_t g = int64_t(src % uint32_t(n_cap));
    const int64_t r = int64_t(view) * n_cap + g;
    rec = r;
    const float sc = ldexpf(1.f, -level);
    const double2 m = proj.mean[r];
    const float4 co = proj.cov_o[r];
    const float4 cz = proj.rgb_z[r];
    const float c00 = fmaf(co.x, sc * sc, s.dilation);
    const float c01 = co.y * (sc * sc);
    const float c11 = fmaf(co.z, sc * sc, s.dilation);
    const float det = c00 * c11 - c01 * c01;
    const float idet = 1.f / det;
    const double dsc = double(sc);
    A = make_float4(float(m.x * dsc - ox), float(m.y * dsc - oy), c11 * idet, -c01 * idet);
    B = make_float4(c00 * idet, co.w, cz.x, cz.y);
    blue = cz.z;
}

// Opacity of a staged Gaussian at offset (dx, dy) = mean - pixel.  The same
// instruction sequence serves the forward and the backward, so both take the
// same alpha_min decision.
__device__ __forceinline__ float eval_power(const float4 &A, const float4 &B, float dx, float dy) {
    const float q = fmaf(A.z * dx, dx, B.x * dy * dy);
    return fmaf(-0.5f, q, -(A.w * dx * dy));
}

__global__ void __launch_bounds__(256) render_fwd_kernel(
    gs_settings s, Proj proj, int64_t n_cap, Sorted srt, const gs_target *__restrict__ targets,
    int n_targets, float *__restrict__ out_rgb, float *__restrict__ out_T,
    int32_t *__restrict__ out_last, int32_t *__restrict__ out_nc) {
    __shared__ float4 sA[kTilePix];
    __shared__ float4 sB[kTilePix];
    __shared__ float sC[kTilePix];
    const int tile = blockIdx.x;
    const int tid = threadIdx.x;
    const gs_target t = targets[find_target(targets, n_targets, tile)];
    const int local = tile - t.tile_offset;
    const int tx = local % t.tiles_x, ty = local / t.tiles_x;
    const int px = tx * kTile + (tid % kTile), py = ty * kTile + tid / kTile;
    const bool inside = px < t.width && py < t.height;
    const uint2 range = srt.ranges[tile];
    const double ox = double(tx * kTile), oy = double(ty * kTile);
    const float fpx = float(tid % kTile), fpy = float(tid / kTile);   // relative to the tile origin

    float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
    int32_t nc = 0, last = 0;
    bool done = !inside;
    const int batch = s.batch;
    for (uint32_t b0 = range.x; b0 < range.y; b0 += batch) {
        if (__syncthreads_count(done) == kTilePix) break;
        const uint32_t idx = b0 + tid;
        if (tid < batch && idx < range.y) {
            float4 A, B;
            float blue;
            int64_t rec;
            stage_record(s, proj, n_cap, t.view, t.level, ox, oy, srt.pair_val[idx], A, B, blue, rec);
            sA[tid] = A;
            sB[tid] = B;
            sC[tid] = blue;
        }
        __syncthreads();
        const int cnt = min(uint32_t(batch), range.y - b0);
        if (!done) {
            for (int j = 0; j < cnt; ++j) {
                const float4 A = sA[j];
                const float4 B = sB[j];
                const float dx = A.x - fpx, dy = A.y - fpy;
                const float at = B.y * __expf(eval_power(A, B, dx, dy));
                if (at < s.alpha_min) continue;
                const float alpha = fminf(s.alpha_max, at);
                const float Tn = T * (1.f - alpha);
                if (Tn < s.t_min) { done = true; break; }
                const float w = alpha * T;
                C0 = fmaf(w, B.z, C0);
                C1 = fmaf(w, B.w, C1);
                C2 = fmaf(w, sC[j], C2);
                T = Tn;
                ++nc;
                last = int32_t(b0 - range.x) + j + 1;
            }
        }
    }
    if (inside) {
        const int64_t HW = int64_t(t.width) * t.height;
        const int64_t pix = int64_t(py) * t.width + px;
        float *rgb = out_rgb + 3 * t.pix_offset;
        rgb[pix] = fmaf(T, t.bg[0], C0);
        rgb[HW + pix] = fmaf(T, t.bg[1], C1);
        rgb[2 * HW + pix] = fmaf(T, t.bg[2], C2);
        out_T[t.pix_offset + pix] = T;
        out_last[t.pix_offset + pix] = last;
        if (out_nc) out_nc[t.pix_offset + pix] = nc;
    }
}

__global__ void __launch_bounds__(256) render_bwd_kernel(
    gs_settings s, Proj proj, int64_t n_cap, Sorted srt, const gs_target *__restrict__ targets,
    int n_targets, const float *__restrict__ in_T, const int32_t *__restrict__ in_last,
    const float *__restrict__ dL_drgb, float *__restrict__ acc, int64_t records) {
    __shared__ float4 sA[kTilePix];
    __shared__ float4 sB[kTilePix];
    __shared__ float sC[kTilePix];
    __shared__ int64_t sR[kTilePix];
    __shared__ int sMaxLast;
    const int tile = blockIdx.x;
    const int tid = threadIdx.x;
    const gs_target t = targets[find_target(targets, n_targets, tile)];
    const int local = tile - t.tile_offset;
    const int tx = local % t.tiles_x, ty = local / t.tiles_x;
    const int px = tx * kTile + (tid % kTile), py = ty * kTile + tid / kTile;
    const bool inside = px < t.width && py < t.height;
    const uint2 range = srt.ranges[tile];
    const double ox = double(tx * kTile), oy = double(ty * kTile);
    const float fpx = float(tid % kTile), fpy = float(tid / kTile);   // relative to the tile origin
    const float sc = ldexpf(1.f, -t.level);

    float T = 0.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
    int32_t last = 0;
    if (inside) {
        const int64_t HW = int64_t(t.width) * t.height;
        const int64_t pix = int64_t(py) * t.width + px;
        T = in_T[t.pix_offset + pix];
        last = in_last[t.pix_offset + pix];
        const float *d = dL_drgb + 3 * t.pix_offset;
        g0 = d[pix];
        g1 = d[HW + pix];
        g2 = d[2 * HW + pix];
    }
    // a pixel's restart position never exceeds its tile's list (guards stale input)
    last = min(last, int32_t(range.y - range.x));
    float B0 = t.bg[0], B1 = t.bg[1], B2 = t.bg[2];   // colour behind, unit transmittance
    if (tid == 0) sMaxLast = 0;
    __syncthreads();
    if (last > 0) atomicMax(&sMaxLast, last);
    __syncthreads();
    const int max_last = sMaxLast;
    const int batch = s.batch;

    for (int end = max_last; end > 0; end -= batch) {
        const int start = max(0, end - batch);
        __syncthreads();
        if (tid < end - start) {
            float4 A, Bv;
            float blue;
            int64_t rec;
            stage_record(s, proj, n_cap, t.view, t.level, ox, oy, srt.pair_val[range.x + start + tid],
                         A, Bv, blue, rec);
            sA[tid] = A;
            sB[tid] = Bv;
            sC[tid] = blue;
            sR[tid] = rec;
        }
        __syncthreads();
        for (int j = end - 1; j >= start; --j) {
            const int k = j - start;
            const float4 A = sA[k];
            const float4 Bv = sB[k];
            const float dx = A.x - fpx, dy = A.y - fpy;
            const float ep = __expf(eval_power(A, Bv, dx, dy));
            const float at = Bv.y * ep;
            const bool active = (j < last) && !(at < s.alpha_min);
            float v[kAccRows];
            if (active) {
                const float alpha = fminf(s.alpha_max, at);
                const float oma = 1.f - alpha;
                T = T / oma;                       // transmittance in front of this Gaussian
                const float r = Bv.z, gg = Bv.w, bb = sC[k];
                const float dal = T * ((r - B0) * g0 + (gg - B1) * g1 + (bb - B2) * g2);
                const float w = alpha * T;
                v[6] = w * g0;
                v[7] = w * g1;
                v[8] = w * g2;
                B0 = fmaf(alpha, r, oma * B0);
                B1 = fmaf(alpha, gg, oma * B1);
                B2 = fmaf(alpha, bb, oma * B2);
                const float dat = (at < s.alpha_max) ? dal : 0.f;
                v[5] = ep * dat;
                const float dp = at * dat;
                v[0] = -dp * (A.z * dx + A.w * dy);
                v[1] = -dp * (A.w * dx + Bv.x * dy);
                v[2] = -0.5f * dp * dx * dx;
                v[3] = -dp * dx * dy;
                v[4] = -0.5f * dp * dy * dy;
            } else {
#pragma unroll
                for (int i = 0; i < kAccRows; ++i) v[i] = 0.f;
            }
            if (__ballot(active) == 0) continue;
#pragma unroll
            for (int i = 0; i < kAccRows; ++i) v[i] = wave_sum(v[i]);
            if (lane_id() == 0) {
                // conic gradient -> gradient of the dilated covariance, -K dK K,
                // then back to level-0 units.
                const float a = A.z, b = A.w, c = Bv.x;
                const float ga = v[2], gb = 0.5f * v[3], gc = v[4];
                const float k00 = a * ga + b * gb, k01 = a * gb + b * gc;
                const float k10 = b * ga + c * gb, k11 = b * gb + c * gc;
                const float s2 = sc * sc;
                const float d00 = -(k00 * a + k01 * b) * s2;
                const float d01 = -(k00 * b + k01 * c) * s2;
                const float d11 = -(k10 * b + k11 * c) * s2;
                const int64_t rr = sR[k];
                atomicAdd(&acc[0 * records + rr], v[0] * sc);
                atomicAdd(&acc[1 * records + rr], v[1] * sc);
                atomicAdd(&acc[2 * records + rr], d00);
                atomicAdd(&acc[3 * records + rr], d01);
                atomicAdd(&acc[4 * records + rr], d11);
                atomicAdd(&acc[5 * records + rr], v[5]);
                atomicAdd(&acc[6 * records + rr], v[6]);
                atomicAdd(&acc[7 * records + rr], v[7]);
                atomicAdd(&acc[8 * records + rr], v[8]);
            }
        }
    }
}

__global__ void fill_f32_kernel(float *p, int64_t count, float v) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

gs_status launch_project_backward(const gs_settings &s, const float *params, int64_t n,
                                  int64_t n_cap, const gs_view *views, int32_t n_views,
                                  const float *acc, float *grad, hipStream_t st);

static bool valid_settings(const gs_settings *s) {
    return s && s->sh_degree >= 0 && s->sh_degree <= 3 &&
           (s->batch == 64 || s->batch == 128 || s->batch == 256) && s->alpha_min > 0.f &&
           s->alpha_max <= 1.f && s->alpha_max >= s->alpha_min && s->t_min > 0.f &&
           s->dilation >= 0.f && s->fov_clamp > 0.f;
}

}  // namespace gs

extern "C" gs_status gs_render_fwd(const gs_settings *s, const void *proj_ws, int64_t n_cap,
                                   int32_t n_views, const void *sort_ws, int64_t pair_cap,
                                   const gs_target *targets, int32_t n_targets, int32_t total_tiles,
                                   float *out_rgb, float *out_T, int32_t *out_last,
                                   int32_t *out_ncontrib, void *stream) {
    using namespace gs;
    if (!valid_settings(s) || !proj_ws || !sort_ws || !targets || n_cap <= 0 || n_cap % 64 ||
        n_views <= 0 || n_targets <= 0 || total_tiles <= 0 || pair_cap <= 0 || !out_rgb ||
        !out_T || !out_last)
        return GS_ERR_INVALID_ARGUMENT;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t S = int64_t(n_targets) * n_cap;
    const Sorted srt = sorted_at(sort_ws, S, pair_cap, total_tiles);
    const Proj proj = proj_at(const_cast<void *>(proj_ws), int64_t(n_views) * n_cap);
    hipLaunchKernelGGL(render_fwd_kernel, dim3(total_tiles), dim3(kTilePix), 0, st, *s, proj, n_cap,
                       srt, targets, n_targets, out_rgb, out_T, out_last, out_ncontrib);
    GS_CHECK_LAUNCH();
    return GS_OK;
}

extern "C" gs_status gs_render_bwd(const gs_settings *s, const float *params, int64_t n,
                                   int64_t n_cap, const gs_view *views, int32_t n_views,
                                   const void *proj_ws, const void *sort_ws, int64_t pair_cap,
                                   const gs_target *targets, int32_t n_targets, int32_t total_tiles,
                                   const float *out_T, const int32_t *out_last,
                                   const float *dL_drgb, void *accum_ws, float *grad,
                                   void *stream) {
    using namespace gs;
    if (!valid_settings(s) || !params || !views || !proj_ws || !sort_ws || !targets || !out_T ||
        !out_last || !dL_drgb || !accum_ws || !grad || n < 0 || n_cap <= 0 || n > n_cap ||
        n_cap % 64 || n_views <= 0 || n_targets <= 0 || total_tiles <= 0 || pair_cap <= 0)
        return GS_ERR_INVALID_ARGUMENT;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t records = int64_t(n_views) * n_cap;
    const int64_t S = int64_t(n_targets) * n_cap;
    const Sorted srt = sorted_at(sort_ws, S, pair_cap, total_tiles);
    const Proj proj = proj_at(const_cast<void *>(proj_ws), records);
    float *acc = static_cast<float *>(accum_ws);
    const int64_t acc_n = int64_t(kAccRows) * records;
    hipLaunchKernelGGL(fill_f32_kernel, dim3((acc_n + 255) / 256), dim3(256), 0, st, acc, acc_n, 0.f);
    hipLaunchKernelGGL(render_bwd_kernel, dim3(total_tiles), dim3(kTilePix), 0, st, *s, proj, n_cap,
                       srt, targets, n_targets, out_T, out_last, dL_drgb, acc, records);
    GS_CHECK_LAUNCH();
    return launch_project_backward(*s, params, n, n_cap, views, n_views, acc, grad, st);
}

extern "C" gs_status gs_fill(float *dst, int64_t count, float value, void *stream) {
    if (!dst || count < 0) return GS_ERR_INVALID_ARGUMENT;
    if (count == 0) return GS_OK;
    hipLaunchKernelGGL(gs::fill_f32_kernel, dim3((count + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), dst, count, value);
    GS_CHECK_LAUNCH();
    return GS_OK;
}
