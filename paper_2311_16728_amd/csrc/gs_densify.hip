// Gradient-driven densification of the map (Section 3.3.1 keeps the split /
// clone rule of 3D Gaussian splatting, Kerbl et al. 2023, Sec. 5.2): the
// gradient statistic, the split / clone / prune decision with compaction
// into new buffers, and the opacity reset.
//
// gs_densify is three launches over blocks of 256 primitives, one per
// thread: count (decisions and per-block totals), a one-workgroup scan of
// the block totals, and scatter (the decisions again, block-local ranks,
// stores).  A decision reads 6 floats per primitive, so making it twice costs
// less than storing it.  The whole pass moves about 1.4 KB per primitive (59
// rows of parameters and of both moments, read and written) and is bound by
// HBM: the copy loops keep several rows in flight per thread, and the stores
// of a wave land on consecutive columns because the ranks are a scan.

#include "gs_internal.hpp"

#include <cmath>

namespace gs {
namespace {

constexpr int kDenThreads = 256;          // one primitive per thread
constexpr int kDenBlock = kDenThreads;
constexpr int kDenRows = 16;              // rows in flight per thread in the copy loops

// Outcome for one original primitive.
struct Fate {
    bool keep;    // the original survives
    bool split;   // densified by splitting (else by cloning when nnew > 0)
    int nnew;     // new primitives it adds: 0, 1 (copy) or 2 (children)
};

__device__ __forceinline__ Fate decide(const gs_densify_rule &r, float s0, float s1, float l0,
                                       float l1, float l2, float logit) {
    const float avg = s1 > 0.f ? s0 / s1 : 0.f;
    const float maxls = fmaxf(fmaxf(l0, l1), l2);
    const bool faint = logit < r.logit_min;
    const bool prune = faint || maxls > r.log_big;
    Fate f{!prune, false, 0};
    if (avg >= r.grad_threshold) {
        if (maxls <= r.log_dense) {
            f.nnew = prune ? 0 : 1;
        } else {
            f.keep = false;
            f.split = true;
            const bool child_big = (maxls - r.log_shrink) > r.log_big;
            f.nnew = (faint || child_big) ? 0 : 2;
        }
    }
    return f;
}

// Fate of primitive g (nothing for g >= n).
__device__ __forceinline__ Fate fate_of(const gs_densify_rule &r, const float *__restrict__ P,
                                        const float *__restrict__ stats, int64_t n, int64_t n_cap,
                                        int64_t g) {
    if (g >= n) return Fate{false, false, 0};
    return decide(r, stats[g], stats[n_cap + g], P[3 * n_cap + g], P[4 * n_cap + g],
                  P[5 * n_cap + g], P[10 * n_cap + g]);
}

__global__ void __launch_bounds__(kDenThreads) densify_count_kernel(
    gs_densify_rule r, const float *__restrict__ P, const float *__restrict__ stats, int64_t n,
    int64_t n_cap, int64_t n_blocks, int4 *__restrict__ blk) {
    const int64_t b = xcd_tile(blockIdx.x, n_blocks);
    if (b >= n_blocks) return;
    const int64_t g = b * kDenBlock + threadIdx.x;
    const Fate f = fate_of(r, P, stats, n, n_cap, g);
    // kept originals, new primitives, copies made, splits
    int c[4] = {f.keep, f.nnew, !f.split && f.nnew > 0, f.split};
    __shared__ int part[kDenThreads / kWave][4];
    const int wave = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int s = wave_sum(c[k]);
        if (lane_id() == 0) part[wave][k] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int t[4] = {0, 0, 0, 0};
        for (int w = 0; w < kDenThreads / kWave; ++w)
            for (int k = 0; k < 4; ++k) t[k] += part[w][k];
        blk[b] = make_int4(t[0], t[1], t[2], t[3]);
    }
}

// One workgroup: exclusive offsets of the kept originals (x) and new
// primitives (y) of every block, in place; totals to tot[0..1] and d_counts.
// Each thread takes kScanItems consecutive blocks per round.
__global__ void __launch_bounds__(kScanThreads) densify_scan_kernel(int4 *__restrict__ blk,
                                                                    int64_t n_blocks, int64_t n,
                                                                    int64_t *__restrict__ tot,
                                                                    int64_t *__restrict__ d_counts) {
    __shared__ uint32_t lds[8];
    int64_t carry_k = 0, carry_n = 0, copies = 0, splits = 0;
    for (int64_t c0 = 0; c0 < n_blocks; c0 += kScanTile) {
        const int64_t b0 = c0 + int64_t(threadIdx.x) * kScanItems;
        int4 e[kScanItems];
        uint32_t sk = 0, sn = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            e[i] = b0 + i < n_blocks ? blk[b0 + i] : make_int4(0, 0, 0, 0);
            sk += uint32_t(e[i].x);
            sn += uint32_t(e[i].y);
            copies += e[i].z;
            splits += e[i].w;
        }
        uint32_t tk, tn;
        uint32_t ek = block_exclusive_scan(sk, lds, &tk);
        uint32_t en = block_exclusive_scan(sn, lds, &tn);
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if (b0 + i < n_blocks)
                blk[b0 + i] = make_int4(int(carry_k + ek), int(carry_n + en), e[i].z, e[i].w);
            ek += uint32_t(e[i].x);
            en += uint32_t(e[i].y);
        }
        carry_k += tk;
        carry_n += tn;
    }
    copies = wave_sum(copies);
    splits = wave_sum(splits);
    __shared__ int64_t red[2][kScanThreads / kWave];
    const int wave = threadIdx.x / kWave;
    if (lane_id() == 0) { red[0][wave] = copies; red[1][wave] = splits; }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t cs = 0, ss = 0;
        for (int w = 0; w < kScanThreads / kWave; ++w) { cs += red[0][w]; ss += red[1][w]; }
        tot[0] = carry_k;
        tot[1] = carry_n;
        d_counts[0] = carry_k + carry_n;
        d_counts[1] = cs;
        d_counts[2] = ss;
        d_counts[3] = n - ss - carry_k;
    }
}

// Stores of one output column's value for row `row`: the surviving original,
// then its copy or its two children (child values given).
__device__ __forceinline__ void put(float *__restrict__ o, const Fate &f, int64_t dk, int64_t dn,
                                    float x, float c0, float c1) {
    if (f.keep) o[dk] = x;
    if (f.nnew == 1) o[dn] = x;
    if (f.nnew == 2) { o[dn] = c0; o[dn + 1] = c1; }
}

__global__ void __launch_bounds__(kDenThreads) densify_scatter_kernel(
    gs_densify_rule r, const float *__restrict__ P, const float *__restrict__ m,
    const float *__restrict__ v, const float *__restrict__ stats, const float *__restrict__ noise,
    int64_t n, int64_t n_cap, float *__restrict__ oP, float *__restrict__ om, float *__restrict__ ov,
    int64_t out_cap, int64_t n_blocks, const int4 *__restrict__ blk, const int64_t *__restrict__ tot) {
    // neighbouring blocks write the two ends of the same cache lines: keep
    // them on one XCD (one L2)
    const int64_t b = xcd_tile(blockIdx.x, n_blocks);
    const int64_t K = tot[0];
    if (b >= n_blocks || K + tot[1] > out_cap) return;   // uniform per block
    const int64_t g = b * kDenBlock + threadIdx.x;
    const Fate f = fate_of(r, P, stats, n, n_cap, g);
    __shared__ uint32_t lds[8];
    uint32_t tk, tn;
    const uint32_t ek = block_exclusive_scan(uint32_t(f.keep), lds, &tk);
    const uint32_t en = block_exclusive_scan(uint32_t(f.nnew), lds, &tn);
    if (!f.keep && f.nnew == 0) return;   // also every g >= n
    const int4 off = blk[b];
    const int64_t dk = int64_t(off.x) + ek, dn = K + int64_t(off.y) + en;

    // rows 0-5: children move their centre by Rq (s * z_c) and shrink
    {
        float raw[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) raw[k] = P[int64_t(k) * n_cap + g];
        float d0[3] = {0.f, 0.f, 0.f}, d1[3] = {0.f, 0.f, 0.f};
        if (f.nnew == 2) {
            float z[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) z[k] = noise[int64_t(k) * n_cap + g];
            float w = raw[6], x = raw[7], y = raw[8], zz = raw[9];
            const float inv = 1.f / sqrtf(w * w + x * x + y * y + zz * zz);
            w *= inv; x *= inv; y *= inv; zz *= inv;
            const float R[9] = {1.f - 2.f * (y * y + zz * zz), 2.f * (x * y - w * zz), 2.f * (x * zz + w * y),
                                2.f * (x * y + w * zz), 1.f - 2.f * (x * x + zz * zz), 2.f * (y * zz - w * x),
                                2.f * (x * zz - w * y), 2.f * (y * zz + w * x), 1.f - 2.f * (x * x + y * y)};
            const float s[3] = {expf(raw[3]), expf(raw[4]), expf(raw[5])};
            const float u0[3] = {s[0] * z[0], s[1] * z[1], s[2] * z[2]};
            const float u1[3] = {s[0] * z[3], s[1] * z[4], s[2] * z[5]};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                d0[a] = R[3 * a] * u0[0] + R[3 * a + 1] * u0[1] + R[3 * a + 2] * u0[2];
                d1[a] = R[3 * a] * u1[0] + R[3 * a + 1] * u1[1] + R[3 * a + 2] * u1[2];
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
            put(oP + int64_t(a) * out_cap, f, dk, dn, raw[a], raw[a] + d0[a], raw[a] + d1[a]);
#pragma unroll
        for (int a = 3; a < 6; ++a) {
            const float y = raw[a] - r.log_shrink;
            put(oP + int64_t(a) * out_cap, f, dk, dn, raw[a], y, y);
        }
#pragma unroll
        for (int a = 6; a < 10; ++a) put(oP + int64_t(a) * out_cap, f, dk, dn, raw[a], raw[a], raw[a]);
    }
    // rows 10-58: copies, kDenRows loads in flight
    for (int row = 10; row < kRows; row += kDenRows) {
        float x[kDenRows];
#pragma unroll
        for (int k = 0; k < kDenRows; ++k)
            if (row + k < kRows) x[k] = P[int64_t(row + k) * n_cap + g];
#pragma unroll
        for (int k = 0; k < kDenRows; ++k)
            if (row + k < kRows) put(oP + int64_t(row + k) * out_cap, f, dk, dn, x[k], x[k], x[k]);
    }
    // moments: survivors keep theirs, new primitives start at zero
    for (int row = 0; row < kRows; row += kDenRows / 2) {
        float a[kDenRows / 2], b[kDenRows / 2];
#pragma unroll
        for (int k = 0; k < kDenRows / 2; ++k)
            if (row + k < kRows && f.keep) {
                a[k] = m[int64_t(row + k) * n_cap + g];
                b[k] = v[int64_t(row + k) * n_cap + g];
            }
#pragma unroll
        for (int k = 0; k < kDenRows / 2; ++k) {
            if (row + k >= kRows) continue;
            float *o1 = om + int64_t(row + k) * out_cap, *o2 = ov + int64_t(row + k) * out_cap;
            if (f.keep) { o1[dk] = a[k]; o2[dk] = b[k]; }
            for (int c = 0; c < f.nnew; ++c) { o1[dn + c] = 0.f; o2[dn + c] = 0.f; }
        }
    }
}

__global__ void densify_stats_kernel(const float *__restrict__ acc, int64_t n, int64_t n_cap,
                                     const gs_view *__restrict__ views, int32_t n_views,
                                     float *__restrict__ stats) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= n) return;
    float s0 = stats[g], s1 = stats[n_cap + g];
    for (int vi = 0; vi < n_views; ++vi) {
        const float *a = acc + (int64_t(vi) * n_cap + g) * kAccRows;
        float x[kAccRows];
        bool any = false;
#pragma unroll
        for (int k = 0; k < kAccRows; ++k) { x[k] = a[k]; any |= (x[k] != 0.f); }
        if (!any) continue;
        const float gx = x[0] * (0.5f * float(views[vi].width));
        const float gy = x[1] * (0.5f * float(views[vi].height));
        s0 += sqrtf(gx * gx + gy * gy);
        s1 += 1.f;
    }
    stats[g] = s0;
    stats[n_cap + g] = s1;
}

__global__ void reset_opacity_kernel(float *__restrict__ P, float *__restrict__ m,
                                     float *__restrict__ v, int64_t n, int64_t n_cap, float cap) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int64_t i = 10 * n_cap + g;
    if (P[i] > cap) P[i] = cap;
    if (m) m[i] = 0.f;
    if (v) v[i] = 0.f;
}

struct DensifyWs {
    size_t blk, tot, bytes;
    static DensifyWs make(int64_t n) {
        DensifyWs L;
        const int64_t nb = (n + kDenBlock - 1) / kDenBlock;
        L.blk = 0;
        L.tot = align_up(sizeof(int4) * (nb > 0 ? nb : 1), 256);
        L.bytes = L.tot + 256;
        return L;
    }
};

}  // namespace
}  // namespace gs

using namespace gs;

extern "C" gs_status gs_densify_rule_make(double extent, double grad_threshold, double percent_dense,
                                          double min_opacity, double big_fraction, double shrink,
                                          gs_densify_rule *out) {
    if (!out || !(extent > 0) || !(percent_dense > 0) || !(shrink > 0) || !(min_opacity > 0) ||
        !(min_opacity < 1) || !std::isfinite(grad_threshold))
        return GS_ERR_INVALID_ARGUMENT;
    out->grad_threshold = float(grad_threshold);
    out->log_dense = float(std::log(percent_dense * extent));
    out->log_big = big_fraction > 0 ? float(std::log(big_fraction * extent)) : INFINITY;
    out->logit_min = float(std::log(min_opacity / (1.0 - min_opacity)));
    out->log_shrink = float(std::log(shrink));
    return GS_OK;
}

extern "C" gs_status gs_densify_stats(const void *accum_ws, int64_t n, int64_t n_cap,
                                      const gs_view *views, int32_t n_views, float *stats,
                                      void *stream) {
    if (!accum_ws || !views || !stats || n < 0 || n > n_cap || n_cap % 64 || n_views <= 0)
        return GS_ERR_INVALID_ARGUMENT;
    if (n == 0) return GS_OK;
    hipLaunchKernelGGL(densify_stats_kernel, dim3((n + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), static_cast<const float *>(accum_ws), n,
                       n_cap, views, n_views, stats);
    GS_CHECK_LAUNCH();
    return GS_OK;
}

extern "C" size_t gs_densify_workspace_bytes(int64_t n) {
    return DensifyWs::make(n < 0 ? 0 : n).bytes;
}

extern "C" gs_status gs_densify(const gs_densify_rule *rule, const float *params, const float *m,
                                const float *v, const float *stats, const float *noise, int64_t n,
                                int64_t n_cap, float *out_params, float *out_m, float *out_v,
                                int64_t out_cap, void *ws, int64_t *d_counts, void *stream) {
    if (!rule || !params || !m || !v || !stats || !noise || !out_params || !out_m || !out_v || !ws ||
        !d_counts || n < 0 || n > n_cap || n_cap % 64 || out_cap < 0 || out_cap % 64 ||
        n_cap >= (int64_t(1) << 31) || out_cap >= (int64_t(1) << 31))
        return GS_ERR_INVALID_ARGUMENT;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const DensifyWs L = DensifyWs::make(n);
    char *b = static_cast<char *>(ws);
    int4 *blk = reinterpret_cast<int4 *>(b + L.blk);
    int64_t *tot = reinterpret_cast<int64_t *>(b + L.tot);
    const int64_t nb = (n + kDenBlock - 1) / kDenBlock;
    if (nb > 0)
        hipLaunchKernelGGL(densify_count_kernel, dim3(xcd_grid(nb)), dim3(kDenThreads), 0, st, *rule,
                           params, stats, n, n_cap, nb, blk);
    hipLaunchKernelGGL(densify_scan_kernel, dim3(1), dim3(kScanThreads), 0, st, blk, nb, n, tot,
                       d_counts);
    if (nb > 0)
        hipLaunchKernelGGL(densify_scatter_kernel, dim3(xcd_grid(nb)), dim3(kDenThreads), 0, st, *rule,
                           params, m, v, stats, noise, n, n_cap, out_params, out_m, out_v, out_cap, nb,
                           blk, tot);
    GS_CHECK_LAUNCH();
    return GS_OK;
}

extern "C" gs_status gs_reset_opacity(float *params, float *m, float *v, int64_t n, int64_t n_cap,
                                      double max_opacity, void *stream) {
    if (!params || n < 0 || n > n_cap || !(max_opacity > 0) || !(max_opacity < 1))
        return GS_ERR_INVALID_ARGUMENT;
    if (n == 0) return GS_OK;
    const float cap = float(std::log(max_opacity / (1.0 - max_opacity)));
    hipLaunchKernelGGL(reset_opacity_kernel, dim3((n + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), params, m, v, n, n_cap, cap);
    GS_CHECK_LAUNCH();
    return GS_OK;
}
