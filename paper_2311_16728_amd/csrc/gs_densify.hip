// Gradient-driven densification of the map (Section 3.3.1 keeps the split /
// clone rule of 3D Gaussian splatting, Kerbl et al. 2023, Sec. 5.2): the
// gradient statistic, the split / clone / prune decision with compaction
// into new buffers, and the opacity reset.
//
// gs_densify is three launches over blocks of 1024 primitives, four
// consecutive ones per thread so that every row is read with one 16-byte
// load per thread: count (decisions and per-block totals), a one-workgroup
// scan of the block totals, and scatter (the decisions again, block-local
// ranks, stores).  A decision reads 6 floats per primitive, so making it
// twice costs less than storing it.  The whole pass moves about 1.4 KB per
// primitive (59 rows of parameters and of both moments, read and written)
// and is bound by HBM.

#include "gs_internal.hpp"

#include <cmath>

namespace gs {
namespace {

constexpr int kDenThreads = 256;
constexpr int kDenPer = 4;
constexpr int kDenBlock = kDenThreads * kDenPer;

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

__device__ __forceinline__ float4 row4(const float *__restrict__ a, int row, int64_t n_cap,
                                       int64_t base) {
    return *reinterpret_cast<const float4 *>(a + int64_t(row) * n_cap + base);
}

__device__ __forceinline__ float lane4(const float4 &v, int i) {
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

// Fates of the (up to) four primitives base..base+3 below n.
__device__ __forceinline__ void fates(const gs_densify_rule &r, const float *__restrict__ P,
                                      const float *__restrict__ stats, int64_t n, int64_t n_cap,
                                      int64_t base, Fate (&f)[kDenPer]) {
#pragma unroll
    for (int i = 0; i < kDenPer; ++i) f[i] = Fate{false, false, 0};
    if (base >= n) return;
    const float4 s0 = row4(stats, 0, n_cap, base), s1 = row4(stats, 1, n_cap, base);
    const float4 l0 = row4(P, 3, n_cap, base), l1 = row4(P, 4, n_cap, base);
    const float4 l2 = row4(P, 5, n_cap, base), op = row4(P, 10, n_cap, base);
#pragma unroll
    for (int i = 0; i < kDenPer; ++i)
        if (base + i < n)
            f[i] = decide(r, lane4(s0, i), lane4(s1, i), lane4(l0, i), lane4(l1, i), lane4(l2, i),
                          lane4(op, i));
}

__global__ void __launch_bounds__(kDenThreads) densify_count_kernel(
    gs_densify_rule r, const float *__restrict__ P, const float *__restrict__ stats, int64_t n,
    int64_t n_cap, int4 *__restrict__ blk) {
    const int64_t base = int64_t(blockIdx.x) * kDenBlock + int64_t(threadIdx.x) * kDenPer;
    Fate f[kDenPer];
    fates(r, P, stats, n, n_cap, base, f);
    int c[4] = {0, 0, 0, 0};   // kept originals, new primitives, copies made, splits
#pragma unroll
    for (int i = 0; i < kDenPer; ++i) {
        c[0] += f[i].keep;
        c[1] += f[i].nnew;
        c[2] += (!f[i].split && f[i].nnew > 0);
        c[3] += f[i].split;
    }
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
        blk[blockIdx.x] = make_int4(t[0], t[1], t[2], t[3]);
    }
}

// One workgroup: exclusive offsets of the kept originals (x) and new
// primitives (y) of every block, in place; totals to tot[0..1] and d_counts.
__global__ void __launch_bounds__(kScanThreads) densify_scan_kernel(int4 *__restrict__ blk,
                                                                    int64_t n_blocks, int64_t n,
                                                                    int64_t *__restrict__ tot,
                                                                    int64_t *__restrict__ d_counts) {
    __shared__ uint32_t lds[8];
    int64_t carry_k = 0, carry_n = 0, copies = 0, splits = 0;
    for (int64_t c0 = 0; c0 < n_blocks; c0 += kScanThreads) {
        const int64_t b = c0 + threadIdx.x;
        const int4 v = b < n_blocks ? blk[b] : make_int4(0, 0, 0, 0);
        uint32_t tk, tn;
        const uint32_t ek = block_exclusive_scan(uint32_t(v.x), lds, &tk);
        const uint32_t en = block_exclusive_scan(uint32_t(v.y), lds, &tn);
        if (b < n_blocks) blk[b] = make_int4(int(carry_k + ek), int(carry_n + en), v.z, v.w);
        carry_k += tk;
        carry_n += tn;
        copies += v.z;
        splits += v.w;
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

__global__ void __launch_bounds__(kDenThreads) densify_scatter_kernel(
    gs_densify_rule r, const float *__restrict__ P, const float *__restrict__ m,
    const float *__restrict__ v, const float *__restrict__ stats, const float *__restrict__ noise,
    int64_t n, int64_t n_cap, float *__restrict__ oP, float *__restrict__ om, float *__restrict__ ov,
    int64_t out_cap, const int4 *__restrict__ blk, const int64_t *__restrict__ tot) {
    const int64_t K = tot[0];
    if (K + tot[1] > out_cap) return;   // the same for every thread of the grid
    const int64_t base = int64_t(blockIdx.x) * kDenBlock + int64_t(threadIdx.x) * kDenPer;
    Fate f[kDenPer];
    fates(r, P, stats, n, n_cap, base, f);
    uint32_t kc = 0, nc = 0;
#pragma unroll
    for (int i = 0; i < kDenPer; ++i) { kc += f[i].keep; nc += f[i].nnew; }
    __shared__ uint32_t lds[8];
    uint32_t tk, tn;
    const uint32_t ek = block_exclusive_scan(kc, lds, &tk);
    const uint32_t en = block_exclusive_scan(nc, lds, &tn);
    if (base >= n) return;
    const int4 off = blk[blockIdx.x];
    int64_t dk[kDenPer], dn[kDenPer];
    {
        int64_t k = int64_t(off.x) + ek, q = K + int64_t(off.y) + en;
#pragma unroll
        for (int i = 0; i < kDenPer; ++i) {
            dk[i] = k; k += f[i].keep;
            dn[i] = q; q += f[i].nnew;
        }
    }
    bool any_split = false;
#pragma unroll
    for (int i = 0; i < kDenPer; ++i) any_split |= (f[i].split && f[i].nnew == 2);

    // child offsets Rq (s * z_c), only where a split is written
    float off3[kDenPer][2][3];
#pragma unroll
    for (int i = 0; i < kDenPer; ++i)
#pragma unroll
        for (int c = 0; c < 2; ++c) off3[i][c][0] = off3[i][c][1] = off3[i][c][2] = 0.f;
    if (any_split) {
        float4 q4[4], ls4[3], z4[6];
#pragma unroll
        for (int k = 0; k < 4; ++k) q4[k] = row4(P, 6 + k, n_cap, base);
#pragma unroll
        for (int k = 0; k < 3; ++k) ls4[k] = row4(P, 3 + k, n_cap, base);
#pragma unroll
        for (int k = 0; k < 6; ++k) z4[k] = row4(noise, k, n_cap, base);
#pragma unroll
        for (int i = 0; i < kDenPer; ++i) {
            if (!(f[i].split && f[i].nnew == 2)) continue;
            float w = lane4(q4[0], i), x = lane4(q4[1], i), y = lane4(q4[2], i), z = lane4(q4[3], i);
            const float inv = 1.f / sqrtf(w * w + x * x + y * y + z * z);
            w *= inv; x *= inv; y *= inv; z *= inv;
            const float R[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                                2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                                2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
            const float s[3] = {expf(lane4(ls4[0], i)), expf(lane4(ls4[1], i)), expf(lane4(ls4[2], i))};
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const float u[3] = {s[0] * lane4(z4[3 * c], i), s[1] * lane4(z4[3 * c + 1], i),
                                    s[2] * lane4(z4[3 * c + 2], i)};
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    off3[i][c][a] = R[3 * a] * u[0] + R[3 * a + 1] * u[1] + R[3 * a + 2] * u[2];
            }
        }
    }

    // parameters: rows 0-2 and 3-5 differ for children, the rest are copies
#pragma unroll 1
    for (int row = 0; row < kRows; ++row) {
        const float4 pv = row4(P, row, n_cap, base);
        float *o = oP + int64_t(row) * out_cap;
#pragma unroll
        for (int i = 0; i < kDenPer; ++i) {
            const float x = lane4(pv, i);
            if (f[i].keep) o[dk[i]] = x;
            if (f[i].nnew == 0) continue;
            if (!f[i].split) {
                o[dn[i]] = x;
            } else if (row < 3) {
                o[dn[i]] = x + off3[i][0][row];
                o[dn[i] + 1] = x + off3[i][1][row];
            } else if (row < 6) {
                const float y = x - r.log_shrink;
                o[dn[i]] = y;
                o[dn[i] + 1] = y;
            } else {
                o[dn[i]] = x;
                o[dn[i] + 1] = x;
            }
        }
    }
    // moments: survivors keep theirs, new primitives start at zero
#pragma unroll 1
    for (int row = 0; row < kRows; ++row) {
        const float4 mv = row4(m, row, n_cap, base), vv = row4(v, row, n_cap, base);
        float *o1 = om + int64_t(row) * out_cap, *o2 = ov + int64_t(row) * out_cap;
#pragma unroll
        for (int i = 0; i < kDenPer; ++i) {
            if (f[i].keep) { o1[dk[i]] = lane4(mv, i); o2[dk[i]] = lane4(vv, i); }
            for (int c = 0; c < f[i].nnew; ++c) { o1[dn[i] + c] = 0.f; o2[dn[i] + c] = 0.f; }
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
    // rows are read with 16-byte loads
    for (const void *p : {static_cast<const void *>(params), static_cast<const void *>(m),
                          static_cast<const void *>(v), static_cast<const void *>(stats),
                          static_cast<const void *>(noise)})
        if (reinterpret_cast<uintptr_t>(p) % 16) return GS_ERR_INVALID_ARGUMENT;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const DensifyWs L = DensifyWs::make(n);
    char *b = static_cast<char *>(ws);
    int4 *blk = reinterpret_cast<int4 *>(b + L.blk);
    int64_t *tot = reinterpret_cast<int64_t *>(b + L.tot);
    const int64_t nb = (n + kDenBlock - 1) / kDenBlock;
    if (nb > 0)
        hipLaunchKernelGGL(densify_count_kernel, dim3(nb), dim3(kDenThreads), 0, st, *rule, params,
                           stats, n, n_cap, blk);
    hipLaunchKernelGGL(densify_scan_kernel, dim3(1), dim3(kScanThreads), 0, st, blk, nb, n, tot,
                       d_counts);
    if (nb > 0)
        hipLaunchKernelGGL(densify_scatter_kernel, dim3(nb), dim3(kDenThreads), 0, st, *rule, params,
                           m, v, stats, noise, n, n_cap, out_params, out_m, out_v, out_cap, blk, tot);
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
