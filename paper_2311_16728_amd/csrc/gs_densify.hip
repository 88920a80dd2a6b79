// Gradient-driven densification of the map (Section 3.3.1 keeps the split /
// clone rule of 3D Gaussian splatting, Kerbl et al. 2023, Sec. 5.2): the
// gradient statistic, the split / clone / prune decision with compaction
// into new buffers, and the opacity reset.
//
// gs_densify is four launches.  Count, over blocks of 256 primitives, one
// per thread: the decisions, kept as three 256-bit masks per block (survives;
// the two bits of the number of new primitives) and per-block totals.  A
// one-workgroup scan of the totals into output offsets.  Tables: per 256-wide
// output tile, the source block holding its first column.  Gather, one output
// column per thread: it finds its source primitive by a search over the block
// offsets and a rank select in the block's mask, then copies.  The whole pass
// moves about 1.4 KB per primitive (59 rows of parameters and of both moments,
// read and written) and is bound by HBM; gathering makes every workgroup's
// stores fill 256 consecutive columns of each row, so the writes (the larger
// half of the traffic) are whole cache lines.

#include "gs_internal.hpp"

#include <cmath>
#include <mutex>

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

// Per block of 256 primitives, bit i of word i / 64: the original survives
// (keep), and the two bits of its number of new primitives (lo, hi).
struct BlockMasks {
    uint64_t keep[4], lo[4], hi[4];
};

__global__ void __launch_bounds__(kDenThreads) densify_count_kernel(
    gs_densify_rule r, const float *__restrict__ P, const float *__restrict__ stats, int64_t n,
    int64_t n_cap, int64_t n_blocks, int4 *__restrict__ blk, BlockMasks *__restrict__ masks) {
    const int64_t b = xcd_tile(blockIdx.x, n_blocks);
    if (b >= n_blocks) return;
    const int64_t g = b * kDenBlock + threadIdx.x;
    const Fate f = fate_of(r, P, stats, n, n_cap, g);
    // kept originals, new primitives, copies made, splits
    int c[4] = {f.keep, f.nnew, !f.split && f.nnew > 0, f.split};
    __shared__ int part[kDenThreads / kWave][4];
    const int wave = threadIdx.x / kWave;
    {
        const uint64_t km = __ballot(f.keep), lm = __ballot(f.nnew & 1), hm = __ballot(f.nnew >> 1);
        if (lane_id() == 0) {
            masks[b].keep[wave] = km;
            masks[b].lo[wave] = lm;
            masks[b].hi[wave] = hm;
        }
    }
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

// First source block of every 256-column output tile, for the surviving
// originals (first_keep) and the new primitives (first_new, tiles counted
// from the first new column).  One thread per source block writes the tiles
// whose first column it holds.
__global__ void __launch_bounds__(kDenThreads) densify_tables_kernel(
    const int4 *__restrict__ blk, int64_t n_blocks, const int64_t *__restrict__ tot,
    int32_t *__restrict__ first_keep, int32_t *__restrict__ first_new) {
    const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= n_blocks) return;
    const int4 e = blk[b];
    const int64_t k1 = b + 1 < n_blocks ? blk[b + 1].x : tot[0];
    const int64_t n1 = b + 1 < n_blocks ? blk[b + 1].y : tot[1];
    for (int64_t o = (int64_t(e.x) + kDenBlock - 1) / kDenBlock; o * kDenBlock < k1; ++o)
        first_keep[o] = int32_t(b);
    for (int64_t o = (int64_t(e.y) + kDenBlock - 1) / kDenBlock; o * kDenBlock < n1; ++o)
        first_new[o] = int32_t(b);
}

// Index of the r-th set bit (0-based) of the 256-bit mask m.
__device__ __forceinline__ int select_bit(const uint64_t (&m)[4], uint32_t r) {
    int w = 0;
    while (w < 3 && r >= uint32_t(__popcll(m[w]))) { r -= uint32_t(__popcll(m[w])); ++w; }
    uint64_t x = m[w];
    int pos = 0;
#pragma unroll
    for (int sft = 32; sft >= 1; sft >>= 1) {
        const uint32_t c = uint32_t(__popcll(x & ((uint64_t(1) << sft) - 1)));
        if (r >= c) { r -= c; x >>= sft; pos += sft; }
    }
    return w * 64 + pos;
}

// Item i and child c (r = new primitives before i + c) for per-item counts
// lo_i + 2 hi_i over the 256 items.
__device__ __forceinline__ int select_new(const uint64_t (&lo)[4], const uint64_t (&hi)[4], uint32_t r,
                                          uint32_t &child) {
    int w = 0;
    while (w < 3) {
        const uint32_t c = uint32_t(__popcll(lo[w]) + 2 * __popcll(hi[w]));
        if (r < c) break;
        r -= c;
        ++w;
    }
    uint64_t xl = lo[w], xh = hi[w];
    int pos = 0;
#pragma unroll
    for (int sft = 32; sft >= 1; sft >>= 1) {
        const uint64_t msk = (uint64_t(1) << sft) - 1;
        const uint32_t c = uint32_t(__popcll(xl & msk) + 2 * __popcll(xh & msk));
        if (r >= c) { r -= c; xl >>= sft; xh >>= sft; pos += sft; }
    }
    child = r;
    return w * 64 + pos;
}

// One output column per thread: the surviving original it copies, or the
// original whose copy or child it is.  Stores of a workgroup fill 256
// consecutive columns of every row (whole cache lines for the survivors).
__global__ void __launch_bounds__(kDenThreads) densify_gather_kernel(
    gs_densify_rule r, const float *__restrict__ P, const float *__restrict__ m,
    const float *__restrict__ v, const float *__restrict__ noise, int64_t n_cap,
    float *__restrict__ oP, float *__restrict__ om, float *__restrict__ ov, int64_t out_cap,
    int64_t n_blocks, int64_t keep_tiles, const int4 *__restrict__ blk,
    const BlockMasks *__restrict__ masks, const int32_t *__restrict__ first_keep,
    const int32_t *__restrict__ first_new, const int64_t *__restrict__ tot) {
    const int64_t K = tot[0], N = tot[1];
    if (K + N > out_cap) return;   // the same for every thread of the grid
    const bool kept = int64_t(blockIdx.x) < keep_tiles;
    const int64_t tile = kept ? int64_t(blockIdx.x) : int64_t(blockIdx.x) - keep_tiles;
    const int64_t j = tile * kDenBlock + threadIdx.x;   // column among survivors or new ones
    if (j >= (kept ? K : N)) return;
    // source block: the last one whose first column is at or before j, between
    // the blocks holding this tile's first column and the next tile's
    const int32_t *first = kept ? first_keep : first_new;
    const int64_t n_out_tiles = ((kept ? K : N) + kDenBlock - 1) / kDenBlock;
    int64_t b = first[tile];
    int64_t hi = tile + 1 < n_out_tiles ? int64_t(first[tile + 1]) : n_blocks - 1;
    while (b < hi) {
        const int64_t mid = (b + hi + 1) >> 1;
        const int4 e = blk[mid];
        if (int64_t(kept ? e.x : e.y) <= j) b = mid; else hi = mid - 1;
    }
    const BlockMasks bm = masks[b];
    uint32_t child = 0;
    int nnew = 0;
    int item;
    if (kept) {
        item = select_bit(bm.keep, uint32_t(j - blk[b].x));
    } else {
        item = select_new(bm.lo, bm.hi, uint32_t(j - blk[b].y), child);
        nnew = int((bm.lo[item >> 6] >> (item & 63)) & 1) + 2 * int((bm.hi[item >> 6] >> (item & 63)) & 1);
    }
    const int64_t g = b * kDenBlock + item;
    const int64_t col = kept ? j : K + j;

    // rows 0-9: a child moves its centre by Rq (s * z_child) and shrinks
    {
        float raw[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) raw[k] = P[int64_t(k) * n_cap + g];
        if (nnew == 2) {
            float z[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) z[k] = noise[int64_t(3 * child + k) * n_cap + g];
            float w = raw[6], x = raw[7], y = raw[8], zz = raw[9];
            const float inv = 1.f / sqrtf(w * w + x * x + y * y + zz * zz);
            w *= inv; x *= inv; y *= inv; zz *= inv;
            const float R[9] = {1.f - 2.f * (y * y + zz * zz), 2.f * (x * y - w * zz), 2.f * (x * zz + w * y),
                                2.f * (x * y + w * zz), 1.f - 2.f * (x * x + zz * zz), 2.f * (y * zz - w * x),
                                2.f * (x * zz - w * y), 2.f * (y * zz + w * x), 1.f - 2.f * (x * x + y * y)};
            const float u[3] = {expf(raw[3]) * z[0], expf(raw[4]) * z[1], expf(raw[5]) * z[2]};
#pragma unroll
            for (int a = 0; a < 3; ++a)
                raw[a] = raw[a] + (R[3 * a] * u[0] + R[3 * a + 1] * u[1] + R[3 * a + 2] * u[2]);
#pragma unroll
            for (int a = 3; a < 6; ++a) raw[a] = raw[a] - r.log_shrink;
        }
#pragma unroll
        for (int k = 0; k < 10; ++k) oP[int64_t(k) * out_cap + col] = raw[k];
    }
    // rows 10-58: copies, kDenRows loads in flight
    for (int row = 10; row < kRows; row += kDenRows) {
        float x[kDenRows];
#pragma unroll
        for (int k = 0; k < kDenRows; ++k)
            if (row + k < kRows) x[k] = P[int64_t(row + k) * n_cap + g];
#pragma unroll
        for (int k = 0; k < kDenRows; ++k)
            if (row + k < kRows) oP[int64_t(row + k) * out_cap + col] = x[k];
    }
    // moments: survivors keep theirs, new primitives start at zero
    if (kept) {
        for (int row = 0; row < kRows; row += kDenRows / 2) {
            float a[kDenRows / 2], c[kDenRows / 2];
#pragma unroll
            for (int k = 0; k < kDenRows / 2; ++k)
                if (row + k < kRows) {
                    a[k] = m[int64_t(row + k) * n_cap + g];
                    c[k] = v[int64_t(row + k) * n_cap + g];
                }
#pragma unroll
            for (int k = 0; k < kDenRows / 2; ++k)
                if (row + k < kRows) {
                    om[int64_t(row + k) * out_cap + col] = a[k];
                    ov[int64_t(row + k) * out_cap + col] = c[k];
                }
        }
    } else {
#pragma unroll 4
        for (int row = 0; row < kRows; ++row) {
            om[int64_t(row) * out_cap + col] = 0.f;
            ov[int64_t(row) * out_cap + col] = 0.f;
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

// Workspace: per source block its totals / offsets and masks; the first
// source block of every output tile (at most n survivors and 2n new
// primitives); the totals.
struct DensifyWs {
    size_t blk, masks, first_keep, first_new, tot, bytes;
    int64_t nb, keep_tiles, new_tiles;
    static constexpr DensifyWs make(int64_t n) {
        DensifyWs L{};
        L.nb = (n + kDenBlock - 1) / kDenBlock;
        L.keep_tiles = L.nb;
        L.new_tiles = (2 * n + kDenBlock - 1) / kDenBlock;
        const int64_t nb1 = L.nb > 0 ? L.nb : 1;
        size_t o = 0;
        L.blk = o;        o = align_up(o + sizeof(int4) * nb1, 256);
        L.masks = o;      o = align_up(o + sizeof(BlockMasks) * nb1, 256);
        L.first_keep = o; o = align_up(o + sizeof(int32_t) * (L.keep_tiles + 1), 256);
        L.first_new = o;  o = align_up(o + sizeof(int32_t) * (L.new_tiles + 1), 256);
        L.tot = o;        o = align_up(o + 2 * sizeof(int64_t), 256);
        L.bytes = o;
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

namespace gs {
namespace {

// One densification pass (count, scan, tables, gather) with its workspace at b
// (DensifyWs::make(n) bytes).  Arguments already validated.
void densify_launch(const gs_densify_rule &rule, const float *params, const float *m, const float *v,
                    const float *stats, const float *noise, int64_t n, int64_t n_cap, float *out_params,
                    float *out_m, float *out_v, int64_t out_cap, char *b, int64_t *d_counts,
                    hipStream_t st) {
    const DensifyWs L = DensifyWs::make(n);
    int4 *blk = reinterpret_cast<int4 *>(b + L.blk);
    BlockMasks *masks = reinterpret_cast<BlockMasks *>(b + L.masks);
    int32_t *first_keep = reinterpret_cast<int32_t *>(b + L.first_keep);
    int32_t *first_new = reinterpret_cast<int32_t *>(b + L.first_new);
    int64_t *tot = reinterpret_cast<int64_t *>(b + L.tot);
    const int64_t nb = L.nb;
    if (nb > 0)
        hipLaunchKernelGGL(densify_count_kernel, dim3(xcd_grid(nb)), dim3(kDenThreads), 0, st, rule,
                           params, stats, n, n_cap, nb, blk, masks);
    hipLaunchKernelGGL(densify_scan_kernel, dim3(1), dim3(kScanThreads), 0, st, blk, nb, n, tot,
                       d_counts);
    if (nb > 0) {
        hipLaunchKernelGGL(densify_tables_kernel, dim3((nb + kDenThreads - 1) / kDenThreads),
                           dim3(kDenThreads), 0, st, blk, nb, tot, first_keep, first_new);
        hipLaunchKernelGGL(densify_gather_kernel, dim3(L.keep_tiles + L.new_tiles), dim3(kDenThreads), 0,
                           st, rule, params, m, v, noise, n_cap, out_params, out_m, out_v, out_cap, nb,
                           L.keep_tiles, blk, masks, first_keep, first_new, tot);
    }
}

bool densify_args_ok(const gs_densify_rule *rule, const float *params, const float *m, const float *v,
                     const float *stats, const float *noise, int64_t n, int64_t n_cap,
                     const float *out_params, const float *out_m, const float *out_v, int64_t out_cap,
                     const int64_t *d_counts) {
    return rule && params && m && v && stats && noise && out_params && out_m && out_v && d_counts &&
           n >= 0 && n <= n_cap && n_cap % 64 == 0 && out_cap >= 0 && out_cap % 64 == 0 &&
           n_cap < (int64_t(1) << 31) && out_cap < (int64_t(1) << 31);
}

// Workspace of gs_densify_noalloc: a pass over up to GS_DENSIFY_NOALLOC_MAX_N
// primitives.  Nothing in it has to start cleared (every word a pass reads is
// written earlier in the same pass).  In host code `scratch` names a host-side
// stand-in; kernels get the device address that hipGetSymbolAddress returns
// for the current device.
constexpr size_t kNoAllocScratchBytes = DensifyWs::make(GS_DENSIFY_NOALLOC_MAX_N).bytes;
static_assert(kNoAllocScratchBytes == 8127232, "the header states the scratch size");
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::once_flag scratch_once[kMaxDevices];
void *scratch_ptr[kMaxDevices];
hipError_t scratch_err[kMaxDevices];

// Device address of this device's scratch array, looked up once per device
// (with that device current).
gs_status scratch_address(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GS_ERR_HIP;
    std::call_once(scratch_once[dev], [dev] {
        void *ptr = nullptr;
        scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        scratch_ptr[dev] = ptr;
    });
    if (scratch_err[dev] != hipSuccess || !scratch_ptr[dev]) return GS_ERR_HIP;
    *out = scratch_ptr[dev];
    return GS_OK;
}

}  // namespace
}  // namespace gs

extern "C" gs_status gs_densify(const gs_densify_rule *rule, const float *params, const float *m,
                                const float *v, const float *stats, const float *noise, int64_t n,
                                int64_t n_cap, float *out_params, float *out_m, float *out_v,
                                int64_t out_cap, void *ws, int64_t *d_counts, void *stream) {
    if (!ws || !densify_args_ok(rule, params, m, v, stats, noise, n, n_cap, out_params, out_m, out_v,
                                out_cap, d_counts))
        return GS_ERR_INVALID_ARGUMENT;
    densify_launch(*rule, params, m, v, stats, noise, n, n_cap, out_params, out_m, out_v, out_cap,
                   static_cast<char *>(ws), d_counts, static_cast<hipStream_t>(stream));
    GS_CHECK_LAUNCH();
    return GS_OK;
}

extern "C" gs_status gs_densify_noalloc(const gs_densify_rule *rule, const float *params,
                                        const float *m, const float *v, const float *stats,
                                        const float *noise, int64_t n, int64_t n_cap,
                                        float *out_params, float *out_m, float *out_v,
                                        int64_t out_cap, int64_t *d_counts, void *stream) {
    if (!densify_args_ok(rule, params, m, v, stats, noise, n, n_cap, out_params, out_m, out_v, out_cap,
                         d_counts))
        return GS_ERR_INVALID_ARGUMENT;
    if (n > GS_DENSIFY_NOALLOC_MAX_N) return GS_ERR_CAPACITY;
    void *ws = nullptr;
    const gs_status st = scratch_address(&ws);
    if (st != GS_OK) return st;
    densify_launch(*rule, params, m, v, stats, noise, n, n_cap, out_params, out_m, out_v, out_cap,
                   static_cast<char *>(ws), d_counts, static_cast<hipStream_t>(stream));
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
