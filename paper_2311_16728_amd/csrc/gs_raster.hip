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
// transmittance back out Gaussian by Gaussian, and keeps a running dot
// product of what lies behind with dL/dC, so no per-pixel list is stored.
// Per Gaussian it sums over the tile's pixels the moments of dL/d(exponent)
// over the pixel offsets and the opacity and colour terms (registers, DPP
// and LDS), turns the moments into the gradients of the nine 2D quantities,
// and commits them with one atomic per quantity per tile.
#include "gs_internal.hpp"

#include <atomic>

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
// 1e-7 px.  thr = ln(alpha_min / opacity): a pixel composites the Gaussian iff
// its exponent reaches thr.
__device__ __forceinline__ void stage_record(const gs_settings &s, const Proj &proj, int64_t n_cap,
                                             int view, int level, double ox, double oy, uint32_t src,
                                             float4 &A, float4 &B, float2 &C, int64_t &rec) {
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
    C = make_float2(cz.z, __logf(s.alpha_min / co.w));
}

// Minimum of the quadratic form q(d) = a dx^2 + 2 b dx dy + c dy^2, d = p - m,
// over pixel centres p in [0, hx] x [0, hy] (tile-relative), relaxed to the
// rectangle.
__device__ __forceinline__ float qmin_tile(const float4 &A, const float4 &B, float hx, float hy) {
    const float mx = A.x, my = A.y, a = A.z, b = A.w, c = B.x;
    const float lo = 0.f;
    if (mx >= lo && mx <= hx && my >= lo && my <= hy) return 0.f;
    float best = 3.4e38f;
    // edges x = const: minimise over dy
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float dx = (e ? hx : lo) - mx;
        const float dy = fminf(fmaxf(-b * dx / c, lo - my), hy - my);
        best = fminf(best, a * dx * dx + 2.f * b * dx * dy + c * dy * dy);
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float dy = (e ? hy : lo) - my;
        const float dx = fminf(fmaxf(-b * dy / a, lo - mx), hx - mx);
        best = fminf(best, a * dx * dx + 2.f * b * dx * dy + c * dy * dy);
    }
    return best;
}

// True when some pixel of the tile (ts) may reach the cutoff (conservative).
__device__ __forceinline__ bool touches_tile(const float4 &A, const float4 &B, const float2 &C,
                                             const TileShape &ts) {
    const float tq = -2.f * C.y;   // q <= tq  <=>  exponent >= thr
    return qmin_tile(A, B, float(ts.w - 1), float(ts.h - 1)) <= tq * 1.0001f + 1e-3f;
}

// alpha = min(opacity x exp(power), alpha_max) for the non-negative first
// argument, as one median instruction (an fminf canonicalises its operands
// on every use); forward and backward use the same instruction.
__device__ __forceinline__ float clamp_alpha(float at, float amax) {
    return __builtin_amdgcn_fmed3f(at, 0.f, amax);
}

// Staged records hold the conic in base-2 exponent form: A.z = -a log2(e) / 2,
// A.w = -b log2(e), B.x = -c log2(e) / 2 for the conic (a, b, c) of
// stage_record, and the cutoff C.y = ln(alpha_min / opacity) log2(e), so the
// exponent in base 2, -(a dx^2 + 2 b dx dy + c dy^2) log2(e) / 2, takes five
// operations and goes to the hardware exp2 as it is.  conic_a/b/c give the
// conic back (to a rounding or two: the gradients use it, the compositing
// decisions do not).
constexpr float kLog2e = 1.44269504088896341f, kLn2 = 0.693147180559945309f;
__device__ __forceinline__ void to_exponent_form(float4 &A, float4 &B, float2 &C) {
    A.z *= -0.5f * kLog2e;
    A.w *= -kLog2e;
    B.x *= -0.5f * kLog2e;
    C.y *= kLog2e;
}
__device__ __forceinline__ float conic_a(const float4 &A) { return A.z * (-2.f * kLn2); }
__device__ __forceinline__ float conic_b(const float4 &A) { return A.w * -kLn2; }
__device__ __forceinline__ float conic_c(const float4 &B) { return B.x * (-2.f * kLn2); }

// Base-2 exponent of a staged Gaussian at offset (dx, dy) = mean - pixel:
// dx (A.z dx) + dy (A.w dx + B.x dy).  The same instruction sequence serves
// the forward and the backward, so both take the same alpha_min decision.
__device__ __forceinline__ float eval_power(const float4 &A, const float4 &B, float dx, float dy) {
    const float u = fmaf(A.w, dx, B.x * dy);
    return fmaf(A.z * dx, dx, u * dy);
}

// Block-wide count of `flag` for kThreads threads (a multiple of 64): the
// number of threads before this one where it holds (ballots, no scan), and
// the block total.
template <int kThreads>
__device__ __forceinline__ uint32_t block_count_n(bool flag, uint32_t *lds, uint32_t *total) {
    constexpr int kW = kThreads / kWave;
    const uint64_t m = __ballot(flag);
    const uint32_t below = uint32_t(mask_rank(m));
    if (kW == 1) {
        *total = uint32_t(__popcll(m));
        return below;
    }
    const int wave = threadIdx.x / kWave;
    if (lane_id() == 0) lds[wave] = uint32_t(__popcll(m));
    __syncthreads();
    uint32_t base = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kW; ++w) {
        const uint32_t s = lds[w];
        base += (w < wave) ? s : 0u;
        all += s;
    }
    __syncthreads();
    *total = all;
    return base + below;
}

// Per-pixel transmittance store of the store-all variant (the comparison
// point of the recompute backward): the transmittance in front of a pixel's
// k-th composited Gaussian sits at base[tile] + k * 256 + (pixel in tile), so
// each compositing step of a tile writes 256 consecutive floats.  base has
// total_tiles + 1 entries (the last is the floats needed); nothing is stored
// or read when that exceeds cap.
struct TStore {
    const int64_t *base;   // [total_tiles + 1]
    const int64_t *need;   // base + total_tiles: floats the store needs
    float *T;
    int64_t cap;
};

// kCount: per-pixel composited and evaluated counts (and, with tile_max, the
// largest composited count of each tile); kStore: the transmittance store.
template <bool kCount, bool kStore = false, bool kQueued = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) render_fwd_kernel(
    gs_settings s, Proj proj, int64_t n_cap, Sorted srt, const gs_target *__restrict__ targets,
    int n_targets, float *__restrict__ out_rgb, float *__restrict__ out_T,
    int32_t *__restrict__ out_last, int32_t *__restrict__ out_nc, int32_t *__restrict__ out_ne,
    int32_t *__restrict__ tile_max = nullptr, TStore ts_store = TStore{nullptr, nullptr, nullptr, 0},
    const uint32_t *__restrict__ order = nullptr, uint32_t *__restrict__ queue = nullptr, int total_tiles = 0) {
    __shared__ float4 sA[kTilePix];
    __shared__ float4 sB[kTilePix];
    __shared__ float2 sC[kTilePix];
    __shared__ int32_t sPos[kTilePix];
    __shared__ uint32_t scan_lds[8];
    constexpr bool queued = kQueued;
    const float amax = __builtin_canonicalizef(s.alpha_max);   // (once per launch)
    for (int round = 0;; ++round) {
        int tile;
        if (queued) {   // next tile of the cost-ordered queue
            __shared__ int s_item;
            if (threadIdx.x == 0) s_item = int(atomicAdd(&queue[kQueueNextFwd], 1u));
            __syncthreads();
            const int item = s_item;
            __syncthreads();
            if (item >= total_tiles) break;
            tile = int(order[item]);
            if (tile < 0 || tile >= total_tiles) continue;   // not a tile: order not built
        } else {
            if (round > 0) break;
            tile = blockIdx.x;
        }
        const int tid = threadIdx.x;
        const gs_target t = targets[find_target(targets, n_targets, tile)];
        const int local = tile - t.tile_offset;
        const int tx = local % t.tiles_x, ty = local / t.tiles_x;
        const TileShape ts = tile_shape(t.tile_w);
        const int lxp = tid & (ts.w - 1), lyp = tid >> ts.wlog;   // pixel inside the tile
        const int px = tx * ts.w + lxp, py = ty * ts.h + lyp;
        const bool inside = px < t.width && py < t.height;
        const uint2 range = srt.ranges[tile];
        const double ox = double(tx * ts.w), oy = double(ty * ts.h);
        const float fpx = float(lxp), fpy = float(lyp);   // relative to the tile origin

        float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
        int32_t nc = 0, ne = 0, last = 0;
        bool done = !inside;
        float *store_at = nullptr;   // this pixel's first slot (kStore), or none
        if (kStore && *ts_store.need <= ts_store.cap) store_at = ts_store.T + ts_store.base[tile] + tid;
        const int batch = s.batch;
        for (uint32_t b0 = range.x; b0 < range.y; b0 += batch) {
            if (__syncthreads_count(done) == kTilePix) break;
            // stage the batch, keeping only Gaussians whose cutoff ellipse meets the tile
            const uint32_t idx = b0 + tid;
            float4 A, B;
            float2 Cc;
            int64_t rec;
            bool keep = false;
            if (tid < batch && idx < range.y) {
                stage_record(s, proj, n_cap, t.view, t.level, ox, oy, srt.pair_val[idx], A, B, Cc, rec);
                keep = touches_tile(A, B, Cc, ts);
                to_exponent_form(A, B, Cc);
            }
            uint32_t cnt;
            const uint32_t at_pos = block_count_n<kTilePix>(keep, scan_lds, &cnt);
            if (keep) {
                sA[at_pos] = A;
                sB[at_pos] = B;
                sC[at_pos] = Cc;
                sPos[at_pos] = int32_t(idx - range.x);
            }
            __syncthreads();
            if (!done) {
                int lj = -1;   // staged index of this batch's last composited Gaussian
                // Straight-line body: every lane evaluates every staged
                // Gaussian and keeps the result only where it composites (a
                // wave runs the exponential whenever one of its lanes does);
                // a lane that stops compositing stays in the loop as a no-op
                // until all of the wave's lanes have stopped (checked every
                // four Gaussians; the loop is unrolled by hand, four at a time).
                auto step = [&](int j) {
                    const float4 A = sA[j];
                    const float4 B = sB[j];
                    const float2 Cj = sC[j];
                    const float dx = A.x - fpx, dy = A.y - fpy;
                    const float pw = eval_power(A, B, dx, dy);
                    if (kCount) ne += done ? 0 : 1;
                    const bool hit = !done && !(pw < Cj.y);
                    const float alpha = clamp_alpha(B.y * __builtin_amdgcn_exp2f(pw), amax);
                    const float Tn = T * (1.f - alpha);
                    const bool stop = hit && Tn < s.t_min;
                    const bool comp = hit && !stop;
                    if (kStore && store_at && comp) store_at[int64_t(nc) * kTilePix] = T;
                    // a Gaussian that does not composite adds 0 x colour:
                    // colours and sums are finite and >= 0, so the sums keep
                    // their bits
                    const float w = comp ? alpha * T : 0.f;
                    C0 = fmaf(w, B.z, C0);
                    C1 = fmaf(w, B.w, C1);
                    C2 = fmaf(w, Cj.x, C2);
                    T = comp ? Tn : T;
                    if (kCount || kStore) nc += comp ? 1 : 0;
                    lj = comp ? j : lj;
                    done = done || stop;
                };
                const int n_staged = __builtin_amdgcn_readfirstlane(int(cnt));   // (uniform)
                int j = 0;
                for (; j + 4 <= n_staged; j += 4) {
                    step(j);
                    step(j + 1);
                    step(j + 2);
                    step(j + 3);
                    if (__all(done)) break;
                }
                for (; j < n_staged && !__all(done); ++j) step(j);
                // one past the list position of the last composited Gaussian
                if (lj >= 0) last = sPos[lj] + 1;
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
            if (kCount && out_nc) out_nc[t.pix_offset + pix] = nc;
            if (kCount && out_ne) out_ne[t.pix_offset + pix] = ne;
        }
        if (kCount && tile_max) {
            __shared__ int32_t tmax;
            if (tid == 0) tmax = 0;
            __syncthreads();
            if (nc > 0) atomicMax(&tmax, nc);
            __syncthreads();
            if (tid == 0) tile_max[tile] = tmax;
        }
    }
    if (queued) queue_retire(queue, kQueueNextFwd, kQueueDoneFwd);
}

// Exclusive scan of the per-tile store sizes (256 floats per compositing step
// of the tile's deepest pixel) into base[0..total_tiles]; one workgroup.
__global__ void __launch_bounds__(1024) store_base_kernel(const int32_t *__restrict__ tile_max,
                                                          int64_t total_tiles, int64_t *__restrict__ base) {
    __shared__ int64_t wsum[16];
    const int64_t per = (total_tiles + 1023) / 1024;
    const int64_t lo = int64_t(threadIdx.x) * per;
    int64_t local = 0;
    for (int64_t i = lo; i < lo + per && i < total_tiles; ++i) local += int64_t(tile_max[i]) * kTilePix;
    // inclusive scan over the block in 64 bits
    int64_t inc = local;
    const int lane = lane_id(), wave = threadIdx.x / kWave;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int64_t u = __shfl_up(inc, d, kWave);
        if (lane >= d) inc += u;
    }
    if (lane == kWave - 1) wsum[wave] = inc;
    __syncthreads();
    int64_t before = 0, all = 0;
    for (int w = 0; w < 16; ++w) {
        before += w < wave ? wsum[w] : 0;
        all += wsum[w];
    }
    int64_t run = before + inc - local;
    for (int64_t i = lo; i < lo + per && i < total_tiles; ++i) {
        base[i] = run;
        run += int64_t(tile_max[i]) * kTilePix;
    }
    if (threadIdx.x == 0) base[total_tiles] = all;
}

// Cross-lane add through DPP (full-rate VALU; rows are 16 lanes).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_add(float v) {
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, kRowMask, 0xf, false));
}


// Backward raster with kWaves waves per 16x16 tile; every lane owns
// kPix = 4 / kWaves pixels (rows spaced by 4 * kWaves), so the per-Gaussian
// wave reduction is shared by kPix pixels.  Entries are staged kThreads at a
// time, back to front.
// Per-Gaussian sums over a wave without a full butterfly per value: each quad
// of lanes adds its values with two DPP steps, one lane per quad stores them
// in an LDS transpose buffer, and once kGroup Gaussians are buffered every
// lane sums the 16 quad partials of one of the kGroup * 9 values.  About 31
// instructions per Gaussian instead of 72 for nine 64-lane reductions.
constexpr int kGroup = 7;                      // 7 * 9 = 63 values <= 64 lanes
constexpr int kQuads = kWave / 4;
constexpr int kTStride = kQuads + 1;           // odd row stride: conflict-free reads

// kStored: the store-all variant, which reads each composited Gaussian's
// transmittance from the forward's store (in_nc: per-pixel composited counts)
// instead of dividing it back out.
template <int kWaves, bool kStored = false, bool kQueued = false>
__global__ void __launch_bounds__(64 * kWaves) render_bwd_kernel(
    gs_settings s, Proj proj, int64_t n_cap, Sorted srt, const gs_target *__restrict__ targets,
    int n_targets, const float *__restrict__ in_T, const int32_t *__restrict__ in_last,
    const float *__restrict__ dL_drgb, float *__restrict__ acc,
    const int32_t *__restrict__ in_nc = nullptr, TStore ts_store = TStore{nullptr, nullptr, nullptr, 0},
    const uint32_t *__restrict__ order = nullptr, uint32_t *__restrict__ queue = nullptr, int total_tiles = 0) {
    constexpr int kThreads = 64 * kWaves;
    constexpr int kPix = kTilePix / kThreads;
    __shared__ float4 sA[kThreads];
    __shared__ float4 sB[kThreads];
    __shared__ float2 sC[kThreads];
    __shared__ uint32_t sR[kThreads];   // record view * n_cap + g (< 2^32)
    __shared__ int32_t sPos[kThreads];
    __shared__ uint32_t scan_lds[8];
    __shared__ float red[kWaves][kThreads][kAccRows];
    __shared__ float tbuf[kWaves][kGroup * kAccRows * kTStride];
    __shared__ int32_t sK[kWaves][kGroup];
    __shared__ int sMaxLast;
    if (kStored && !(*ts_store.need <= ts_store.cap)) return;   // the forward stored nothing
    constexpr bool queued = kQueued;
    const float amax = __builtin_canonicalizef(s.alpha_max);   // (once per launch)
    for (int round = 0;; ++round) {
        int tile;
        if (queued) {   // next tile of the cost-ordered queue
            __shared__ int s_item;
            if (threadIdx.x == 0) s_item = int(atomicAdd(&queue[kQueueNextBwd], 1u));
            __syncthreads();
            const int item = s_item;
            __syncthreads();
            if (item >= total_tiles) break;
            tile = int(order[item]);
            if (tile < 0 || tile >= total_tiles) continue;   // not a tile: order not built
        } else {
            if (round > 0) break;
            tile = blockIdx.x;
        }
        const int tid = threadIdx.x;
        const int wave = tid / kWave;
        const int lane = lane_id();
        const gs_target t = targets[find_target(targets, n_targets, tile)];
        const int local = tile - t.tile_offset;
        const int tx = local % t.tiles_x, ty = local / t.tiles_x;
        const TileShape ts = tile_shape(t.tile_w);
        const uint2 range = srt.ranges[tile];
        const double ox = double(tx * ts.w), oy = double(ty * ts.h);
        const float sc = ldexpf(1.f, -t.level);
        const int64_t HW = int64_t(t.width) * t.height;
        const float *dLt = dL_drgb + 3 * t.pix_offset;
        float *tb = tbuf[wave];

        // S: the colour behind the current Gaussian (what the pixel shows
        // from there on, background included, at unit transmittance) dotted
        // with dL/dC; only that dot product enters the gradient, so the
        // colour itself is never formed
        float T[kPix], g0[kPix], g1[kPix], g2[kPix], S[kPix], fpy[kPix];
        int32_t last[kPix];
        int32_t kc[kPix];             // kStored: composited Gaussians not yet walked back
        const float *srow = nullptr;  // kStored: this tile's store
        int32_t steps = 0;            // kStored: compositing steps stored for the tile
        if (kStored) {
            srow = ts_store.T + ts_store.base[tile];
            steps = int32_t((ts_store.base[tile + 1] - ts_store.base[tile]) / kTilePix);
        }
        // the tile width divides 64, so a lane keeps its column in every row it owns
        const float fpx = float(tid & (ts.w - 1));
        int my_max = 0;
    #pragma unroll
        for (int i = 0; i < kPix; ++i) {
            const int lp = tid + i * kThreads;   // tile-local pixel index
            const int ly = lp >> ts.wlog;
            fpy[i] = float(ly);
            const int px = tx * ts.w + (lp & (ts.w - 1)), py = ty * ts.h + ly;
            T[i] = 0.f; g0[i] = g1[i] = g2[i] = 0.f; last[i] = 0;
            kc[i] = 0;
            if (px < t.width && py < t.height) {
                const int64_t pix = int64_t(py) * t.width + px;
                if (kStored)
                    kc[i] = min(in_nc[t.pix_offset + pix], steps);
                else
                    T[i] = in_T[t.pix_offset + pix];
                last[i] = in_last[t.pix_offset + pix];
                g0[i] = dLt[pix];
                g1[i] = dLt[HW + pix];
                g2[i] = dLt[2 * HW + pix];
            }
            // a restart position never exceeds the tile's list (guards stale input)
            last[i] = min(last[i], int32_t(range.y - range.x));
            my_max = max(my_max, last[i]);
            S[i] = fmaf(t.bg[0], g0[i], fmaf(t.bg[1], g1[i], t.bg[2] * g2[i]));   // the background
        }
        if (tid == 0) sMaxLast = 0;
        __syncthreads();
        if (my_max > 0) atomicMax(&sMaxLast, my_max);
        __syncthreads();
        const int max_last = sMaxLast;

        // Orders this wave's LDS accesses around a hand-over between its lanes.
        auto wave_sync = [] {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };
        // sums the buffered Gaussians' values: lane m < n * 9 owns value m
        auto flush = [&](int n) {
            wave_sync();
            if (lane < n * kAccRows) {
                const float *row = tb + lane * kTStride;
                float sum = -0.f;
    #pragma unroll
                for (int q = 0; q < kQuads; ++q) sum += row[q];
                const int slot = lane / kAccRows;
                red[wave][sK[wave][slot]][lane - slot * kAccRows] = sum;
            }
            wave_sync();
        };

        for (int end = max_last; end > 0; end -= kThreads) {
            const int start = max(0, end - kThreads);
            __syncthreads();
            float4 A, Bv;
            float2 Cc;
            int64_t rec;
            bool keep = false;
            if (tid < end - start) {
                stage_record(s, proj, n_cap, t.view, t.level, ox, oy, srt.pair_val[range.x + start + tid],
                             A, Bv, Cc, rec);
                keep = touches_tile(A, Bv, Cc, ts);
                to_exponent_form(A, Bv, Cc);
            }
            uint32_t cnt;
            const uint32_t at_pos = block_count_n<kThreads>(keep, scan_lds, &cnt);
            if (keep) {
                sA[at_pos] = A;
                sB[at_pos] = Bv;
                sC[at_pos] = Cc;
                sR[at_pos] = uint32_t(rec);
                sPos[at_pos] = start + tid;
            }
            __syncthreads();
            int slots = 0;   // Gaussians buffered in tb (wave-uniform)
            for (int k = int(cnt) - 1; k >= 0; --k) {
                const float4 A = sA[k];
                const float4 Bv = sB[k];
                const float2 Ck = sC[k];
                const int pos = sPos[k];
                // sums start at -0: -0 + x and -0 - x are exactly x and -x,
                // so the first pixel's terms need no add (from +0 they would:
                // +0 + -0 is +0)
                float v[kAccRows];
    #pragma unroll
                for (int i = 0; i < kAccRows; ++i) v[i] = -0.f;
                bool any = false;
    #pragma unroll
                for (int i = 0; i < kPix; ++i) {
                    const float dx = A.x - fpx, dy = A.y - fpy[i];
                    const float pw = eval_power(A, Bv, dx, dy);
                    if (pos < last[i] && !(pw < Ck.y)) {
                        any = true;
                        const float ep = __builtin_amdgcn_exp2f(pw);
                        const float at = Bv.y * ep;
                        const float alpha = clamp_alpha(at, amax);
                        const float oma = 1.f - alpha;
                        if (kStored) {   // transmittance in front of it, as stored
                            kc[i] = max(kc[i] - 1, 0);
                            T[i] = srow[int64_t(kc[i]) * kTilePix + tid + i * kThreads];
                        } else {
                            T[i] = T[i] * __builtin_amdgcn_rcpf(oma);   // transmittance in front of it
                        }
                        // (the gradient sums use explicit FMAs: the build does
                        // not contract, so that both passes take the cutoff
                        // decisions with the same instructions)
                        // dL/dalpha = T (c - colour behind) . dL/dC
                        const float cg = fmaf(Bv.z, g0[i], fmaf(Bv.w, g1[i], Ck.x * g2[i]));
                        const float dal = T[i] * (cg - S[i]);
                        const float w = alpha * T[i];
                        v[6] = fmaf(w, g0[i], v[6]);
                        v[7] = fmaf(w, g1[i], v[7]);
                        v[8] = fmaf(w, g2[i], v[8]);
                        S[i] = fmaf(alpha, cg, oma * S[i]);
                        const float dat = (at < amax) ? dal : 0.f;
                        v[5] = fmaf(ep, dat, v[5]);
                        // ndp = dL/d(exponent); the sums 0-4 are its moments
                        // over the pixel offsets (sum ndp d, sum ndp d d^T),
                        // which the conic turns into the mean and conic
                        // gradients once per Gaussian
                        const float ndp = -(at * dat);
                        const float nx = ndp * dx, ny = ndp * dy;
                        v[0] += nx;
                        v[1] += ny;
                        v[2] = fmaf(nx, dx, v[2]);
                        v[3] = fmaf(nx, dy, v[3]);
                        v[4] = fmaf(ny, dy, v[4]);
                    }
                }
                const uint64_t act = __ballot(any);
                float *slot_out = red[wave][k];
                if (act == 0) {
                    if (lane == kWave - 1) {
    #pragma unroll
                        for (int i = 0; i < kAccRows; ++i) slot_out[i] = 0.f;
                    }
                    continue;
                }
                if (__popcll(act) == 1) {
                    // one lane of this wave touches the Gaussian: it holds the sums
                    if (act & (uint64_t(1) << lane)) {
    #pragma unroll
                        for (int i = 0; i < kAccRows; ++i) slot_out[i] = v[i];
                    }
                    continue;
                }
                // quad sums, then one lane per quad into the transpose buffer
    #pragma unroll
                for (int i = 0; i < kAccRows; ++i) {
                    v[i] = dpp_add<0xB1, 0xf>(v[i]);   // quad_perm [1,0,3,2]
                    v[i] = dpp_add<0x4E, 0xf>(v[i]);   // quad_perm [2,3,0,1]
                }
                {   // all four lanes of a quad hold the same bits ((a+b)+(c+d) and
                    // its reorderings by commutation) and all store them to the
                    // quad's slot: the second DPP add then stays one instruction
                    // for the whole wave (kept behind a branch of the quads'
                    // first lanes it became a move, a copy and an add)
                    float *col = tb + slots * kAccRows * kTStride + (lane >> 2);
    #pragma unroll
                    for (int i = 0; i < kAccRows; ++i) col[i * kTStride] = v[i];
                }
                if (lane == 0) sK[wave][slots] = k;
                if (++slots == kGroup) {
                    flush(kGroup);
                    slots = 0;
                }
            }
            if (slots > 0) flush(slots);
            __syncthreads();
            // The waves' sums are added, the conic gradient becomes the gradient of
            // the dilated covariance (-K dK K), and both go back to level-0 units
            // (in place, in red[0]) ...
            for (int k = tid; k < int(cnt); k += kThreads) {
                float v[kAccRows];
    #pragma unroll
                for (int i = 0; i < kAccRows; ++i) {
                    float sum = -0.f;
    #pragma unroll
                    for (int w = 0; w < kWaves; ++w) sum += red[w][k][i];
                    v[i] = sum;
                }
                const float a = conic_a(sA[k]), b = conic_b(sA[k]), c = conic_c(sB[k]);
                // mean gradient K (sum ndp d); conic gradient (sum ndp d d^T) / 2
                const float P = v[0], Q = v[1];
                const float ga = 0.5f * v[2], gb = 0.5f * v[3], gc = 0.5f * v[4];
                const float k00 = a * ga + b * gb, k01 = a * gb + b * gc;
                const float k10 = b * ga + c * gb, k11 = b * gb + c * gc;
                const float s2 = sc * sc;
                v[0] = (a * P + b * Q) * sc;
                v[1] = (b * P + c * Q) * sc;
                v[2] = -(k00 * a + k01 * b) * s2;
                v[3] = -(k00 * b + k01 * c) * s2;
                v[4] = -(k10 * b + k11 * c) * s2;
    #pragma unroll
                for (int i = 0; i < kAccRows; ++i) red[0][k][i] = v[i];
            }
            __syncthreads();
            // ... then one atomic per (Gaussian, quantity) for the whole tile, with
            // consecutive threads on consecutive accumulators of a record (a
            // record's nine accumulators are contiguous)
            for (int idx = tid; idx < int(cnt) * kAccRows; idx += kThreads) {
                const int k = idx / kAccRows, i = idx - k * kAccRows;
                const float v = red[0][k][i];
                if (v != 0.f) atomicAdd(&acc[int64_t(sR[k]) * kAccRows + i], v);   // sR unsigned
            }
        }
    }
    if (queued) queue_retire(queue, kQueueNextBwd, kQueueDoneBwd);
}

__global__ void fill_f32_kernel(float *p, int64_t count, float v) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// Four floats per thread, one 16-byte store each (p 16-byte aligned); the
// last thread also writes a tail of fewer than four.
__global__ void fill_f32x4_kernel(float *p, int64_t count, float v) {
    const int64_t e = 4 * (int64_t(blockIdx.x) * blockDim.x + threadIdx.x);
    if (e + 4 <= count) {
        *reinterpret_cast<float4 *>(p + e) = make_float4(v, v, v, v);
    } else {
        for (int64_t k = e; k < count; ++k) p[k] = v;
    }
}

// Workgroups of a persistent launch: as many as the chip holds at once (CUs x
// resident workgroups per CU for the kernel), looked up once per kernel.  Any
// count is correct (workgroups only take tiles from the queue); this one
// keeps every CU busy with no workgroup left waiting for a slot.
template <class Kernel>
static int persistent_grid(Kernel kernel, int threads) {
    static std::atomic<int> cached{0};
    int g = cached.load(std::memory_order_relaxed);
    if (g > 0) return g;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || cus <= 0 ||
        per_cu <= 0)
        return 2048;
    g = cus * per_cu;
    cached.store(g, std::memory_order_relaxed);
    return g;
}

static void launch_fill(float *p, int64_t count, float v, hipStream_t st) {
    if (reinterpret_cast<uintptr_t>(p) % 16 == 0)
        hipLaunchKernelGGL(fill_f32x4_kernel, dim3((count + 1023) / 1024), dim3(256), 0, st, p, count, v);
    else
        hipLaunchKernelGGL(fill_f32_kernel, dim3((count + 255) / 256), dim3(256), 0, st, p, count, v);
}

gs_status launch_project_backward(const gs_settings &s, const float *params, int64_t n,
                                  int64_t n_cap, const gs_view *views, int32_t n_views,
                                  const float *acc, float *grad, hipStream_t st);
gs_status launch_project_backward_adam(const gs_settings &s, float *params, int64_t n, int64_t n_cap,
                                       const gs_view *views, int32_t n_views, const float *acc,
                                       float *m, float *v, const float *lr_rows, double beta1,
                                       double beta2, double eps, int32_t step, const int32_t *d_step,
                                       void *proj_out, hipStream_t st);

}  // namespace gs

extern "C" gs_status gs_render_fwd(const gs_settings *s, const void *proj_ws, int64_t n_cap,
                                   int32_t n_views, const void *sort_ws, int64_t pair_cap,
                                   const gs_target *targets, int32_t n_targets, int32_t total_tiles,
                                   float *out_rgb, float *out_T, int32_t *out_last,
                                   int32_t *out_ncontrib, int32_t *out_nevals, void *stream) {
    using namespace gs;
    if (!valid_settings(s) || !proj_ws || !sort_ws || !targets || n_cap <= 0 || n_cap % 64 ||
        n_views <= 0 || n_targets <= 0 || total_tiles <= 0 || pair_cap <= 0 || !out_rgb ||
        !out_T || !out_last || pair_cap > kMaxPairs || int64_t(n_views) * n_cap > kMaxRecords)
        return GS_ERR_INVALID_ARGUMENT;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Sorted srt = sorted_at(sort_ws, n_views, n_targets, n_cap, pair_cap, total_tiles);
    const Proj proj = proj_at(const_cast<void *>(proj_ws), int64_t(n_views) * n_cap);
    if (out_ncontrib || out_nevals)
        hipLaunchKernelGGL(render_fwd_kernel<true>, dim3(total_tiles), dim3(kTilePix), 0, st, *s, proj, n_cap,
                           srt, targets, n_targets, out_rgb, out_T, out_last, out_ncontrib, out_nevals);
    else if (s->schedule == 1)
        hipLaunchKernelGGL((render_fwd_kernel<false, false, true>),
                           dim3(persistent_grid(render_fwd_kernel<false, false, true>, kTilePix)), dim3(kTilePix), 0, st, *s,
                           proj, n_cap, srt, targets, n_targets, out_rgb, out_T, out_last, nullptr, nullptr,
                           nullptr, TStore{nullptr, nullptr, nullptr, 0}, srt.order, srt.queue, total_tiles);
    else
        hipLaunchKernelGGL(render_fwd_kernel<false>, dim3(total_tiles), dim3(kTilePix), 0, st, *s, proj, n_cap,
                           srt, targets, n_targets, out_rgb, out_T, out_last, nullptr, nullptr);
    GS_CHECK_LAUNCH();
    return GS_OK;
}

extern "C" gs_status gs_raster_bwd(const gs_settings *s, const void *proj_ws, int64_t n_cap,
                                   int32_t n_views, const void *sort_ws, int64_t pair_cap,
                                   const gs_target *targets, int32_t n_targets, int32_t total_tiles,
                                   const float *out_T, const int32_t *out_last,
                                   const float *dL_drgb, void *accum_ws, void *stream) {
    using namespace gs;
    if (!valid_settings(s) || !proj_ws || !sort_ws || !targets || !out_T || !out_last || !dL_drgb ||
        !accum_ws || n_cap <= 0 || n_cap % 64 || n_views <= 0 || n_targets <= 0 ||
        total_tiles <= 0 || pair_cap <= 0 || pair_cap > kMaxPairs ||
        int64_t(n_views) * n_cap > kMaxRecords)
        return GS_ERR_INVALID_ARGUMENT;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t records = int64_t(n_views) * n_cap;
    const Sorted srt = sorted_at(sort_ws, n_views, n_targets, n_cap, pair_cap, total_tiles);
    const Proj proj = proj_at(const_cast<void *>(proj_ws), records);
    float *acc = static_cast<float *>(accum_ws);
    const int64_t acc_n = int64_t(kAccRows) * records;
    launch_fill(acc, acc_n, 0.f, st);
    const TStore none{nullptr, nullptr, nullptr, 0};
    if (s->schedule >= 1) {   // persistent workgroups over the cost-ordered tile queue
        switch (s->bwd_waves) {
            case 1:
                hipLaunchKernelGGL((render_bwd_kernel<1, false, true>),
                                   dim3(persistent_grid(render_bwd_kernel<1, false, true>, 64)), dim3(64), 0, st,
                                   *s, proj, n_cap, srt, targets, n_targets, out_T, out_last, dL_drgb, acc,
                                   nullptr, none, srt.order, srt.queue, total_tiles);
                break;
            case 2:
                hipLaunchKernelGGL((render_bwd_kernel<2, false, true>),
                                   dim3(persistent_grid(render_bwd_kernel<2, false, true>, 128)), dim3(128), 0, st,
                                   *s, proj, n_cap, srt, targets, n_targets, out_T, out_last, dL_drgb, acc,
                                   nullptr, none, srt.order, srt.queue, total_tiles);
                break;
            default:
                hipLaunchKernelGGL((render_bwd_kernel<4, false, true>),
                                   dim3(persistent_grid(render_bwd_kernel<4, false, true>, 256)), dim3(256), 0, st,
                                   *s, proj, n_cap, srt, targets, n_targets, out_T, out_last, dL_drgb, acc,
                                   nullptr, none, srt.order, srt.queue, total_tiles);
                break;
        }
    } else {
        switch (s->bwd_waves) {
            case 1:
                hipLaunchKernelGGL(render_bwd_kernel<1>, dim3(total_tiles), dim3(64), 0, st, *s, proj, n_cap,
                                   srt, targets, n_targets, out_T, out_last, dL_drgb, acc);
                break;
            case 2:
                hipLaunchKernelGGL(render_bwd_kernel<2>, dim3(total_tiles), dim3(128), 0, st, *s, proj, n_cap,
                                   srt, targets, n_targets, out_T, out_last, dL_drgb, acc);
                break;
            default:
                hipLaunchKernelGGL(render_bwd_kernel<4>, dim3(total_tiles), dim3(256), 0, st, *s, proj, n_cap,
                                   srt, targets, n_targets, out_T, out_last, dL_drgb, acc);
                break;
        }
    }
    GS_CHECK_LAUNCH();
    return GS_OK;
}

extern "C" gs_status gs_render_fwd_store(const gs_settings *s, const void *proj_ws, int64_t n_cap,
                                         int32_t n_views, const void *sort_ws, int64_t pair_cap,
                                         const gs_target *targets, int32_t n_targets,
                                         int32_t total_tiles, float *out_rgb, float *out_T,
                                         int32_t *out_last, int32_t *out_ncontrib, int32_t *tile_steps,
                                         int64_t *store_base, float *store, int64_t store_cap,
                                         void *stream) {
    using namespace gs;
    if (!valid_settings(s) || !proj_ws || !sort_ws || !targets || n_cap <= 0 || n_cap % 64 ||
        n_views <= 0 || n_targets <= 0 || total_tiles <= 0 || pair_cap <= 0 || !out_rgb || !out_T ||
        !out_last || !out_ncontrib || !tile_steps || !store_base || !store || store_cap < 0 ||
        pair_cap > kMaxPairs || int64_t(n_views) * n_cap > kMaxRecords)
        return GS_ERR_INVALID_ARGUMENT;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Sorted srt = sorted_at(sort_ws, n_views, n_targets, n_cap, pair_cap, total_tiles);
    const Proj proj = proj_at(const_cast<void *>(proj_ws), int64_t(n_views) * n_cap);
    // counts, the store layout, then the forward again writing the store
    hipLaunchKernelGGL(render_fwd_kernel<true>, dim3(total_tiles), dim3(kTilePix), 0, st, *s, proj, n_cap, srt,
                       targets, n_targets, out_rgb, out_T, out_last, out_ncontrib, nullptr, tile_steps,
                       TStore{nullptr, nullptr, nullptr, 0});
    hipLaunchKernelGGL(store_base_kernel, dim3(1), dim3(1024), 0, st, tile_steps, int64_t(total_tiles), store_base);
    hipLaunchKernelGGL((render_fwd_kernel<false, true>), dim3(total_tiles), dim3(kTilePix), 0, st, *s, proj,
                       n_cap, srt, targets, n_targets, out_rgb, out_T, out_last, nullptr, nullptr, nullptr,
                       TStore{store_base, store_base + total_tiles, store, store_cap});
    GS_CHECK_LAUNCH();
    return GS_OK;
}

extern "C" gs_status gs_raster_bwd_stored(const gs_settings *s, const void *proj_ws, int64_t n_cap,
                                          int32_t n_views, const void *sort_ws, int64_t pair_cap,
                                          const gs_target *targets, int32_t n_targets,
                                          int32_t total_tiles, const int32_t *out_last,
                                          const int32_t *out_ncontrib, const int64_t *store_base,
                                          const float *store, int64_t store_cap, const float *dL_drgb,
                                          void *accum_ws, void *stream) {
    using namespace gs;
    if (!valid_settings(s) || !proj_ws || !sort_ws || !targets || !out_last || !out_ncontrib ||
        !store_base || !store || store_cap < 0 || !dL_drgb || !accum_ws || n_cap <= 0 || n_cap % 64 ||
        n_views <= 0 || n_targets <= 0 || total_tiles <= 0 || pair_cap <= 0 || pair_cap > kMaxPairs ||
        int64_t(n_views) * n_cap > kMaxRecords)
        return GS_ERR_INVALID_ARGUMENT;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t records = int64_t(n_views) * n_cap;
    const Sorted srt = sorted_at(sort_ws, n_views, n_targets, n_cap, pair_cap, total_tiles);
    const Proj proj = proj_at(const_cast<void *>(proj_ws), records);
    float *acc = static_cast<float *>(accum_ws);
    launch_fill(acc, int64_t(kAccRows) * records, 0.f, st);
    const TStore ts{store_base, store_base + total_tiles, const_cast<float *>(store), store_cap};
    switch (s->bwd_waves) {
        case 1:
            hipLaunchKernelGGL((render_bwd_kernel<1, true>), dim3(total_tiles), dim3(64), 0, st, *s, proj, n_cap,
                               srt, targets, n_targets, nullptr, out_last, dL_drgb, acc, out_ncontrib, ts);
            break;
        case 2:
            hipLaunchKernelGGL((render_bwd_kernel<2, true>), dim3(total_tiles), dim3(128), 0, st, *s, proj, n_cap,
                               srt, targets, n_targets, nullptr, out_last, dL_drgb, acc, out_ncontrib, ts);
            break;
        default:
            hipLaunchKernelGGL((render_bwd_kernel<4, true>), dim3(total_tiles), dim3(256), 0, st, *s, proj, n_cap,
                               srt, targets, n_targets, nullptr, out_last, dL_drgb, acc, out_ncontrib, ts);
            break;
    }
    GS_CHECK_LAUNCH();
    return GS_OK;
}

extern "C" gs_status gs_project_bwd(const gs_settings *s, const float *params, int64_t n,
                                    int64_t n_cap, const gs_view *views, int32_t n_views,
                                    const void *accum_ws, float *grad, void *stream) {
    using namespace gs;
    if (!valid_settings(s) || !params || !views || !accum_ws || !grad || n < 0 || n_cap <= 0 ||
        n > n_cap || n_cap % 64 || n_views <= 0)
        return GS_ERR_INVALID_ARGUMENT;
    return launch_project_backward(*s, params, n, n_cap, views, n_views,
                                   static_cast<const float *>(accum_ws), grad,
                                   static_cast<hipStream_t>(stream));
}

extern "C" gs_status gs_project_bwd_adam(const gs_settings *s, float *params, int64_t n,
                                         int64_t n_cap, const gs_view *views, int32_t n_views,
                                         const void *accum_ws, float *m, float *v,
                                         const float *lr_rows, double beta1, double beta2,
                                         double eps, int32_t step, const int32_t *d_step,
                                         void *proj_out, void *stream) {
    using namespace gs;
    if (!valid_settings(s) || !params || !views || !accum_ws || !m || !v || !lr_rows || n < 0 ||
        n_cap <= 0 || n > n_cap || n_cap % 64 || n_views <= 0 || (step < 1 && !d_step) ||
        !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps >= 0.0))
        return GS_ERR_INVALID_ARGUMENT;
    return launch_project_backward_adam(*s, params, n, n_cap, views, n_views,
                                        static_cast<const float *>(accum_ws), m, v, lr_rows, beta1,
                                        beta2, eps, step, step < 1 ? d_step : nullptr, proj_out,
                                        static_cast<hipStream_t>(stream));
}

extern "C" gs_status gs_render_bwd(const gs_settings *s, const float *params, int64_t n,
                                   int64_t n_cap, const gs_view *views, int32_t n_views,
                                   const void *proj_ws, const void *sort_ws, int64_t pair_cap,
                                   const gs_target *targets, int32_t n_targets, int32_t total_tiles,
                                   const float *out_T, const int32_t *out_last,
                                   const float *dL_drgb, void *accum_ws, float *grad,
                                   void *stream) {
    if (!params || !grad || n < 0 || n > n_cap || !views) return GS_ERR_INVALID_ARGUMENT;
    gs_status r = gs_raster_bwd(s, proj_ws, n_cap, n_views, sort_ws, pair_cap, targets, n_targets,
                                total_tiles, out_T, out_last, dL_drgb, accum_ws, stream);
    if (r != GS_OK) return r;
    return gs_project_bwd(s, params, n, n_cap, views, n_views, accum_ws, grad, stream);
}

extern "C" gs_status gs_render_bwd_adam(const gs_settings *s, float *params, int64_t n,
                                        int64_t n_cap, const gs_view *views, int32_t n_views,
                                        const void *proj_ws, const void *sort_ws, int64_t pair_cap,
                                        const gs_target *targets, int32_t n_targets,
                                        int32_t total_tiles, const float *out_T,
                                        const int32_t *out_last, const float *dL_drgb,
                                        void *accum_ws, float *m, float *v, const float *lr_rows,
                                        double beta1, double beta2, double eps, int32_t step,
                                        const int32_t *d_step, void *proj_out, void *stream) {
    if (!params || !m || !v || !lr_rows || n < 0 || n > n_cap || !views || (step < 1 && !d_step))
        return GS_ERR_INVALID_ARGUMENT;
    gs_status r = gs_raster_bwd(s, proj_ws, n_cap, n_views, sort_ws, pair_cap, targets, n_targets,
                                total_tiles, out_T, out_last, dL_drgb, accum_ws, stream);
    if (r != GS_OK) return r;
    return gs_project_bwd_adam(s, params, n, n_cap, views, n_views, accum_ws, m, v, lr_rows, beta1,
                               beta2, eps, step, d_step, proj_out, stream);
}

namespace gs {
__global__ void step_advance_kernel(int32_t *d_step) {
    if (threadIdx.x == 0) *d_step += 1;
}
}  // namespace gs

extern "C" gs_status gs_step_advance(int32_t *d_step, void *stream) {
    if (!d_step) return GS_ERR_INVALID_ARGUMENT;
    hipLaunchKernelGGL(gs::step_advance_kernel, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream),
                       d_step);
    GS_CHECK_LAUNCH();
    return GS_OK;
}

extern "C" gs_status gs_fill(float *dst, int64_t count, float value, void *stream) {
    if (!dst || count < 0) return GS_ERR_INVALID_ARGUMENT;
    if (count == 0) return GS_OK;
    gs::launch_fill(dst, count, value, static_cast<hipStream_t>(stream));
    GS_CHECK_LAUNCH();
    return GS_OK;
}
