// Tile binning for the tile-based renderer (Section 3.3): every (target,
// Gaussian) whose cutoff ellipse touches a 16x16 tile becomes a (tile,
// Gaussian) pair, and each tile's pairs are put in front-to-back order.
//
// The order is built in two stable sorts instead of one wide-key sort:
// (1) the visible (view, Gaussian) records (visible in any target of the
// view: the pyramid levels of a keyframe share one record and one depth) are
// compacted and radix-sorted by their camera depth (27-bit keys, three 9-bit
// passes over V records); (2) the records emit their pairs, for every target
// of their view, in that depth order and the pairs are sorted by global tile
// index alone: one counting pass whose digit is the whole tile index up to
// 4096 tiles (3225 at 1200x680), else 8- or 9-bit radix passes.  Because
// both sorts are stable and records are compacted in (view, Gaussian) order,
// each tile's list is ordered by (depth, Gaussian index).
// Pair counts are data dependent; every kernel reads them from device
// counters so the whole sequence is launch-shape static and graph-capturable.
#include "gs_internal.hpp"

namespace gs {

// Conservative pixel bounding box of {alpha >= alpha_min} for a record at a
// pyramid level.  Returns false when the record cannot reach any pixel; records
// behind the near plane carry opacity 0 and are rejected by the opacity test.
struct Rect {
    int x0, x1, y0, y1;   // inclusive tile ranges
};

__device__ __forceinline__ bool tile_rect(const gs_settings &s, double2 md, float4 cov_o,
                                          const gs_target &t, Rect &r) {
    const float o = cov_o.w;
    if (!(o >= s.alpha_min)) return false;
    const float sc = ldexpf(1.f, -t.level);
    const float mx = float(md.x) * sc, my = float(md.y) * sc;
    const float c00 = cov_o.x * sc * sc + s.dilation;
    const float c11 = cov_o.z * sc * sc + s.dilation;
    const float tq = 2.f * logf(o / s.alpha_min);
    float ex = sqrtf(tq * c00), ey = sqrtf(tq * c11);
    ex += 0.05f + 1e-3f * ex;
    ey += 0.05f + 1e-3f * ey;
    const float fx0 = ceilf(mx - ex), fx1 = floorf(mx + ex);
    const float fy0 = ceilf(my - ey), fy1 = floorf(my + ey);
    if (!(fx1 >= 0.f) || !(fy1 >= 0.f) || !(fx0 <= float(t.width - 1)) ||
        !(fy0 <= float(t.height - 1)) || !(fx0 <= fx1) || !(fy0 <= fy1))
        return false;
    const int px0 = max(0, int(fx0)), px1 = min(t.width - 1, int(fx1));
    const int py0 = max(0, int(fy0)), py1 = min(t.height - 1, int(fy1));
    const TileShape ts = tile_shape(t.tile_w);
    r.x0 = px0 >> ts.wlog; r.x1 = px1 >> ts.wlog;
    r.y0 = py0 / ts.h; r.y1 = py1 / ts.h;
    return true;
}

// Set-up of a binning call: counters to zero, tile ranges to empty, and
// (block 0) the targets of each view as a CSR list in target order.
// Clears the counters and the tile ranges, and lists the targets of every
// view: view_off[v] = number of targets of views before v, view_list holds
// the targets view by view in index order.  Workgroup 0 does the lists from
// the targets' view indices staged in LDS, kSetupChunk at a time: the offset
// of view v counts the targets of smaller views, a target's place adds the
// earlier targets of its own view (targets of a view outside [0, n_views) are
// left out).
constexpr int kSetupChunk = 1024;

__global__ void __launch_bounds__(256) sort_setup_kernel(const gs_target *__restrict__ targets,
                                                         int32_t n_targets, int32_t n_views,
                                                         uint32_t *__restrict__ counters,
                                                         uint32_t *__restrict__ view_off,
                                                         uint32_t *__restrict__ view_list,
                                                         uint2 *__restrict__ ranges, int64_t total_tiles,
                                                         uint32_t *__restrict__ queue) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < total_tiles) ranges[i] = make_uint2(0u, 0u);
    if (blockIdx.x != 0) return;
    const int tid = threadIdx.x;
    if (tid < kNumCounters) counters[tid] = 0u;
    if (tid < kQueueWords) queue[tid] = 0u;
    __shared__ int32_t tv[kSetupChunk];
    auto stage = [&](int32_t c0) {
        __syncthreads();
        for (int k = tid; k < kSetupChunk; k += 256) {
            const int32_t t = c0 + k;
            const int32_t v = t < n_targets ? targets[t].view : -1;
            tv[k] = (v >= 0 && v < n_views) ? v : -1;
        }
        __syncthreads();
    };
    for (int32_t v0 = 0; v0 <= n_views; v0 += 256) {
        const int32_t v = v0 + tid;
        uint32_t below = 0;
        for (int32_t c0 = 0; c0 < n_targets; c0 += kSetupChunk) {
            stage(c0);
            const int m = n_targets - c0 < kSetupChunk ? n_targets - c0 : kSetupChunk;
#pragma unroll 8
            for (int k = 0; k < m; ++k) below += uint32_t(tv[k] >= 0 && tv[k] < v);
        }
        if (v <= n_views) view_off[v] = below;
    }
    for (int32_t t0 = 0; t0 < n_targets; t0 += 256) {
        const int32_t t = t0 + tid;
        int32_t mv = -1;
        if (t < n_targets) {
            const int32_t v = targets[t].view;
            mv = (v >= 0 && v < n_views) ? v : -1;
        }
        uint32_t place = 0;
        for (int32_t c0 = 0; c0 < n_targets; c0 += kSetupChunk) {
            stage(c0);
            const int m = n_targets - c0 < kSetupChunk ? n_targets - c0 : kSetupChunk;
#pragma unroll 8
            for (int k = 0; k < m; ++k) {
                const int32_t w = tv[k];
                place += uint32_t(w >= 0 && (w < mv || (w == mv && c0 + k < t)));
            }
        }
        if (mv >= 0) view_list[place] = uint32_t(t);
    }
}

// A tile rectangle that holds no tile (x0 = 1 > x1 = 0): count 0.
constexpr uint32_t kEmptyRectX = 1u;

__device__ __forceinline__ uint32_t rect_count(uint2 rc) {
    const uint32_t w = (rc.x >> 16) - (rc.x & 0xffffu) + 1u;
    const uint32_t h = (rc.y >> 16) - (rc.y & 0xffffu) + 1u;
    return w * h;
}

// Index of this workgroup in the count and compaction grids (n_cap / 256
// rounded up, n_views) of 256-thread workgroups: workgroups in record order.
__device__ __forceinline__ int64_t group_slot() {
    return int64_t(blockIdx.y) * gridDim.x + blockIdx.x;
}

// Number of lanes of the workgroup where `flag` holds, summed over the waves
// before this one (*before) and over all of them (returned).  Every thread
// of the workgroup takes part.
__device__ __forceinline__ uint32_t group_count(bool flag, uint32_t *lds4, uint32_t *before) {
    const int wave = threadIdx.x / kWave;
    const uint32_t c = uint32_t(__popcll(__ballot(flag)));
    if (lane_id() == 0) lds4[wave] = c;
    __syncthreads();
    uint32_t b = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        const uint32_t x = lds4[w];
        b += w < wave ? x : 0u;
        all += x;
    }
    *before = b;
    return all;
}

// For record (v, g): counts[v * n_cap + g] = its number of tiles over the
// targets of view v, and its tile rectangle in the q-th target packed as
// (x0 | x1 << 16, y0 | y1 << 16) (empty when it touches none) at
// rects[view_off[v] * n_cap + g * m_v + q] (m_v targets in view v: a record's
// rectangles are adjacent).
// kOne: a single target in the call.  Its view's list is that target, and
// the count kernel also does the set-up's other work (counters, the work
// queue and the tile ranges to zero), so no set-up kernel runs.
template <bool kOne>
__global__ void __launch_bounds__(256) count_kernel(gs_settings s, Proj proj, int64_t n, int64_t n_cap,
                                                    const gs_target *__restrict__ targets,
                                                    const uint32_t *__restrict__ view_off,
                                                    const uint32_t *__restrict__ view_list,
                                                    uint32_t *__restrict__ counts,
                                                    uint2 *__restrict__ rects,
                                                    uint32_t *__restrict__ group_vis,
                                                    uint32_t *__restrict__ counters, uint32_t *__restrict__ queue,
                                                    uint2 *__restrict__ ranges, int64_t total_tiles) {
    __shared__ uint32_t lds4[kScanThreads / kWave];
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int v = blockIdx.y;
    const int64_t r = int64_t(v) * n_cap + g;
    int one_view = -1;   // kOne: the target's view (-1: outside [0, n_views), no list)
    if (kOne) {
        const int64_t gid = group_slot() * blockDim.x + threadIdx.x;
        const int64_t nthreads = int64_t(gridDim.x) * gridDim.y * blockDim.x;
        for (int64_t i = gid; i < total_tiles; i += nthreads) ranges[i] = make_uint2(0u, 0u);
        if (gid < kNumCounters) counters[gid] = 0u;
        if (gid < kQueueWords) queue[gid] = 0u;
        const int tv = targets[0].view;
        one_view = (tv >= 0 && tv < int(gridDim.y)) ? tv : -1;
    }
    uint32_t total = 0;
    if (g < n) {   // (n <= n_cap)
        const double2 md = proj.mean[r];
        const float4 co = proj.cov_o[r];
        const uint32_t q0 = kOne ? uint32_t(one_view >= 0 && v > one_view) : view_off[v];
        const uint32_t m = kOne ? uint32_t(v == one_view) : view_off[v + 1] - q0;
        uint2 *out = rects + int64_t(q0) * n_cap + g * m;
        for (uint32_t q = 0; q < m; ++q) {
            const gs_target t = targets[kOne ? 0u : view_list[q0 + q]];
            Rect rc;
            uint2 packed = make_uint2(kEmptyRectX, 0u);
            if (tile_rect(s, md, co, t, rc)) {
                total += uint32_t(rc.x1 - rc.x0 + 1) * uint32_t(rc.y1 - rc.y0 + 1);
                packed = make_uint2(uint32_t(rc.x0) | (uint32_t(rc.x1) << 16),
                                    uint32_t(rc.y0) | (uint32_t(rc.y1) << 16));
            }
            out[q] = packed;   // streamed for every record: cheaper than sparse writes
        }
    }
    if (g < n_cap) counts[r] = total;
    uint32_t before;
    const uint32_t vis = group_count(total != 0u, lds4, &before);
    if (threadIdx.x == 0) group_vis[group_slot()] = vis;
}

// ---------------------------------------------------------------------------
// Scan helpers
// ---------------------------------------------------------------------------
// 64-bit wave scans for the pair offsets: a sum of per-record pair counts may
// pass 2^32, and is then saturated (a total past pair_cap <= 2^31 - 1 is an
// overflow, reported as such) instead of wrapping.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
    return (uint64_t(dpp_u32<kCtrl, kRowMask>(uint32_t(v >> 32))) << 32) | dpp_u32<kCtrl, kRowMask>(uint32_t(v));
}
// (the DPP steps of wave_inclusive_scan, on both halves)
__device__ __forceinline__ uint64_t wave_inclusive_scan64(uint64_t v) {
    v += dpp_u64<0x111, 0xf>(v);
    v += dpp_u64<0x112, 0xf>(v);
    v += dpp_u64<0x114, 0xf>(v);
    v += dpp_u64<0x118, 0xf>(v);
    v += dpp_u64<0x142, 0xa>(v);
    v += dpp_u64<0x143, 0xc>(v);
    return v;
}
__device__ __forceinline__ uint32_t sat32(uint64_t v) {
    return v > 0xffffffffull ? 0xffffffffu : uint32_t(v);
}

// Exclusive scan over a 256-thread block in 64 bits; block total to *total.
// lds needs 4 words.
__device__ __forceinline__ uint64_t block_exclusive_scan64(uint64_t v, uint64_t *lds, uint64_t *total) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const uint64_t inc = wave_inclusive_scan64(v);
    if (lane == kWave - 1) lds[wave] = inc;
    __syncthreads();
    uint64_t base = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        const uint64_t x = lds[w];
        base += w < wave ? x : 0u;
        all += x;
    }
    __syncthreads();
    *total = all;
    return base + inc - v;
}

// Exclusive scan of the per-workgroup visible-record counts bsum[0..nb) in
// place (one block of 1024 threads); the total goes to *total_out.  Every
// partial sum counts records, so it fits 32 bits.  Wave w takes the w-th of
// 16 consecutive runs of 64-entry chunks, its lanes reading consecutive
// entries.  Runs of up to kBsumBatch chunks are loaded once and kept in
// registers; longer ones are read twice, kBsumBatch chunks at a time.
constexpr int kBsumWaves = 16, kBsumBatch = 16;
__global__ void __launch_bounds__(kBsumWaves * kWave) scan_bsums_kernel(uint32_t *bsum, int64_t nb,
                                                                       uint32_t *total_out) {
    __shared__ uint32_t lds[kBsumWaves];
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const int64_t chunks = (nb + kWave - 1) / kWave;
    const int64_t per = (chunks + kBsumWaves - 1) / kBsumWaves;   // chunks per wave
    const int64_t c0 = wave * per, c1 = c0 + per < chunks ? c0 + per : chunks;
    auto load = [&](int64_t c, uint32_t (&v)[kBsumBatch]) {
#pragma unroll
        for (int j = 0; j < kBsumBatch; ++j) {
            const int64_t i = (c + j) * kWave + lane;
            v[j] = (c + j < c1 && i < nb) ? bsum[i] : 0u;
        }
    };
    auto store = [&](int64_t c, const uint32_t (&v)[kBsumBatch], uint32_t &run) {
#pragma unroll
        for (int j = 0; j < kBsumBatch; ++j) {
            const int64_t i = (c + j) * kWave + lane;
            const uint32_t inc = wave_inclusive_scan(v[j]);
            if (c + j < c1 && i < nb) bsum[i] = run + inc - v[j];
            run += uint32_t(__builtin_amdgcn_readlane(int(inc), kWave - 1));
        }
    };
    auto cross_waves = [&](uint32_t local, uint32_t &run, uint32_t &all) {
        const uint32_t wtotal = wave_sum(local);
        if (lane == 0) lds[wave] = wtotal;
        __syncthreads();
        run = 0u;
        all = 0u;
#pragma unroll
        for (int w = 0; w < kBsumWaves; ++w) {
            const uint32_t x = lds[w];
            run += w < wave ? x : 0u;
            all += x;
        }
    };
    uint32_t run, all;
    if (per <= kBsumBatch) {   // uniform: every wave holds its run
        uint32_t v[kBsumBatch], local = 0u;
        load(c0, v);
#pragma unroll
        for (int j = 0; j < kBsumBatch; ++j) local += v[j];
        cross_waves(local, run, all);
        store(c0, v, run);
    } else {
        uint32_t local = 0u;
        for (int64_t c = c0; c < c1; c += kBsumBatch) {
            uint32_t v[kBsumBatch];
            load(c, v);
#pragma unroll
            for (int j = 0; j < kBsumBatch; ++j) local += v[j];
        }
        cross_waves(local, run, all);
        for (int64_t c = c0; c < c1; c += kBsumBatch) {
            uint32_t v[kBsumBatch];
            load(c, v);
            store(c, v, run);
        }
    }
    if (threadIdx.x == 0) *total_out = all;
}


// Depth sort key of a visible record: the bit pattern of its (positive,
// float) depth minus that of the near plane, which orders depths exactly as
// the floats do while they stay within 2^27 ulps of the near plane (below
// znear * 2^16: 13 km at znear 0.2 m); deeper ones share the largest key and
// keep record order.  27 bits: three 9-bit radix passes.
constexpr int kDepthKeyBits = 27;
__device__ __forceinline__ uint32_t depth_key(float z, float znear) {
    const uint32_t a = __float_as_uint(z), b = __float_as_uint(znear);
    const uint32_t d = a > b ? a - b : 0u;
    return d < (1u << kDepthKeyBits) ? d : (1u << kDepthKeyBits) - 1u;
}

// Compaction of the visible records (pair count > 0) in record order: keys =
// depth keys, values = record indices, and the counts alongside.  Same grid
// as count_kernel; a workgroup's records land after those of the workgroups
// before it, in thread order.
// kFold (at most kFoldGroups count workgroups): each workgroup sums the
// visible counts of the workgroups before it itself (at most four 16-byte
// loads per thread, from L2), and the last one stores the number of visible
// records to *n_visible, so no scan of the counts runs in between.
// Otherwise group_vis holds the counts' exclusive scan (scan_bsums_kernel).
constexpr int64_t kFoldGroups = 4096;
template <bool kFold>
__global__ void __launch_bounds__(256) compact_scatter_kernel(const uint32_t *__restrict__ counts,
                                                              int64_t n_cap, Proj proj, float znear,
                                                              const uint32_t *__restrict__ group_vis,
                                                              int64_t groups,
                                                              uint32_t *__restrict__ vis_key,
                                                              uint32_t *__restrict__ vis_val,
                                                              uint32_t *__restrict__ vis_cnt,
                                                              uint32_t *__restrict__ n_visible) {
    __shared__ uint32_t lds4[kScanThreads / kWave];
    __shared__ uint32_t fold4[kScanThreads / kWave];
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t r = int64_t(blockIdx.y) * n_cap + g;
    const int64_t gs = group_slot();
    const uint32_t c = g < n_cap ? counts[r] : 0u;
    if constexpr (kFold) {
        // entries [0, gs) in 16-byte pieces (group_vis is 256-byte aligned and
        // padded to a multiple of 4 entries); pieces past gs read piece 0
        constexpr int kIt = int(kFoldGroups / (4 * kScanThreads));
        const uint4 *gv = reinterpret_cast<const uint4 *>(group_vis);
        uint4 q[kIt];
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            const int64_t j = threadIdx.x + k * kScanThreads;
            q[k] = gv[4 * j < gs ? j : 0];
        }
        uint32_t sum = 0u;
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            const int64_t i = 4 * (threadIdx.x + k * kScanThreads);
            sum += (i < gs ? q[k].x : 0u) + (i + 1 < gs ? q[k].y : 0u) + (i + 2 < gs ? q[k].z : 0u) +
                   (i + 3 < gs ? q[k].w : 0u);
        }
        sum = wave_sum(sum);
        if (lane_id() == 0) fold4[threadIdx.x / kWave] = sum;   // (read after group_count's barrier)
    }
    uint32_t before;
    const uint32_t all = group_count(c != 0u, lds4, &before);
    uint32_t gbase;
    if constexpr (kFold) {
        gbase = fold4[0] + fold4[1] + fold4[2] + fold4[3];
        if (gs == groups - 1 && threadIdx.x == 0) *n_visible = gbase + all;
    } else {
        gbase = group_vis[gs];
    }
    const uint64_t mask = __ballot(c != 0u);
    if (c != 0u) {
        const uint32_t at = gbase + before + uint32_t(mask_rank(mask));
        vis_key[at] = depth_key(proj.rgb_z[r].w, znear);
        vis_val[at] = uint32_t(r);
        vis_cnt[at] = c;
    }
}

// q = k / w, r = k % w for k < 2^24, w >= 1: a float reciprocal estimate
// corrected by one step (exact: the estimate is off by at most one).
__device__ __forceinline__ void divmod_small(uint32_t k, uint32_t w, uint32_t &q, uint32_t &r) {
    q = uint32_t(float(k) * __builtin_amdgcn_rcpf(float(w)));
    int32_t rr = int32_t(k) - int32_t(q * w);
    if (rr < 0) { --q; rr += int32_t(w); }
    else if (rr >= int32_t(w)) { ++q; rr -= int32_t(w); }
    r = uint32_t(rr);
}

// Pair emission over chunks of kEmitChunk consecutive pair slots, kEmitPer
// consecutive slots per thread.  The records covering a chunk (at most one per
// slot, each has >= 1 pair) start at chunk_first[] (one entry per 256 slots,
// written by the last depth pass).  Every record after the first marks the slot
// where it starts, and a block scan of the marks gives each slot its record,
// so near-camera Gaussians that cover thousands of tiles are spread over many
// threads; a thread reuses its record's data across its slots and stores its
// keys and values as one vector each.
constexpr int kEmitPer = 4;
constexpr int kEmitChunk = kScanThreads * kEmitPer;
constexpr int kEmitCache = 4;   // targets per view held in registers (pyramid levels)
constexpr int kEmitTab = 256;   // views and listed targets staged in LDS

// 64 VGPRs: eight waves per SIMD for this latency-bound kernel (66 and seven
// waves otherwise, measured slower in spite of a small spill)
// kOne: a single target in the call, so every visible record has exactly one
// rectangle, rects[g] with g = record - target view * n_cap.
template <bool kOne>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
emit_kernel(int64_t n_cap, int32_t n_views, const gs_target *__restrict__ targets,
            uint32_t *__restrict__ counters,
            const uint32_t *__restrict__ vis_val, const uint32_t *__restrict__ vis_off,
            const uint2 *__restrict__ rects, const uint32_t *__restrict__ view_off,
            const uint32_t *__restrict__ view_list, const uint32_t *__restrict__ chunk_first,
            int64_t pair_cap, uint32_t *__restrict__ pkey, uint32_t *__restrict__ pval,
            uint32_t *__restrict__ d_status) {
    __shared__ uint32_t off[kEmitChunk];
    __shared__ uint32_t srcs[kEmitChunk];            // record ids, staged with the offsets
    __shared__ uint2 srect[kOne ? kEmitChunk : 1];   // kOne: the records' tile rectangles
    __shared__ uint32_t mark[kEmitChunk / 32];       // bit per slot: a record starts there
    __shared__ uint32_t lds[8];
    // the view offsets and, per listed target, its tile offset and row length,
    // staged once (indices beyond the tables read global memory)
    __shared__ uint32_t s_voff[kEmitTab + 1];
    __shared__ uint2 s_tgt[kEmitTab];
    const uint32_t V = counters[kVisible];
    const uint32_t P = counters[kPairs];
    const uint32_t Pc = int64_t(P) > pair_cap ? uint32_t(pair_cap) : P;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        counters[kPairsClamped] = Pc;
        if (Pc != P && d_status) atomicOr(d_status, GS_STATUS_PAIR_OVERFLOW);
    }
    if (V == 0) return;   // no visible record, no pair (Pc == 0)
    // the grid is sized for the pair capacity: workgroups without a chunk
    // leave before staging the tables
    if (int64_t(blockIdx.x) * kEmitChunk >= int64_t(Pc)) return;
    const int tid = threadIdx.x;
    // lim_v / lim_t entries are in LDS, the rest in global memory
    uint32_t lim_v = 0, lim_t = 0;
    uint32_t one_toff = 0, one_tx = 0, one_vbase = 0;   // kOne: the target
    if (kOne) {
        const gs_target t0 = targets[0];
        one_toff = uint32_t(t0.tile_offset);
        one_tx = uint32_t(t0.tiles_x);
        one_vbase = uint32_t(t0.view) * uint32_t(n_cap);   // (records are indexed by uint32)
    } else {
        const int nv = n_views < kEmitTab ? n_views : kEmitTab;
        for (int i = tid; i <= nv; i += kScanThreads) s_voff[i] = view_off[i];
        const uint32_t listed = view_off[n_views];   // targets in the lists
        lim_v = uint32_t(nv) + 1u;
        lim_t = listed < uint32_t(kEmitTab) ? listed : uint32_t(kEmitTab);
        for (uint32_t i = tid; i < lim_t; i += kScanThreads) {
            const gs_target &t = targets[view_list[i]];
            s_tgt[i] = make_uint2(uint32_t(t.tile_offset), uint32_t(t.tiles_x));
        }
        __syncthreads();
    }
    auto voff_of = [&](uint32_t v) { return v < lim_v ? s_voff[v] : view_off[v]; };
    auto tgt_of = [&](uint32_t i) {
        if (i < lim_t) return s_tgt[i];
        const gs_target &t = targets[view_list[i]];
        return make_uint2(uint32_t(t.tile_offset), uint32_t(t.tiles_x));
    };
    for (int64_t chunk = blockIdx.x; chunk * kEmitChunk < Pc; chunk += gridDim.x) {
        const uint32_t o0 = uint32_t(chunk * kEmitChunk);
        const uint32_t j0 = chunk_first[chunk * (kEmitChunk / kScanThreads)];   // record holding slot o0
        // the record holding the next chunk's first slot is the last one this
        // chunk can touch: only the offsets up to it are loaded
        const uint32_t j1 = (chunk + 1) * kEmitChunk < Pc
                                ? chunk_first[(chunk + 1) * (kEmitChunk / kScanThreads)]
                                : V - 1u;
        __syncthreads();
        if (tid < kEmitChunk / 32) mark[tid] = 0u;
        uint32_t sv[kEmitPer];
#pragma unroll
        for (int r = 0; r < kEmitPer; ++r) {
            const int i = tid + r * kScanThreads;
            const uint32_t j = j0 + uint32_t(i);
            const bool in = j <= j1 && j < V;
            off[i] = in ? vis_off[j] : 0xffffffffu;
            sv[r] = in ? vis_val[j] : 0u;
            srcs[i] = sv[r];
        }
        if (kOne) {   // every record's rectangle, loaded once per chunk with the others in flight
#pragma unroll
            for (int r = 0; r < kEmitPer; ++r) {
                const int i = tid + r * kScanThreads;
                const uint32_t j = j0 + uint32_t(i);
                const bool in = j <= j1 && j < V;
                const uint2 rc = rects[in ? sv[r] - one_vbase : 0u];
                srect[i] = in ? rc : make_uint2(kEmptyRectX, 0u);
            }
        }
        __syncthreads();
        // records after the first start strictly after o0
#pragma unroll
        for (int r = 0; r < kEmitPer; ++r) {
            const int i = tid + r * kScanThreads;
            const uint32_t rel = off[i] - o0;
            if (i > 0 && j0 + uint32_t(i) < V && rel < uint32_t(kEmitChunk))
                atomicOr(&mark[rel >> 5], 1u << (rel & 31u));
        }
        __syncthreads();
        static_assert(32 % kEmitPer == 0, "a thread's slots lie in one mark word");
        const uint32_t mword = mark[(tid * kEmitPer) >> 5] >> ((tid * kEmitPer) & 31);
        uint32_t mk[kEmitPer], msum = 0;
#pragma unroll
        for (int i = 0; i < kEmitPer; ++i) { mk[i] = (mword >> i) & 1u; msum += mk[i]; }
        uint32_t total;
        uint32_t rec = block_exclusive_scan(msum, lds, &total);   // records started before my slots
        uint32_t key[kEmitPer], val[kEmitPer];
        uint32_t cur = 0xffffffffu, src = 0, base = 0, v = 0, g = 0, q0 = 0, mv = 0;
        const uint2 *rc_v = rects;
        // the record's first kEmitCache targets: rectangle, tile count, tile
        // offset and row length, loaded once per record
        uint2 rcc[kEmitCache];
        uint32_t cnt[kEmitCache], toff[kEmitCache], tx[kEmitCache];
#pragma unroll
        for (int i = 0; i < kEmitPer; ++i) {
            rec += mk[i];
            const uint32_t o = o0 + uint32_t(tid * kEmitPer + i);
            key[i] = 0u;
            val[i] = 0u;
            if (o >= Pc) continue;
            if (kOne) {
                if (rec != cur) {
                    cur = rec;
                    src = srcs[rec];
                    base = off[rec];
                    rcc[0] = srect[rec];
                }
                const uint32_t k = o - base;
                const uint32_t x0 = rcc[0].x & 0xffffu, x1 = rcc[0].x >> 16, y0 = rcc[0].y & 0xffffu;
                uint32_t dy, dx;
                divmod_small(k, x1 - x0 + 1, dy, dx);
                key[i] = one_toff + (y0 + dy) * one_tx + x0 + dx;
                val[i] = src;
                continue;
            }
            if (rec != cur) {   // first slot of this thread in a record
                cur = rec;
                src = srcs[rec];   // record v * n_cap + g
                base = off[rec];
                v = src / uint32_t(n_cap);
                g = src - v * uint32_t(n_cap);
                q0 = voff_of(v);
                mv = voff_of(v + 1) - q0;
                rc_v = rects + int64_t(q0) * n_cap + int64_t(g) * mv;
#pragma unroll
                for (int q = 0; q < kEmitCache; ++q) {
                    rcc[q] = make_uint2(1u, 0u);
                    cnt[q] = toff[q] = tx[q] = 0u;
                    if (uint32_t(q) < mv) {
                        rcc[q] = rc_v[q];
                        cnt[q] = rect_count(rcc[q]);
                        const uint2 tg = tgt_of(q0 + q);
                        toff[q] = tg.x;
                        tx[q] = tg.y;
                    }
                }
            }
            // the k-th pair of the record: targets of its view in order, tiles row-major
            uint32_t k = o - base;
            bool found = false;
#pragma unroll
            for (int q = 0; q < kEmitCache; ++q) {
                if (found || uint32_t(q) >= mv) continue;
                if (k < cnt[q]) {
                    const uint32_t x0 = rcc[q].x & 0xffffu, x1 = rcc[q].x >> 16, y0 = rcc[q].y & 0xffffu;
                    uint32_t dy, dx;
                    divmod_small(k, x1 - x0 + 1, dy, dx);
                    key[i] = toff[q] + (y0 + dy) * tx[q] + x0 + dx;
                    found = true;
                } else {
                    k -= cnt[q];
                }
            }
            for (uint32_t q = kEmitCache; !found && q < mv; ++q) {
                const uint2 rc = rc_v[q];
                const uint32_t c = rect_count(rc);
                if (k < c) {
                    const uint32_t x0 = rc.x & 0xffffu, x1 = rc.x >> 16, y0 = rc.y & 0xffffu;
                    uint32_t dy, dx;
                    divmod_small(k, x1 - x0 + 1, dy, dx);
                    const uint2 tg = tgt_of(q0 + q);
                    key[i] = tg.x + (y0 + dy) * tg.y + x0 + dx;
                    found = true;
                }
                k -= c;
            }
            val[i] = src;
        }
        const uint32_t o_first = o0 + uint32_t(tid * kEmitPer);
        if (o_first + kEmitPer <= Pc) {
            *reinterpret_cast<uint4 *>(pkey + o_first) = make_uint4(key[0], key[1], key[2], key[3]);
            *reinterpret_cast<uint4 *>(pval + o_first) = make_uint4(val[0], val[1], val[2], val[3]);
        } else {
#pragma unroll
            for (int i = 0; i < kEmitPer; ++i)
                if (o_first + uint32_t(i) < Pc) { pkey[o_first + i] = key[i]; pval[o_first + i] = val[i]; }
        }
    }
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort pass (kBits-bit digit at `shift`) over n = *n_ptr
// elements.  A sort block owns kItems * 256 consecutive elements; wave w of
// it owns the contiguous quarter [w * kItems * 64, (w + 1) * kItems * 64).
// The grids are grid-stride over the sort blocks, so a capacity-sized launch
// does not start thousands of idle workgroups.
// ---------------------------------------------------------------------------
// Weighted (kW): also the sum of the weights w[] of each digit's elements per
// block, formed in 64 bits and stored saturated at 2^32 - 1 in
// whist[digit * wstride + block].
template <int kItems, int kBits, bool kW = false>
__global__ void __launch_bounds__(256) radix_hist_kernel(const uint32_t *__restrict__ n_ptr,
                                                         const uint32_t *__restrict__ keys, int shift,
                                                         uint32_t *__restrict__ hist,
                                                         int64_t max_blocks,
                                                         const uint32_t *__restrict__ w = nullptr,
                                                         uint32_t *__restrict__ whist = nullptr,
                                                         int64_t wstride = 0) {
    constexpr int kBins = 1 << kBits, kTileN = kItems * kScanThreads;
    __shared__ uint32_t h[kBins];
    __shared__ unsigned long long hw[kW ? kBins : 1];
    const uint32_t n = *n_ptr;
    const int64_t nb = (int64_t(n) + kTileN - 1) / kTileN;
    for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        __syncthreads();
        for (int i = threadIdx.x; i < kBins; i += kScanThreads) {
            h[i] = 0;
            if (kW) hw[i] = 0ull;
        }
        __syncthreads();
        const int64_t base = b * kTileN;
        uint32_t kk[kItems], ww[kItems];   // every load in flight before the first LDS atomic
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const int64_t e = base + k * kScanThreads + threadIdx.x;
            kk[k] = e < n ? keys[e] : 0u;
            ww[k] = (kW && e < n) ? w[e] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const int64_t e = base + k * kScanThreads + threadIdx.x;
            if (e < n) {
                const uint32_t d = (kk[k] >> shift) & (kBins - 1);
                atomicAdd(&h[d], 1u);
                if (kW) atomicAdd(&hw[d], static_cast<unsigned long long>(ww[k]));
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < kBins; i += kScanThreads) {
            hist[int64_t(i) * max_blocks + b] = h[i];
            if (kW) whist[int64_t(i) * wstride + b] = sat32(hw[i]);
        }
    }
}

// Block d: exclusive scan of row d of hist over the active blocks; row total
// to digit[d].  Weighted (kW): the same for row d of whist, in 64 bits,
// stored saturated, total to wdigit[d].
template <int kItems, bool kW = false>
__global__ void __launch_bounds__(256) radix_rowscan_kernel(const uint32_t *__restrict__ n_ptr,
                                                            uint32_t *__restrict__ hist,
                                                            int64_t max_blocks,
                                                            uint32_t *__restrict__ digit,
                                                            uint32_t *__restrict__ whist = nullptr,
                                                            int64_t wstride = 0,
                                                            uint32_t *__restrict__ wdigit = nullptr) {
    __shared__ uint32_t lds[8];
    __shared__ uint64_t lds64[kScanThreads / kWave];
    const int64_t nb = (int64_t(*n_ptr) + kItems * kScanThreads - 1) / (kItems * kScanThreads);
    uint32_t *row = hist + int64_t(blockIdx.x) * max_blocks;
    uint32_t *wrow = kW ? whist + int64_t(blockIdx.x) * wstride : nullptr;
    uint32_t run = 0;
    uint64_t wrun = 0;
    for (int64_t c = 0; c < nb; c += 256) {
        const int64_t i = c + threadIdx.x;
        const uint32_t v = (i < nb) ? row[i] : 0u;
        uint32_t total;
        const uint32_t pre = block_exclusive_scan(v, lds, &total);
        if (i < nb) row[i] = run + pre;
        run += total;
        if (kW) {
            const uint64_t x = (i < nb) ? wrow[i] : 0u;
            uint64_t wtotal;
            const uint64_t wpre = block_exclusive_scan64(x, lds64, &wtotal);
            if (i < nb) wrow[i] = sat32(wrun + wpre);
            wrun += wtotal;
        }
    }
    if (threadIdx.x == 0) {
        digit[blockIdx.x] = run;
        if (kW) wdigit[blockIdx.x] = sat32(wrun);
    }
}

// Outputs of the last depth pass in offsets mode: the pair-count sums per
// (digit, block) after their row scan and per digit, where the total pair
// count goes, and the first record of every 256-slot emission chunk.
struct PairOffsets {
    const uint32_t *whist;
    int64_t wstride;
    const uint32_t *wdigit;
    uint32_t *total;
    uint32_t *chunk_first;
    int64_t n_chunks;
};

// Scatter.  Ranks are found per wave with no workgroup barrier per element:
// a wave walks its quarter in order, groups equal digits with kBits ballots,
// and keeps a running count per digit in its own LDS row.  One barrier later
// the rows are turned into per-wave offsets, the block's elements are laid out
// in digit order in LDS and written so that consecutive threads write
// consecutive addresses of each digit's run.  Order inside a digit is the
// input order (stable).
// kCarry: a second value array (cin -> cout) moves with the keys.
// kOffsets (with kCarry; the last pass of the record sort): cin holds the
// records' pair counts, and cout receives instead each record's pair offset,
// the exclusive sum of the counts in the final order: counts of smaller
// digits (per-digit sums) + of the digit in earlier blocks (weighted row scan)
// + of the digit's run in this block before the record (a block scan of the
// counts laid out in digit order).  The record holding slot 256 q is written
// to chunk_first[q], and workgroup 0 stores the total pair count.  Sums are
// formed in 64 bits and stored saturated.
template <int kItems, int kBits, bool kCarry, bool kOffsets = false>
__global__ void __launch_bounds__(256) radix_scatter_kernel(
    const uint32_t *__restrict__ n_ptr, const uint32_t *__restrict__ kin,
    const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
    const uint32_t *__restrict__ cin, uint32_t *__restrict__ cout,
    int shift, const uint32_t *__restrict__ hist, int64_t max_blocks,
    const uint32_t *__restrict__ digit, PairOffsets po = PairOffsets{}) {
    static_assert(!kOffsets || kCarry, "offsets mode reads the counts as the carried values");
    constexpr int kBins = 1 << kBits, kPer = kBins / kScanThreads;
    constexpr int kWaves = kScanThreads / kWave;
    constexpr int kTileN = kItems * kScanThreads, kWaveN = kItems * kWave;
    static_assert(kPer >= 1 && kBins % kScanThreads == 0, "digit bins per thread");
    __shared__ uint32_t dbase[kBins];         // start of each digit over all blocks
    __shared__ uint32_t gbase[kBins];         // global start of each digit's run of this block
    __shared__ uint32_t lstart[kBins];        // start of each digit inside the block
    __shared__ uint32_t wcnt[kWaves][kBins];  // per-wave digit counts, then per-wave offsets
    __shared__ uint32_t skey[kTileN];
    __shared__ uint32_t sval[kTileN];
    __shared__ uint32_t scar[kCarry ? kTileN : 1];
    __shared__ uint32_t lds[8];
    __shared__ uint64_t wdbase[kOffsets ? kBins : 1];   // pair offset of each digit's first record
    __shared__ uint64_t wgbase[kOffsets ? kBins : 1];   // ... of its first record in this block
    __shared__ uint64_t wstart[kOffsets ? kBins : 1];   // block-scan value at the run's start
    __shared__ uint64_t lds64[kScanThreads / kWave];
    const uint32_t n = *n_ptr;
    const int64_t nb = (int64_t(n) + kTileN - 1) / kTileN;
    // each XCD takes consecutive sort blocks, whose digit runs meet in the same
    // cache lines, so the partial lines at run ends are completed in one L2.
    // The first T workgroups share the blocks (T a multiple of the XCD count,
    // as is the grid, and no larger than the blocks need, so that every XCD
    // gets some when there are fewer blocks than workgroups).
    const int64_t nb8 = (nb + kXcds - 1) / kXcds * kXcds;
    const int64_t T = nb8 < int64_t(gridDim.x) ? nb8 : int64_t(gridDim.x);
    if (int64_t(blockIdx.x) >= T) return;
    const int64_t w0 = xcd_tile(blockIdx.x, T);
    if (w0 >= nb) return;   // uniform over the workgroup
    const int tid = threadIdx.x, wave = tid / kWave, lane = lane_id();
    {
        uint32_t v[kPer], sum = 0, total;
#pragma unroll
        for (int j = 0; j < kPer; ++j) { v[j] = digit[tid * kPer + j]; sum += v[j]; }
        uint32_t pre = block_exclusive_scan(sum, lds, &total);
#pragma unroll
        for (int j = 0; j < kPer; ++j) { dbase[tid * kPer + j] = pre; pre += v[j]; }
    }
    if constexpr (kOffsets) {
        uint64_t v[kPer], sum = 0, total;
#pragma unroll
        for (int j = 0; j < kPer; ++j) { v[j] = po.wdigit[tid * kPer + j]; sum += v[j]; }
        uint64_t pre = block_exclusive_scan64(sum, lds64, &total);
#pragma unroll
        for (int j = 0; j < kPer; ++j) { wdbase[tid * kPer + j] = pre; pre += v[j]; }
        if (blockIdx.x == 0 && tid == 0) *po.total = sat32(total);
    }
    for (int64_t b = w0; b < nb; b += T) {
        const int64_t base = b * kTileN;
#pragma unroll
        for (int j = 0; j < kPer; ++j)
#pragma unroll
            for (int w = 0; w < kWaves; ++w) wcnt[w][tid * kPer + j] = 0;
        __syncthreads();
        uint32_t key[kItems], val[kItems], car[kItems], pos[kItems];
        const int64_t wbase = base + int64_t(wave) * kWaveN;
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const int64_t e = wbase + k * kWave + lane;
            const bool valid = e < n;
            key[k] = valid ? kin[e] : 0u;
            val[k] = valid ? vin[e] : 0u;
            car[k] = (kCarry && valid) ? cin[e] : 0u;
        }
        // The lowest lane of each digit group adds the group's size to the
        // wave's running count of that digit and gets the count before it.
        // A wave's LDS atomics execute in program order, so the counts follow
        // the element order (stable) while the atomics of all items are in
        // flight together; the leaders' counts then go to their groups.
        // pos[k] holds, until the hand-over, the leader's count (bits 0-15; a
        // wave's counts stay below kItems * 64), the leader lane (bits 16-21)
        // and this lane's rank in its group (bits 24-29).
        static_assert(kItems * kWave < (1 << 16), "counts fit 16 bits");
        // (items in groups of kRankGroup, which bounds the registers in flight)
        constexpr int kRankGroup = 4;
        static_assert(kItems % kRankGroup == 0, "items in whole groups");
#pragma unroll
        for (int k0 = 0; k0 < kItems; k0 += kRankGroup) {
#pragma unroll
            for (int k = k0; k < k0 + kRankGroup; ++k) {
                const bool valid = wbase + k * kWave + lane < n;
                const uint32_t d = (key[k] >> shift) & (kBins - 1);
                uint64_t peers = __ballot(valid);
#pragma unroll
                for (int bit = 0; bit < kBits; ++bit) {
                    const bool set = (d >> bit) & 1u;
                    const uint64_t m = __ballot(set);
                    peers &= set ? m : ~m;
                }
                const uint32_t rank = uint32_t(mask_rank(peers));
                const uint32_t leader = peers ? uint32_t(__builtin_ctzll(peers)) : uint32_t(lane);
                const uint32_t c =
                    (valid && rank == 0) ? atomicAdd(&wcnt[wave][d], uint32_t(__popcll(peers))) : 0u;
                pos[k] = c | (leader << 16) | (rank << 24);
            }
#pragma unroll
            for (int k = k0; k < k0 + kRankGroup; ++k)
                pos[k] = (uint32_t(__shfl(int(pos[k]), int((pos[k] >> 16) & 63u), kWave)) & 0xffffu) +
                         (pos[k] >> 24);
        }
        __syncthreads();
        {
            uint32_t cnt[kPer], sum = 0, total;
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                const int d = tid * kPer + j;
                uint32_t r = 0;
#pragma unroll
                for (int w = 0; w < kWaves; ++w) {
                    const uint32_t c = wcnt[w][d];
                    wcnt[w][d] = r;
                    r += c;
                }
                cnt[j] = r;
                sum += r;
            }
            uint32_t pre = block_exclusive_scan(sum, lds, &total);
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                const int d = tid * kPer + j;
                lstart[d] = pre;
                gbase[d] = dbase[d] + hist[int64_t(d) * max_blocks + b];
                if (kOffsets) wgbase[d] = wdbase[d] + po.whist[int64_t(d) * po.wstride + b];
                pre += cnt[j];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (wbase + k * kWave + lane < n) {
                const uint32_t d = (key[k] >> shift) & (kBins - 1);
                const uint32_t p = lstart[d] + wcnt[wave][d] + pos[k];
                skey[p] = key[k];
                sval[p] = val[k];
                if (kCarry) scar[p] = car[k];
            }
        }
        __syncthreads();
        const int cnt = int(min(int64_t(kTileN), int64_t(n) - base));
        if constexpr (kOffsets) {
            // element i = tid * kItems + j of the block in digit order
            static_assert(kTileN == kItems * kScanThreads, "block layout");
            uint64_t wl[kItems], wp[kItems], s = 0, tot;
#pragma unroll
            for (int j = 0; j < kItems; ++j) {
                const int i = tid * kItems + j;
                wl[j] = i < cnt ? scar[i] : 0u;
                s += wl[j];
            }
            uint64_t pre = block_exclusive_scan64(s, lds64, &tot);
#pragma unroll
            for (int j = 0; j < kItems; ++j) {
                const int i = tid * kItems + j;
                wp[j] = pre;
                pre += wl[j];
                if (i < cnt) {
                    const uint32_t d = (skey[i] >> shift) & (kBins - 1);
                    if (uint32_t(i) == lstart[d]) wstart[d] = wp[j];
                }
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kItems; ++j) {
                const int i = tid * kItems + j;
                if (i < cnt) {
                    const uint32_t k2 = skey[i];
                    const uint32_t d = (k2 >> shift) & (kBins - 1);
                    const uint32_t p = gbase[d] + (uint32_t(i) - lstart[d]);
                    kout[p] = k2;
                    vout[p] = sval[i];
                    const uint64_t o = wgbase[d] + (wp[j] - wstart[d]);
                    cout[p] = sat32(o);
                    // this record holds the first slot of every chunk starting in [o, o + count)
                    const uint64_t end = o + wl[j];
                    for (uint64_t q = (o + 255) / 256; q * 256 < end && int64_t(q) < po.n_chunks; ++q)
                        po.chunk_first[q] = p;
                }
            }
        } else {
            for (int i = tid; i < cnt; i += kScanThreads) {
                const uint32_t k2 = skey[i];
                const uint32_t d = (k2 >> shift) & (kBins - 1);
                const uint32_t p = gbase[d] + (uint32_t(i) - lstart[d]);
                kout[p] = k2;
                vout[p] = sval[i];
                if (kCarry) cout[p] = scar[i];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Tile counting sort: one stable pass over the emitted pairs whose digit is
// the whole tile index (up to kTileCountMax tiles).  Blocks of kTileSortN
// consecutive pairs; hist[b * stride + t] counts the pairs of tile t in block
// b.  Rows are contiguous, so a block writes its counts in one coalesced
// sweep; tile_colscan_kernel turns every column into the exclusive count over
// the blocks before b and leaves the tile totals in digit[].  The scatter
// ranks each block's pairs per tile (per wave, in order) and writes the values
// straight to their final slots; its workgroup 0 also writes every tile's
// range.  Keys >= total_tiles (never emitted) are dropped by both sides, and
// total_tiles <= 2^bits, so `bits` ballots tell every two tiles apart.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) tile_hist_kernel(const uint32_t *__restrict__ n_ptr,
                                                        const uint32_t *__restrict__ keys, int32_t total_tiles,
                                                        int64_t stride, uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[kTileCountMax];
    const uint32_t n = *n_ptr;
    const int64_t nb = (int64_t(n) + kTileSortN - 1) / kTileSortN;
    const int tid = threadIdx.x;
    for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        __syncthreads();
        for (int i = tid; i < stride; i += kScanThreads) h[i] = 0u;
        __syncthreads();
        const int64_t base = b * kTileSortN;
        uint32_t kk[kTileSortItems];   // every key load in flight before the first LDS atomic
#pragma unroll
        for (int k = 0; k < kTileSortItems; ++k) {
            const int64_t e = base + k * kScanThreads + tid;
            kk[k] = e < n ? keys[e] : 0xffffffffu;
        }
#pragma unroll
        for (int k = 0; k < kTileSortItems; ++k)
            if (kk[k] < uint32_t(total_tiles)) atomicAdd(&h[kk[k]], 1u);
        __syncthreads();
        uint32_t *row = hist + b * stride;
        for (int i = tid; i < stride; i += kScanThreads) row[i] = h[i];
    }
}

// Exclusive scan of every column of hist over the active blocks, in place;
// column totals to digit[t].  A workgroup takes 64 tiles, one per lane, so
// each load is a contiguous 256-byte piece of a row, and its kColWaves waves
// take consecutive runs of blocks.  Each wave sums its run, the run sums are
// scanned across the waves in LDS, and the wave writes the prefixes.  Runs of
// up to kColHold blocks stay in registers between the two steps (one batch of
// loads); longer runs are read twice, kColBatch loads at a time.
// Grid: stride / 64 workgroups.
constexpr int kColWaves = 16, kColHold = 32, kColBatch = 16;
__global__ void __launch_bounds__(kColWaves * kWave) tile_colscan_kernel(const uint32_t *__restrict__ n_ptr,
                                                                         uint32_t *__restrict__ hist,
                                                                         int64_t stride,
                                                                         uint32_t *__restrict__ digit) {
    __shared__ uint32_t wsum[kColWaves][kWave];
    const uint32_t n = *n_ptr;
    const int64_t nb = (int64_t(n) + kTileSortN - 1) / kTileSortN;
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    uint32_t *col = hist + int64_t(blockIdx.x) * kWave + lane;
    const int64_t per = (nb + kColWaves - 1) / kColWaves;
    const int64_t b0 = wave * per, b1 = b0 + per < nb ? b0 + per : nb;
    auto cross_waves = [&](uint32_t s, uint32_t &run, uint32_t &all) {
        wsum[wave][lane] = s;
        __syncthreads();
        run = 0u;
        all = 0u;
#pragma unroll
        for (int w = 0; w < kColWaves; ++w) {
            const uint32_t x = wsum[w][lane];
            run += w < wave ? x : 0u;
            all += x;
        }
    };
    uint32_t run, all;
    if (per <= kColHold) {   // uniform over the workgroup
        // 32-bit element offsets from the run's first entry (a run spans at
        // most kColHold rows of at most kTileCountMax entries)
        uint32_t *c0 = col + b0 * stride;
        const uint32_t st = uint32_t(stride), cnt = uint32_t(b1 > b0 ? b1 - b0 : 0);
        uint32_t v[kColHold], s = 0u;
#pragma unroll
        for (int j = 0; j < kColHold; ++j) {
            v[j] = uint32_t(j) < cnt ? c0[uint32_t(j) * st] : 0u;
            s += v[j];
        }
        cross_waves(s, run, all);
#pragma unroll
        for (int j = 0; j < kColHold; ++j) {
            if (uint32_t(j) < cnt) c0[uint32_t(j) * st] = run;
            run += v[j];
        }
    } else {
        uint32_t s = 0u;
        for (int64_t b = b0; b < b1; b += kColBatch) {
            uint32_t v[kColBatch];
#pragma unroll
            for (int j = 0; j < kColBatch; ++j) v[j] = b + j < b1 ? col[(b + j) * stride] : 0u;
#pragma unroll
            for (int j = 0; j < kColBatch; ++j) s += v[j];
        }
        cross_waves(s, run, all);
        for (int64_t b = b0; b < b1; b += kColBatch) {
            uint32_t v[kColBatch];
#pragma unroll
            for (int j = 0; j < kColBatch; ++j) v[j] = b + j < b1 ? col[(b + j) * stride] : 0u;
#pragma unroll
            for (int j = 0; j < kColBatch; ++j) {
                if (b + j < b1) col[(b + j) * stride] = run;
                run += v[j];
            }
        }
    }
    if (wave == 0) digit[int64_t(blockIdx.x) * kWave + lane] = all;
}

// Scatter of the counting sort.  Wave w of a block owns the contiguous
// quarter [w * kTileSortItems * 64, (w + 1) * kTileSortItems * 64) and ranks
// its pairs row by row (64 consecutive pairs per row), in element order, with
// one LDS atomic per tile: the per-wave counts are 16-bit fields, two tiles to
// a word (a wave holds 2048 pairs, a block 8192, so no field carries into its
// neighbour).  Most rows hold each tile at most once (a row spans a few
// records, whose tile rectangles seldom meet): every lane writes its lane
// number into a per-wave tag byte of its tile and reads it back, and when no
// lane finds another's number each lane adds 1 to its own tile's field.
// Otherwise the row falls back to grouping equal tiles with `bits` ballots,
// the lowest lane of a group adding the group's size (the radix scatter's
// scheme).  A pair's slot = start of its tile + count of its tile in earlier
// blocks (hist after the column scan) + in earlier waves of its block + its
// rank in its wave.  The values are then laid out in LDS in slot order with
// their slots, and written by consecutive threads: each tile's run of the
// block goes out as consecutive addresses.  All loads of a block are issued
// before the first wait.  LDS: one 64 KB pool holding the tile starts, the
// per-wave counts and the tags while ranking, then the block-local tile
// starts, then the staged values and slots.
__global__ void __launch_bounds__(256) tile_scatter_kernel(
    const uint32_t *__restrict__ n_ptr, const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint32_t *__restrict__ vout, int32_t total_tiles, int64_t stride, int bits,
    const uint32_t *__restrict__ hist, const uint32_t *__restrict__ digit, uint2 *__restrict__ ranges) {
    constexpr int kWaves = kScanThreads / kWave, kPer = kTileCountMax / kScanThreads;
    constexpr int kWaveN = kTileSortItems * kWave;
    static_assert(kTileSortN < (1 << 16), "a block's counts fit 16 bits");
    __shared__ uint32_t pool[2 * kTileSortN];
    static_assert(kTileCountMax + kWaves * kTileCountMax / 2 + kWaves * kTileCountMax / 4 == 2 * kTileSortN,
                  "pool layout");
    uint32_t *bstart = pool;                              // first slot of each tile's run of this block
    uint32_t (*wc)[kTileCountMax / 2] =                   // per-wave counts, then offsets (16-bit fields)
        reinterpret_cast<uint32_t (*)[kTileCountMax / 2]>(pool + kTileCountMax);
    uint32_t *tag_words = pool + kTileCountMax + kWaves * kTileCountMax / 2;
    uint8_t (*tags)[kTileCountMax] =                      // per-wave tile tags (lane numbers) ...
        reinterpret_cast<uint8_t (*)[kTileCountMax]>(tag_words);
    uint32_t *lstart = tag_words;                         // ... then block-local tile starts
    uint32_t *sval = pool, *sdst = pool + kTileSortN;     // finally the values in slot order
    __shared__ uint32_t lds[8];
    const uint32_t n = *n_ptr;
    const int tid = threadIdx.x, wave = tid / kWave, lane = lane_id();
    const uint32_t nt = uint32_t(total_tiles);
    const int64_t nb = (int64_t(n) + kTileSortN - 1) / kTileSortN;
    // consecutive blocks to one XCD, whose runs of a tile meet in the same
    // cache lines (as in the radix scatter).  The grid is sized for the pair
    // capacity: workgroups without a block leave at once, except workgroup 0,
    // which writes the ranges.
    const int64_t nb8 = (nb + kXcds - 1) / kXcds * kXcds;
    const int64_t T = nb8 < int64_t(gridDim.x) ? nb8 : int64_t(gridDim.x);
    const int64_t w0 = int64_t(blockIdx.x) < T ? xcd_tile(blockIdx.x, T) : nb;
    if (w0 >= nb && blockIdx.x != 0) return;   // uniform over the workgroup
    const int half = int((stride + 1) / 2);
    bool first = true;
    for (int64_t b = w0; first || b < nb; b += T) {
        const bool has = b < nb;   // false only for workgroup 0 with no block
        // tile totals and this block's counts of tile t = tid * kPer + j, and
        // the block's keys and values
        // (16-byte loads: stride is a multiple of 64 and both arrays are
        // 256-byte aligned).  Out-of-range lanes load entry 0 and discard it,
        // so that every load is unconditional.
        uint32_t dv[kPer], hv[kPer];
        const uint32_t *hrow = hist + (has ? b : 0) * stride;
#pragma unroll
        for (int j = 0; j < kPer; j += 4) {
            const int t = tid * kPer + j;
            const bool tin = t < stride;
            const uint4 d4 = *reinterpret_cast<const uint4 *>(digit + (tin ? t : 0));
            const uint4 h4 = *reinterpret_cast<const uint4 *>(hrow + (tin ? t : 0));
            const bool hin = has && tin;
            dv[j] = tin ? d4.x : 0u; dv[j + 1] = tin ? d4.y : 0u;
            dv[j + 2] = tin ? d4.z : 0u; dv[j + 3] = tin ? d4.w : 0u;
            hv[j] = hin ? h4.x : 0u; hv[j + 1] = hin ? h4.y : 0u;
            hv[j + 2] = hin ? h4.z : 0u; hv[j + 3] = hin ? h4.w : 0u;
        }
        const int64_t wbase = b * kTileSortN + int64_t(wave) * kWaveN;
        uint32_t key[kTileSortItems], val[kTileSortItems], pos[kTileSortItems];
#pragma unroll
        for (int k = 0; k < kTileSortItems; ++k) {
            const int64_t e = wbase + k * kWave + lane;
            const bool in = has && e < n;
            const int64_t ec = in ? e : 0;
            const uint32_t kv = kin[ec], vv = vin[ec];
            key[k] = in ? kv : 0xffffffffu;
            val[k] = in ? vv : 0u;
        }
#pragma unroll
        for (int w = 0; w < kWaves; ++w)
            for (int i = tid; i < half; i += kScanThreads) wc[w][i] = 0u;
        {
            uint32_t sum = 0, total;
#pragma unroll
            for (int j = 0; j < kPer; ++j) sum += dv[j];
            uint32_t pre = block_exclusive_scan(sum, lds, &total);   // (barriers inside)
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                const int t = tid * kPer + j;
                if (first && blockIdx.x == 0 && t < total_tiles) ranges[t] = make_uint2(pre, pre + dv[j]);
                bstart[t] = pre + hv[j];
                pre += dv[j];
            }
        }
        first = false;
        if (!has) return;
        __syncthreads();
        constexpr int kRankGroup = 4;
        static_assert(kTileSortItems % kRankGroup == 0, "items in whole groups");
#pragma unroll
        for (int k0 = 0; k0 < kTileSortItems; k0 += kRankGroup) {
            // Each row writes its tags and reads them back before the next row
            // writes (a wave's LDS operations execute in order; relaxed atomics
            // keep the compiler from reusing the written value).  A tile held
            // by several lanes of the row keeps one lane's number, so at least
            // one of them reads another's: no clash is missed.
            uint64_t clash[kRankGroup];
#pragma unroll
            for (int j = 0; j < kRankGroup; ++j) {
                const uint32_t d = key[k0 + j];
                if (d < nt)
                    __hip_atomic_store(&tags[wave][d], uint8_t(lane), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                const uint8_t got = d < nt ? __hip_atomic_load(&tags[wave][d], __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_WORKGROUP)
                                           : uint8_t(lane);
                clash[j] = __ballot(got != uint8_t(lane));
            }
#pragma unroll
            for (int j = 0; j < kRankGroup; ++j) {
                const int k = k0 + j;
                const uint32_t d = key[k];
                const bool valid = d < nt;
                const uint32_t sh = (d & 1u) * 16u;
                if (clash[j] == 0) {
                    pos[k] = valid ? (atomicAdd(&wc[wave][d >> 1], 1u << sh) >> sh) & 0xffffu : 0u;
                } else {
                    uint64_t peers = __ballot(valid);
                    for (int bit = 0; bit < bits; ++bit) {
                        const bool set = (d >> bit) & 1u;
                        const uint64_t m = __ballot(set);
                        peers &= set ? m : ~m;
                    }
                    const uint32_t rank = uint32_t(mask_rank(peers));
                    const uint32_t leader = peers ? uint32_t(__builtin_ctzll(peers)) : uint32_t(lane);
                    uint32_t c = 0u;
                    if (valid && rank == 0)
                        c = (atomicAdd(&wc[wave][d >> 1], uint32_t(__popcll(peers)) << sh) >> sh) & 0xffffu;
                    pos[k] = (uint32_t(__shfl(int(c), int(leader), kWave)) & 0xffffu) + rank;
                }
            }
        }
        __syncthreads();
        // per-wave counts -> counts of the earlier waves (both fields at once:
        // a field's sum stays below 2^16), and the block-local start of every
        // tile (thread tid takes words [8 tid, 8 tid + 8): tiles 16 tid ...)
        constexpr int kWords = kTileCountMax / 2 / kScanThreads;
        uint32_t placed;   // the block's pairs with a valid tile
        {
            uint32_t tot[kWords], sum = 0u;
#pragma unroll
            for (int j = 0; j < kWords; ++j) {
                const int i = tid * kWords + j;
                uint32_t r = 0u;
                if (i < half) {
#pragma unroll
                    for (int w = 0; w < kWaves; ++w) {
                        const uint32_t c = wc[w][i];
                        wc[w][i] = r;
                        r += c;
                    }
                }
                tot[j] = r;
                sum += (r & 0xffffu) + (r >> 16);
            }
            uint32_t pre = block_exclusive_scan(sum, lds, &placed);   // (barriers inside)
#pragma unroll
            for (int j = 0; j < kWords; ++j) {
                const int i = tid * kWords + j;
                lstart[2 * i] = pre;
                pre += tot[j] & 0xffffu;
                lstart[2 * i + 1] = pre;
                pre += tot[j] >> 16;
            }
        }
        __syncthreads();
        uint32_t li[kTileSortItems];   // slot inside the block's staging
#pragma unroll
        for (int k = 0; k < kTileSortItems; ++k) {
            const uint32_t d = key[k];
            if (d < nt) {
                const uint32_t before = (wc[wave][d >> 1] >> ((d & 1u) * 16u)) & 0xffffu;
                li[k] = lstart[d] + before + pos[k];
                pos[k] = bstart[d] + before + pos[k];   // the global slot
            }
        }
        __syncthreads();   // the pool is free: stage the values in slot order
#pragma unroll
        for (int k = 0; k < kTileSortItems; ++k) {
            if (key[k] < nt) {
                sval[li[k]] = val[k];
                sdst[li[k]] = pos[k];
            }
        }
        __syncthreads();
        for (uint32_t i = tid; i < placed; i += kScanThreads) vout[sdst[i]] = sval[i];
        __syncthreads();   // LDS reads done before the next block's writes
    }
}

// Work queue of the persistent raster launches: tiles in order of decreasing
// list length, by length class floor(log2(length)) + 1 (0 for an empty tile),
// larger classes first; the order inside a class is arbitrary (any order
// gives the same images: tiles are independent).
__device__ __forceinline__ int length_class(uint2 r) {
    const uint32_t len = r.y - r.x;
    return len ? 32 - __clz(len) : 0;
}

__global__ void __launch_bounds__(256) tile_class_count_kernel(const uint2 *__restrict__ ranges, int64_t T,
                                                               uint32_t *__restrict__ queue) {
    __shared__ uint32_t h[kQueueClasses];
    if (threadIdx.x < kQueueClasses) h[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < T) atomicAdd(&h[length_class(ranges[i])], 1u);
    __syncthreads();
    if (threadIdx.x < kQueueClasses && h[threadIdx.x]) atomicAdd(&queue[kQueueCount + threadIdx.x], h[threadIdx.x]);
}

__global__ void __launch_bounds__(256) tile_order_kernel(const uint2 *__restrict__ ranges, int64_t T,
                                                         uint32_t *__restrict__ queue, uint32_t *__restrict__ order) {
    __shared__ uint32_t h[kQueueClasses], start[kQueueClasses];
    if (threadIdx.x < kQueueClasses) {
        h[threadIdx.x] = 0u;
        uint32_t before = 0;   // tiles of the larger classes
        for (int c = kQueueClasses - 1; c > int(threadIdx.x); --c) before += queue[kQueueCount + c];
        start[threadIdx.x] = before;
    }
    __syncthreads();
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int c = 0;
    uint32_t rank = 0;
    if (i < T) {
        c = length_class(ranges[i]);
        rank = atomicAdd(&h[c], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kQueueClasses && h[threadIdx.x])
        start[threadIdx.x] += atomicAdd(&queue[kQueueCursor + threadIdx.x], h[threadIdx.x]);
    __syncthreads();
    if (i < T) order[start[c] + rank] = uint32_t(i);
}

struct SortBufs {
    uint32_t *counters, *counts, *vk[2], *vv[2], *voff, *pk[2], *pv[2], *bsum, *hist, *digit, *chunk_first,
        *view_off, *view_list;
    uint2 *ranges, *rects;
    uint32_t *order, *queue, *thist, *whist, *wdigit;
    int64_t max_blocks, tile_blocks, tile_stride, wstride;
};

static SortBufs sort_bufs(void *ws, int32_t n_views, int32_t n_targets, int64_t n_cap, int64_t pair_cap,
                          int32_t total_tiles) {
    SortLayout L = SortLayout::make(n_views, n_targets, n_cap, pair_cap, total_tiles);
    char *b = static_cast<char *>(ws);
    auto u = [&](size_t o) { return reinterpret_cast<uint32_t *>(b + o); };
    SortBufs B;
    B.counters = u(L.counters);
    B.counts = u(L.counts);
    B.vk[0] = u(L.vis_key0); B.vk[1] = u(L.vis_key1);
    B.vv[0] = u(L.vis_val0); B.vv[1] = u(L.vis_val1);
    B.voff = u(L.vis_off);
    B.pk[0] = u(L.pair_key0); B.pk[1] = u(L.pair_key1);
    B.pv[0] = u(L.pair_val0); B.pv[1] = u(L.pair_val1);
    B.bsum = u(L.bsum);
    B.hist = u(L.hist);
    B.digit = u(L.digit);
    B.chunk_first = u(L.chunk_first);
    B.view_off = u(L.view_off);
    B.view_list = u(L.view_list);
    B.ranges = reinterpret_cast<uint2 *>(b + L.ranges);
    B.rects = reinterpret_cast<uint2 *>(b + L.rects);
    B.max_blocks = L.max_blocks;
    B.thist = u(L.thist);
    B.whist = u(L.whist);
    B.wdigit = u(L.wdigit);
    B.wstride = L.wstride;
    B.tile_blocks = L.tile_blocks;
    B.tile_stride = L.tile_stride;
    B.order = u(L.order);
    B.queue = u(L.queue);
    return B;
}

// Sorts (kbuf[cur], vbuf[cur]) through the two buffers over `passes` kBits
// digits starting at bit first_bit; returns the buffer index holding the result.
// With kCarry, cbuf[cur] moves along as a second value array.
template <int kItems, int kBits, bool kCarry = false>
static int radix_sort(const uint32_t *n_ptr, uint32_t *kbuf[2], uint32_t *vbuf[2], int cur,
                      int first_bit, int passes, int64_t capacity, const SortBufs &B,
                      hipStream_t st, uint32_t *const *cbuf = nullptr) {
    const int64_t blocks = (capacity + kItems * kScanThreads - 1) / (kItems * kScanThreads);
    const int64_t grid = blocks < kRadixPersist ? blocks : kRadixPersist;
    for (int p = 0; p < passes; ++p) {
        const int shift = first_bit + p * kBits;
        hipLaunchKernelGGL((radix_hist_kernel<kItems, kBits>), dim3(grid), dim3(256), 0, st, n_ptr,
                           kbuf[cur], shift, B.hist, B.max_blocks, nullptr, nullptr, int64_t(0));
        hipLaunchKernelGGL((radix_rowscan_kernel<kItems>), dim3(1 << kBits), dim3(256), 0, st, n_ptr, B.hist,
                           B.max_blocks, B.digit, nullptr, int64_t(0), nullptr);
        hipLaunchKernelGGL((radix_scatter_kernel<kItems, kBits, kCarry>), dim3(xcd_grid(grid)), dim3(256), 0, st,
                           n_ptr, kbuf[cur], vbuf[cur], kbuf[cur ^ 1], vbuf[cur ^ 1],
                           kCarry ? cbuf[cur] : nullptr, kCarry ? cbuf[cur ^ 1] : nullptr, shift, B.hist,
                           B.max_blocks, B.digit, PairOffsets{});
        cur ^= 1;
    }
    return cur;
}

__global__ void __launch_bounds__(256) ranges_kernel(const uint32_t *__restrict__ counters,
                                                     const uint32_t *__restrict__ keys,
                                                     uint2 *__restrict__ ranges) {
    // four consecutive keys per thread (one 16-byte load) and the keys on
    // either side; 0xffffffff (never a tile index) stands beyond both ends
    constexpr uint32_t kNone = 0xffffffffu;
    const int64_t P = counters[kPairsClamped];
    const int64_t groups = (P + 3) / 4;
    for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < groups;
         q += int64_t(gridDim.x) * blockDim.x) {
        const int64_t e0 = 4 * q;
        uint32_t k[6];
        k[0] = e0 > 0 ? keys[e0 - 1] : kNone;
        if (e0 + 4 <= P) {
            const uint4 v = *reinterpret_cast<const uint4 *>(keys + e0);
            k[1] = v.x; k[2] = v.y; k[3] = v.z; k[4] = v.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) k[1 + j] = e0 + j < P ? keys[e0 + j] : kNone;
        }
        k[5] = e0 + 4 < P ? keys[e0 + 4] : kNone;
#pragma unroll
        for (int j = 1; j <= 4; ++j) {
            const int64_t e = e0 + j - 1;
            if (e >= P) break;
            if (k[j - 1] != k[j]) ranges[k[j]].x = uint32_t(e);
            if (k[j + 1] != k[j]) ranges[k[j]].y = uint32_t(e + 1);
        }
    }
}

}  // namespace gs

extern "C" gs_status gs_bin_sort(const gs_settings *s, const void *proj_ws, int64_t n,
                                 int64_t n_cap, int32_t n_views, const gs_target *targets,
                                 int32_t n_targets, int32_t total_tiles, void *sort_ws,
                                 int64_t pair_cap, uint32_t *d_status, void *stream) {
    using namespace gs;
    if (!valid_settings(s) || !proj_ws || !targets || !sort_ws || n < 0 || n_cap <= 0 || n > n_cap ||
        n_cap % 64 || n_views <= 0 || n_targets <= 0 || total_tiles <= 0 || pair_cap <= 0 ||
        pair_cap > kMaxPairs || int64_t(n_views) * n_cap > kMaxRecords)
        return GS_ERR_INVALID_ARGUMENT;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t S = int64_t(n_views) * n_cap;   // (view, Gaussian) records
    SortBufs B = sort_bufs(sort_ws, n_views, n_targets, n_cap, pair_cap, total_tiles);
    Proj proj = proj_at(const_cast<void *>(proj_ws), S);

    const int64_t cgx = (n_cap + 255) / 256;   // count / compaction grid: (cgx, n_views)
    if (n_targets == 1) {   // the set-up folded into the count kernel
        hipLaunchKernelGGL(count_kernel<true>, dim3(cgx, n_views), dim3(256), 0, st, *s, proj, n, n_cap, targets,
                           B.view_off, B.view_list, B.counts, B.rects, B.bsum, B.counters, B.queue, B.ranges,
                           int64_t(total_tiles));
    } else {
        hipLaunchKernelGGL(sort_setup_kernel, dim3((int64_t(total_tiles) + 255) / 256), dim3(256), 0, st, targets,
                           n_targets, n_views, B.counters, B.view_off, B.view_list, B.ranges, int64_t(total_tiles),
                           B.queue);
        hipLaunchKernelGGL(count_kernel<false>, dim3(cgx, n_views), dim3(256), 0, st, *s, proj, n, n_cap, targets,
                           B.view_off, B.view_list, B.counts, B.rects, B.bsum, B.counters, B.queue, B.ranges,
                           int64_t(0));
    }
    // compact visible records: the count kernel left each workgroup's number
    // of visible records in bsum, which place the workgroups (summed by the
    // compaction itself up to kFoldGroups workgroups, else scanned first)
    // the visible records' pair counts move with them through compaction and
    // the depth sort, in two S-sized buffers that are free meanwhile: vis_off
    // (written by no other step) and counts (read only by the compaction)
    uint32_t *cnt_buf[2] = {B.voff, B.counts};
    const int64_t groups = cgx * n_views;
    if (groups <= kFoldGroups) {
        hipLaunchKernelGGL(compact_scatter_kernel<true>, dim3(cgx, n_views), dim3(256), 0, st, B.counts, n_cap, proj,
                           s->znear, B.bsum, groups, B.vk[0], B.vv[0], cnt_buf[0], B.counters + kVisible);
    } else {
        hipLaunchKernelGGL(scan_bsums_kernel, dim3(1), dim3(1024), 0, st, B.bsum, groups, B.counters + kVisible);
        hipLaunchKernelGGL(compact_scatter_kernel<false>, dim3(cgx, n_views), dim3(256), 0, st, B.counts, n_cap, proj,
                           s->znear, B.bsum, groups, B.vk[0], B.vv[0], cnt_buf[0], B.counters + kVisible);
    }
    // depth order (three 9-bit passes over the 27-bit keys); the last pass
    // also turns the pair counts into pair offsets (in `counts`), writes the
    // emission chunks' first records and the total pair count
    static_assert(kDepthKeyBits == 3 * 9, "depth key width");
    int cur = radix_sort<4, 9, true>(B.counters + kVisible, B.vk, B.vv, 0, 0, 2, S, B, st, cnt_buf);
    const int64_t n_chunks = pair_chunks(pair_cap);
    {
        const int64_t blocks = (S + 1023) / 1024;
        const int64_t grid = blocks < kRadixPersist ? blocks : kRadixPersist;
        const uint32_t *nv = B.counters + kVisible;
        hipLaunchKernelGGL((radix_hist_kernel<4, 9, true>), dim3(grid), dim3(256), 0, st, nv, B.vk[cur], 18, B.hist,
                           B.max_blocks, cnt_buf[cur], B.whist, B.wstride);
        hipLaunchKernelGGL((radix_rowscan_kernel<4, true>), dim3(512), dim3(256), 0, st, nv, B.hist, B.max_blocks,
                           B.digit, B.whist, B.wstride, B.wdigit);
        const PairOffsets po{B.whist, B.wstride, B.wdigit, B.counters + kPairs, B.chunk_first, n_chunks};
        hipLaunchKernelGGL((radix_scatter_kernel<4, 9, true, true>), dim3(xcd_grid(grid)), dim3(256), 0, st, nv,
                           B.vk[cur], B.vv[cur], B.vk[cur ^ 1], B.vv[cur ^ 1], cnt_buf[cur], cnt_buf[cur ^ 1], 18,
                           B.hist, B.max_blocks, B.digit, po);
        cur ^= 1;
    }
    const uint32_t *vis_off = cnt_buf[cur];
    const int64_t persistent = 256 * 16;   // 16 workgroups per CU, grid-stride beyond
    const int64_t emit_chunks = (pair_cap + kEmitChunk - 1) / kEmitChunk;
    const dim3 egrid(emit_chunks < persistent ? emit_chunks : persistent);
    if (n_targets == 1)
        hipLaunchKernelGGL(emit_kernel<true>, egrid, dim3(256), 0, st, n_cap, n_views, targets, B.counters,
                           B.vv[cur], vis_off, B.rects, B.view_off, B.view_list, B.chunk_first, pair_cap, B.pk[0],
                           B.pv[0], d_status);
    else
        hipLaunchKernelGGL(emit_kernel<false>, egrid, dim3(256), 0, st, n_cap, n_views, targets, B.counters,
                           B.vv[cur], vis_off, B.rects, B.view_off, B.view_list, B.chunk_first, pair_cap, B.pk[0],
                           B.pv[0], d_status);
    // tile order
    const TileSortPlan plan = tile_sort_plan(total_tiles);
    if (plan.counting) {   // one pass, pairs pk[0] / pv[0] -> values pv[1] and the ranges
        const int64_t tb = B.tile_blocks < kRadixPersist ? B.tile_blocks : kRadixPersist;
        hipLaunchKernelGGL(tile_hist_kernel, dim3(tb), dim3(256), 0, st, B.counters + kPairsClamped, B.pk[0],
                           total_tiles, B.tile_stride, B.thist);
        hipLaunchKernelGGL(tile_colscan_kernel, dim3(B.tile_stride / kWave), dim3(kColWaves * kWave), 0, st,
                           B.counters + kPairsClamped, B.thist, B.tile_stride, B.digit);
        hipLaunchKernelGGL(tile_scatter_kernel, dim3(xcd_grid(tb)), dim3(256), 0, st, B.counters + kPairsClamped,
                           B.pk[0], B.pv[0], B.pv[1], total_tiles, B.tile_stride, plan.bits, B.thist, B.digit,
                           B.ranges);
    } else {
        // 9-bit digits come with many tiles and pairs: 8192-element sort blocks keep
        // each digit's run per block long enough for full write segments
        const int pc = plan.bits == 9 ? radix_sort<32, 9>(B.counters + kPairsClamped, B.pk, B.pv, 0, 0,
                                                          plan.passes, pair_cap, B, st)
                                      : radix_sort<16, 8>(B.counters + kPairsClamped, B.pk, B.pv, 0, 0,
                                                          plan.passes, pair_cap, B, st);
        hipLaunchKernelGGL(ranges_kernel, dim3(n_chunks < persistent ? n_chunks : persistent), dim3(256), 0, st,
                           B.counters, B.pk[pc], B.ranges);
    }
    if (s->schedule >= 1) {   // the raster work queue
        const int64_t tg = (int64_t(total_tiles) + 255) / 256;
        hipLaunchKernelGGL(tile_class_count_kernel, dim3(tg), dim3(256), 0, st, B.ranges, int64_t(total_tiles),
                           B.queue);
        hipLaunchKernelGGL(tile_order_kernel, dim3(tg), dim3(256), 0, st, B.ranges, int64_t(total_tiles), B.queue,
                           B.order);
    }
    GS_CHECK_LAUNCH();
    return GS_OK;
}
