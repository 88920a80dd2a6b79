// Internal definitions shared by the libgs HIP sources (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs.h"

namespace gs {

constexpr int kWave = 64;
constexpr int kRows = GS_NUM_ROWS;
constexpr int kTile = GS_TILE;                   // default tile width
constexpr int kTilePix = GS_TILE_PIXELS;         // 256 pixels per tile, one thread each
static_assert(kTile * kTile == kTilePix, "the default tile is square");

// A target's tile: tile_w x (256 / tile_w) pixels (set by gs_targets_layout).
struct TileShape {
    int w, h, wlog;   // width, height, log2(width)
};
__host__ __device__ __forceinline__ TileShape tile_shape(int tile_w) {
    // widths other than 8, 16, 32 (rejected by gs_targets_layout) read as 16
    const int wlog = tile_w == 8 ? 3 : tile_w == 32 ? 5 : 4;
    return TileShape{1 << wlog, kTilePix >> wlog, wlog};
}
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;   // 4096 elements per block
constexpr int kRadixBitsMax = 9;              // widest radix digit (depth sort, large tile sorts)
constexpr int kRadixBinsMax = 1 << kRadixBitsMax;
constexpr int kRadixPersist = 2048;           // workgroups of the grid-stride radix kernels
// Tile counting sort: one stable pass whose digit is the whole tile index,
// for up to kTileCountMax tiles (one LDS table), over blocks of kTileSortN
// pairs (kTileSortItems per thread).
constexpr int kTileCountMax = 4096;
constexpr int kTileSortItems = 32;
constexpr int kTileSortN = kTileSortItems * kScanThreads;   // 8192 pairs per block

static constexpr size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Size limits of the interface: records are indexed by uint32, pair slots by
// uint32 with the total kept below 2^31 (so a count past it is seen, not wrapped).
constexpr int64_t kMaxRecords = 0xffffffffLL;
constexpr int64_t kMaxPairs = 0x7fffffffLL;

// Host-side validation of the rasteriser settings shared by every entry point.
static inline bool valid_settings(const gs_settings *s) {
    return s && s->sh_degree >= 0 && s->sh_degree <= 3 &&
           (s->batch == 64 || s->batch == 128 || s->batch == 256) &&
           (s->bwd_waves == 1 || s->bwd_waves == 2 || s->bwd_waves == 4) && s->alpha_min > 0.f &&
           s->alpha_max <= 1.f && s->alpha_max >= s->alpha_min && s->t_min > 0.f &&
           s->dilation >= 0.f && s->fov_clamp > 0.f && s->znear > 0.f &&
           (s->checked == 0 || (s->checked == 1 && s->status != nullptr)) &&
           (s->schedule >= 0 && s->schedule <= 2);
}

// ---------------------------------------------------------------------------
// Workspace layouts.  All sub-buffers are 256-byte aligned.
// ---------------------------------------------------------------------------
struct ProjLayout {
    size_t mean, cov_o, rgb_z, bytes;   // double2, float4, float4 per record
    static ProjLayout make(int64_t records) {
        ProjLayout L;
        size_t o = 0;
        L.mean = o;  o = align_up(o + sizeof(double) * 2 * records, 256);
        L.cov_o = o; o = align_up(o + sizeof(float) * 4 * records, 256);
        L.rgb_z = o; o = align_up(o + sizeof(float) * 4 * records, 256);
        L.bytes = o;
        return L;
    }
};

struct Proj {
    double2 *mean;   // level-0 2D mean (pixels), kept in FP64 so that pixel
                     // offsets staged relative to a tile carry ~1e-6 px error
    float4 *cov_o;   // undilated 2D covariance (s00, s01, s11) and opacity
    float4 *rgb_z;   // colour and camera depth (depth <= 0 marks invalid)
};

static inline Proj proj_at(void *ws, int64_t records) {
    ProjLayout L = ProjLayout::make(records);
    char *b = static_cast<char *>(ws);
    return Proj{reinterpret_cast<double2 *>(b + L.mean), reinterpret_cast<float4 *>(b + L.cov_o),
                reinterpret_cast<float4 *>(b + L.rgb_z)};
}

// Work queue of the persistent raster launches (settings.schedule 1 or 2): the
// tiles in order of decreasing list length (order, built by gs_bin_sort) and
// a control block: per length class (floor(log2(length)) + 1, 0 for empty)
// its count and a cursor, then the next-item and finished-workgroup counters
// of the forward and the backward.  The last workgroup of a launch resets its
// two counters, so every launch starts at item 0.
constexpr int kQueueClasses = 34;
enum QueueWord {
    kQueueCount = 0, kQueueCursor = kQueueClasses, kQueueNextFwd = 2 * kQueueClasses, kQueueDoneFwd,
    kQueueNextBwd, kQueueDoneBwd, kQueueWords = 128
};

// Counters at the head of the sort workspace.
enum Counter { kVisible = 0, kPairs = 1, kPairsClamped = 2, kNumCounters = 16 };

// Pair emission works in chunks of 256 consecutive pair slots.
static inline int64_t pair_chunks(int64_t pair_cap) { return (pair_cap + 255) / 256; }

struct SortLayout {
    size_t counters, counts, rects, vis_key0, vis_key1, vis_val0, vis_val1, vis_off, pair_key0,
        pair_key1, pair_val0, pair_val1, ranges, bsum, hist, digit, chunk_first, view_off, view_list,
        order, queue, thist, whist, wdigit, bytes;
    int64_t sources, pair_cap, max_blocks;
    // row stride of the pair-count sums per (digit, block) of the last depth
    // pass (whist), which turn the counts into pair offsets
    int64_t wstride;
    // tile counting sort: blocks of pairs and the row stride of its per-block
    // tile counts (rows of tile_stride >= total_tiles entries; 0 when the
    // tiles are too many for it)
    int64_t tile_blocks, tile_stride;
    // sources: (view, Gaussian) records, n_views * n_cap; rects: one per
    // (target, Gaussian), n_targets * n_cap
    static SortLayout make(int64_t n_views, int64_t n_targets, int64_t n_cap, int64_t pair_cap,
                           int64_t total_tiles) {
        SortLayout L;
        const int64_t sources = n_views * n_cap;
        L.sources = sources;
        L.pair_cap = pair_cap;
        // radix blocks: 1024 keys per block for the record sort, 4096 for pairs
        const int64_t rb = (sources + 1023) / 1024, pb = (pair_cap + kScanTile - 1) / kScanTile;
        L.max_blocks = (rb > pb ? rb : pb) + 1;
        size_t o = 0;
        auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
        L.counters = take(sizeof(uint32_t) * kNumCounters);
        L.counts = take(sizeof(uint32_t) * sources);
        L.rects = take(sizeof(uint32_t) * 2 * n_targets * n_cap);
        L.vis_key0 = take(sizeof(uint32_t) * sources);
        L.vis_key1 = take(sizeof(uint32_t) * sources);
        L.vis_val0 = take(sizeof(uint32_t) * sources);
        L.vis_val1 = take(sizeof(uint32_t) * sources);
        L.vis_off = take(sizeof(uint32_t) * (sources + 1));
        L.pair_key0 = take(sizeof(uint32_t) * pair_cap);
        L.pair_key1 = take(sizeof(uint32_t) * pair_cap);
        L.pair_val0 = take(sizeof(uint32_t) * pair_cap);
        L.pair_val1 = take(sizeof(uint32_t) * pair_cap);
        L.ranges = take(sizeof(uint32_t) * 2 * (total_tiles > 0 ? total_tiles : 1));
        // block sums; also one visible-record count per workgroup of the count
        // grid (padded to whole 16-byte pieces, which the compaction reads)
        const int64_t groups = n_views * ((n_cap + 255) / 256);
        L.bsum = take(sizeof(uint32_t) * ((L.max_blocks > groups ? L.max_blocks : groups) + 4));
        L.hist = take(sizeof(uint32_t) * kRadixBinsMax * L.max_blocks);
        L.digit = take(sizeof(uint32_t) * ((kRadixBinsMax > kTileCountMax ? kRadixBinsMax : kTileCountMax) + 1));
        // first sorted record of every 256-pair emission chunk
        L.chunk_first = take(sizeof(uint32_t) * (pair_chunks(pair_cap) + 1));
        // targets of each view (CSR)
        L.view_off = take(sizeof(uint32_t) * (n_views + 1));
        L.view_list = take(sizeof(uint32_t) * n_targets);
        L.order = take(sizeof(uint32_t) * (total_tiles > 0 ? total_tiles : 1));
        L.queue = take(sizeof(uint32_t) * kQueueWords);
        const bool counting = total_tiles > 0 && total_tiles <= kTileCountMax;
        L.tile_blocks = (pair_cap + kTileSortN - 1) / kTileSortN;
        L.tile_stride = counting ? int64_t(align_up(size_t(total_tiles), 64)) : 0;
        L.thist = take(counting ? sizeof(uint32_t) * L.tile_blocks * L.tile_stride : sizeof(uint32_t));
        L.wstride = rb + 1;
        L.whist = take(sizeof(uint32_t) * kRadixBinsMax * L.wstride);
        L.wdigit = take(sizeof(uint32_t) * (kRadixBinsMax + 1));
        L.bytes = o;
        return L;
    }
};

// How the pairs are put in tile order.  Up to kTileCountMax tiles: one
// counting pass whose digit is the whole tile index (bits = the index width,
// counting = true).  Beyond: stable radix passes over the global tile index,
// 8-bit digits, or 9-bit ones where they save a pass (17 or 18 bits: two
// passes instead of three).
struct TileSortPlan {
    int bits, passes;
    bool counting;
};
static inline TileSortPlan tile_sort_plan(int32_t total_tiles) {
    int bits = 1;
    while ((int64_t(1) << bits) < total_tiles) ++bits;
    if (total_tiles <= kTileCountMax) return TileSortPlan{bits, 1, true};
    const int p8 = (bits + 7) / 8, p9 = (bits + 8) / 9;
    return p9 < p8 ? TileSortPlan{9, p9, false} : TileSortPlan{8, p8, false};
}

// Sorted pair buffers after binning: the tile sort ends in buffer (passes & 1).
struct Sorted {
    const uint32_t *pair_val;   // record index view * n_cap + g, per pair
    const uint2 *ranges;        // [start, end) of each global tile
    const uint32_t *order;      // tiles by decreasing list length (schedule 1)
    uint32_t *queue;            // work-queue control block (schedule 1)
};

static inline Sorted sorted_at(const void *ws, int64_t n_views, int64_t n_targets, int64_t n_cap,
                               int64_t pair_cap, int32_t total_tiles) {
    SortLayout L = SortLayout::make(n_views, n_targets, n_cap, pair_cap, total_tiles);
    const char *b = static_cast<const char *>(ws);
    const int passes = tile_sort_plan(total_tiles).passes;
    size_t val = (passes & 1) ? L.pair_val1 : L.pair_val0;
    return Sorted{reinterpret_cast<const uint32_t *>(b + val), reinterpret_cast<const uint2 *>(b + L.ranges),
                  reinterpret_cast<const uint32_t *>(b + L.order),
                  reinterpret_cast<uint32_t *>(const_cast<char *>(b) + L.queue)};
}

// Per-row learning rates (kernel argument).
struct LrRows {
    float lr[kRows];
};

// Per-(view, Gaussian) accumulators of 2D gradients, [records][9] so that the
// nine atomics of one record share a cache line: d mean x, d mean y (level-0
// pixels), d cov00, d cov01, d cov11 (undilated level-0 covariance,
// symmetric-matrix entries), d opacity, d r, d g, d b.
constexpr int kAccRows = 9;
static inline size_t accum_bytes(int64_t records) {
    return align_up(sizeof(float) * kAccRows * records, 256);
}

// Loss workspace: per-tile partial sums (L1, SSIM) and three SSIM partial maps
// per pixel and channel.
// per-target losses in double (a target has at least one tile)
struct LossLayout {
    size_t partial, maps, tloss, bytes;
    static LossLayout make(int64_t total_pixels, int64_t total_tiles) {
        LossLayout L;
        size_t o = 0;
        const int64_t tiles = total_tiles > 0 ? total_tiles : 1;
        L.partial = o; o = align_up(o + sizeof(float) * 2 * tiles, 256);
        L.maps = o;    o = align_up(o + sizeof(float) * 9 * total_pixels, 256);
        L.tloss = o;   o = align_up(o + sizeof(double) * tiles, 256);
        L.bytes = o;
        return L;
    }
};

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0));
}

// Number of set bits of mask below this lane.
__device__ __forceinline__ int mask_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0));
}

// Checked mode: the lowest lane of the wave on which `bad` holds ORs
// GS_STATUS_NUMERIC into the status word (the guards' only device write).
__device__ __forceinline__ void report_numeric(uint32_t *status, bool bad) {
    const uint64_t b = __ballot(bad);
    if (b != 0 && lane_id() == __builtin_ctzll(b)) atomicOr(status, GS_STATUS_NUMERIC);
}

// Cross-lane move through DPP: lanes whose source is outside their row, or
// whose row kRowMask leaves out, read 0.  Control words: row_shr:n = 0x110 + n
// (within rows of 16 lanes), row_bcast:15 = 0x142 (lane 15 of each row to the
// next row), row_bcast:31 = 0x143 (lane 31 to rows 2 and 3).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), kCtrl, kRowMask, 0xf, false));
}

// Inclusive scan over the wave in six DPP adds (no LDS round trips): prefix
// sums inside each row of 16 lanes by shifts of 1, 2, 4 and 8, then row 0's
// total into row 1 and row 2's into row 3, then the first two rows' total
// into rows 2 and 3.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
    v += dpp_u32<0x111, 0xf>(v);
    v += dpp_u32<0x112, 0xf>(v);
    v += dpp_u32<0x114, 0xf>(v);
    v += dpp_u32<0x118, 0xf>(v);
    v += dpp_u32<0x142, 0xa>(v);
    v += dpp_u32<0x143, 0xc>(v);
    return v;
}

// End of a persistent launch over the work queue: each workgroup counts
// itself out once it has found the queue empty; the last one resets the
// next-item and finished counters for the next launch.
__device__ __forceinline__ void queue_retire(uint32_t *queue, int next, int done) {
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&queue[done], 1u) == gridDim.x - 1) {
            queue[next] = 0u;
            queue[done] = 0u;
        }
    }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Workgroups of a launch are handed to the chip's 8 XCDs in turn, and each
// XCD has its own L2.  A grid of xcd_grid(T) workgroups with tile xcd_tile(b)
// gives every XCD one contiguous eighth of the T tiles, so neighbouring tiles
// that read the same lines (image halos) share an L2.  Workgroups with
// xcd_tile(b) >= T have nothing to do.
constexpr int kXcds = 8;
static inline int64_t xcd_grid(int64_t T) { return kXcds * ((T + kXcds - 1) / kXcds); }
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t T) {
    return (b % kXcds) * ((T + kXcds - 1) / kXcds) + b / kXcds;
}

// Exclusive scan over a 256-thread block; returns the prefix of this thread
// and writes the block total to *total.  lds needs 4 + 1 words.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds,
                                                         uint32_t *total) {
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    uint32_t inc = wave_inclusive_scan(v);
    if (lane == kWave - 1) lds[wave] = inc;
    __syncthreads();
    uint32_t base = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        uint32_t s = lds[w];
        base += (w < wave) ? s : 0u;
        all += s;
    }
    __syncthreads();
    *total = all;
    return base + inc - v;
}

}  // namespace gs

#define GS_CHECK_LAUNCH()                                   \
    do {                                                    \
        if (hipGetLastError() != hipSuccess) return GS_ERR_HIP; \
    } while (0)
