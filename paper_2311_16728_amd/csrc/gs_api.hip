// Host-side helpers of the C interface: status strings, default settings,
// target layout and workspace sizing.  No device work happens here.
#include "gs_internal.hpp"

extern "C" const char *gs_status_string(gs_status s) {
    switch (s) {
        case GS_OK: return "ok";
        case GS_ERR_INVALID_ARGUMENT: return "invalid argument";
        case GS_ERR_CAPACITY: return "capacity exceeded";
        case GS_ERR_NOT_SUPPORTED: return "not supported";
        case GS_ERR_HIP: return "HIP launch error";
        case GS_ERR_NUMERIC: return "non-finite value";
    }
    return "unknown status";
}

extern "C" void gs_default_settings(gs_settings *s) {
    if (!s) return;
    s->alpha_min = 1.f / 255.f;
    s->alpha_max = 0.99f;
    s->t_min = 1e-4f;
    s->znear = 0.2f;
    s->dilation = 0.3f;
    s->fov_clamp = 1.3f;
    s->sh_degree = 3;
    s->batch = 256;
    s->bwd_waves = 2;
    s->checked = 0;
    s->schedule = 0;
    s->status = nullptr;
}

extern "C" gs_status gs_status_word(uint32_t word) {
    if (word & ~(GS_STATUS_PAIR_OVERFLOW | GS_STATUS_NUMERIC)) return GS_ERR_INVALID_ARGUMENT;
    if (word & GS_STATUS_NUMERIC) return GS_ERR_NUMERIC;
    if (word & GS_STATUS_PAIR_OVERFLOW) return GS_ERR_CAPACITY;
    return GS_OK;
}

extern "C" gs_status gs_targets_layout(const gs_view *views, int32_t n_views, gs_target *targets,
                                       int32_t n_targets, int64_t *total_pixels,
                                       int32_t *total_tiles) {
    if (!views || !targets || n_views <= 0 || n_targets <= 0 || !total_pixels || !total_tiles)
        return GS_ERR_INVALID_ARGUMENT;
    int64_t pix = 0, tiles = 0;
    for (int i = 0; i < n_targets; ++i) {
        gs_target &t = targets[i];
        if (t.view < 0 || t.view >= n_views || t.level < 0 || t.level > 15)
            return GS_ERR_INVALID_ARGUMENT;
        int w = views[t.view].width, h = views[t.view].height;
        if (w <= 0 || h <= 0) return GS_ERR_INVALID_ARGUMENT;
        for (int l = 0; l < t.level; ++l) {
            w = (w + 1) / 2;
            h = (h + 1) / 2;
        }
        if (t.tile_w == 0) t.tile_w = gs::kTile;
        if (t.tile_w != 8 && t.tile_w != 16 && t.tile_w != 32)
            return GS_ERR_INVALID_ARGUMENT;
        const int tw = t.tile_w, th = gs::kTilePix / tw;
        t.width = w;
        t.height = h;
        t.tiles_x = (w + tw - 1) / tw;
        t.tiles_y = (h + th - 1) / th;
        t.tile_offset = int32_t(tiles);
        t.pix_offset = pix;
        tiles += int64_t(t.tiles_x) * t.tiles_y;
        pix += int64_t(w) * h;
        if (tiles > 0x7fffffff) return GS_ERR_CAPACITY;
    }
    *total_pixels = pix;
    *total_tiles = int32_t(tiles);
    return GS_OK;
}

extern "C" gs_status gs_workspace_query(const gs_settings *s, int64_t n_cap, int32_t n_views,
                                        const gs_target *targets, int32_t n_targets,
                                        int64_t pair_cap, gs_sizes *out) {
    if (!gs::valid_settings(s) || !targets || !out || n_cap <= 0 || n_cap % 64 || n_views <= 0 ||
        n_targets <= 0 || pair_cap <= 0 || pair_cap > gs::kMaxPairs ||
        int64_t(n_views) * n_cap > gs::kMaxRecords)
        return GS_ERR_INVALID_ARGUMENT;
    int64_t pix = 0, tiles = 0;
    for (int i = 0; i < n_targets; ++i) {
        pix += int64_t(targets[i].width) * targets[i].height;
        tiles += int64_t(targets[i].tiles_x) * targets[i].tiles_y;
    }
    const int64_t records = int64_t(n_views) * n_cap;
    out->proj_bytes = gs::ProjLayout::make(records).bytes;
    out->sort_bytes = gs::SortLayout::make(n_views, n_targets, n_cap, pair_cap, tiles).bytes;
    out->accum_bytes = gs::accum_bytes(records);
    out->loss_bytes = gs::LossLayout::make(pix, tiles).bytes;
    return GS_OK;
}
