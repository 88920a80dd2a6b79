/*
 * libgs - the photorealistic-mapping hot path of Photo-SLAM (Huang et al.,
 * CVPR 2024, arXiv 2311.16728) for AMD Instinct MI355X (gfx950).
 *
 * The mapper optimises a map of 3D Gaussian primitives (position, rotation,
 * scale, density and spherical-harmonic colour; Section 3.1) by rendering
 * keyframes with a tile-based rasteriser (Section 3.3, Eq. 3), scoring them
 * with the photometric loss of Eq. 4 against a Gaussian pyramid of the
 * keyframe image (Section 3.4, Eq. 5), back-propagating, and taking a
 * fixed-learning-rate gradient step (Section 4.1).  Each call below is one
 * step of that loop; all of them run on the GPU.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Device pointers are marked (device); host pointers (host).  Every device
 *   buffer is owned by the caller; the library never allocates or frees
 *   device memory and keeps no state between calls (one exception:
 *   gs_densify_noalloc keeps its workspace in a fixed device array).
 * - `stream` is a hipStream_t passed as void*.  Calls only enqueue work on it
 *   (stream-ordered, asynchronous) and never synchronise, so a sequence of
 *   calls can be captured into a HIP graph.  NULL means the default stream.
 * - Parameter store `params`: float32 [59][n_cap] (structure of arrays, row r
 *   of Gaussian g at params[r * n_cap + g]).  Rows 0-2 mean (world, metres),
 *   3-5 log-scale, 6-9 rotation quaternion (w, x, y, z; need not be
 *   normalised), 10 opacity logit, 11 + 3k + ch SH coefficient k (0..15) of
 *   colour channel ch (R, G, B).  Columns n..n_cap-1 are ignored.
 *   n_cap must be a positive multiple of 64 and n <= n_cap.
 * - Cameras: pinhole, world-to-camera rotation R (row-major) and translation
 *   t, +z forward, +y down; pixel (i, j) has its centre at (i, j).
 * - Images: planar float32 [3][H][W] per target, packed back to back at
 *   3 * pix_offset floats; per-pixel planes [H][W] at pix_offset.
 * - Errors: every call validates its arguments on the host and returns a
 *   non-zero gs_status without enqueuing anything when they are invalid.
 *   Launch failures return GS_ERR_HIP.  Conditions only the device can see
 *   (tile-pair buffer overflow; non-finite values in checked mode) are OR-ed
 *   into a device status word (uint32) that the caller reads after the stream
 *   has synchronised and maps to a status with gs_status_word.  No C++
 *   exception crosses this interface.
 * - Sizes: n_views * n_cap (projection records) is at most 2^32 - 1 and
 *   pair_cap at most 2^31 - 1.
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GS_OK = 0,
    GS_ERR_INVALID_ARGUMENT = 1,
    GS_ERR_CAPACITY = 2,      /* a buffer is too small for the request */
    GS_ERR_NOT_SUPPORTED = 3,
    GS_ERR_HIP = 4,
    GS_ERR_NUMERIC = 5        /* a non-finite value was met (checked mode) */
} gs_status;

/* Bits of a device status word.  GS_STATUS_PAIR_OVERFLOW: gs_bin_sort found
 * more tile pairs than pair_cap.  GS_STATUS_NUMERIC: a checked-mode call
 * (settings.checked = 1) met a NaN or infinity. */
#define GS_STATUS_PAIR_OVERFLOW 1u
#define GS_STATUS_NUMERIC 2u

#define GS_NUM_ROWS 59
#define GS_TILE 16            /* default tile width (square 16 x 16 tiles) */
#define GS_TILE_PIXELS 256    /* pixels per tile, whatever its shape */

/* Rasteriser settings.  Defaults (gs_default_settings): alpha_min 1/255,
 * alpha_max 0.99, t_min 1e-4, znear 0.2, dilation 0.3 px^2, fov_clamp 1.3,
 * sh_degree 3, batch 256, bwd_waves 2, checked 0, schedule 0.  A pixel composites a Gaussian iff its opacity
 * there, o * exp(power), reaches alpha_min; the contribution uses
 * min(alpha_max, .); compositing stops before the Gaussian that would take
 * the transmittance below t_min (Eq. 3).
 *
 * Checked mode (checked = 1, status a device uint32 word, required): the
 * guards below OR GS_STATUS_NUMERIC into *status; every kernel still runs to
 * its end.  gs_preprocess checks the 59 parameters of every column < n and
 * the record it computes; a column with a non-finite value gets the record
 * of a culled Gaussian (opacity 0), so nothing downstream composites it.
 * gs_project_bwd checks every gradient it adds; gs_project_bwd_adam checks
 * every gradient and updated parameter, and writes the next records (when
 * asked) through the guarded projection.  With checked = 0 no guard runs and
 * status is ignored. */
typedef struct {
    float alpha_min, alpha_max, t_min, znear, dilation, fov_clamp;
    int32_t sh_degree;   /* 0..3 */
    int32_t batch;       /* forward: Gaussians staged per LDS round: 64, 128 or 256 */
    int32_t bwd_waves;   /* backward: waves per tile, 1, 2 or 4 (4, 2 or 1 pixels per lane) */
    int32_t checked;     /* 0 or 1: NaN / infinity guards */
    int32_t schedule;    /* raster launch: 0 one workgroup per tile; 1 persistent workgroups
                            taking tiles from a queue in order of decreasing list length
                            in the forward and the backward; 2 the queue in the backward
                            only.  The queue is built by gs_bin_sort called with schedule
                            1 or 2, which gs_render_fwd / gs_raster_bwd then need */
    uint32_t *status;    /* (device) status word of the guards; NULL when checked = 0 */
} gs_settings;

/* A keyframe pose with its level-0 intrinsics and image size. */
typedef struct {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int32_t width, height;
} gs_view;

/* A render target: one pyramid level of one view.  Level l renders at
 * ceil(size / 2^l) with intrinsics divided by 2^l (Eq. 5).  Its image is cut
 * into tiles of tile_w x (256 / tile_w) pixels (tile_w 8, 16 or 32; 0
 * means 16).  tile_offset and pix_offset are filled by gs_targets_layout. */
typedef struct {
    int32_t view;        /* index into the view array */
    int32_t level;       /* pyramid level, 0 = full resolution */
    int32_t width, height;
    int32_t tiles_x, tiles_y;
    int32_t tile_offset; /* first global tile index of this target */
    int32_t tile_w;      /* tile width in pixels (set by the caller; 0 -> 16) */
    int64_t pix_offset;  /* first pixel of this target in packed images */
    float bg[3];         /* background colour */
    float weight;        /* weight of this target's loss in the total */
} gs_target;

/* Workspace sizes in bytes (from gs_workspace_query). */
typedef struct {
    size_t proj_bytes;   /* per-(view, Gaussian) projection records */
    size_t sort_bytes;   /* binning + radix sort + tile ranges */
    size_t accum_bytes;  /* per-(view, Gaussian) 2D gradient accumulators */
    size_t loss_bytes;   /* loss partial sums and SSIM maps */
} gs_sizes;

/* Human-readable name of a status code (static string). */
const char *gs_status_string(gs_status s);

/* (host) The status a device status word stands for, once the caller has read
 * it back: GS_ERR_NUMERIC when GS_STATUS_NUMERIC is set, else
 * GS_ERR_CAPACITY when GS_STATUS_PAIR_OVERFLOW is set, else GS_OK (unknown
 * bits: GS_ERR_INVALID_ARGUMENT). */
gs_status gs_status_word(uint32_t word);

/* Fills *s with the defaults listed above. */
void gs_default_settings(gs_settings *s);

/* (host) Completes targets[0..n_targets): derives width/height from the
 * view's size and the level, the tile grid for the target's tile_w (0 becomes
 * 16; other values than 8, 16, 32 are rejected), tile_offset and
 * pix_offset (targets packed in order).  Writes the totals.  views is host
 * memory.  The tile shape changes no rendered value (a pixel composites the
 * same Gaussians in the same order whatever tile holds it). */
gs_status gs_targets_layout(const gs_view *views, int32_t n_views, gs_target *targets,
                            int32_t n_targets, int64_t *total_pixels, int32_t *total_tiles);

/* (host) Workspace sizes for a problem: n_cap Gaussian columns, n_views
 * views, targets (host array, already laid out), pair_cap tile/Gaussian
 * pairs. */
gs_status gs_workspace_query(const gs_settings *s, int64_t n_cap, int32_t n_views,
                             const gs_target *targets, int32_t n_targets, int64_t pair_cap,
                             gs_sizes *out);

/* Projection (Eq. 3's splat G, Section 3.3): for every view v and Gaussian
 * g < n, the camera-frame depth, the level-0 2D mean, the undilated 2D
 * covariance J W Sigma W^T J^T, the opacity sigmoid(raw) and the SH colour
 * seen from the view's centre (max(0, 0.5 + sum_k Y_k c_k)).  Gaussians with
 * depth <= znear are marked invalid (zero record: opacity 0, depth 0).
 * params (device) as above; views (device) n_views entries; proj_ws (device)
 * proj_bytes. */
gs_status gs_preprocess(const gs_settings *s, const float *params, int64_t n, int64_t n_cap,
                        const gs_view *views, int32_t n_views, void *proj_ws, void *stream);

/* Tile binning of the tile-based renderer (Section 3.3: the keyframe is
 * rendered tile by tile; Eq. 3's sum runs front to back over depth): for
 * every target, each valid Gaussian whose cutoff ellipse
 * {alpha >= alpha_min} overlaps a tile of the target is paired with that tile; the
 * pairs are sorted by (target tile, depth, Gaussian index) with a device
 * radix sort and each tile's range of pairs is recorded.  targets (device,
 * laid out), total_tiles from gs_targets_layout.  sort_ws (device)
 * sort_bytes.  d_status (device, uint32): GS_STATUS_PAIR_OVERFLOW is OR-ed in
 * when the pairs exceed pair_cap (the tile lists are then incomplete; retry
 * with a larger pair_cap).  d_status is not cleared by the call. */
gs_status gs_bin_sort(const gs_settings *s, const void *proj_ws, int64_t n, int64_t n_cap,
                      int32_t n_views, const gs_target *targets, int32_t n_targets,
                      int32_t total_tiles, void *sort_ws, int64_t pair_cap, uint32_t *d_status,
                      void *stream);

/* Forward rasterisation (Eq. 3): front-to-back alpha compositing of every
 * tile's sorted list, one pixel per thread.  proj_ws and sort_ws as filled by
 * gs_preprocess and gs_bin_sort with the same n_cap, n_views, targets and
 * pair_cap.  Writes, per target,
 * out_rgb (device, 3 * total_pixels floats, C + T_final * bg), out_T (device,
 * total_pixels, final transmittance), out_last (device, total_pixels, one
 * past the tile-list position of the last composited Gaussian; the backward
 * restarts from it) and, when not NULL, out_ncontrib (device, total_pixels,
 * number of composited Gaussians) and out_nevals (device, total_pixels,
 * number of (pixel, Gaussian) pairs the pixel evaluated: Gaussians of its
 * tile's list that reach the tile, up to its early stop). */
gs_status gs_render_fwd(const gs_settings *s, const void *proj_ws, int64_t n_cap,
                        int32_t n_views, const void *sort_ws, int64_t pair_cap,
                        const gs_target *targets,
                        int32_t n_targets, int32_t total_tiles, float *out_rgb, float *out_T,
                        int32_t *out_last, int32_t *out_ncontrib, int32_t *out_nevals,
                        void *stream);

/* Backward of the rasteriser (reverse mode of Eq. 3 per pixel): recomputes
 * compositing back to front from out_T and out_last (no per-pixel lists are
 * stored) and accumulates, per (view, Gaussian), the gradients of the loss
 * with respect to the 2D mean (level-0 pixels), the undilated 2D covariance
 * (entries 00, 01, 11 of the symmetric matrix gradient), the opacity and the
 * colour into accum_ws (device, accum_bytes; float32 [n_views * n_cap][9],
 * the nine values of a record in that order; cleared by this call).  dL_drgb (device) has the layout
 * of out_rgb.  proj_ws, sort_ws, out_T, out_last as left by the forward. */
gs_status gs_raster_bwd(const gs_settings *s, const void *proj_ws, int64_t n_cap,
                        int32_t n_views, const void *sort_ws, int64_t pair_cap,
                        const gs_target *targets, int32_t n_targets, int32_t total_tiles,
                        const float *out_T, const int32_t *out_last, const float *dL_drgb,
                        void *accum_ws, void *stream);

/* Store-all variant of the rasteriser, the comparison point of the recompute
 * backward above (back-propagation of Eq. 3, Section 3.3): the forward keeps
 * the transmittance in front of every composited (pixel, Gaussian) pair and
 * the backward reads it instead of dividing it back out of the final
 * transmittance.
 *
 * gs_render_fwd_store: the forward of gs_render_fwd (same out_rgb, out_T,
 * out_last; out_ncontrib required), then the store.  tile_steps (device,
 * int32 [total_tiles]) receives the largest composited count of each tile;
 * store_base (device, int64 [total_tiles + 1]) the start of each tile's
 * stretch of the store, base[total_tiles] being the floats the store needs.
 * The transmittance in front of a pixel's k-th composited Gaussian is at
 * store[base[tile] + 256 k + (pixel index in the tile)].  store (device,
 * store_cap floats): when base[total_tiles] > store_cap nothing is stored
 * (read base[total_tiles] after the stream has synchronised, re-size, call
 * again).  The call runs the forward twice (counts, then the store).
 *
 * gs_raster_bwd_stored: gs_raster_bwd reading the store (out_last,
 * out_ncontrib, store_base, store as left by gs_render_fwd_store).  When the
 * store was too small it leaves accum_ws cleared. */
gs_status gs_render_fwd_store(const gs_settings *s, const void *proj_ws, int64_t n_cap,
                              int32_t n_views, const void *sort_ws, int64_t pair_cap,
                              const gs_target *targets, int32_t n_targets, int32_t total_tiles,
                              float *out_rgb, float *out_T, int32_t *out_last, int32_t *out_ncontrib,
                              int32_t *tile_steps, int64_t *store_base, float *store, int64_t store_cap,
                              void *stream);
gs_status gs_raster_bwd_stored(const gs_settings *s, const void *proj_ws, int64_t n_cap,
                               int32_t n_views, const void *sort_ws, int64_t pair_cap,
                               const gs_target *targets, int32_t n_targets, int32_t total_tiles,
                               const int32_t *out_last, const int32_t *out_ncontrib,
                               const int64_t *store_base, const float *store, int64_t store_cap,
                               const float *dL_drgb, void *accum_ws, void *stream);

/* Chain rule from the per-view 2D gradients in accum_ws to the raw parameters
 * (through the 2D covariance, projection Jacobian with its field-of-view clamp,
 * rotation/scale, opacity sigmoid and the SH basis including its view
 * direction), summed over views and ADDED to grad (device, [59][n_cap]). */
gs_status gs_project_bwd(const gs_settings *s, const float *params, int64_t n, int64_t n_cap,
                         const gs_view *views, int32_t n_views, const void *accum_ws, float *grad,
                         void *stream);

/* gs_project_bwd fused with the Adam step of gs_adam_step: each parameter is
 * updated in place (params, m, v: device [59][n_cap]) as soon as its gradient
 * is known, so no gradient buffer is written, read or cleared.  Every column
 * < n is stepped (Gaussians no view touched get a zero gradient); the result
 * equals gs_project_bwd into a zeroed gradient followed by gs_adam_step.
 * proj_out (device, proj_bytes, optional): when non-NULL, the projection
 * records of the updated parameters for the same views are also written there,
 * equal to what gs_preprocess of the updated parameters writes, so the next
 * iteration can skip gs_preprocess; it may be the proj_ws of the iteration
 * (this call does not read projection records). */
gs_status gs_project_bwd_adam(const gs_settings *s, float *params, int64_t n, int64_t n_cap,
                              const gs_view *views, int32_t n_views, const void *accum_ws,
                              float *m, float *v, const float *lr_rows, double beta1,
                              double beta2, double eps, int32_t step, const int32_t *d_step,
                              void *proj_out, void *stream);

/* gs_raster_bwd followed by gs_project_bwd (the full backward to the raw
 * parameters, ADDED to grad). */
gs_status gs_render_bwd(const gs_settings *s, const float *params, int64_t n, int64_t n_cap,
                        const gs_view *views, int32_t n_views, const void *proj_ws,
                        const void *sort_ws, int64_t pair_cap, const gs_target *targets,
                        int32_t n_targets, int32_t total_tiles, const float *out_T,
                        const int32_t *out_last, const float *dL_drgb, void *accum_ws,
                        float *grad, void *stream);

/* gs_raster_bwd followed by gs_project_bwd_adam (one optimiser step); proj_out
 * as there (it may be proj_ws: the raster backward has read it by then). */
gs_status gs_render_bwd_adam(const gs_settings *s, float *params, int64_t n, int64_t n_cap,
                             const gs_view *views, int32_t n_views, const void *proj_ws,
                             const void *sort_ws, int64_t pair_cap, const gs_target *targets,
                             int32_t n_targets, int32_t total_tiles, const float *out_T,
                             const int32_t *out_last, const float *dL_drgb, void *accum_ws,
                             float *m, float *v, const float *lr_rows, double beta1, double beta2,
                             double eps, int32_t step, const int32_t *d_step, void *proj_out, void *stream);

/* Gaussian pyramid of one planar image (Section 3.4): level l+1 is level l
 * smoothed by the 5x5 binomial kernel (1 4 6 4 1)^2/256 with mirrored
 * borders (edge sample not repeated) and decimated to even rows and columns,
 * sizes ceil(H/2) x ceil(W/2).  img (device) [C][H][W]; out (device) receives
 * levels 0..levels-1 packed back to back (level 0 is a copy). */
gs_status gs_pyramid_build(const float *img, int32_t C, int32_t H, int32_t W, int32_t levels,
                           float *out, void *stream);

/* Photometric loss of Eq. 4 for every target:
 *   L_t = (1 - lambda) mean|I_r - I_gt| + lambda (1 - mean SSIM(I_r, I_gt)),
 * SSIM with an 11x11 Gaussian window (sigma 1.5) and zero padding, per
 * channel, C1 = 0.01^2, C2 = 0.03^2.  render, target (device) packed like
 * out_rgb.  Writes d_loss (device, n_targets floats, L_t) and d_total
 * (device, 1 float, sum_t weight_t L_t) and dL_drender (device, like render,
 * the gradient of the total).  loss_ws (device) loss_bytes. */
gs_status gs_pyramid_loss(const float *render, const float *target, const gs_target *targets,
                          int32_t n_targets, int32_t total_tiles, int64_t total_pixels,
                          float lambda, void *loss_ws, float *d_loss, float *d_total,
                          float *dL_drender, void *stream);

/* Adam step on the parameter store (Section 4.1 fixed learning rate; torch's
 * bias-corrected update): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr[row] * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * params, grad, m, v (device) [59][n_cap]; lr_rows (host) 59 floats;
 * beta1, beta2 in [0, 1), eps >= 0 (double so 1 - beta is formed before
 * rounding); step >= 1, or step = 0 with d_step (device int32) holding the
 * step, read on the device (for graph replay; see gs_step_advance).  Only
 * columns < n are updated. */
gs_status gs_adam_step(float *params, const float *grad, float *m, float *v, int64_t n,
                       int64_t n_cap, const float *lr_rows, double beta1, double beta2, double eps,
                       int32_t step, const int32_t *d_step, void *stream);

/* Adds 1 to the device step counter d_step (device int32) on the stream.  With
 * step = 0 and d_step set, the Adam entry points read the step from d_step on
 * the device, so a captured graph that advances it and then steps replays
 * correctly. */
gs_status gs_step_advance(int32_t *d_step, void *stream);

/* ---------------------------------------------------------------------------
 * Initialisation of newly densified primitives.  Section 3.3.1 creates
 * temporary primitives at inactive keypoints of each new keyframe, placed with
 * the keypoint's depth.  A small MLP proposes their scale, rotation, opacity
 * and colour; the heuristic below is its fallback and its baseline.
 * Keypoints kp (device float [B][4]): pixel u, v, depth (metres) and scale
 * 1.2^octave.
 * ------------------------------------------------------------------------- */

/* Network input per keypoint (device BF16 [B][160]): the 7x7 RGB patch of img
 * (device float [3][H][W], edge-clamped) around the rounded pixel, channel
 * major, then depth, scale, a one-hot of the octave round(log_1.2 scale)
 * clamped to 0..7, the heuristic log-scale (row 3 of heuristic, device float
 * [59][B], optional: 0 when NULL) and log depth (159 values), zero-padded to
 * 160. */
gs_status gs_init_features(const float *img, int32_t H, int32_t W, const float *kp, int32_t B,
                           const float *heuristic, void *x_bf16, void *stream);

/* MLP 160 -> 128 -> 128 -> 16 with ReLU hidden layers, BF16 weights and
 * activations on the matrix cores, FP32 accumulation.  w_bf16 (device, 38912
 * BF16): W1 [128][160], W2 [128][128], W3 [16][128] row-major [out][in], in
 * that order; bias (device, 272 floats): b1, b2, b3.  x_bf16 (device BF16
 * [B][160]); y (device float [B][16]: log-scale correction (3), camera-frame
 * quaternion (4), opacity logit, SH DC correction (3), 5 unused); act_ws (device,
 * 2 * B * 128 BF16) keeps the hidden activations for the backward. */
gs_status gs_init_mlp_fwd(const void *w_bf16, const float *bias, const void *x_bf16, int32_t B,
                          float *y, void *act_ws, void *stream);

/* Backward of sum over rows of <dy, y> (dy device float [B][16]): ADDS the
 * weight gradient to dw (device float, layout of w_bf16) and the bias
 * gradient to db (device float [272]).  BF16 operands (dy and the hidden
 * gradients rounded where they enter a product), FP32 accumulation. */
gs_status gs_init_mlp_bwd(const void *w_bf16, const void *x_bf16, const void *act_ws,
                          const float *dy, int32_t B, float *dw, float *db, void *stream);

/* Adam on the MLP's FP32 master weights (device, 38912) and biases (device,
 * 272), moments m, v (device, 39184 each, weights then biases); refreshes the
 * BF16 weight copy (round to nearest even). */
gs_status gs_init_mlp_adam(float *w_master, float *b_master, void *w_bf16, const float *dw,
                           const float *db, float *m, float *v, float lr, double beta1,
                           double beta2, double eps, int32_t step, void *stream);

/* FP32 to BF16 (round to nearest even), count values, device to device. */
gs_status gs_to_bf16(const float *src, void *dst, int64_t count, void *stream);

/* Heuristic initial parameters (device float [59][B]) for new means new_mu
 * (device float [3][B], world) with pixel colours new_rgb (device [3][B]):
 * log-scale = log(mean distance to the 3 nearest means among the n existing
 * ones in params and the other new ones), isotropic; quaternion (1, 0, 0, 0);
 * opacity logit ln(0.1/0.9); SH DC = (rgb - 0.5) / Y_0; other SH 0. */
gs_status gs_init_heuristic(const float *new_mu, const float *new_rgb, int32_t B,
                            const float *params, int64_t n, int64_t n_cap, float *out,
                            void *stream);

/* World-frame parameters (device float [59][B]) from MLP outputs y for
 * keypoints kp seen by view (host struct, level 0), relative to the heuristic
 * columns (device [59][B]): mean = back-projection of (u, v) at the depth;
 * log-scale = heuristic log-scale + y[0..2]; quaternion = rotation of the
 * camera-to-world transform composed with y[3..6]; opacity logit = y[7];
 * SH DC = heuristic DC + y[8..10]; other SH 0.  Where sigmoid(y[7]) < 0.01
 * the heuristic column is used unchanged and used_fallback (device int32
 * [B], optional) is set to 1. */
gs_status gs_init_decode(const float *y, const float *kp, const gs_view *view, int32_t B,
                         const float *heuristic, float *out, int32_t *used_fallback,
                         void *stream);

/* Appends B new columns (device float [59][B]) to params at column n
 * (n + B <= n_cap); the Adam moments m, v (optional) of those columns are
 * zeroed. */
gs_status gs_append(float *params, float *m, float *v, int64_t n, int64_t n_cap,
                    const float *new_params, int32_t B, void *stream);

/* Fills dst (device, count floats) with value (a kernel, not a memset, so a
 * captured graph replays it faithfully). */
gs_status gs_fill(float *dst, int64_t count, float value, void *stream);

/* ---------------------------------------------------------------------------
 * Gradient-driven densification (Section 3.3.1: split or clone primitives
 * with large loss gradients, as in 3D Gaussian splatting, Kerbl et al. 2023,
 * Sec. 5.2), plus the pruning and the opacity reset of the same rule.
 * ------------------------------------------------------------------------- */

/* Thresholds of the rule, in the float32 form the kernels compare against. */
typedef struct {
    float grad_threshold; /* mean NDC gradient norm at or above which a primitive is densified */
    float log_dense;      /* clone if the largest log-scale is <= this, else split */
    float log_big;        /* prune if the largest log-scale is > this (+inf: never) */
    float logit_min;      /* prune if the opacity logit is < this */
    float log_shrink;     /* subtracted from the log-scales of a split's children */
} gs_densify_rule;

/* (host) Rule for a scene of the given extent (e.g. the radius of the
 * keyframe centres): grad_threshold; log_dense = ln(percent_dense * extent);
 * log_big = ln(big_fraction * extent), or +inf when big_fraction <= 0;
 * logit_min = ln(min_opacity / (1 - min_opacity)); log_shrink = ln(shrink);
 * each computed in double and rounded to float.  The usual values are
 * 2e-4, 0.01, 0.005, 0.1 and 1.6.  Invalid arguments (extent, percent_dense
 * or shrink <= 0, min_opacity outside (0, 1)) return GS_ERR_INVALID_ARGUMENT. */
gs_status gs_densify_rule_make(double extent, double grad_threshold, double percent_dense,
                               double min_opacity, double big_fraction, double shrink,
                               gs_densify_rule *out);

/* Adds one backward pass to the densification statistic stats (device float
 * [2][n_cap]): for every view v and primitive g < n whose accumulator record
 * in accum_ws (as left by gs_raster_bwd; [n_views * n_cap][9]) holds any
 * nonzero value, row 0 gains the norm of its 2D-mean gradient in normalised
 * device coordinates, |(dx * W_v / 2, dy * H_v / 2)| with W_v, H_v the view's
 * level-0 size, and row 1 gains 1.  views: device gs_view[n_views]. */
gs_status gs_densify_stats(const void *accum_ws, int64_t n, int64_t n_cap, const gs_view *views,
                           int32_t n_views, float *stats, void *stream);

/* Bytes of device workspace gs_densify needs for n primitives. */
size_t gs_densify_workspace_bytes(int64_t n);

/* Applies the rule to primitives 0..n-1 of params, m, v (device [59][n_cap])
 * with the statistic stats (device [2][n_cap]; mean = row 0 / row 1, 0 where
 * row 1 is 0) and writes the result to out_params, out_m, out_v (device
 * [59][out_cap], out_cap a multiple of 64, not overlapping the inputs):
 *   - densified (mean >= grad_threshold) and largest log-scale <= log_dense:
 *     cloned (the original and an identical copy);
 *   - densified and larger: split into two children with the parent's
 *     values except mean + Rq (exp(log-scale) * z_c) and log-scale -
 *     log_shrink (Rq the rotation of the normalised quaternion, z_0 = noise
 *     rows 0-2, z_1 = rows 3-5 of the parent's column; noise: device float
 *     [6][n_cap] standard normals); the parent is dropped;
 *   - any primitive, original or new, with opacity logit < logit_min or
 *     largest log-scale > log_big is dropped.
 * Output order: the surviving originals in order, then for each original in
 * order its surviving copy or children.  Survivors keep their moments, new
 * primitives get zero moments.  d_counts (device int64[4]) receives the
 * output count, the copies made, the primitives split and the originals
 * pruned.  If the output count exceeds out_cap nothing is written to the
 * outputs (d_counts[0] still tells the count required).  ws: device,
 * gs_densify_workspace_bytes(n).  The statistic is not cleared (the caller
 * restarts it for the new layout).  Columns >= the output count are not
 * written. */
gs_status gs_densify(const gs_densify_rule *rule, const float *params, const float *m,
                     const float *v, const float *stats, const float *noise, int64_t n,
                     int64_t n_cap, float *out_params, float *out_m, float *out_v,
                     int64_t out_cap, void *ws, int64_t *d_counts, void *stream);

/* Largest n that gs_densify_noalloc accepts. */
#define GS_DENSIFY_NOALLOC_MAX_N 16777216

/* gs_densify without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same kernels, arguments (less ws) and results as
 * gs_densify.  Its workspace is a fixed device array inside the library,
 * 8,127,232 bytes (the workspace of n = GS_DENSIFY_NOALLOC_MAX_N), which each
 * device holds from the first call on it until the process ends; nothing in it
 * needs to start cleared, and the call allocates nothing.  n above
 * GS_DENSIFY_NOALLOC_MAX_N returns GS_ERR_CAPACITY and enqueues nothing.  All
 * calls on one device share that device's array: calls that may overlap on the
 * same device (other streams, other host threads) race on it and must be
 * ordered by the caller. */
gs_status gs_densify_noalloc(const gs_densify_rule *rule, const float *params, const float *m,
                             const float *v, const float *stats, const float *noise, int64_t n,
                             int64_t n_cap, float *out_params, float *out_m, float *out_v,
                             int64_t out_cap, int64_t *d_counts, void *stream);

/* Opacity reset of the same rule: the opacity logit of every primitive < n is
 * lowered to ln(max_opacity / (1 - max_opacity)) (computed in double, rounded
 * to float) where it is above, and the opacity row of m and v (optional) is
 * zeroed. */
gs_status gs_reset_opacity(float *params, float *m, float *v, int64_t n, int64_t n_cap,
                           double max_opacity, void *stream);

/* ---------------------------------------------------------------------------
 * Loop-closure correction of the primitives (Section 3.5: keyframes and map
 * points move by similarity corrections when a loop is closed; the hyper
 * primitives follow).
 * ------------------------------------------------------------------------- */

/* The similarity x' = s R(q) x + t: q a quaternion (w, x, y, z; normalised by
 * the library), s > 0. */
typedef struct {
    float q[4];
    float t[3];
    float s;
} gs_sim3;

/* Bytes of device workspace gs_sim3_apply needs for n_transforms transforms. */
size_t gs_sim3_workspace_bytes(int32_t n_transforms);

/* Moves primitives 0..n-1 of params (device [59][n_cap], in place) by
 * transforms[assign[g]] (transforms: device gs_sim3[n_transforms]; assign:
 * device int32 [n], or NULL for transform 0 everywhere): mean -> s R mean + t,
 * log-scale -> log-scale + ln s, quaternion -> q_R * q (Hamilton product,
 * q_R the normalised transform quaternion), opacity unchanged, and every
 * colour channel's SH bands 1-3 rotated so that the colour seen along d
 * equals the old colour seen along R^T d (band l: c -> D_l(R)^T c with
 * Y_l(R^T d) = D_l(R) Y_l(d); band 0 unchanged).  Primitives whose index is
 * outside [0, n_transforms), or whose transform has s <= 0 or a zero
 * quaternion, are left unchanged.  Adam moments are not touched.
 * ws: device, gs_sim3_workspace_bytes(n_transforms). */
gs_status gs_sim3_apply(float *params, int64_t n, int64_t n_cap, const gs_sim3 *transforms,
                        int32_t n_transforms, const int32_t *assign, void *ws, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
