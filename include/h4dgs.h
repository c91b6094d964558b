/*
 * h4dgs.h - C ABI of the MI355X (gfx950) hybrid 3D/4D Gaussian rasterizer.
 *
 * The library renders a scene made of two Gaussian sets - static 3D Gaussians
 * and dynamic 4D Gaussians - at given cameras and timestamps, differentiates
 * the images with respect to every raw parameter, converts temporally
 * invariant 4D Gaussians to 3D ones and applies Adam steps.  It follows the
 * rasterization problem statement of "Hybrid 3D-4D Gaussian Splatting for Fast
 * Dynamic Scene Representation" (Alg. 1: Rasterize(w, h, M4D, S4D, M3D, S3D,
 * A, V, s)) and its conversion pass (Sec. 4.1-4.2).
 *
 * Conventions shared by every entry point
 *  - All parameter, image and gradient arrays are DEVICE pointers to float32,
 *    structure-of-arrays, component-major: component c of Gaussian i is at
 *    a[c * n + i].  Arrays marked "host" are host memory.
 *  - The caller owns every buffer.  No call allocates device memory: each
 *    reports the sizes it needs (h4dgs_workspace_size) and works inside the
 *    caller's `state` and `scratch` buffers, except h4dgs_render_infer_noalloc,
 *    which works inside a fixed workspace of the library's device code (a
 *    static array loaded with it).  Device buffers must be 256-byte aligned
 *    (any hipMalloc / PyTorch allocation is).
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream)
 *    and returns before it completes, except where a call says it synchronises.
 *  - Errors are return codes; nothing is thrown across the ABI.
 *    h4dgs_last_error() gives a message for the last failing call on a context.
 *    Argument errors are found on the host before anything is enqueued.
 *  - A context is a small host object (tuning cache, error text); use one
 *    context from one host thread at a time.
 */
#ifndef H4DGS_H
#define H4DGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define H4DGS_MAX_VIEWS 32
#define H4DGS_SH_ROWS 48 /* degree-3 SH: 16 coefficients x RGB, row k*3 + channel */

typedef enum {
    H4D_OK = 0,
    H4D_ERR_INVALID_ARG = 1, /* bad pointer, size, tile size, view ... (host-side check) */
    H4D_ERR_CAPACITY = 2,    /* the (Gaussian, tile) pairs did not fit: see h4dgs_check */
    H4D_ERR_HIP = 3,         /* a HIP runtime call failed */
    H4D_ERR_NONFINITE = 4,   /* reserved */
    H4D_ERR_UNSUPPORTED = 5  /* valid request this build does not handle */
} h4d_status;

typedef struct h4d_ctx h4d_ctx;

/* Static 3D Gaussians (Sec. 3.1): mean[3][n], log_scale[3][n] (scale = exp),
 * quat[4][n] (w,x,y,z, any norm > 0: normalised inside), opacity[n] (logit:
 * sigmoid inside), sh[48][n]. */
typedef struct {
    int32_t n;
    const float *mean, *log_scale, *quat, *opacity, *sh;
} h4d_g3d;

/* Dynamic 4D Gaussians (Sec. 3.2, Eq. 4-7): spatial mean[3][n], temporal
 * mean mean_t[n], log_scale[4][n] (x, y, z, t), quat_l[4][n] = (a,b,c,d) and
 * quat_r[4][n] = (p,q,r,s) of the left/right isoclinic rotations, opacity[n]
 * (logit), sh[48][n].
 * Optional time-varying colour (the cosine terms of 4D Gaussian splatting's
 * colour model, which the paper's 4D Gaussians inherit, end of Sec. 3.2):
 * with sh_t_degree D in {1, 2}, sh_t[48 D][n] and a period T = sh_t_period,
 * the SH coefficients at view time t are sh + sum_{k=1..D} cos(2 pi k (t -
 * mean_t) / T) sh_t[k - 1]; D = 0 (sh_t ignored) is plain SH. */
typedef struct {
    int32_t n;
    const float *mean, *mean_t, *log_scale, *quat_l, *quat_r, *opacity, *sh;
    int32_t sh_t_degree;
    float sh_t_period;
    const float *sh_t;
} h4d_g4d;

/* Writable mirrors: gradients (overwritten by h4dgs_render_bwd) and the
 * outputs of h4dgs_convert_static.  Field meaning and layout as above; for a
 * 4D input with time coefficients the mirror's sh_t must be given (its
 * degree and period fields are not read). */
typedef struct {
    int32_t n;
    float *mean, *log_scale, *quat, *opacity, *sh;
} h4d_g3d_mut;
typedef struct {
    int32_t n;
    float *mean, *mean_t, *log_scale, *quat_l, *quat_r, *opacity, *sh;
    int32_t sh_t_degree;
    float sh_t_period;
    float *sh_t;
} h4d_g4d_mut;

/* One rendered view (host struct): pinhole camera, world -> camera [R | t]
 * row-major (camera x right, y down, z forward), focal lengths and principal
 * point in pixels, image size, timestamp t at which the 4D set is sliced, and
 * the background colour.  Pixel (i, j) is sampled at (i + 0.5, j + 0.5). */
typedef struct {
    float world_to_cam[12];
    float fx, fy, cx, cy;
    int32_t width, height;
    float t;
    float bg[3];
} h4d_view;

/* Launch configuration.  tile: tile edge in pixels (8, 16 or 32); chunk:
 * list entries staged in LDS per round of the blending kernels (64, 128, 256
 * or 512); batched: 0 = views processed one after another,
 * 1 = the views of a call in one pass per stage (several passes only when
 * their super-tiles exceed 65536); in a batched call whose views repeat a
 * camera (same pose, intrinsics and size) at several times, the 3D Gaussians
 * are projected, sorted and binned once per camera and each view's tiles merge
 * that list with the view's own 4D list (the 3D Gaussians do not depend on
 * t); cull: 0 = a tile's list holds
 * every splat whose pixel square overlaps the tile (Alg. 1), 1 = in addition a
 * splat is left out of tiles in which no pixel centre can reach
 * alpha >= 1/255 (tested in FP64 with a margin far above the FP32 evaluation
 * error, so no pixel's blending changes); pair_capacity: capacity of the
 * call's binning in (Gaussian, tile) slots, summed over its views: the
 * workspace holds pair_capacity / S^2 (Gaussian, super-tile) entries, a
 * super-tile being S x S tiles (S = 4; 2 for 32-pixel tiles) and each entry
 * standing for its S^2 tiles, so this exceeds the number of (Gaussian, tile)
 * pairs.  A view may span at most 65536 super-tiles (16384 x 16384 pixels at
 * 16- and 32-pixel tiles, 8192 x 8192 at 8; H4D_ERR_UNSUPPORTED otherwise).
 * Images do not depend on tile, chunk, batched or cull (a pixel's
 * contributors are fixed by its own square and alpha tests), so these are
 * pure performance knobs. */
typedef struct {
    int32_t tile;
    int32_t chunk;
    int32_t batched;
    int32_t cull;
    int64_t pair_capacity;
} h4d_config;

h4d_status h4dgs_create(h4d_ctx **out);
h4d_status h4dgs_destroy(h4d_ctx *ctx);
const char *h4dgs_last_error(const h4d_ctx *ctx);
/* Build identification string (static storage). */
const char *h4dgs_version(void);

/* Bytes of `state` (kept from render_fwd to render_bwd: the caller leaves it
 * unchanged in between; the backward accumulates into its gradient records)
 * and of `scratch` (free between calls) for n3 + n4 Gaussians, the given host
 * array of n_views views and the configuration.  Pure host arithmetic.  An
 * inference render needs only a leading part of the state (no gradient
 * records: N x n_views x 64 bytes less). */
h4d_status h4dgs_workspace_size(h4d_ctx *ctx, int32_t n3, int32_t n4, const h4d_view *views, int32_t n_views,
                                const h4d_config *cfg, size_t *state_bytes, size_t *scratch_bytes);

/* Forward (Alg. 1, Sec. 4.3): per view, slice every 4D Gaussian at the view's t
 * (Eq. 5-6, opacity times the temporal marginal), merge with the 3D set
 * (index order [4D | 3D]), cull, EWA-project, colour by SH, duplicate into
 * (tile, depth) keys, sort, find tile ranges and blend front to back (Eq. 3).
 * images: host array of n_views device pointers, each float[3][H][W] (planar
 * RGB, written).  A (Gaussian, tile) pair-capacity overflow is not reported by
 * the return code (it is known only on the device): call h4dgs_check. */
h4d_status h4dgs_render_fwd(h4d_ctx *ctx, const h4d_g3d *g3, const h4d_g4d *g4, const h4d_view *views,
                            int32_t n_views, const h4d_config *cfg, float *const *images, void *state,
                            size_t state_bytes, void *scratch, size_t scratch_bytes, void *stream);

/* Inference render (the paper's rendering speed claims, Tables 1-2): the
 * forward of render_fwd (same arguments, same images, bit for bit) without the
 * state only the backward reads (per-pixel final transmittance, last
 * contributor and output colour; per-tile adjoint cost), for rendering without
 * training.  `state` still holds the records, lists and status (h4dgs_check
 * applies as after render_fwd).  render_bwd must not follow it: it would
 * combine this call's records and tile lists with the per-pixel state of an
 * earlier render_fwd (or uninitialised memory), so its gradients are
 * meaningless; its reads stay inside each tile's list and the records. */
h4d_status h4dgs_render_infer(h4d_ctx *ctx, const h4d_g3d *g3, const h4d_g4d *g4, const h4d_view *views,
                              int32_t n_views, const h4d_config *cfg, float *const *images, void *state,
                              size_t state_bytes, void *scratch, size_t scratch_bytes, void *stream);

/* Allocation-free inference render, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and images as h4dgs_render_infer, but the
 * call's state and scratch live in a fixed workspace of H4DGS_NOALLOC_BYTES
 * inside the library: one copy per GPU, allocated when the library's device
 * code is loaded on that GPU and held until the process ends.  The call itself
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 * status_out (device, may be NULL): receives two uint64 words, the status
 * flags (bit 0 = the (Gaussian, tile) pairs exceeded cfg->pair_capacity; the
 * images are then incomplete) and the number of pairs the call needed;
 * written on `stream` after the render.
 * Errors: H4D_ERR_CAPACITY (on the host, before anything is enqueued) when
 * the call's workspace (h4dgs_workspace_size: state rounded up to 256 bytes
 * plus the forward's part of scratch) exceeds H4DGS_NOALLOC_BYTES; the
 * arguments are checked as for h4dgs_render_infer.
 * Every call on one GPU shares that GPU's workspace and leaves its contents
 * behind (each call clears what it needs cleared): calls that overlap on one
 * GPU (other streams, other host threads) race and give undefined images;
 * serialise them.  No backward can follow (there is no state handle). */
#define H4DGS_NOALLOC_BYTES ((size_t)256 << 20)
h4d_status h4dgs_render_infer_noalloc(h4d_ctx *ctx, const h4d_g3d *g3, const h4d_g4d *g4, const h4d_view *views,
                                      int32_t n_views, const h4d_config *cfg, float *const *images,
                                      uint64_t *status_out, void *stream);

/* Backward (the training step's fast adjoint, which Sec. 5.2 adopts from
 * prior work without describing it): the exact adjoint of render_fwd
 * through blending (Eq. 3), projection, slicing (Eq. 5-6), covariance (Eq. 2
 * and its 4D analogue), rotation (Eq. 4) and the activations; per-pixel
 * transmittance is recomputed front to back, not stored.  dl_dimages: host
 * array of n_views device pointers to float[3][H][W] (dL/dC, loss weighting
 * included).  The gradients of every raw parameter (grad3/grad4: device
 * arrays laid out as the parameters) are OVERWRITTEN with
 * sum_v J_v^T dl_dimages_v.  Same g3, g4, views and cfg as the forward; state
 * as the forward left it (unchanged in between by the caller; the backward
 * accumulates screen-space gradients in it, and a further backward on the
 * same state clears them first, so it gives the same gradients); scratch as
 * sized by h4dgs_workspace_size.  Argument errors: H4D_ERR_INVALID_ARG before
 * anything is enqueued.  After a forward whose pairs overflowed, the blending kernels
 * find empty tile lists and the gradients hold only what no pair needs. */
h4d_status h4dgs_render_bwd(h4d_ctx *ctx, const h4d_g3d *g3, const h4d_g4d *g4, const h4d_view *views,
                            int32_t n_views, const h4d_config *cfg, const float *const *dl_dimages,
                            void *state, size_t state_bytes, void *scratch, size_t scratch_bytes,
                            h4d_g3d_mut *grad3, h4d_g4d_mut *grad4, void *stream);

/* Per-Gaussian statistics of a backward call, for the optimiser's
 * visibility mask and for densification (device arrays of one set's n rows;
 * any pointer may be NULL):
 *   grad_norm[n]  += sum, over the call's views in which the Gaussian's pixel
 *                    square meets the image, of the norm of the loss gradient
 *                    with respect to its projected centre in normalised device
 *                    coordinates (the pixel-space gradient times half the
 *                    image width and height), the statistic 3D Gaussian
 *                    Splatting densifies by;
 *   visible[n]    += the number of those views;
 *   step_visible[n] = 1 if there is at least one such view, else 0. */
typedef struct {
    float *grad_norm;
    float *visible;
    uint8_t *step_visible;
} h4d_set_stats;

/* h4dgs_render_bwd (same arguments, same gradients) that also accumulates
 * the statistics above for the 3D and the 4D set (Sec. 4.3: densification
 * and pruning run on each set separately). */
h4d_status h4dgs_render_bwd_stats(h4d_ctx *ctx, const h4d_g3d *g3, const h4d_g4d *g4, const h4d_view *views,
                                  int32_t n_views, const h4d_config *cfg, const float *const *dl_dimages,
                                  void *state, size_t state_bytes, void *scratch, size_t scratch_bytes,
                                  h4d_g3d_mut *grad3, h4d_g4d_mut *grad4, const h4d_set_stats *stats3,
                                  const h4d_set_stats *stats4, void *stream);

/* Synchronises `stream`, then reads the status the last render_fwd left in
 * `state`.  Returns H4D_OK or H4D_ERR_CAPACITY; *pairs_needed (host, may be
 * NULL) receives the number of pairs the call needed. */
h4d_status h4dgs_check(h4d_ctx *ctx, const void *state, size_t state_bytes, int64_t *pairs_needed, void *stream);

/* Alg. 1 from CreateTiles to BlendInOrder alone, on given screen-space splats: n splats with centre
 * u[n], v[n], conic[3][n] (inverse 2D covariance entries 00, 01, 11), effective
 * opacity[n], rgb[3][n], integer radius[n], depth key[n] and visible[n] (uint8).
 * Splat i covers pixel (x, y) iff |x + 0.5 - u| <= r and |y + 0.5 - v| <= r.
 * Writes image[3][H][W], T_final[H][W] (may be NULL) and, if sorted_ids and
 * ranges are not NULL, the per-tile depth-ordered splat ids
 * (sorted_ids[pair_capacity]) with tile ranges (ranges[2 * tiles]: start,
 * end): tile t's list is sorted_ids[ranges[2t] .. ranges[2t+1]), the lists
 * one after another in tile order, as h4dgs_tile_lists writes them.  Uses the
 * same kernels as render_fwd.
 * Workspace: h4dgs_workspace_size(n3 = n, n4 = 0, one view of W x H). */
h4d_status h4dgs_rasterize_splats(h4d_ctx *ctx, int32_t n, const float *u, const float *v, const float *conic,
                                  const float *opacity, const float *rgb, const int32_t *radius,
                                  const float *depth, const uint8_t *visible, int32_t width, int32_t height,
                                  const float *bg /* host, 3 */, const h4d_config *cfg, float *image,
                                  float *T_final, uint32_t *sorted_ids, int64_t *ranges, void *state,
                                  size_t state_bytes, void *scratch, size_t scratch_bytes, void *stream);

/* The tile lists (Alg. 1: the depth-ordered splats of every tile, the lists
 * BlendInOrder traverses) of the last render_fwd / render_infer on `state`,
 * written out for inspection: the blending kernels never store them, they
 * compact each tile's entries from its super-tile's sorted list as they go;
 * this call walks every list the same way.  Same n3, n4, views and cfg as
 * that call; scratch as sized by h4dgs_workspace_size (overwritten).
 * ids (device, ids_capacity words): the splat ids (indices into the merged
 * set [4D | 3D]) of every tile, one list after another in global tile order
 * (views in order), entries from position ids_capacity on left unwritten;
 * ranges (device, int64[2 * total tiles]): start and end of each tile's
 * list (the last end is the number of entries; a shared static list counts
 * once per view that uses it).  Enqueued on `stream`. */
h4d_status h4dgs_tile_lists(h4d_ctx *ctx, int32_t n3, int32_t n4, const h4d_view *views, int32_t n_views,
                            const h4d_config *cfg, const void *state, size_t state_bytes, void *scratch,
                            size_t scratch_bytes, uint32_t *ids, uint64_t ids_capacity, int64_t *ranges,
                            void *stream);

/* Static identification and 4D -> 3D conversion (Sec. 4.1-4.2, Eq. 7-9).
 * Row i of in4 is static iff (double)log_scale_t[i] > log((double)tau).  out4
 * receives the non-static rows in their order (capacity in4->n); out3
 * receives the rows of in3 followed by the converted rows in ascending 4D
 * index (capacity in3->n + in4->n).  A converted row keeps mean, the three
 * spatial log-scales, opacity and SH bit-exactly and gets the Eq. 9
 * quaternion of the top-left 3x3 block of R_l R_r (not renormalised).
 * perm[n4] (device, int32): new 4D row, or -(1 + new 3D row).  Synchronises
 * `stream`; *n4_out and *n3_out are host pointers.  out3/out4 must not alias
 * in3/in4.  scratch: at least h4dgs_convert_scratch_bytes(n4). */
size_t h4dgs_convert_scratch_bytes(int32_t n4);
h4d_status h4dgs_convert_static(h4d_ctx *ctx, const h4d_g4d *in4, const h4d_g3d *in3, float tau,
                                h4d_g4d_mut *out4, h4d_g3d_mut *out3, int32_t *perm, int32_t *n4_out,
                                int32_t *n3_out, void *scratch, size_t scratch_bytes, void *stream);

/* Adaptive densification and pruning, run on the 3D and the 4D set
 * separately with limits of their own (Sec. 4.3 adopts the clone / split /
 * prune scheme of 3D Gaussian Splatting and applies it to each set; the paper
 * uses no opacity reset).  Per row i of a set, with g = stats->grad_norm[i],
 * c = stats->visible[i] and L = the largest of its three spatial log-scales:
 *   selected  iff c > 0 and (double)g >= (double)grad_threshold * (double)c;
 *   cloned    iff selected and L <= log_dense_scale;
 *   split     iff selected and L >  log_dense_scale;
 *   a row is pruned iff (double)opacity_logit < opacity_logit_min or
 *   L > log_max_scale (all compared in double, exactly).
 * Output rows (out3 / out4, row stride = their n, the capacity, which must be
 * at least max(2, split_n) times the input count): the rows that are not
 * split and not pruned, in order; then the clones (exact copies) that are not
 * pruned, in order; then for k = 0 .. split_n - 1 the k-th child of every split
 * row, in order, unless pruned.  A child copies its parent except for its
 * log-scales, fl32((double)ls - log_shrink) for every component (the prune
 * test uses these), and its centre: the parent's plus the parent's rotation
 * applied to exp(ls) * z, with z the row's k-th draw from noise (standard
 * normal, caller-drawn): 3D: noise3[split_n][3][n3], rotation R(q) (Eq. 2),
 * centre = mean; 4D: noise4[split_n][4][n4], rotation R_l R_r (Eq. 4) on
 * (x, y, z, t), centre = (mean, mean_t), so children spread in space and
 * time.  src3 / src4 (device int32, capacity rows): the source row of each
 * output row, or -(1 + parent) for a new row (clone or child).  *n3_out and
 * *n4_out (host) receive the row counts; the call synchronises `stream`.
 * scratch: at least h4dgs_densify_scratch_bytes(n3, n4).  The statistics are
 * not reset here (the caller zeroes them for the new rows). */
typedef struct {
    float grad_threshold;     /* 3DGS: 2e-4 */
    int32_t split_n;          /* children per split row, 1 .. 8 (3DGS: 2) */
    double log_dense_scale;   /* 3DGS: log(0.01 * scene extent) */
    double opacity_logit_min; /* 3DGS: logit(0.005) */
    double log_max_scale;     /* +inf: no size pruning */
    double log_shrink;        /* 3DGS: log(0.8 * split_n) */
} h4d_densify_params;
size_t h4dgs_densify_scratch_bytes(int32_t n3, int32_t n4);
h4d_status h4dgs_densify(h4d_ctx *ctx, const h4d_g3d *in3, const h4d_g4d *in4, const h4d_set_stats *stats3,
                         const h4d_set_stats *stats4, const float *noise3, const float *noise4,
                         const h4d_densify_params *p3, const h4d_densify_params *p4, h4d_g3d_mut *out3,
                         h4d_g4d_mut *out4, int32_t *src3, int32_t *src4, int32_t *n3_out, int32_t *n4_out,
                         void *scratch, size_t scratch_bytes, void *stream);

/* Optimiser state across densification: out row r of a set takes row
 * src[r] of the input arrays (laid out as the parameters) when src[r] >= 0,
 * zeros otherwise (a new row's moments start at zero); rows3 / rows4 output
 * rows (<= the outputs' n, which is their row stride); src as h4dgs_densify
 * wrote it (a value outside [0, n) reads as zeros).  Enqueued on `stream`. */
h4d_status h4dgs_gather_rows(h4d_ctx *ctx, const h4d_g3d *in3, const h4d_g4d *in4, const int32_t *src3,
                             int32_t rows3, const int32_t *src4, int32_t rows4, h4d_g3d_mut *out3,
                             h4d_g4d_mut *out4, void *stream);

/* Optimiser state across the static conversion: moves one set of per-
 * parameter arrays (an Adam moment, laid out exactly as the parameters) the
 * way h4dgs_convert_static moved the parameters, following its perm (device,
 * [in4->n], from a convert_static call on the same sets).  A kept 4D row takes
 * all its entries; a converted row takes those of the fields the conversion
 * copies (mean, the three spatial log-scales, opacity, SH) and gets zeros for
 * its new quaternion (Eq. 9 makes a new parameter, whose moments start from
 * zero); the 3D rows are copied.  in4/in3: the moment arrays of the old sets;
 * out4/out3: capacities and row strides as for convert_static (out4->n >=
 * in4->n, out3->n >= in3->n + in4->n), rows past the new counts are left
 * unwritten.  Enqueued on `stream`; errors as for convert_static. */
h4d_status h4dgs_convert_moments(h4d_ctx *ctx, const h4d_g4d *in4, const h4d_g3d *in3, const int32_t *perm,
                                 h4d_g4d_mut *out4, h4d_g3d_mut *out3, void *stream);

/* One bias-corrected Adam step (Kingma & Ba) over up to 16 float32 segments:
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2, p -= lr * m_hat / (sqrt(v_hat)
 * + eps), in place.  Host arrays of n_seg device pointers / sizes / learning
 * rates; the constants are taken in double so that 1 - b is formed exactly
 * before rounding to float32.  step >= 1 is the 1-based step count. */
h4d_status h4dgs_adam(h4d_ctx *ctx, int32_t n_seg, float *const *params, const float *const *grads,
                      float *const *m, float *const *v, const int64_t *sizes, const float *lrs, double beta1,
                      double beta2, double eps, int32_t step, void *stream);

/* h4dgs_adam with a visibility mask per segment (the sparse update that
 * leaves Gaussians outside the step's views untouched, so that a step costs
 * what its visible Gaussians need): masks (host array of n_seg device
 * pointers, each may be NULL = no mask) and rows (host, per segment): element
 * e of a masked segment belongs to Gaussian e % rows (the component-major
 * layout) and is updated only where mask[e % rows] != 0; elsewhere the
 * parameter and both moments keep their values.  size must be a multiple of
 * rows.  The bias correction uses the global step. */
h4d_status h4dgs_adam_masked(h4d_ctx *ctx, int32_t n_seg, float *const *params, const float *const *grads,
                             float *const *m, float *const *v, const int64_t *sizes, const float *lrs,
                             const uint8_t *const *masks, const int64_t *rows, double beta1, double beta2,
                             double eps, int32_t step, void *stream);

/* L1 photometric loss of n_views images against targets (both float[3][H][W]
 * per view, host arrays of device pointers): dl_dimages_v = sign(C - target) /
 * (3 W H n_views) (sign(0) = 0), the gradient of the mean over views of the
 * per-view mean absolute error.  loss (device float, may be NULL) receives that
 * mean.  Reading: the paper does not state its loss; L1 is the plain choice. */
h4d_status h4dgs_l1_loss_grad(h4d_ctx *ctx, int32_t n_views, const float *const *images,
                              const float *const *targets, const h4d_view *views, float *const *dl_dimages,
                              float *loss, void *stream);

/* ---- workspace self-check (host arithmetic only, no device work) ---------
 * Every radix sort pass of the binning writes 2^nbits counts per sort block
 * and segment into a histogram buffer of the scratch workspace.  The forward
 * checks each pass against the buffer sizes of its workspace layout on the
 * host before launching anything (and the launcher again per pass); these two
 * calls expose that arithmetic so that it can be tested without a GPU.
 * h4dgs_radix_hist_words: histogram words one pass over `capacity` keys in
 * n_seg segments with nbits-bit digits and `items` keys per thread (8 or 2)
 * needs.  h4dgs_radix_pass_check: H4D_OK if such a pass fits histogram /
 * digit-total buffers of hist_words / totals_words 32-bit words, else
 * H4D_ERR_INVALID_ARG (also for nbits outside [1, 11] or other items). */
size_t h4dgs_radix_hist_words(uint64_t capacity, int32_t n_seg, int32_t nbits, int32_t items);
h4d_status h4dgs_radix_pass_check(uint64_t capacity, int32_t n_seg, int32_t nbits, int32_t items,
                                  size_t hist_words, size_t totals_words);

/* ---- instrumentation ---------------------------------------------------- */
typedef enum {
    H4D_STAGE_PREPROCESS = 0,     /* per-Gaussian FP64 geometry, records, depth keys */
    H4D_STAGE_DEPTH_SORT = 1,     /* radix sort of the depth keys */
    H4D_STAGE_BINNING = 2,        /* pair offsets, emission, tile sort, tile ranges */
    H4D_STAGE_BLEND_FWD = 3,      /* front-to-back blending */
    H4D_STAGE_BLEND_BWD = 4,      /* blending adjoint */
    H4D_STAGE_PREPROCESS_BWD = 5, /* per-Gaussian FP64 adjoint */
    H4D_STAGE_ADAM = 6,
    H4D_STAGE_LOSS = 7,
    H4D_STAGE_COUNT = 8
} h4d_stage;

/* Timing of later calls with HIP events (host objects; no device memory):
 * enable 0: off.
 * enable 1: each stage's kernels are bracketed by two events recorded on the
 *           call's stream; every stage reports, at the price of the idle time
 *           such event commands add between stages.
 * enable 2: only the blending kernels (H4D_STAGE_BLEND_FWD / _BWD) report,
 *           timed from their own dispatch (start and end of the kernel itself);
 *           nothing is added to the stream.
 * enable 3 / 4: as 2, the forward / the backward blending kernel only.
 * Any other value: H4D_ERR_INVALID_ARG. */
h4d_status h4dgs_profile(h4d_ctx *ctx, int32_t enable);
/* Waits for the recorded events and writes, per stage, the summed milliseconds
 * and the number of bracketed launches since the previous read (arrays of
 * H4D_STAGE_COUNT entries), then forgets them. */
h4d_status h4dgs_profile_read(h4d_ctx *ctx, double *ms, int64_t *launches);

/* enable != 0: later render calls use counting variants of the blending
 * kernels (slower; for measurement only).  h4dgs_stats_read synchronises
 * `stream` and reads, from the state the last forward/backward used, seven
 * counts (out: host array of at least 7):
 * out[0] (pixel, splat) evaluations of the forward blend (pixel inside the
 * splat's square, before the pixel stopped), out[1] blended ones,
 * out[2] evaluations of the backward blend, out[3] blended ones,
 * out[4] entries of the forward's tile lists ((Gaussian, tile) pairs),
 * out[5] list entries the blending traverses (each tile's list up to its last
 * contributor, summed over tiles), out[6] (Gaussian, view) records whose pixel
 * square meets the image.  out[4..6] are summed over the forward's views. */
h4d_status h4dgs_stats(h4d_ctx *ctx, int32_t enable);
h4d_status h4dgs_stats_read(h4d_ctx *ctx, const void *state, size_t state_bytes, int64_t *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* H4DGS_H */
