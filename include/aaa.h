/*
 * aaa.h -- C ABI of the MI355X (gfx950) AAA-Gaussians rasteriser.
 *
 * Renders a cloud of anisotropic 3D Gaussians through a pinhole camera with
 * the method of "AAA-Gaussians: Anti-Aliased and Artifact-Free 3D Gaussian
 * Rendering" (arXiv 2504.12811):
 *   - every Gaussian is evaluated in 3D at its point of maximum response
 *     along the pixel's line (Sec. 3.1, Eq. 4-5);
 *   - an adaptive 3D smoothing filter with perpendicular amplitude
 *     normalisation and the training-frequency clamp (Sec. 3.2, Eq. 6-13);
 *   - view-space angular bounding that survives Gaussians crossing the
 *     camera plane (Sec. 3.3, Eq. 14-17) and a camera-inside discard;
 *   - 3D frustum culling of each (Gaussian, tile) pair and of the whole view
 *     (Sec. 3.4, Eq. 18);
 *   - hierarchical ordering: tiles sorted by a per-tile 3D depth, then a
 *     bounded per-ray window (Sec. 3.1 "Blending Sort Order", Sec. 4);
 *   - front-to-back alpha blending with early termination.
 *
 * Conventions shared by every entry point:
 *   - Arrays marked DEVICE are device memory on the context's GPU, owned by
 *     the caller; the library never frees or retains them past the call's
 *     stream work.  Structs passed by pointer are host memory, read during
 *     the call only.
 *   - Scene arrays are float32 structure-of-arrays (index [k][i] is element
 *     k*n + i).  Images are float32 planar: rgb [3][H][W], T [H][W].
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued on it; calls return after enqueueing, except where noted.
 *   - Every call returns an aaa_status.  On failure nothing was enqueued
 *     unless the status is AAA_ERR_HIP; aaa_last_error() gives a message
 *     (thread-local, valid until the next call on the same thread).
 *   - A context, a workspace or a scene is used by one call at a time; calls
 *     on different contexts/workspaces may overlap.
 */
#ifndef AAA_H
#define AAA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AAA_OK = 0,
    AAA_ERR_INVALID = 1,        /* bad argument (NULL, size, degree) */
    AAA_ERR_WORKSPACE = 2,      /* workspace smaller than aaa_workspace_size() */
    AAA_ERR_PAIR_OVERFLOW = 3,  /* more (Gaussian, tile) pairs than max_pairs; stats->pairs holds the need */
    AAA_ERR_HIP = 4,            /* a HIP runtime call failed */
    AAA_ERR_UNSUPPORTED = 5     /* e.g. sh_degree > 3 */
} aaa_status;

/* Scene (Sec. 3.1): mean mu, log-scale (s = exp), rotation quaternion
 * (w,x,y,z; normalised inside), opacity logit (alpha = sigmoid), real
 * spherical-harmonic colour coefficients of degree <= 3 (colour =
 * max(0, 0.5 + sum Y_lm(d) c_lm), d = unit camera->mean direction), and the
 * per-Gaussian maximum training sampling frequency v_train of Sec. 3.2
 * (Eq. 6, 13) in pixels per world unit (NULL: no clamp).  All DEVICE. */
typedef struct {
    int64_t n;
    int32_t sh_degree;
    int32_t _pad;
    const float *means;          /* [3][n] */
    const float *log_scales;     /* [3][n] */
    const float *quats;          /* [4][n] */
    const float *opacity_logits; /* [n] */
    const float *sh;             /* [(sh_degree+1)^2][3][n] */
    const float *v_train;        /* [n] or NULL; values > 0, +inf allowed */
} aaa_scene;

/* Gradients, same layouts as aaa_scene; DEVICE; accumulated (+=). */
typedef struct {
    float *means;
    float *log_scales;
    float *quats;
    float *opacity_logits;
    float *sh;
} aaa_scene_grad;

/* Pinhole camera (Sec. 3.1: viewport * projection * view).  viewmat is the
 * rigid world->view matrix, row-major, view axes +x right, +y down, +z
 * forward; pixel (i, j) has centre (i + 0.5, j + 0.5); screen x = cx + fx X/Z.
 * znear: smallest depth of a contributing maximum (pixels only blend a
 * Gaussian whose maximum along the line lies at depth >= znear).  Host. */
typedef struct {
    double viewmat[16];
    double fx, fy, cx, cy;
    int32_t width, height;
    double znear;
    double bg[3];
} aaa_camera;

#define AAA_FILTER_OFF 1u      /* no 3D smoothing filter (alpha~ = alpha) */
#define AAA_FILTER_VOLUME 2u   /* volume-normalised amplitude (Eq. 7-8) instead of Eq. 12 */
#define AAA_NO_TILE_CULL 4u    /* keep every tile of the bounding rectangle (no Eq. 18 per tile) */
#define AAA_STATS 8u           /* count evaluations / contributors (small overhead) */
#define AAA_TIMING 16u         /* time each stage with HIP events on `stream` (see aaa_stage_times) */
#define AAA_LONG_ALL 32u       /* diagnostic: every tile takes the long-list blend path (same results) */
#define AAA_WIDE_RANKS 64u     /* diagnostic: the backward replay keeps 32-bit contributor ranks (same results) */
/* The middle level of the hierarchical sort (Sec. 3.1, blending sort order;
 * Sec. 4): every 8x8 sub-tile gets its own list, holding the Gaussians whose
 * screen box reaches it (sub-tile culling), in the exact order of their depth
 * of maximum response on the sub-tile-centre line (ties by index), before the
 * per-ray window.  Without it the tile's list is ordered by the depth on the
 * tile-centre line.  Keys carry the sub-tile number 4 tile + q (q = 2 qy +
 * qx); the long-list route is not taken. */
#define AAA_SUBTILE_SORT 128u

/* Method settings.  filter_k: filter size k (0.3 in Sec. 4).  ray_window:
 * capacity K of the per-ray re-sort window (0 = blend in tile order; the
 * supported values are 0, 1, 2, 4, 8, 16, 32).  alpha_min: contribution
 * threshold (a Gaussian contributes to a pixel iff min(alpha_max, alpha~
 * exp(-rho^2/2)) >= alpha_min); alpha_max: opacity clamp, below 1 also
 * after rounding to float (the backward divides by 1 - alpha; 0.99 in the
 * 3DGS lineage); t_min: blending stops before the first entry that would
 * take transmittance below t_min.  Calls reject settings outside
 * 0 < alpha_min < alpha_max < 1, 0 <= t_min < 1 with AAA_ERR_INVALID.
 * Host. */
typedef struct {
    double filter_k;
    int32_t ray_window;
    uint32_t flags;
    double alpha_min, alpha_max, t_min;
} aaa_settings;

/* Per-frame counters, host. */
typedef struct {
    uint64_t pairs;          /* (Gaussian, tile) pairs after culling */
    uint64_t visible;        /* Gaussians that survived preprocessing */
    uint64_t evaluations;    /* pixel x list-entry evaluations (AAA_STATS) */
    uint64_t contributors;   /* evaluations that passed the contribution test (AAA_STATS) */
    uint64_t candidate_tiles;/* tile tests executed by the pair emitter (AAA_STATS) */
    uint64_t near;           /* evaluations that passed the rho^2 prefilter (AAA_STATS) */
    uint64_t wave_steps;     /* list entries visited by 64-pixel wavefronts of the blend (AAA_STATS) */
    uint64_t wave_near_steps;    /* ... of which some pixel passed the prefilter (AAA_STATS) */
    uint64_t wave_contrib_steps; /* ... of which some pixel had a contribution (AAA_STATS) */
} aaa_stats;

/* Stages timed under AAA_TIMING, in launch order. */
enum {
    AAA_STAGE_PREPROCESS = 0, AAA_STAGE_COUNT = 1, AAA_STAGE_SCAN = 2, AAA_STAGE_WRITE = 3, AAA_STAGE_SORT = 4,
    AAA_STAGE_RANGES = 5, AAA_STAGE_BLEND = 6, AAA_STAGE_FRAME = 7, AAA_NUM_STAGES = 8
};

typedef struct aaa_ctx aaa_ctx;

/* Create a context on HIP device `device` (makes it current on this thread). */
int aaa_create(aaa_ctx **out, int device);
void aaa_destroy(aaa_ctx *ctx);
const char *aaa_last_error(void);
/* Library version string, static storage. */
const char *aaa_version(void);

/* Bytes of workspace needed to render `scene` through `cam` with room for
 * max_pairs (Gaussian, tile) pairs and 8 * max_pairs candidate tile tests
 * (the tiles of the Gaussians' screen rectangles).  Host-only computation. */
int aaa_workspace_size(const aaa_scene *scene, const aaa_camera *cam, const aaa_settings *settings,
                       uint64_t max_pairs, size_t *bytes_out);

/* Render one view.  out_rgb [3][H][W] = blended colour + T * bg,
 * out_T [H][W] = final transmittance (DEVICE, written).  The workspace
 * (DEVICE, >= aaa_workspace_size bytes, 256-byte aligned) keeps the frame's
 * per-Gaussian records, sorted pairs and per-pixel state until it is used
 * again; aaa_render_backward reads them.  The call synchronises `stream`
 * once to learn the pair count; on AAA_ERR_PAIR_OVERFLOW stats->pairs is the
 * max_pairs needed (the pair count, or an eighth of the candidate tile tests
 * when that is larger: a workspace holds the tests of 8 per pair) and the
 * outputs are not written.  stats (host) may be NULL. */
int aaa_render(aaa_ctx *ctx, const aaa_scene *scene, const aaa_camera *cam, const aaa_settings *settings,
               void *ws, size_t ws_bytes, uint64_t max_pairs, void *stream, float *out_rgb, float *out_T,
               aaa_stats *stats);

/* Gradient of a scalar loss L given dL/d(out_rgb) [3][H][W] (DEVICE) for the
 * last aaa_render into `ws` with the same scene, camera and settings; out_rgb
 * is that render's output (DEVICE, read).  Accumulates (+=) into `grad`
 * (DEVICE arrays, same layouts as the scene; any pointer may be NULL to skip
 * it).  The blend state is recomputed per tile from the stored sorted pairs
 * (no per-pixel lists are kept by the forward).  `scratch` (DEVICE, 256-byte
 * aligned) holds 8-byte slots, for each 8x8 pixel quadrant of each tile 64
 * per contributor of the quadrant's busiest pixel in the forward; its size
 * comes from aaa_backward_scratch_size and it needs no clearing.  Decisions (culls, thresholds,
 * the window order, the alpha clamp, min(v_train, v), the colour clamp) are
 * held fixed; their gradients are zero or one-sided.  The forward state is
 * left intact (backward may be called again).  Synchronises `stream`. */
int aaa_render_backward(aaa_ctx *ctx, const aaa_scene *scene, const aaa_camera *cam, const aaa_settings *settings,
                        void *ws, size_t ws_bytes, uint64_t max_pairs, void *stream, const float *out_rgb,
                        const float *dL_drgb, void *scratch, size_t scratch_bytes, aaa_scene_grad *grad);

/* Bytes of backward scratch for the last render into `ws` (single view:
 * n_views = 1, cams = &cam).  Runs a scan on `stream` and synchronises it. */
int aaa_backward_scratch_size(aaa_ctx *ctx, const aaa_scene *scene, int n_views, const aaa_camera *cams,
                              const aaa_settings *settings, void *ws, size_t ws_bytes, uint64_t max_pairs,
                              void *stream, size_t *bytes_out);

/* ---- batches of views (serving, multi-view steps) ---------------------- */

/* A batch renders n_views (1..256) views of the same resident scene in one
 * sequence of launches: the per-Gaussian stages run over (Gaussian, view)
 * items, the sort key carries a global tile index across views, and the
 * blend covers every view's tiles.  Each view's image is bit-identical to
 * rendering that view alone.  cams: host array [n_views]; out_rgb, out_T:
 * host arrays of n_views DEVICE pointers.  n * n_views must be < 2^32.  The
 * single-view calls above are the batch of one view. */
int aaa_workspace_size_batch(const aaa_scene *scene, int n_views, const aaa_camera *cams,
                             const aaa_settings *settings, uint64_t max_pairs, size_t *bytes_out);
int aaa_render_batch(aaa_ctx *ctx, const aaa_scene *scene, int n_views, const aaa_camera *cams,
                     const aaa_settings *settings, void *ws, size_t ws_bytes, uint64_t max_pairs, void *stream,
                     float *const *out_rgb, float *const *out_T, aaa_stats *stats);
/* Backward of the last aaa_render_batch into `ws`: the gradient of
 * sum_v sum(dL_drgb[v] * out_rgb[v]) accumulated (+=) into `grad`
 * (a multi-view training step).  Synchronises `stream` before returning. */
int aaa_render_backward_batch(aaa_ctx *ctx, const aaa_scene *scene, int n_views, const aaa_camera *cams,
                              const aaa_settings *settings, void *ws, size_t ws_bytes, uint64_t max_pairs,
                              void *stream, const float *const *out_rgb, const float *const *dL_drgb,
                              void *scratch, size_t scratch_bytes, aaa_scene_grad *grad);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): aaa_render_backward
 * without the caller's `scratch`.  The per-contributor slots live in a static
 * device array of AAA_STATIC_SLOT_BYTES (64 MiB) per device, held from the
 * library's first use on that device until the process ends; the call
 * allocates nothing.  A frame whose slots exceed it (8 bytes x 64 per
 * contributor of each 8x8 quadrant's busiest pixel: about 128x128 pixels with
 * tens of contributors per pixel fit) returns AAA_ERR_WORKSPACE and computes
 * nothing.  The slots need no clearing (each one read is written first in the
 * same call).  All calls on one device share the array: within a process the
 * library runs them one at a time (the call returns after synchronising
 * `stream`); anything else that used the array concurrently would race.
 * Arguments, results and errors otherwise as aaa_render_backward. */
#define AAA_STATIC_SLOT_BYTES (64ull << 20)
int aaa_render_backward_noalloc(aaa_ctx *ctx, const aaa_scene *scene, const aaa_camera *cam,
                                const aaa_settings *settings, void *ws, size_t ws_bytes, uint64_t max_pairs,
                                void *stream, const float *out_rgb, const float *dL_drgb, aaa_scene_grad *grad);

/* Accumulated stage times (milliseconds, HIP events on the render stream) of
 * every aaa_render with AAA_TIMING since the last reset, and the number of
 * such frames.  Waits for the last timed frame to finish.  ms [AAA_NUM_STAGES]
 * (host); the last entry is the whole frame (first to last kernel).  reset != 0
 * clears the totals after reading. */
int aaa_stage_times(aaa_ctx *ctx, double *ms, uint64_t *frames, int reset);

/* ---- stage outputs of the last aaa_render into `ws` (for checks) ------ */

/* Per-Gaussian preprocessing results (DEVICE outputs, each may be NULL):
 * status [n] (0 visible, 1 invalid input, 2 alpha~ < alpha_min, 3 camera
 * inside the level set, 4 outside the view / empty bounds), alpha_t [n]
 * (filtered opacity alpha~), tau [n] (rho^2 level where alpha~ exp(-rho^2/2)
 * = alpha_min), color [3][n], rect [4][n] (tile rectangle tx0, tx1, ty0,
 * ty1, half-open). */
int aaa_read_gaussians(const aaa_scene *scene, const aaa_camera *cam, uint64_t max_pairs, const void *ws,
                       size_t ws_bytes, void *stream, int32_t *status, float *alpha_t, float *tau, float *color,
                       int32_t *rect);

/* Sorted pairs of the last frame: keys [pairs] (tile id << 32 | order key of
 * the tile depth), values [pairs] (Gaussian index), and tile ranges
 * [tiles][2] (start, end).  DEVICE outputs sized by the caller (cap pairs);
 * *n_pairs (host) receives the count.  Synchronises `stream`. */
int aaa_read_pairs(const aaa_scene *scene, const aaa_camera *cam, uint64_t max_pairs, const void *ws,
                   size_t ws_bytes, void *stream, uint64_t *keys, uint32_t *values, uint32_t *ranges, uint64_t cap,
                   uint64_t *n_pairs);

/* Stable LSD radix sort of (key, value) pairs by the low `key_bits` bits of
 * the keys (1..64), in place (DEVICE arrays of n).  tmp: DEVICE scratch of
 * aaa_sort_tmp_size(n) bytes. */
int aaa_sort_tmp_size(uint64_t n, size_t *bytes_out);
int aaa_sort_pairs(uint64_t *keys, uint32_t *values, uint64_t n, int key_bits, void *tmp, size_t tmp_bytes,
                   void *stream);

/* ---- training sampling frequency (K7) ---------------------------------- */

#define AAA_MAX_TRAIN_CAMERAS 4096

/* The 3D smoothing filter's stored per-Gaussian frequency (Sec. 3.2: the
 * maximum of f / d over the N_c training cameras, f the focal length in
 * pixels, d the view-space depth of the mean; Eq. 13 clamps the render-time
 * frequency to it).  A camera counts when the mean lies in front of its near
 * plane and projects inside the image (border included); when no camera sees
 * the mean, every camera with the mean in front of the near plane counts;
 * with none of those the value is +inf (no clamp).  f = fx.
 * means: [3][n] DEVICE float32 (read).  cams: HOST array of n_cams
 * (0..AAA_MAX_TRAIN_CAMERAS) cameras; viewmat, fx, fy, cx, cy, width, height
 * and znear are used.  v_train: [n] DEVICE float32, written (it may be passed
 * as aaa_scene.v_train afterwards).  FP64 with a fixed operation order and no
 * fused multiply-add, rounded to float once, so the result is reproducible
 * bit for bit.  The camera table goes through the context's pinned staging;
 * the call synchronises `stream`.  Errors: AAA_ERR_INVALID for null pointers,
 * n < 0, too many cameras or an invalid camera. */
int aaa_training_frequency(aaa_ctx *ctx, const float *means, int64_t n, const aaa_camera *cams, int n_cams,
                           void *stream, float *v_train);

/* ---- optimiser step of a training step ---------------------------------- */

/* Adam with bias correction (Kingma & Ba, Algorithm 1), in place on n float32
 * parameters (DEVICE arrays param, m, v updated; grad read):
 *   m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
 *   param -= lr (m / c1) / (sqrt(v / c2) + eps),  c1 = 1 - b1^step,
 *   c2 = 1 - b2^step (c1, c2, 1 - b1 and 1 - b2 computed in double on the host,
 *   then applied in float).
 * step counts from 1.  Enqueued on `stream` (no synchronisation).  Errors:
 * AAA_ERR_INVALID for n < 0, null arrays, step < 1, betas outside [0, 1)
 * or eps <= 0. */
int aaa_adam_step(float *param, const float *grad, float *m, float *v, int64_t n, int64_t step, double lr, double beta1,
                  double beta2, double eps, void *stream);

/* ---- machine rates (for roofline fractions) ----------------------------- */

/* Measures, on `stream`, the device's FP32 fused multiply-add rate (non-packed;
 * out[0], TFLOP/s at 2 flops per FMA), its v_exp_f32 rate (out[1], G/s) and
 * its copy bandwidth (out[2], GB/s counting bytes read plus written, a copy
 * between the two halves of `buf`), each the best of `reps` timed runs after
 * one warm-up, with HIP events.  buf: DEVICE scratch of `bytes` (>= 1 MiB,
 * 256-byte aligned; ~1 GiB gives a steady copy rate), overwritten.
 * Synchronises `stream`.  Errors: AAA_ERR_INVALID for bad arguments,
 * AAA_ERR_HIP. */
int aaa_measure_peaks(void *buf, size_t bytes, int reps, void *stream, double *out);

#ifdef __cplusplus
}
#endif

#endif /* AAA_H */
