/*
 * gs2d.h - C ABI of the MI355X (gfx950) 2D-Gaussian frame fitter.
 *
 * The library fits N 2D Gaussians to one RGB frame, the per-frame encoding
 * loop of "Neural Video Compression using 2D Gaussian Splatting"
 * (Sec. 3.1-3.2): each Gaussian has a mean mu (2 floats), a Cholesky vector
 * l = (l1, l2, l3) with Sigma = L L^T, L = [[l1, 0], [l2, l3]] (Eq. 1), and a
 * colour c' (3 floats).  A frame is rendered by the accumulated sum of
 * Eq. 2, C(p) = sum_n c'_n exp(-q/2), q = d^T Sigma^-1 d, d = (x+1/2, y+1/2)
 * - mu, over the Gaussians with q <= 9 (3-sigma cutoff, inclusive); the
 * loop minimises the mean squared error to the target with Adam.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - All array arguments are DEVICE pointers to contiguous buffers owned by
 *    the caller; the library never allocates device memory for them and keeps
 *    no pointer after a call returns (except inside a gs2d_ctx's cached
 *    graphs, below).  Scratch space is one caller-provided workspace of
 *    gs2d_workspace_bytes() bytes (256-byte aligned).  Its contents (tile
 *    lists, status words) carry over from call to call: a caller may zero
 *    or reallocate it between calls, but writes nothing else into it.
 *  - Parameter layout (structure of arrays, FP32): xy [N][2] (x, y in pixel
 *    units, origin at the top-left corner of the frame), chol [N][3]
 *    (l1, l2, l3), rgb [N][3].  Images are planar FP32 [3][H][W].
 *  - `stream` is a hipStream_t passed as void*; NULL means the default
 *    stream.  Calls only enqueue work on it and return (results are ready
 *    when the stream reaches them) unless their comment says that they
 *    synchronise it.
 *  - Every call returns a gs2d_status and never aborts.  Invalid arguments
 *    return GS2D_EINVAL before anything is enqueued (except where a call's
 *    comment says it checks one after the work).  Conditions found on the
 *    device are reported in the workspace status word (gs2d_bins.status):
 *    bit 0 = tile-pair capacity overflow (lists truncated, no out-of-bounds
 *    write), bit 1 = at least one Gaussian culled (non-finite mean or
 *    Cholesky vector, or |l1| or |l3| < 2^-14), bit 2 = a lazy tile-list
 *    rebuild (gs2d_fit_opts.bin_skin > 0) gave up its bounded device-side
 *    wait and kept the previous lists (gs2d_fit_frame then returns
 *    GS2D_EHIP).
 *  - Limits: 1 <= W, H; 1 <= N <= 65536; tile in {8, 16, 32};
 *    ceil(W/tile) * ceil(H/tile) <= 65536; 1 <= max_pairs <= 2^30.
 */
#ifndef GS2D_H
#define GS2D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GS2D_OK = 0,
  GS2D_EINVAL = -1,    /* bad shape, NULL pointer, unsupported tile size   */
  GS2D_ENOSPACE = -2,  /* workspace smaller than gs2d_workspace_bytes()    */
  GS2D_EOVERFLOW = -3, /* tile pairs exceeded max_pairs (fit loop only)    */
  GS2D_EHIP = -4       /* a HIP runtime call failed                        */
} gs2d_status;

/* One frame's problem size.  max_pairs is the capacity of the tile-pair
 * list (pairs of (tile, Gaussian) whose 3-sigma box meets the tile).
 * px_per_lane selects the raster kernel variant: each wavefront covers an
 * 8 x (8 * px_per_lane) pixel block, i.e. tile^2 / (64 * px_per_lane)
 * wavefronts per tile; 1, 2 or 4 with 8 * px_per_lane <= tile, 0 = 1. */
typedef struct {
  int32_t W, H, N, tile, max_pairs, px_per_lane;
} gs2d_shape;

/* Device views into a workspace after gs2d_project_bin (read-only for the
 * caller).  Sorted pair keys are (tile << 16) | gaussian_index, ascending;
 * tile = ty * ceil(W/tile) + tx.  tile_start[t] is the first pair whose tile
 * is >= t (n_tiles + 1 entries).  n_pairs is min(total pairs, max_pairs). */
typedef struct {
  const float *geom;          /* [N][8] per-Gaussian derived geometry      */
  const int32_t *counts;      /* [N] tiles touched by each Gaussian        */
  const int32_t *offsets;     /* [N+1] exclusive prefix sum of counts      */
  const uint32_t *keys;       /* [max_pairs] sorted (tile, index) keys     */
  const int32_t *tile_start;  /* [n_tiles + 1]                             */
  const int32_t *n_pairs;     /* scalar                                    */
  const uint32_t *status;     /* scalar status word (bits above)           */
  const int32_t *n_culled;    /* scalar count of culled Gaussians          */
  int32_t n_tiles, tiles_x, tiles_y;
} gs2d_bins;

/* Adam hyper-parameters; lr per parameter group (0 = mean, 1 = Cholesky
 * vector, 2 = colour). */
typedef struct {
  float lr[3];
  float beta1, beta2, eps;
} gs2d_adam_cfg;

/* Bit depths of the uniform quantisers of the Cholesky vector and the colour
 * (gs2d_ptq, and quantisation-aware fitting through gs2d_fit_opts.qat). */
typedef struct gs2d_quant_cfg_s {
  int32_t bits_chol, bits_rgb;
} gs2d_quant_cfg;

typedef struct {
  int32_t iters;        /* maximum iterations                               */
  int32_t check_every;  /* iterations per launched chunk / PSNR check (>=1) */
  float psnr_target;    /* stop at the first check with PSNR >= target; <=0 off */
  int32_t use_graph;    /* 1: capture each chunk in a hipGraph and replay    */
  gs2d_adam_cfg adam;
  /* [N] device uint8 or NULL: only Gaussians with active[n] != 0 are
   * updated; the others keep their parameters and moments bit for bit and
   * their gradients are not accumulated (P-frame selective optimisation,
   * Sec. 3.2.C).  The render and the loss always use every Gaussian.
   * gs2d_fit_batch requires NULL. */
  const uint8_t *active;
  /* Host pointer or NULL: quantisation-aware fitting (Sec. 3.3.A, QAT).
   * Every iteration renders the parameters after the gs2d_ptq quantisers
   * (ranges taken from the current parameters, so they follow the fit) and
   * applies the gradients at the quantised point to the FP32 parameters
   * (straight-through estimator).  The loss trace is the quantised
   * render's.  gs2d_fit_batch and gs2d_fit_frame_static require NULL. */
  const gs2d_quant_cfg *qat;
  /* Lazy tile binning, 0 <= bin_skin <= 64 pixels; 0: the tile lists are
   * rebuilt every iteration.  With bin_skin > 0 (frames of at most 2048
   * tiles; with qat, the quantised Gaussians) each Gaussian is binned into
   * the tiles its 3-sigma box grown by bin_skin pixels meets, and the lists
   * are rebuilt only when some Gaussian's exact tile rectangle has left the
   * one it was binned with (or it became culled), and at the first
   * iteration of a call unless the workspace still holds the complete lists
   * of an earlier lazy fit of the same shape (not truncated at max_pairs,
   * and no other binning into it since; the call's parameters may differ,
   * since the test above covers them).  In between, the projection still
   * runs every iteration and the lists of the last rebuild are a superset
   * of the exact ones in the same (tile, index) order.  Every pixel's sum
   * tests each pair against the cutoff, so the render, the loss and the
   * gradients are those of exact binning.  gs2d_fit_batch applies it frame
   * by frame (a frame rebuilds its lists when one of its Gaussians has left
   * its rectangle, and at the first iteration of every call). */
  float bin_skin;
  /* gs2d_fit_batch's raster launch: 0 = one workgroup per (frame, tile)
   * item of the frame-area-ordered queue, with exact block masks (the
   * faster, default); 1 = one persistent launch of the device's resident
   * capacity whose workgroups pop the items from that queue with one
   * atomic each (box masks: the exact ones do not fit its registers).
   * Ignored by gs2d_fit_frame. */
  int32_t batch_persistent;
} gs2d_fit_opts;

typedef struct {
  int32_t iters_run;        /* iterations executed                          */
  int32_t iter_hit_target;  /* first iteration whose loss met the target, -1 */
  float final_loss;         /* MSE of the last evaluated iteration          */
  float final_psnr;
  double seconds;           /* host wall time of the call                   */
  uint32_t status;          /* OR of the status words of the tile lists used */
  int32_t n_culled;         /* culled Gaussians when the lists were built   */
  int32_t rebins;           /* lazy binning: tile-list rebuilds in the call
                               (0 if it kept the workspace's earlier lists
                               throughout); 0 without lazy binning          */
} gs2d_fit_stats;

/* Human-readable name of a status code (static string). */
const char *gs2d_status_str(int status);

/* Bytes of workspace needed for `shape`; 0 if the shape is invalid. */
size_t gs2d_workspace_bytes(const gs2d_shape *shape);

/* Fill `out` with device views into workspace `ws`.  Host-only. */
int gs2d_bins_view(const gs2d_shape *shape, void *ws, size_t ws_bytes, gs2d_bins *out);

/* Projection and tile binning (the setup a tile-based rasteriser needs,
 * Sec. 3.1, rendering of Eq. 2): per Gaussian the culling test, inverse
 * diagonal of L, the 3-sigma box (half-widths 3|l1| and 3 sqrt(l2^2+l3^2)),
 * the tile rectangle it meets and its tile count; an exclusive scan of the
 * counts; one key (tile << 16 | index) per (Gaussian, tile); a stable device
 * radix sort of the keys by tile; and the per-tile ranges.  The result is
 * bit-identical for identical inputs.  Box and rectangle are evaluated in
 * FP32 without contraction, in the order
 *   r = sqrt(l2*l2 + l3*l3); ry = 3*r; rx = 3*|l1|; xlo = mx - rx; ...
 *   tx0 = max(floor(xlo/tile), 0); tx1 = min(floor(xhi/tile), TX-1) ...
 * xy, chol: device [N][2], [N][3].  ws: workspace. */
int gs2d_project_bin(const gs2d_shape *shape, const float *xy, const float *chol,
                     void *ws, size_t ws_bytes, void *stream);

/* Forward render of Eq. 2 over the tile lists built by gs2d_project_bin
 * (which must have run on the same workspace with the same xy/chol).
 *   rgb     [N][3] colours c'.
 *   target  [3][H][W] or NULL.  With a target the call also computes the
 *           residual r = C - target, dl_dimg = 2 r / (3HW) and the MSE.
 *   img     [3][H][W] output or NULL (not written).
 *   dl_dimg [3][H][W] output or NULL; requires target.
 *   loss    device float scalar output (MSE) or NULL; requires target.
 * Pixels with no Gaussian in range render exactly 0. */
int gs2d_render_fwd(const gs2d_shape *shape, void *ws, size_t ws_bytes, const float *rgb,
                    const float *target, float *img, float *dl_dimg, float *loss,
                    void *stream);

/* Backward render: given g = dLoss/dC ([3][H][W]), the gradients of the loss
 * w.r.t. every parameter, by the chain rule through Eq. 2 and Eq. 1 with the
 * cutoff indicator held fixed:
 *   dL/dc'_k = sum_p g_k w;  with s = (g . c') w, u = L^-1 d, v = L^-T u:
 *   dL/dmu = s v;  dL/dl1 = s v1 u1;  dL/dl2 = s v2 u1;  dL/dl3 = s v2 u2.
 * g_xy [N][2], g_chol [N][3], g_rgb [N][3] are overwritten.  Per-tile partial
 * sums are reduced across the wavefront first and then added with atomics,
 * so the summation order (and the last bits) may vary between runs. */
int gs2d_render_bwd(const gs2d_shape *shape, void *ws, size_t ws_bytes, const float *rgb,
                    const float *dl_dimg, float *g_xy, float *g_chol, float *g_rgb,
                    void *stream);

/* Forward render, MSE and backward render in one pass per tile, the form the
 * fitting loop runs: Eq. 2 is an order-free sum and every Gaussian that
 * reaches a pixel is in that pixel's tile list, so each tile renders its
 * pixels, forms dL/dC = 2 (C - target) / (3HW) in registers and back-
 * propagates it without dL/dC touching memory.  Gradients (same formulas as
 * gs2d_render_bwd) are ADDED to g_xy/g_chol/g_rgb: zero them first for plain
 * gradients.  loss: device float scalar (MSE) or NULL; with NULL the call is
 * exactly one kernel launch.  Requires gs2d_project_bin on the same
 * workspace. */
int gs2d_render_fused(const gs2d_shape *shape, void *ws, size_t ws_bytes, const float *rgb,
                      const float *target, float *g_xy, float *g_chol, float *g_rgb, float *loss,
                      void *stream);

/* Number of (pixel, Gaussian) pairs inside the frame with q <= 9 (the terms
 * the sum of Eq. 2 contains) for the tile lists in `ws`, written to the
 * device uint64 *out (8-byte aligned).  Used to state the algorithmic work
 * of a render. */
int gs2d_count_pairs(const gs2d_shape *shape, void *ws, size_t ws_bytes, uint64_t *out,
                     void *stream);

/* One Adam step (Kingma & Ba, bias-corrected, eps added to sqrt(v_hat)) on
 * all 8N parameters, the optimiser of the fitting loop (Sec. 3.2, encoding
 * optimisation steps).  m, v: [8N] moments laid out as [xy 2N | chol 3N |
 * rgb 3N].  step: device int32 scalar, the number of steps taken so far;
 * the call increments it and uses the new value as t.  active: [N] uint8 or
 * NULL; a Gaussian with
 * active[n] == 0 keeps its parameters and moments bit-for-bit.
 * zero_grads != 0 clears g_* after reading them. */
int gs2d_adam_step(int32_t N, float *xy, float *chol, float *rgb, float *g_xy, float *g_chol,
                   float *g_rgb, float *m, float *v, int32_t *step, const gs2d_adam_cfg *cfg,
                   const uint8_t *active, int32_t zero_grads, void *stream);

/* P-frame selective optimisation (Sec. 3.2.C): the pixels that changed since
 * the reference frame by more than a user-defined threshold, and the
 * reference Gaussians that influence one of them; a P-frame fits only those
 * (pass `active` to gs2d_fit_frame through gs2d_fit_opts.active).  Both are
 * integer decisions taken in FP32, in this order, without contraction:
 *   pixel (x, y) changed  iff  |frame - prev| > tau on some channel;
 *   Gaussian n influences it  iff  q <= 9, with dx = (x + 1/2) - mx,
 *   dy = (y + 1/2) - my, u1 = dx / l1, u2 = (dy - l2 u1) / l3,
 *   q = u1 u1 + u2 u2 (the Gaussian's 3-sigma cutoff, as in Eq. 2).
 * xy, chol: the reference Gaussians [N][2], [N][3], which gs2d_project_bin
 *   must have binned into ws (their tile lists are the pixel-to-Gaussian
 *   mapping; culled Gaussians influence nothing).
 * frame, prev: [3][H][W] FP32, the current and the reference source frame.
 * active: [N] uint8 output, 1 for a selected Gaussian, else 0.
 * counts: nullable device int32 [2] output = {changed pixels, selected
 *   Gaussians}. */
int gs2d_select_changed(const gs2d_shape *shape, void *ws, size_t ws_bytes, const float *xy,
                        const float *chol, const float *frame, const float *prev, float tau,
                        uint8_t *active, int32_t *counts, void *stream);

/* Post-training quantisation of a frame's Gaussians and its bit count
 * (Sec. 3.3.A: distinct quantisers for mean, Cholesky vector and colour;
 * Sec. 3.3.B: vanilla entropy coding of an I-frame).  Means: IEEE binary16
 * (round to nearest even).  Cholesky components and colour channels: per
 * component a uniform min-max quantiser with bits_chol / bits_rgb bits
 * (1..12) over the frame's range, in FP32 in this order without
 * contraction: lo = min, hi = max, L = 2^b - 1, inv = L / (hi - lo) (0 if
 * hi == lo), step = (hi - lo) / L, code = clamp(rint((x - lo) inv), 0, L)
 * (ties to even), dequantised x^ = lo + code step.  Inputs must be finite.
 *   q_xy [N][2], q_chol [N][3], q_rgb [N][3]: dequantised parameters.
 *   codes (nullable) [N][8] uint16: binary16 bits of x, y, then the six codes.
 *   ranges (nullable) [6][2]: lo, hi of l1, l2, l3, r, g, b.
 *   bits (nullable) [7] double: N * H (empirical entropy of the codes, the
 *     size an ideal static entropy coder reaches) for each of the six
 *     components, then the frame total 32 N + sum + 6 * 64 (side info).
 *   ws: gs2d_ptq_workspace_bytes(N) bytes, 256-byte aligned. */
size_t gs2d_ptq_workspace_bytes(int32_t N);
int gs2d_ptq(int32_t N, const float *xy, const float *chol, const float *rgb,
             const gs2d_quant_cfg *cfg, float *q_xy, float *q_chol, float *q_rgb,
             uint16_t *codes, float *ranges, double *bits, void *ws, size_t ws_bytes,
             void *stream);

/* --------------------------------------------------------------- context --
 * Opaque host object holding the instantiated hipGraphs of fitting chunks
 * (gs2d_fit_frame / gs2d_fit_batch with use_graph), keyed by every pointer,
 * size, chunk length and Adam setting baked into them.  A video encoder fits
 * every frame of a sequence with the same buffers (Sec. 3.2: I-frames from an
 * initialisation, P-frames warm-started from the previous frame), so a chunk
 * is captured and instantiated once per sequence, not once per frame.  The
 * context belongs to one device and serves one host thread at a time; it
 * keeps at most 16 graphs (least recently used dropped) and keeps the cached
 * pointers until it is destroyed or the entry is dropped, so buffers freed
 * and reallocated at the same address are re-used by a cached graph.
 *   gs2d_ctx_create: *out = new context for `device` (GS2D_EINVAL for an
 *   invalid device; the current device is left unchanged).  It holds a
 *   capture stream and 64 bytes of pinned host memory for the status words a
 *   fitting call reads back.
 *   gs2d_ctx_destroy: frees it (NULL is ignored); no fitting call may be in
 *   flight.
 *   gs2d_ctx_stats: graphs cached now and graphs instantiated so far (each
 *   output nullable). */
typedef struct gs2d_ctx gs2d_ctx;
int gs2d_ctx_create(gs2d_ctx **out, int32_t device);
void gs2d_ctx_destroy(gs2d_ctx *ctx);
int gs2d_ctx_stats(const gs2d_ctx *ctx, int32_t *cached, int64_t *captures);

/* The whole fitting loop for one frame, the per-frame encoding of Sec. 3.2
 * (optimisation steps of the Gaussians' attributes against an L2 loss, from
 * an initialisation or the previous frame's Gaussians): repeat
 * {project+bin, forward render with fused loss and backward render in one
 * pass per tile, Adam} for opts->iters iterations or until the PSNR of an
 * evaluated iteration reaches opts->psnr_target (checked every
 * opts->check_every iterations).
 *   ctx: graph cache (nullable: graphs are then captured for this call only).
 *   target [3][H][W]; xy/chol/rgb updated in place; m, v [8N] and step as
 *   for gs2d_adam_step (continue from their contents: zero them for a cold
 *   start);
 *   loss_trace [trace_len] device floats: loss_trace[k] = MSE at the
 *   parameters before update k, k = step[0] at that iteration (entries the
 *   call does not reach are left untouched); trace_len must exceed
 *   step[0] + opts->iters (with psnr_target <= 0 this is checked when the
 *   work has run, step[0] being read only then: GS2D_EINVAL, no entry past
 *   trace_len written).
 * Work is enqueued on `stream` (NULL: the default stream) behind whatever the
 * caller enqueued before; the call waits for the stream at each PSNR check
 * (with psnr_target <= 0 only once: all chunks are enqueued back to back)
 * and returns after the work is complete.  Returns GS2D_EOVERFLOW if the
 * tile-pair capacity was exceeded (with psnr_target > 0 the loop stops at
 * the check that finds it; without a target the iterations all run),
 * GS2D_EINVAL if ctx belongs to another device. */
int gs2d_fit_frame(gs2d_ctx *ctx, const gs2d_shape *shape, const float *target, float *xy,
                   float *chol, float *rgb, float *m, float *v, int32_t *step, float *loss_trace,
                   int32_t trace_len, void *ws, size_t ws_bytes, const gs2d_fit_opts *opts,
                   gs2d_fit_stats *stats, void *stream);

/* Instantiate into ctx (required) the graphs that gs2d_fit_frame with the
 * same arguments would replay (chunks of min(check_every, iters) and of the
 * remainder iters % check_every), without launching anything, so that a
 * latency-critical loop starts with its graphs ready.  No-op without
 * use_graph. */
int gs2d_fit_prepare(gs2d_ctx *ctx, const gs2d_shape *shape, const float *target, float *xy,
                     float *chol, float *rgb, float *m, float *v, int32_t *step,
                     float *loss_trace, int32_t trace_len, void *ws, size_t ws_bytes,
                     const gs2d_fit_opts *opts);

/* One-frame autotuner: for each candidate (cand_tile[i], cand_ppl[i]) times
 * `reps` rounds of what gs2d_fit_frame runs per iteration apart from Adam
 * (projection + binning with the default pair capacity max(65536, 16 N +
 * 4 tiles), then the fused forward/loss/backward raster of Eq. 2) with HIP
 * events after one untimed round; out_ms[i] = mean milliseconds per round,
 * *best = index of the fastest.  ws must hold gs2d_workspace_bytes of every
 * candidate; grad_scratch [8N] floats receives accumulated gradients
 * (garbage).  Synchronises `stream`. */
int gs2d_autotune_frame(int32_t W, int32_t H, int32_t N, const float *target, const float *xy,
                        const float *chol, const float *rgb, int32_t n_cand,
                        const int32_t *cand_tile, const int32_t *cand_ppl, int32_t reps,
                        float *grad_scratch, void *ws, size_t ws_bytes, float *out_ms,
                        int32_t *best, void *stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * fitting loop of gs2d_fit_frame with the same arguments apart from the
 * workspace, which is a file-scope device array of
 * GS2D_STATIC_WORKSPACE_BYTES inside the library (one per device, held until
 * the process ends; enough for 1920x1080 with 30,000 Gaussians at every
 * tile size).  Returns GS2D_ENOSPACE when gs2d_workspace_bytes(shape)
 * exceeds it.  The chunks are launched directly (opts->use_graph is
 * ignored) and the call allocates no host or device memory.  Every call on a
 * device shares that device's array and leaves the last call's contents in
 * it; the call clears what must start at zero.  Calls that overlap on one
 * device (other host threads, other streams) race on the array: serialise
 * them. */
#define GS2D_STATIC_WORKSPACE_BYTES (16u << 20)
int gs2d_fit_frame_static(const gs2d_shape *shape, const float *target, float *xy, float *chol,
                          float *rgb, float *m, float *v, int32_t *step, float *loss_trace,
                          int32_t trace_len, const gs2d_fit_opts *opts, gs2d_fit_stats *stats,
                          void *stream);

/* Workspace bytes for gs2d_init_plain on a W x H frame (0 if invalid). */
size_t gs2d_init_workspace_bytes(int32_t W, int32_t H);

/* Content-aware ROI initialisation (Sec. 3.2.A: Gaussians seeded from the
 * region of interest, mean at a content location, colour from the frame),
 * in the form used for synthetic frames: centres are drawn inside the ROI
 * with probability proportional to q + b + 1, where q = floor(1024 |grad Y|)
 * (Y = R+G+B, central differences, FP32) and b = (sum_roi q) // (10 R), and
 * uniformly over the non-ROI pixels outside it.  Draw i of the ROI picks the
 * first ROI pixel (raster order) whose running weight exceeds
 * pick_roi[i] mod (total weight); outside draw j picks the
 * (pick_out[j] mod O)-th non-ROI pixel.  Each Gaussian gets
 *   mu = pixel centre + jitter,  l = (s, 0, s),
 *   s = clamp(0.5 sqrt(1 / (n_region * pmf(pixel))), 0.5, 16),
 *   c' = frame colour * 1 / (2 pi (1/4) (1 - e^-4.5)).
 * An empty ROI makes the whole frame the ROI; a full ROI makes outside draws
 * uniform over the frame.
 *   target [3][H][W] FP32, roi_mask [H][W] uint8 (non-zero = ROI);
 *   pick_* [n] int64 >= 0 and jit_* [n][2] FP32 in [-0.5, 0.5) are the random
 *   draws (caller-supplied);
 *   outputs xy [N][2], chol [N][3], rgb [N][3] with N = n_roi + n_out, ROI
 *   draws first; picked [N] int32 (nullable) receives each draw's pixel index.
 * Synchronises `stream` once (reads the region totals) before the last launch. */
int gs2d_init_plain(int32_t W, int32_t H, const float *target, const uint8_t *roi_mask,
                    int32_t n_roi, const int64_t *pick_roi, const float *jit_roi, int32_t n_out,
                    const int64_t *pick_out, const float *jit_out, float *xy, float *chol,
                    float *rgb, int32_t *picked, void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes for gs2d_init_superpixel (0 if invalid: 1 <= K <= 65536,
 * W * H <= 2^28). */
size_t gs2d_superpixel_workspace_bytes(int32_t W, int32_t H, int32_t K);

/* Superpixel ROI initialisation (Sec. 3.2.A, Fig. 2: the ROI is segmented by
 * K-means superpixels, one Gaussian per segment with the segment's centre,
 * covariance and average colour).  K-means in (x, y, colour) from K seed
 * pixels, SLIC-style:
 *   S = max(1, rint(sqrt(R / K))) with R the ROI pixel count (FP64, ties to
 *   even), w = (m / S)^2 (FP32); ROI pixel p joins the centre k minimising
 *   D = ((dr^2 + dg^2) + db^2) + w (dx^2 + dy^2)   (FP32, this order, no
 *   contraction; d = pixel - centre; pixel position = its centre)
 *   among the centres whose cell (floor(centre / S), FP32 division) is within
 *   one cell of the pixel's (x // S, y // S) on both axes, ties to the lowest
 *   k; a ROI pixel with no such centre gets label -1.  The new centres are
 *   the exact means of their pixels (FP64 from int64 sums of the pixel
 *   indices, plus 1/2, and of the colours in 1/65536 units), rounded to FP32;
 *   an empty segment keeps its centre.  Seed k starts at the centre of pixel
 *   seeds[k] with that pixel's colour rounded to 1/65536.
 * After `iters` rounds, each non-empty segment k writes
 *   xy[k] = mean + 1/2,  chol[k] = Cholesky factor of (covariance + I/12),
 *   rgb[k] = colour sum / (2 pi l1 l3 (1 - e^-4.5)),
 * evaluated in FP64 from the exact integer moments and rounded once, so the
 * Gaussian's rendered mass under the q <= 9 cutoff equals the segment's
 * colour total; an empty segment leaves xy/chol/rgb[k] as passed in.
 *   target [3][H][W] FP32 (device); roi_mask [H][W] uint8 (device, non-zero =
 *   ROI; an all-zero mask means the whole frame);
 *   seeds [K] int32 pixel indices y*W+x (device; values outside [0, W*H) are
 *   clamped into it); 1 <= iters <= 100; compactness m > 0 (finite);
 *   xy [K][2], chol [K][3], rgb [K][3] FP32 (device, in: the Gaussians empty
 *   segments keep, out: the segment Gaussians);
 *   labels [H][W] int32 (device, nullable): the last assignment, -1 outside
 *   the ROI;
 *   centres [2][5][K] FP32 (device, nullable): x, y, r, g, b of every centre
 *   before the last assignment, then after the last update.
 * Enqueued on `stream` without synchronising (no host reads). */
int gs2d_init_superpixel(int32_t W, int32_t H, const float *target, const uint8_t *roi_mask,
                         int32_t K, const int32_t *seeds, int32_t iters, float compactness,
                         float *xy, float *chol, float *rgb, int32_t *labels, float *centres,
                         void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- batches --
 * Many frames of different sizes and Gaussian counts fitted in lockstep (the
 * per-frame encoding loop of Sec. 3.2 applied to independent frames or ROI
 * crops at once).  Frame f has W x H pixels and N Gaussians; its target is
 * the f-th [3][H][W] block of the concatenated `targets`, its parameters the
 * f-th slices of the concatenated xy [sum N][2], chol [sum N][3],
 * rgb [sum N][3], and its Adam moments the matching slices of m, v laid out
 * as [xy 2*sum N | chol 3*sum N | rgb 3*sum N].  Each iteration runs the
 * per-frame binning for all frames, ONE raster launch over the (frame,
 * tile) work items, largest frames first (one workgroup per item, or with
 * gs2d_fit_opts.batch_persistent a resident grid that pulls the items
 * through an atomic counter), and one Adam launch over all parameters.  Every frame's tile
 * lists and image are those of the one-frame path.  `tile` and
 * `px_per_lane` are as in gs2d_shape and apply to all frames; each frame's
 * pair capacity is max(65536, 16 N + 4 tiles). */
typedef struct {
  int32_t W, H, N;
} gs2d_frame;

/* Workspace bytes of a batch (0 if invalid: 1 <= n_frames <= 4096, each
 * frame within the one-frame limits). */
size_t gs2d_batch_workspace_bytes(int32_t n_frames, const gs2d_frame *frames, int32_t tile,
                                  int32_t px_per_lane);

/* Fit all frames of a batch for opts->iters iterations (same rules as
 * gs2d_fit_frame, including ctx and stream; one shared step counter).
 * loss_trace is [trace_rows][n_frames]: row k holds every frame's MSE at
 * iteration k (= step value before the update).  The PSNR stop triggers when every frame has reached
 * opts->psnr_target.  `frames` is a host array. */
int gs2d_fit_batch(gs2d_ctx *ctx, int32_t n_frames, const gs2d_frame *frames, int32_t tile,
                   int32_t px_per_lane, const float *targets, float *xy, float *chol, float *rgb,
                   float *m, float *v, int32_t *step, float *loss_trace, int32_t trace_rows,
                   void *ws, size_t ws_bytes, const gs2d_fit_opts *opts, gs2d_fit_stats *stats,
                   void *stream);

/* Binning and one fused raster pass (one workgroup per item) of a batch without an
 * optimiser step: gradients of every frame's MSE are ADDED to g_* (same
 * layout as the parameters), loss_per_frame [n_frames] (nullable) receives
 * each frame's MSE.  Synchronises `stream`. */
int gs2d_batch_render_grads(int32_t n_frames, const gs2d_frame *frames, int32_t tile,
                            int32_t px_per_lane, const float *targets, const float *xy,
                            const float *chol, const float *rgb, float *g_xy, float *g_chol,
                            float *g_rgb, float *loss_per_frame, void *ws, size_t ws_bytes,
                            void *stream);

/* Device views of frame f's binning inside a batch workspace, in the
 * one-frame gs2d_bins format.  Host-only. */
int gs2d_batch_bins_view(int32_t n_frames, const gs2d_frame *frames, int32_t tile,
                         int32_t px_per_lane, int32_t f, void *ws, size_t ws_bytes,
                         gs2d_bins *out);

/* Autotuner for a batch: times `reps` rounds of batched binning + fused
 * raster (one workgroup per item) for each candidate (cand_tile[i], cand_ppl[i]) with HIP events,
 * writes the mean ms per round to out_ms[i] and the fastest index to *best.
 * ws must be large enough for every candidate; grad_scratch holds
 * 8 * sum(N) floats (overwritten with accumulated garbage gradients). */
int gs2d_autotune_batch(int32_t n_frames, const gs2d_frame *frames, const float *targets,
                        const float *xy, const float *chol, const float *rgb, int32_t n_cand,
                        const int32_t *cand_tile, const int32_t *cand_ppl, int32_t reps,
                        float *grad_scratch, void *ws, size_t ws_bytes, float *out_ms,
                        int32_t *best, void *stream);

/* --------------------------------------------------- learned initialiser --
 * A per-tile convolutional regressor standing in for the paper's Gaussian
 * attribute regressor (Sec. 3.2.B): input [H][W] frame + residual against
 * the previous frame, 4 x (conv3x3 stride 2, 64 channels, ReLU), a conv3x3
 * head with 73 channels per 16x16 tile = 9 count logits (0..8 Gaussians)
 * + 8 slots x 8 parameters (mu_x = x0 + 16 sigmoid(p0), mu_y = y0 + 16
 * sigmoid(p1), l1 = exp(p2), l2 = p3, l3 = exp(p4), colour p5..p7).  It is
 * trained with a per-tile cross-entropy on the count plus a Chamfer set loss
 * on the slots (the paper's remedy for unordered Gaussians), on Gaussians the
 * fitter produced.  BF16 weights and activations, FP32 accumulation on MFMA.
 *
 * Buffers (caller-owned, device): master FP32 weights [param_count]; BF16
 * weight copies [bf16_weight_count] (uint16); workspace
 * [cnn_workspace_bytes] holding activations, the head output, the current
 * training targets, each layer's BF16 output gradient (ReLU applied) and
 * the grad-weight partial sums.  H, W >= 16, H * W <= 2^26.  One workspace
 * serves one call at a time (calls on one stream are ordered). */
size_t gs2d_cnn_param_count(int32_t H, int32_t W);
size_t gs2d_cnn_workspace_bytes(int32_t H, int32_t W);
size_t gs2d_cnn_bf16_weight_count(int32_t H, int32_t W);
/* info[12] = {Hin, Win, Cin, Hout, Wout, Cout, stride, relu, rows, K, w_off,
 * b_off} of layer 0..4; the master weights of a layer are a [rows][K] matrix
 * at w_off with K index = tap * Cin + ci (tap = 3 ky + kx), bias at b_off. */
int gs2d_cnn_layer_info(int32_t H, int32_t W, int32_t layer, int32_t *info);
/* He-normal weights from caller-supplied N(0,1) draws [param_count]; 0 bias. */
int gs2d_cnn_init_params(int32_t H, int32_t W, const float *normal_draws, float *master,
                         void *stream);
/* Refresh the BF16 copies (forward and transposed layouts) from master. */
int gs2d_cnn_sync_weights(int32_t H, int32_t W, const float *master, uint16_t *wbf16,
                          void *stream);
/* Forward pass; frame/prev [3][H][W] FP32 (prev NULL: zero residual);
 * head_out [73][TY][TX] FP32 (nullable; the head also stays in ws). */
int gs2d_cnn_forward(int32_t H, int32_t W, const float *frame, const float *prev,
                     const float *master, const uint16_t *wbf16, float *head_out, void *ws,
                     size_t ws_bytes, void *stream);
/* Per-tile training targets from N fitted Gaussians (stored in ws): the
 * Gaussians whose centre lies in the tile, at most 8, the heaviest by
 * |l1 l3| |c'|^2 (ties to the lower index).  scratch: >= 2*4N + 4*256*G +
 * 4*(tiles+1) + 256 bytes, 256-aligned, in use until the stream reaches the
 * end of the call's work (stream-ordered, no host synchronisation). */
int gs2d_cnn_targets(int32_t H, int32_t W, int32_t N, const float *xy, const float *chol,
                     const float *rgb, void *ws, size_t ws_bytes, void *scratch,
                     size_t scratch_bytes, void *stream);
/* Copy the stored targets out: counts [tiles] int32, vectors [tiles][8][8]
 * (slot s < count: the target in loss units, else 0). */
int gs2d_cnn_read_targets(int32_t H, int32_t W, const void *ws, size_t ws_bytes, int32_t *counts,
                          float *vectors, void *stream);
/* Device view of a tensor the last forward / backward pass left in `ws`
 * (read-only; valid until the next call on that workspace), for inspecting
 * one layer at a time.  which = 0: the input activations of `layer`, BF16
 * channels-last [Hin][Win][Cin] (layer 0: the 3 colour and 3 residual
 * channels padded to 8 with zeros; layer l > 0: layer l-1's ReLU output);
 * which = 1: the gradient of the loss w.r.t. the output of `layer` with the
 * ReLU mask applied, BF16 [Hout][Wout][CoutS] (CoutS = Cout rounded up to
 * 8; the head's entry holds the loss gradient of the 73 head channels).
 * *ptr receives the device address, dims[3] = (rows, columns, channel
 * stride).  Host-only. */
int gs2d_cnn_tensor_view(int32_t H, int32_t W, int32_t layer, int32_t which, const void *ws,
                         size_t ws_bytes, const void **ptr, int32_t *dims);
/* Loss of the last forward pass against the stored targets and the backward
 * pass: weight and bias gradients are ADDED to grad [param_count];
 * loss3 (nullable) = {total, mean CE, mean Chamfer}. */
int gs2d_cnn_backward(int32_t H, int32_t W, const float *master, const uint16_t *wbf16,
                      float *grad, float *loss3, void *ws, size_t ws_bytes, void *stream);
/* Adam on the master weights (step: device int32 counter, incremented) with
 * decoupled weight decay, w <- w - lr (m_hat / (sqrt(v_hat) + 1e-8) + wd w),
 * betas (0.9, 0.999); clears grad, and writes each updated weight to its
 * BF16 copies in the same pass.  wbf16 must have been filled once by
 * gs2d_cnn_sync_weights: the zero padding of the transposed copies is not
 * rewritten here. */
int gs2d_cnn_adam(int32_t H, int32_t W, float *master, float *grad, float *m, float *v,
                  int32_t *step, float lr, float weight_decay, uint16_t *wbf16, void *stream);
/* Decode the last forward pass into N Gaussians: per tile argmax count and
 * that many slots, in tile order; kept up to N and topped up from the plain
 * initialisation plain_* [N]; the plain initialisation is used entirely when
 * fewer than N/2 Gaussians are predicted or any value is non-finite.
 * n_predicted: device int32, the number of predicted Gaussians used. */
int gs2d_cnn_decode(int32_t H, int32_t W, int32_t N, const float *plain_xy,
                    const float *plain_chol, const float *plain_rgb, float *xy, float *chol,
                    float *rgb, int32_t *n_predicted, void *ws, size_t ws_bytes, void *scratch,
                    size_t scratch_bytes, void *stream);

/* Scratch bytes of gs2d_cnn_pframe_replace (0 if invalid: 1 <= N <= 65536). */
size_t gs2d_cnn_pframe_scratch_bytes(int32_t H, int32_t W, int32_t N);

/* Learned re-initialisation of a warm-started P-frame (the regressor of
 * Sec. 3.2.B used at the P-frames of Sec. 3.2.C): the 16 x 16 tiles whose
 * mean squared residual against the previous frame exceeds tau get the
 * network's predictions in place of the warm-started Gaussians centred in
 * them.  Per tile, e = (dr*dr + dg*dg) + db*db per pixel (d = frame - prev),
 * summed over its in-frame pixels in row-major order and divided by their
 * count, in FP32 with every operation rounded once; selected iff e > tau.
 * The Gaussians whose centre lies in a selected tile (floor(mu / 16), FP32)
 * are freed, in increasing index order; the selected tiles' predictions
 * (argmax of the count logits, first maximum; slots 0..k-1; tiles in raster
 * order; decoded as gs2d_cnn_decode does) fill the freed slots in that
 * order.  Freed slots beyond the predictions keep their Gaussians and
 * predictions beyond the freed slots are dropped, so N is unchanged; if a
 * raw parameter of any used slot is not finite nothing is replaced.
 *   frame, prev [3][H][W] FP32 (device); tau >= 0 (finite);
 *   head [73][TY][TX] FP32 (device), or NULL for the head the last
 *   gs2d_cnn_forward on `ws` left there (then ws, ws_bytes are required);
 *   xy [N][2], chol [N][3], rgb [N][3] (device, in/out: the warm-started
 *   Gaussians);
 *   stats [4] int32 (device): selected tiles, freed Gaussians, predicted
 *   Gaussians, replaced Gaussians;
 *   tile_sel [TY][TX] uint8 (device, nullable): 1 for a selected tile;
 *   scratch [gs2d_cnn_pframe_scratch_bytes] (device, 256-byte aligned).
 * Enqueued on `stream` without synchronising. */
int gs2d_cnn_pframe_replace(int32_t H, int32_t W, int32_t N, const float *frame,
                            const float *prev, float tau, const float *head, float *xy,
                            float *chol, float *rgb, int32_t *stats, uint8_t *tile_sel, void *ws,
                            size_t ws_bytes, void *scratch, size_t scratch_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GS2D_H */
