/*
 * latentam.h -- C ABI of the MI355X (gfx950) library for the hot path of
 * LatentAM online map optimisation (arXiv 2602.12314):
 *
 *   render_forward   Q = R_f(G, T)                       Sec. III-B, Eq. 4 (blend of Eq. 2)
 *   render_backward  dL/dQ -> dL/d(means, log-scales, quaternions, opacity logits, queries)
 *   render_rgbd_*    the same with colour and depth rendered in the pass     Sec. III-A, Eq. 2
 *   rgbd_l1_loss     the L1 colour and depth terms of the mapping objective   Eq. 7-9
 *   ssim_loss        the SSIM term of the photometric loss                    Eq. 7
 *   decode_loss      F = softmax(Q K^T / sqrt(d)) V, L = mean(1 - cos(F, T)) + lambda ||K - K0||^2,
 *                    and dL/dQ, dL/dK, dL/dV                    Sec. III-B, Eq. 5 and Eq. 6
 *   decode_forward   F alone (inference form of Eq. 5)
 *   decode_backward  the adjoint of decode_forward for a given dL/dF
 *   decode_tied_loss the tied decode and full feature loss as printed   Eq. 5-6
 *   stream_kmeans    dictionary initialisation by streaming K-means     Sec. III-D, Eq. 10
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every call takes a context (lam_ctx, below) made by lam_create for one
 *   HIP device; the calls that launch work must be made with that device
 *   current, otherwise they return LAM_ERR_INVALID_ARG.  The host-only size
 *   queries (*_workspace_size, lam_render_debug_views) also accept NULL,
 *   which stands for a context with the default options.  The context holds
 *   the launch choices (tile schedule, decode block shape, split counts);
 *   they change the speed, never the result beyond the rounding order noted
 *   per option.  Two contexts in one process are independent.
 * - Pointers named as "device" are HIP device pointers; "host" pointers are
 *   read synchronously before the call returns.  Every device buffer belongs
 *   to the caller.  The library performs no device allocation on these paths:
 *   scratch and the state the backward pass needs live in a caller-owned
 *   workspace whose size the *_workspace_size functions report.
 * - All arrays are float32, C-contiguous (row-major).  The row arrays read or
 *   written with 16-byte vector accesses (queries, Q, dQ, target, F, dF) must
 *   be 16-byte aligned; misaligned pointers give LAM_ERR_INVALID_ARG.
 * - ``stream`` is a hipStream_t (NULL = the null stream).  Calls only enqueue
 *   work on it and return; there is no host synchronisation except in the
 *   functions documented as blocking.  Nothing is allocated or freed, and no
 *   memset node is recorded, so the non-blocking calls can be captured into a
 *   HIP graph.
 * - Errors are status codes; nothing is thrown across the ABI.  Invalid
 *   arguments are rejected on the host before any work is enqueued.
 *
 * Gaussians (paper Eq. 1 and Eq. 3): position p (means[N,3]), orientation as
 * a quaternion (quats[N,4], w x y z, any non-zero norm), scale through its
 * logarithm (log_scales[N,3]), opacity through its logit (opacity_logits[N];
 * opacity = sigmoid(logit)), and the compact query vector f_i
 * (queries[N,d], d in {16, 32}).
 *
 * Cameras: host array of n_cams rows of LAM_CAM_FLOATS floats
 *   [width, height, fx, fy, cx, cy, viewmat[16]]
 * with viewmat the row-major 4x4 world->camera transform (x right, y down,
 * z forward).  Pixels sit at integer coordinates.  Views are concatenated in
 * camera order, each row-major, so pixel arrays have P = sum(width*height)
 * rows.  1 <= n_cams <= LAM_MAX_CAMS, 1 <= width, height <= 8192.
 *
 * Rendering follows 3D Gaussian Splatting, which the paper cites for its
 * depth-ordered alpha blending (Eq. 2): EWA projection with a 0.3 px^2
 * dilation, near plane 0.2, 3-sigma square footprint, alpha = min(0.99,
 * o exp(power)), pairs with alpha < 1/255 skipped, blending stops before the
 * transmittance would drop below 1e-4.  Gaussians are ordered per pixel by the
 * float32 camera-space depth of their centre, ties by index; a Gaussian is
 * blended into exactly the pixels inside its footprint, so the result does not
 * depend on the tile shape.
 */
#ifndef LATENTAM_H
#define LATENTAM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LAM_CAM_FLOATS 22
#define LAM_MAX_CAMS 16
#define LAM_VERSION 2
/* bytes of the static per-GPU scratch of lam_decode_forward_noalloc (8 MiB) */
#define LAM_NOALLOC_SCRATCH_BYTES (8u << 20)

typedef enum {
    LAM_OK = 0,
    LAM_ERR_INVALID_ARG = -1, /* null pointer, negative size, workspace too small, ... */
    LAM_ERR_UNSUPPORTED = -2, /* shape outside the supported set (listed per call) */
    LAM_ERR_CAPACITY = -3,    /* reported by lam_render_counters when instances overflowed */
    LAM_ERR_HIP = -4          /* a HIP runtime call failed (launch error, bad stream) */
} lam_status;

typedef enum {
    LAM_FP32 = 0,     /* all products in float32 (MFMA f32) */
    LAM_BF16 = 1,     /* products on bf16 operands, float32 accumulation and softmax */
    LAM_FP8_E4M3 = 2  /* the forward product P V on OCP E4M3 operands: V in E4M3 with a
                         float32 scale per atom (row); the unnormalised softmax weights
                         (which peak at 1 per pixel) times the atom scales, mapped onto
                         the E4M3 range by one factor per call, enter as two E4M3 terms
                         (the rounded value and the rounded residual), so F carries the
                         rounding of V only; the logits Q K^T and every backward product
                         in bf16; float32 accumulation and softmax.  On the 1200x680
                         keyframe of a 2M-Gaussian map (M = D = 1024) the smallest
                         per-pixel cosine of F against exact arithmetic is 0.99966 and
                         dQ, dK, dV are within 1e-2 (relative L2); with a sharper
                         softmax (unit-variance logits) dQ grows to 1-2e-2 */
} lam_precision;

/* Human-readable name of a status code (static storage). */
const char* lam_status_string(int status);

/* Library ABI version (LAM_VERSION). */
int lam_version(void);

/* ----------------------------------------------------------------- context */

typedef struct lam_ctx lam_ctx;

/* Makes a context for HIP device ``device``.  ``options_json`` (nullable) is
 * a flat JSON object of integer options, as an autotuner writes it:
 *   "raster_schedule"  how the compositing kernels walk the tiles:
 *                      0 = one workgroup per tile; 1 = persistent: as many
 *                      workgroups as fit on the device take tiles from a
 *                      counter in the workspace (evens out views of uneven
 *                      size and tiles of uneven list length); 2 = persistent
 *                      only when several cameras are rendered (default 2).
 *                      Results are identical in every mode.
 *   "decode_shape"     workgroup shape of the per-pixel decode kernel:
 *                      0 = 32 pixels with 4 waves (default); 1 = 64 pixels
 *                      with 8 waves, each V fragment feeding two pixel groups
 *                      (BF16 and E4M3 with D a multiple of 256 up to 1024;
 *                      other shapes keep 0).  Results agree to rounding
 *                      (the per-pixel sums over the waves split differently).
 *   "decode_splits"    pixel-range splits of the dV GEMM (the larger of the
 *                      two dictionary-gradient GEMMs; a multiple of 8 in
 *                      [8, 4096], capped at the number of 32-pixel blocks);
 *                      0 = sized to fill the device (default).  dV agrees to
 *                      rounding (the split sums differ); the workspace size
 *                      depends on it.
 * The context queries the device (compute units, occupancy of the persistent
 * kernels) and creates one event; it allocates no device memory.
 * Errors: LAM_ERR_INVALID_ARG (null out, bad device, unknown option or value
 * out of range: checked before the device is touched), LAM_ERR_HIP. */
lam_status lam_create(int device, const char* options_json, lam_ctx** out);

/* Releases a context (NULL is a no-op).  Work it launched must be complete. */
void lam_destroy(lam_ctx* ctx);

/* Changes options of a live context (same JSON as lam_create; fields not
 * named keep their values).  A call already made keeps the options it read;
 * a workspace sized before a change of "decode_splits" may be too small
 * afterwards (the calls then return LAM_ERR_INVALID_ARG).
 * Errors: LAM_ERR_INVALID_ARG (null, unknown option, value out of range). */
lam_status lam_ctx_configure(lam_ctx* ctx, const char* options_json);

/* Reads one option (or "device") of a context.  Errors: LAM_ERR_INVALID_ARG. */
lam_status lam_ctx_get(const lam_ctx* ctx, const char* key, int* value);

/* ------------------------------------------------------------------ render */

/* Bytes of workspace for rendering n_gauss Gaussians with query dimension d
 * into the given cameras with tile_w x tile_h tiles (tile_w * tile_h in
 * {64, 128, 256}, both powers of two) and room for ``instance_capacity``
 * (Gaussian, tile) pairs.  Host-only, never blocks.
 * Errors: LAM_ERR_INVALID_ARG (null out, bad camera rows), LAM_ERR_UNSUPPORTED
 * (tile shape, d, 2^30 or more Gaussian-camera records or pairs of capacity). */
lam_status lam_render_workspace_size(const lam_ctx* ctx, int n_gauss, int d, const float* cams, int n_cams,
                                     int tile_w, int tile_h, uint64_t instance_capacity,
                                     uint64_t* bytes);

/* Forward render of the query map (Eq. 4): projects every (camera, Gaussian)
 * record, bins it to the tiles its footprint touches, sorts each tile's list
 * by depth and blends front to back.
 *   Q        device [P, d]  out: rendered queries
 *   T_final  device [P]     out: transmittance left after blending
 *   ws       device, ws_bytes >= lam_render_workspace_size(...); it keeps the
 *            projected records, sorted tile lists and per-pixel state that
 *            lam_render_backward reads, so it must stay untouched between the
 *            two calls.
 * If the (Gaussian, tile) pairs exceed instance_capacity, the overflow flag in
 * the workspace is set and Q is incomplete: read it with lam_render_counters
 * and call again with a larger workspace.
 * Errors: LAM_ERR_INVALID_ARG, LAM_ERR_UNSUPPORTED, LAM_ERR_HIP. */
lam_status lam_render_forward(lam_ctx* ctx, const float* means, const float* log_scales, const float* quats,
                              const float* opacity_logits, const float* queries, int n_gauss,
                              int d, const float* cams, int n_cams, int tile_w, int tile_h,
                              float* Q, float* T_final, void* ws, uint64_t ws_bytes,
                              uint64_t instance_capacity, void* stream);

/* Backward of lam_render_forward for the upstream gradient dQ (device [P, d]).
 * Transmittance is rebuilt from T_final in reverse order.  Writes (overwrites)
 * the gradients with respect to the raw parameters:
 *   d_means [N,3], d_log_scales [N,3], d_quats [N,4], d_opacity_logits [N],
 *   d_queries [N,d]   (all device).
 * Gaussians culled in every camera get zero gradients.  Arguments other than
 * dQ and the outputs must equal those of the forward call, with the same ws.
 * Errors: LAM_ERR_INVALID_ARG, LAM_ERR_UNSUPPORTED, LAM_ERR_HIP. */
lam_status lam_render_backward(lam_ctx* ctx, const float* means, const float* log_scales, const float* quats,
                               const float* opacity_logits, const float* queries, int n_gauss,
                               int d, const float* cams, int n_cams, int tile_w, int tile_h,
                               const float* dQ, float* d_means, float* d_log_scales,
                               float* d_quats, float* d_opacity_logits, float* d_queries,
                               void* ws, uint64_t ws_bytes, uint64_t instance_capacity,
                               void* stream);

/* Colour and depth rendering (Sec. III-A: view-independent colour c_i blended
 * by Eq. 2; depth blended with the same weights from the camera-space depth
 * of each Gaussian's centre) in the same pass as the query map.  Arguments as
 * lam_render_forward / lam_render_backward plus: colors [N, 3] (device,
 * float32), rgb [P, 3] and depth [P] (device outputs, overwritten); in the
 * backward d_rgb [P, 3] and d_depth [P] (upstream gradients) and d_colors
 * [N, 3] (output, overwritten).  The depth gradient reaches the means through
 * the third row of each view's world->camera transform.  The workspace is the
 * one lam_render_workspace_size reports; the backward reads what the forward
 * of the same call sequence left in it.
 * Errors: LAM_ERR_INVALID_ARG, LAM_ERR_UNSUPPORTED, LAM_ERR_HIP. */
lam_status lam_render_rgbd_forward(lam_ctx* ctx, const float* means, const float* log_scales, const float* quats,
                                   const float* opacity_logits, const float* queries, const float* colors,
                                   int n_gauss, int d, const float* cams, int n_cams, int tile_w, int tile_h,
                                   float* Q, float* rgb, float* depth, float* T_final, void* ws,
                                   uint64_t ws_bytes, uint64_t instance_capacity, void* stream);
lam_status lam_render_rgbd_backward(lam_ctx* ctx, const float* means, const float* log_scales, const float* quats,
                                    const float* opacity_logits, const float* queries, const float* colors,
                                    int n_gauss, int d, const float* cams, int n_cams, int tile_w, int tile_h,
                                    const float* dQ, const float* d_rgb, const float* d_depth, float* d_means,
                                    float* d_log_scales, float* d_quats, float* d_opacity_logits,
                                    float* d_queries, float* d_colors, void* ws, uint64_t ws_bytes,
                                    uint64_t instance_capacity, void* stream);

/* The L1 terms of the mapping objective (Eq. 7-9):
 *   L = lambda_rgb mean_{p,c} |rgb - rgb_obs| + lambda_depth mean_{p: depth_obs > 0} |depth - depth_obs|
 * (an observed depth <= 0 marks a pixel without a measurement; with none the
 * depth term is zero) and dL/drgb, dL/ddepth (the sign, zero at a tie).  The
 * paper's weights: lambda_I1 = 0.2 (times lambda_rgb) and lambda_d = 0.1; its
 * SSIM term is lam_ssim_loss.  Device arrays: rgb, rgb_obs [n, 3], depth,
 * depth_obs [n]; outputs loss [1], d_rgb [n, 3], d_depth [n] (overwritten).
 * Workspace: lam_rgbd_l1_workspace_size bytes.  Deterministic.
 * Errors: LAM_ERR_INVALID_ARG (null pointers, n < 0, a negative weight,
 * workspace too small), LAM_ERR_HIP. */
/* The SSIM term of Eq. 7, read as 3D Gaussian Splatting's: structural
 * similarity per colour channel with an 11 x 11 Gaussian window (standard
 * deviation 1.5, normalised), C1 = 0.01^2, C2 = 0.03^2, zero padding at the
 * border, every view its own image (cams: host camera rows as for the render
 * calls; only width and height are read; rgb rows are the views concatenated,
 * each row-major):
 *   loss = lambda (1 - mean over pixels and channels of SSIM(rgb, rgb_obs))
 * and lambda dSSIM-loss/drgb, written to d_rgb [P, 3] (added to it when
 * accumulate is non-zero, so it can follow lam_rgbd_l1_loss).  The paper's
 * weight: lambda_I2 = 0.8 (times lambda_rgb).  Workspace:
 * lam_ssim_workspace_size bytes (9 floats per pixel).  Deterministic.
 * Errors: LAM_ERR_INVALID_ARG (null pointers, bad camera rows, negative
 * lambda, workspace too small), LAM_ERR_HIP. */
lam_status lam_ssim_workspace_size(const lam_ctx* ctx, const float* cams, int n_cams, uint64_t* bytes);
lam_status lam_ssim_loss(lam_ctx* ctx, const float* rgb, const float* rgb_obs, const float* cams, int n_cams, float lambda,
                         float* loss, float* d_rgb, int accumulate, void* ws, uint64_t ws_bytes, void* stream);

lam_status lam_rgbd_l1_workspace_size(const lam_ctx* ctx, int n, uint64_t* bytes);
lam_status lam_rgbd_l1_loss(lam_ctx* ctx, const float* rgb, const float* rgb_obs, const float* depth, const float* depth_obs,
                            int n, float lambda_rgb, float lambda_depth, float* loss, float* d_rgb,
                            float* d_depth, void* ws, uint64_t ws_bytes, void* stream);

/* BLOCKING: waits for ``stream`` and reads the counters of the last forward
 * call on ``ws``: the number of (Gaussian, tile) pairs it needed and whether
 * it exceeded the capacity (then returns LAM_ERR_CAPACITY).  Returns
 * LAM_ERR_HIP if one of the sorts' bounded waits for an earlier tile's counts
 * ran out (not expected; the binning of that call is then not valid). */
lam_status lam_render_counters(lam_ctx* ctx, const void* ws, void* stream, uint64_t* instances_needed,
                               int* overflowed);

/* Debug / verification view of the workspace of the last forward call: device
 * pointers to its sorted tile keys and record ids ([count] uint32 each),
 * per-tile [start, end) ranges ([tiles, 2] uint32, (0, 0) for an empty tile), per-record depth keys
 * ([n_cams*N] uint32, 0xFFFFFFFF when culled), per-record footprints
 * ([n_cams*N, 2] uint32: x0 | x1 << 16, y0 | y1 << 16) and per-pixel
 * contributor counts ([P] uint32).  Any output pointer may be NULL.
 * Record r = camera * N + Gaussian.  Host-only, never blocks. */
lam_status lam_render_debug_views(const lam_ctx* ctx, const void* ws, int n_gauss, int d, const float* cams,
                                  int n_cams, int tile_w, int tile_h, uint64_t instance_capacity,
                                  const uint32_t** tile_keys, const uint32_t** tile_recs,
                                  const uint32_t** ranges, const uint32_t** depth_keys,
                                  const uint32_t** footprints, const uint32_t** n_contrib);

/* ------------------------------------------------------------------ decode */

/* Bytes of decode workspace for n pixel rows, query dimension d, M atoms,
 * feature dimension D, under the context's options.  Supported: d in
 * {16, 32}; 1 <= M <= 2048 (FP32: the atoms, padded to 64, at most 1024: a
 * 32-pixel block's FP32 softmax weights and feature rows share the 160 KB of
 * LDS of a workgroup); D a multiple of 128 with 128 <= D <= 1024 (a wave
 * accumulates its quarter of a 32-pixel block's feature rows in registers);
 * n >= 0.  Host-only.
 * Errors: LAM_ERR_INVALID_ARG (null out), LAM_ERR_UNSUPPORTED (shape). */
lam_status lam_decode_workspace_size(const lam_ctx* ctx, int precision, int n, int d, int M, int D, uint64_t* bytes);

/* Decode and feature loss, forward and backward in one call (Eq. 5-6):
 *   F   = softmax(Q K^T / sqrt(d)) V                    (softmax over the M atoms)
 *   L   = (1/n) sum_p (1 - F_p.T_p / max(|F_p| |T_p|, 1e-8)) + lambda_tr ||K - K0||_F^2
 * and writes, for dL = 1:
 *   loss   device [1]      L
 *   dQ     device [n, d]   dL/dQ         (nullable: skipped when the queries are fixed)
 *   dK     device [M, d]   dL/dK (includes 2 lambda_tr (K - K0))
 *   dV     device [M, D]   dL/dV
 *   row_cos device [n]     per-pixel cosine (nullable)
 * Q [n,d], K [M,d], V [M,D], target [n,D] and K0 [M,d] are device inputs
 * (K0 may be NULL when lambda_tr == 0).  F itself is not stored.
 * Errors: LAM_ERR_INVALID_ARG, LAM_ERR_UNSUPPORTED, LAM_ERR_HIP. */
lam_status lam_decode_loss(lam_ctx* ctx, int precision, const float* Q, int n, int d, const float* K,
                           const float* V, int M, int D, const float* target, const float* K0,
                           float lambda_tr, float* loss, float* dQ, float* dK, float* dV,
                           float* row_cos, void* ws, uint64_t ws_bytes, void* stream);

/* lam_decode_loss with its second half on another stream: dQ and row_cos are
 * written in order on ``stream``; the dictionary gradients (dK, dV, their
 * split-K reductions) and the loss are computed on ``dict_stream`` (a
 * hipStream_t of default priority; NULL or ``stream`` itself: no second
 * stream), which first waits for the rows kernel on ``stream``.  Work the caller queues on ``stream`` after this call (the render
 * backward, which needs dQ only) then runs beside them.  loss, dK and dV are
 * ready in ``dict_stream`` order; make ``stream`` wait for ``dict_stream``
 * before reading them or passing the same workspace to another call.
 * Otherwise identical to lam_decode_loss (same results bit for bit). */
lam_status lam_decode_loss_overlap(lam_ctx* ctx, int precision, const float* Q, int n, int d, const float* K,
                                   const float* V, int M, int D, const float* target, const float* K0,
                                   float lambda_tr, float* loss, float* dQ, float* dK, float* dV,
                                   float* row_cos, void* ws, uint64_t ws_bytes, void* stream,
                                   void* dict_stream);

/* Inference decode (Eq. 5): F device [n, D] = softmax(Q K^T / sqrt(d)) V.
 * Errors: LAM_ERR_INVALID_ARG, LAM_ERR_UNSUPPORTED, LAM_ERR_HIP. */
lam_status lam_decode_forward(lam_ctx* ctx, int precision, const float* Q, int n, int d, const float* K,
                              const float* V, int M, int D, float* F, void* ws,
                              uint64_t ws_bytes, void* stream);

/* lam_decode_forward for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and the same F bit for bit, but no workspace
 * argument.  Its scratch -- the prepared dictionary: K and V converted to the
 * compute type, V transposed, K permuted for the MFMA layout, the E4M3 row
 * scales -- lives in a static device array of LAM_NOALLOC_SCRATCH_BYTES per
 * GPU, held from library load until the process ends.  The dictionary needs
 *   Mp (d + 2 D + 32) b + 4 (3 Mp + 64) bytes
 * (each of the five parts rounded up to 256 bytes) with Mp = M rounded up to
 * 64 and b = 4 (FP32) or 2 (BF16, E4M3).  That holds every supported BF16 and
 * E4M3 shape except D = 1024 with M > 1920 (d = 32) or M > 1984 (d = 16), and
 * the FP32 shapes with M <= 960 at D = 1024 (M <= 1024 otherwise, the FP32
 * limit of lam_decode_forward).  Larger dictionaries return
 * LAM_ERR_UNSUPPORTED.
 * Every call on one GPU uses the same array, so calls that overlap on one GPU
 * (two streams, two host threads, two contexts) race: serialise them.  Each
 * call rewrites the whole part it reads, so nothing carries over between
 * calls.  Allocates nothing and makes no host synchronisation.
 * Errors: LAM_ERR_INVALID_ARG (no context, null or misaligned pointers),
 * LAM_ERR_UNSUPPORTED (shape, or a dictionary beyond the scratch),
 * LAM_ERR_HIP. */
lam_status lam_decode_forward_noalloc(lam_ctx* ctx, int precision, const float* Q, int n, int d, const float* K,
                                      const float* V, int M, int D, float* F, void* stream);

/* Adjoint of lam_decode_forward: given dF device [n, D] writes dQ [n, d]
 * (nullable), dK [M, d], dV [M, D] (device, overwritten); the softmax is
 * recomputed, not stored.  Errors as above. */
lam_status lam_decode_backward(lam_ctx* ctx, int precision, const float* Q, int n, int d, const float* K,
                               const float* V, int M, int D, const float* dF, float* dQ,
                               float* dK, float* dV, void* ws, uint64_t ws_bytes, void* stream);

/* ------------------------------------------------------ tied decode (paper) */

/* The decode and loss as the paper states them (Sec. III-C, Eq. 5-6):
 *   F^ = Softmax(Q W D^T) D with the softmax taken over the cosine similarity
 *        of the rows of Q W and the atoms D_j, divided by a temperature tau,
 *   L  = lambda_cos mean_p (1 - cos(F^_p, F_p)) + lambda_2 mean_p |F^_p - F_p|^2
 *        + lambda_D sum_j ReLU(|D0_j - D_j| - delta).
 * Norms are guarded as max(|.|, 1e-12), the cosine denominator as
 * max(|F^||F|, 1e-8).  The paper's values: lambda_cos = lambda_2 = 0.5,
 * lambda_D = 0.2, delta = 0.1; it gives no temperature. */
typedef struct {
    float tau;        /* > 0 */
    float lambda_cos; /* >= 0 */
    float lambda_2;   /* >= 0 */
    float lambda_D;   /* >= 0 */
    float delta;      /* >= 0 */
} lam_tied_params;

/* Workspace bytes for lam_decode_tied_loss: n pixel rows, query dimension ds
 * (16 or 32), M atoms, feature dimension df (the decode's D; same limits as
 * lam_decode_workspace_size).  Host-only.
 * Errors: LAM_ERR_INVALID_ARG (null out, n < 0), LAM_ERR_UNSUPPORTED (shape,
 * or a precision other than LAM_FP32 and LAM_BF16). */
lam_status lam_decode_tied_workspace_size(const lam_ctx* ctx, int precision, int n, int ds, int M, int df, uint64_t* bytes);

/* Loss and gradients of the tied decode.  Device inputs (FP32, row-major):
 * Q [n, ds], W [ds, df], D [M, df], target F [n, df], D0 [M, df] (the initial
 * dictionary); params on the host.  Device outputs (overwritten): loss [1],
 * dQ [n, ds] (nullable: the decode-only iterations skip it), dW [ds, df],
 * dD [M, df].  precision selects the attention arithmetic as in
 * lam_decode_loss, LAM_FP32 or LAM_BF16 (LAM_FP8_E4M3 is unsupported: with
 * cosine logits over a small temperature the softmax weights sit on a few
 * atoms, so E4M3 rounding of D is not averaged out and dQ misses its bound);
 * the normalisations and the gradient chain run in FP32.
 * Q, target and dQ rows are read and written 16 bytes at a time (16-byte
 * aligned).  Stream-ordered, no host synchronisation.
 * Errors: LAM_ERR_INVALID_ARG (null or misaligned pointers, workspace too
 * small, tau <= 0 or a negative weight), LAM_ERR_UNSUPPORTED (shape,
 * precision), LAM_ERR_HIP. */
lam_status lam_decode_tied_loss(lam_ctx* ctx, int precision, const float* Q, int n, int ds, const float* W, const float* D,
                                int M, int df, const float* target, const float* D0,
                                const lam_tied_params* params, float* loss, float* dQ, float* dW, float* dD,
                                void* ws, uint64_t ws_bytes, void* stream);

/* -------------------------------------------- streaming K-means (Eq. 10) */

/* The dictionary initialisation of Sec. III-D, D_t0 = StreamKMeans(F_t,
 * D_{t-1}, K), read as the streaming K-means the paper cites: the keyframe's
 * embeddings are summarised into m weighted micro-centres by Lloyd's
 * iteration, merged with the current weighted global centres, and the merged
 * set is re-clustered into K centres.
 *
 * One Lloyd iteration assigns every point to its nearest centre in squared
 * Euclidean distance (ties to the lowest index) and moves every centre to the
 * weighted mean of its points; a centre without points (or with zero total
 * weight) stays where it is.  Iteration counts are fixed (no convergence
 * test), so the calls are stream-ordered and never synchronise.
 *
 * precision selects the distance products: LAM_FP32 (float32 MFMA) or
 * LAM_BF16 (bfloat16 operands, float32 accumulation; an assignment can differ
 * from the float32 one only where two centres are within the bfloat16
 * rounding of the products).  Norms, means and weights are float32; the sums
 * of an update are taken in point-index order per centre, so results do not
 * depend on the launch schedule.
 *
 * Shapes: D a multiple of 32 in [32, 2048] (FP32: up to 1024), 1 <= k <=
 * 65536, fewer than 2^30 points.  Row arrays (points, centres) are float32 row-major and 16-byte
 * aligned.  Otherwise LAM_ERR_UNSUPPORTED (shape) or LAM_ERR_INVALID_ARG. */

/* Workspace bytes for lam_kmeans_assign / lam_kmeans_lloyd with up to n
 * points of dimension D and k centres.  Host-only. */
lam_status lam_kmeans_workspace_size(const lam_ctx* ctx, int precision, int n, int D, int k, uint64_t* bytes);

/* Nearest centre of every point.  Device: X [n, D], C [k, D]; outputs
 * assign [n] (int32, overwritten) and d2 [n] (nullable: the squared distance
 * to that centre, float32, clamped at zero).  Stream-ordered. */
lam_status lam_kmeans_assign(lam_ctx* ctx, int precision, const float* X, int n, int D, const float* C, int k, int32_t* assign,
                             float* d2, void* ws, uint64_t ws_bytes, void* stream);

/* iters >= 1 Lloyd iterations from C0.  Device: X [n, D], weights [n]
 * (nullable: all 1), C0 [k, D]; outputs C [k, D] (may be C0), W [k]
 * (nullable: total weight per centre under the last assignment) and
 * assign [n] (nullable: the last assignment, from which C was computed).
 * Stream-ordered. */
lam_status lam_kmeans_lloyd(lam_ctx* ctx, int precision, const float* X, const float* weights, int n, int D, const float* C0,
                            int k, int iters, float* C, float* W, int32_t* assign, void* ws, uint64_t ws_bytes,
                            void* stream);

/* Workspace bytes for lam_stream_kmeans.  Requires 0 <= m <= n, 0 <= Kp <= K
 * and m >= K - Kp.  Host-only. */
lam_status lam_stream_kmeans_workspace_size(const lam_ctx* ctx, int precision, int n, int D, int Kp, int K, int m, uint64_t* bytes);

/* One streaming step.  Device: F [n, D] the new embeddings (weight 1 each),
 * D_prev [Kp, D] and w_prev [Kp] the global centres and their weights (Kp = 0
 * on the first keyframe: both may be NULL).  Host: seeds [m], distinct
 * indices into F (the random draw), read before the call returns; the
 * micro-centres start at F[seeds].  Steps: iters_local Lloyd iterations of F
 * into the m micro-centres (each weighted by its point count); the merged set
 * [D_prev; micro-centres] with weights [w_prev; counts] then takes
 * iters_global >= 1 weighted Lloyd iterations from [D_prev; the first K - Kp
 * micro-centres].  Outputs D_out [K, D] and W_out [K] (total weight per
 * centre).  Stream-ordered.
 * Errors: LAM_ERR_INVALID_ARG (sizes, null or misaligned pointers, a seed
 * outside [0, n), workspace too small), LAM_ERR_UNSUPPORTED (shape),
 * LAM_ERR_HIP. */
lam_status lam_stream_kmeans(lam_ctx* ctx, int precision, const float* F, int n, int D, const float* D_prev,
                             const float* w_prev, int Kp, int K, const int32_t* seeds, int m, int iters_local,
                             int iters_global, float* D_out, float* W_out, void* ws, uint64_t ws_bytes,
                             void* stream);

/* --------------------------------------------------------------- profiling */

/* Turns per-kernel timing on or off for the calls made through ``ctx`` (off
 * by default).  While on, the main kernels (names: "raster_fwd", "raster_bwd", "decode_rows",
 * "decode_tn", "render_sort", "preprocess", "preprocess_bwd", "tied_prep",
 * "tied_grads", "kmeans", "kmeans_assign", "rgbd_l1", "ssim") are bracketed by
 * HIP events recorded on their launch stream.  Not for use under graph capture. */
lam_status lam_profile_enable(lam_ctx* ctx, int on);

/* BLOCKING: waits for the recorded events of kernel ``name``, returns the sum
 * of their elapsed times (ms) and how many launches were recorded, and clears
 * them.  Unknown names read as zero launches. */
lam_status lam_profile_read(lam_ctx* ctx, const char* name, double* total_ms, int* count);

#ifdef __cplusplus
}
#endif

#endif /* LATENTAM_H */
