/*
 * tcflow.h -- C ABI of the per-frame hot path of streaming temporal
 * consistency ("Interactive Control over Temporal Consistency while
 * Stylizing Video Streams"): a lite coarse-to-fine optical-flow network
 * followed by the consistency step, as HIP kernels for gfx950 (MI355X).
 *
 * Conventions shared by every call
 *   - Every tensor pointer is HIP device memory owned by the caller, dense,
 *     float32, row major.  Frames are NCHW n x 3 x h x w, RGB in [0, 1].
 *     Flows are n x 2 x h x w in pixels: channel 0 = dx, channel 1 = dy,
 *     on the grid of the first frame of the pair.
 *   - Workspaces and pyramid buffers are caller-owned device memory of at
 *     least the size the matching *_bytes query returns, 256-byte aligned.
 *     The library never allocates on a call path and never frees caller
 *     memory.  Outputs must not alias inputs (except where stated).
 *   - Calls that can fail return a tc_status value (as int).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is only
 *     enqueued; nothing synchronises the host.  Argument, shape and
 *     workspace errors are returned before anything is enqueued; a kernel
 *     launch error returns TC_ERR_HIP; faults during execution surface at the
 *     caller's next synchronisation.  Non-finite pixel values propagate and
 *     are not checked.  No C++ exception crosses this boundary.
 *   - A tc_net is immutable after creation: calls on different streams with
 *     distinct workspaces may run concurrently.
 */
#ifndef TCFLOW_H
#define TCFLOW_H

#include <stddef.h>

#include <hip/hip_runtime_api.h> /* hipStream_t */

#ifdef __cplusplus
extern "C" {
#endif

#define TC_API __attribute__((visibility("default")))

typedef enum {
  TC_OK = 0,
  TC_ERR_INVALID_ARG = 1, /* null pointer, n/h/w <= 0, alpha outside [0,1] or NaN */
  TC_ERR_SHAPE = 2,       /* descriptor or weight count inconsistent           */
  TC_ERR_WORKSPACE = 3,   /* workspace / pyramid buffer too small or unaligned */
  TC_ERR_UNSUPPORTED = 4, /* precision or size the library does not handle     */
  TC_ERR_HIP = 5,         /* a HIP runtime call or kernel launch failed        */
  TC_ERR_SCRATCH = 6      /* input too large for the static scratch of
                             tc_flow_estimate_pair_noalloc                      */
} tc_status;

typedef enum { TC_FP32 = 0, TC_BF16 = 1, TC_FP8_E4M3 = 2 } tc_precision;
/* OR-ed into the precision of TC_BF16 or TC_FP8_E4M3 nets: store the pyramid
 * features (the cost volume's inputs) as bfloat16 instead of float16, and
 * correlate them in float32 (the form measured beside the float16 cost
 * volume). */
#define TC_PREC_BF16_FEATURES 0x100

/* Network descriptor.  levels L in [1, 8]; ch[l-1] = channels of pyramid
 * level l (multiples of 8, at most 128); dec = widths of the three decoder
 * conv layers (multiples of 16, at most 128, with dec[1] + dec[2] <= 128:
 * the head's input [h2 | h3]); radius = cost-volume radius
 * (4 gives 81 displacements); leaky = LeakyReLU slope.
 * Variants of Sec. 3.2 ("Optimized Network Architecture"): finest = the
 * finest level with a flow estimator, in [1, L] (1: every level; 2: the
 * finest estimator removed, the flow of level 2 is upsampled to the input);
 * ref_layers in [0, 8] depthwise separable refinement layers ("-sepref") on
 * that level, layer j with ref_ch[j] outputs (multiples of 8, at most 128;
 * the last one 2) and dilation ref_dil[j] in [1, 64]. */
typedef struct {
  int levels;
  int ch[8];
  int dec[3];
  int radius;
  float leaky;
  int finest;
  int ref_layers;
  int ref_ch[8];
  int ref_dil[8];
} tc_net_desc;

typedef struct tc_net tc_net; /* opaque */

TC_API const char* tc_status_str(int status);
TC_API const char* tc_version(void);

/* Host-side float -> FP8 E4M3 encoder used for the FP8 weights (OCP 8-bit
 * floating point "E4M3FN": bias 7, no infinities, largest finite 448; round
 * to nearest even, saturating).  Plain host memory, n values. */
TC_API void tc_fp8_e4m3_encode(const float* in, unsigned char* out, size_t n);

/* Number of float32 values of the weight blob for `desc`.  Blob layout,
 * layer after layer: W[cout][cin][3][3] then b[cout]; order: pyramid convs
 * of level 1..L (stride 2: C_{l-1} -> C_l with C_0 = 3, then stride 1:
 * C_l -> C_l), then the decoders of level finest..L: c1 ((2r+1)^2 + C_l + 2
 * -> dec0), c2 (dec0 -> dec1), c3 (dec1 -> dec2), head (dec1 + dec2 -> 2),
 * then per refinement layer j: depthwise W[c][3][3], b[c] and pointwise
 * W[ref_ch[j]][c], b[ref_ch[j]] (c = dec1 + dec2 + 2 for j = 0, else
 * ref_ch[j-1]). */
TC_API size_t tc_weight_floats(const tc_net_desc* desc);

/* Copies the host weight blob to the current HIP device, packed for the
 * kernels of `precision`: TC_FP32 (FP32 activations, FP32 MFMA); TC_BF16
 * (BF16 activations and weights, FP32 accumulation); TC_FP8_E4M3 (BF16
 * activations rounded to FP8 with a per-image, per-tensor scale max|x| / 448
 * when a conv stages them, FP8 weights with per-output-channel scales, FP32
 * accumulation).  In the BF16 and FP8 forms the pyramid features are stored
 * as float16 (bfloat16 with TC_PREC_BF16_FEATURES): the cost volume warps and
 * correlates them with float16 products and float32 sums, and the convs that
 * read them convert to their operand type when staging.  In every form the
 * flows, their upsampling and accumulation and the warp coordinates are FP32,
 * and the cost volume accumulates in FP32.  Paper, Sec. 3.2: PWC-Net-shaped
 * network with light estimators (a conv feature pyramid, warping, correlation
 * and a CNN flow estimator per level).  *out is set only on TC_OK;
 * TC_ERR_UNSUPPORTED for an unknown precision. */
TC_API int tc_net_create(const tc_net_desc* desc, const float* host_weights, size_t n_floats,
                         int precision, tc_net** out);
TC_API void tc_net_destroy(tc_net* net);

/* ---- feature pyramids (cacheable per frame) ---------------------------- */

/* Bytes of the buffer that holds the feature pyramid of n frames of h x w
 * (levels at resolution ceil-to-2^L / 2^l, NHWC) plus its build scratch. */
TC_API size_t tc_pyramid_bytes(const tc_net* net, int n, int h, int w);

/* Feature pyramid of `frames` (n x 3 x h x w): the frame is edge-replicated
 * up to a multiple of 2^L, then each level applies a stride-2 and a stride-1
 * 3x3 conv, each followed by LeakyReLU.  Writes into `pyr`. */
TC_API int tc_pyramid(const tc_net* net, const float* frames, int n, int h, int w, void* pyr,
                      size_t pyr_bytes, hipStream_t stream);

/* ---- flow -------------------------------------------------------------- */

/* Scratch bytes of tc_flow_from_pyramids for n pairs (both directions). */
TC_API size_t tc_decoder_workspace_bytes(const tc_net* net, int n, int h, int w);

/* Coarse-to-fine flow from the frames of pyramid `pyr1` to those of `pyr2`
 * (flow12, n x 2 x h x w) and, if flow21 is not NULL, the opposite direction
 * in the same batched pass.  Per level l = L..f (f = desc.finest):
 * U = 2 up2(flow_{l+1}) (U_L = 0), warp the second pyramid's features by U,
 * 81-channel cost volume, light estimator on [cost volume | F1 | U] ->
 * increment, flow_l = U + increment; with refinement layers,
 * flow_f += refine([h2 | h3 | flow_f]) (each layer: dilated depthwise 3x3,
 * bias, LeakyReLU, pointwise, bias, LeakyReLU except on the last); output =
 * 2^f upsample(flow_f, 2^f) (bilinear, half-pixel centres) cropped to h x w.
 * Paper, Sec. 3.2 and supplementary S1. */
TC_API int tc_flow_from_pyramids(const tc_net* net, const void* pyr1, const void* pyr2, int n,
                                 int h, int w, float* flow12, float* flow21, void* ws,
                                 size_t ws_bytes, hipStream_t stream);

/* Continuous batching over streams: one decoder pass for n (<= 16) frame
 * pairs whose pyramids live in separate one-image buffers (tc_pyramid with
 * n = 1 and the same h, w): flow_fw[i] = flow(prev i -> cur i),
 * flow_bw[i] = flow(cur i -> prev i), each 1 x 2 x h x w.  Every image is
 * computed exactly as in a one-pair call.  TC_FP32 and TC_BF16 nets. */
TC_API size_t tc_decoder_list_workspace_bytes(const tc_net* net, int n, int h, int w);
TC_API int tc_flow_from_pyramid_list(const tc_net* net, const void* const* pyr_prev,
                                     const void* const* pyr_cur, int n, int h, int w,
                                     float* const* flow_fw, float* const* flow_bw, void* ws,
                                     size_t ws_bytes, hipStream_t stream);

/* Scratch bytes of tc_flow_estimate / tc_flow_estimate_pair (two pyramids
 * plus the decoder scratch). */
TC_API size_t tc_flow_workspace_bytes(const tc_net* net, int n, int h, int w);

/* flow_estimate(prev, cur) -> flow from prev to cur on prev's grid, in
 * pixels (paper Sec. 3.1: the input video I and the optical flow between
 * consecutive frames that warps the previous output; Sec. 3.2: the flow
 * network).  prev, cur: n x 3 x h x w; flow: n x 2 x h x w (caller-owned
 * device memory); ws: at least tc_flow_workspace_bytes(net, n, h, w) bytes,
 * 256-byte aligned.  Builds both pyramids, then the coarse-to-fine decoder
 * as tc_flow_from_pyramids.  TC_ERR_INVALID_ARG for null pointers or
 * n, h, w < 1; TC_ERR_WORKSPACE for a small or misaligned workspace. */
TC_API int tc_flow_estimate(const tc_net* net, const float* prev, const float* cur, int n, int h,
                            int w, float* flow, void* ws, size_t ws_bytes, hipStream_t stream);

/* flow_fw = flow(prev -> cur), flow_bw = flow(cur -> prev), sharing both
 * pyramids and one batched decoder pass: the two flows the consistency step
 * needs (paper Sec. 3.1, Eq. 4 warps O_{t-1} with the flow from t to t-1;
 * the forward-backward test of the mask compares both; Sec. 3.2 network).
 * Arguments, workspace and errors as for tc_flow_estimate; flow_bw must
 * not be NULL. */
TC_API int tc_flow_estimate_pair(const tc_net* net, const float* prev, const float* cur, int n,
                                 int h, int w, float* flow_fw, float* flow_bw, void* ws,
                                 size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * tc_flow_estimate_pair without a workspace argument.  The scratch (two
 * pyramids and the decoder buffers) is a static device array of
 * TC_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held until the
 * process ends; the call itself allocates nothing.  The inputs and outputs
 * are as for tc_flow_estimate_pair and stay caller-owned.  Returns
 * TC_ERR_SCRATCH, before enqueueing anything, when
 * tc_flow_workspace_bytes(net, n, h, w) > TC_NOALLOC_SCRATCH_BYTES (e.g. the
 * 5-level 16..128-channel FP32 network fits up to about 640 x 360 per pair).
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (different streams or host threads without ordering) race and give
 * undefined results; calls ordered on one stream are safe.  The array keeps
 * the last call's contents; nothing the kernels read is assumed to start at
 * zero (what must be zero, e.g. the FP8 scale slots, is cleared by a kernel
 * at the start of each call).  The device is the stream's (the current
 * device for the NULL stream); the net must live on it. */
#define TC_NOALLOC_SCRATCH_BYTES (256u << 20)
TC_API int tc_flow_estimate_pair_noalloc(const tc_net* net, const float* prev, const float* cur,
                                         int n, int h, int w, float* flow_fw, float* flow_bw,
                                         hipStream_t stream);

/* Flow pair of the paper's fast preset (Sec. 4.1, implementation details:
 * optical flow computed on half-sized inputs).  Each frame is reduced to
 * h2 x w2 = ceil(h/2) x ceil(w/2) by taking the mean of every 2 x 2 pixel
 * block (a block that runs past the last row or column repeats it), the
 * pair is estimated at that size as by tc_flow_estimate_pair, and each flow
 * is brought back to h x w by bilinear upsampling with half-pixel centres
 * (output pixel i samples the half-size flow at (i + 1/2)/2 - 1/2, clamped
 * to the half-size grid) times 2.  Arguments as for tc_flow_estimate_pair;
 * the workspace (caller-owned device memory, 256-byte aligned) must hold
 * tc_flow_half_workspace_bytes(net, n, h, w).  Errors: TC_ERR_INVALID_ARG
 * for null pointers or n, h, w < 1, TC_ERR_WORKSPACE for a small or
 * misaligned workspace. */
TC_API size_t tc_flow_half_workspace_bytes(const tc_net* net, int n, int h, int w);
TC_API int tc_flow_estimate_pair_half(const tc_net* net, const float* prev, const float* cur,
                                      int n, int h, int w, float* flow_fw, float* flow_bw,
                                      void* ws, size_t ws_bytes, hipStream_t stream);

/* ---- consistency step -------------------------------------------------- */

/* out_t from stylized P_t, previous output O_{t-1}, flow_fw = flow(I_{t-1}
 * -> I_t) and flow_bw = flow(I_t -> I_{t-1}) (paper Sec. 3.1, Eq. 4 and
 * Eq. 5; non-occlusion mask of Sec. 5, Eq. 9).  Per pixel x:
 *   s   = x + flow_bw(x)
 *   G   = bilinear(prev_out, s),  f~ = bilinear(flow_fw, s)
 *   m   = s inside the frame and
 *         |flow_bw + f~|^2 <= 0.01 (|flow_bw|^2 + |f~|^2) + 0.5
 *   w   = alpha * m
 *   out = (1 - w) * stylized + w * G
 * alpha in [0, 1]: 0 returns stylized exactly, 1 returns G where visible.
 * `out` may alias `stylized`; mask_or_null (n x h x w bytes, 1 = visible)
 * is written when not NULL.  For t = 1 the caller sets O_1 = P_1. */
TC_API int tc_consistency_step(const float* stylized, const float* prev_out, const float* flow_fw,
                               const float* flow_bw, float alpha, int n, int h, int w, float* out,
                               unsigned char* mask_or_null, hipStream_t stream);

/* ---- the paper's full consistency step ------------------------------------ */

/* Parameters of Eq. 1-8 (paper Sec. 3.1 and Sec. 4.2): k1, k2 = upper clamps
 * of the previous / next local weights, a_ph = photometric sharpness of the
 * weights' exponentials, lambda = scale of the smoothness weight w_c,
 * eta, kappa = step sizes of the momentum iteration, iterations = its count.
 * tc_paper_default_params fills the paper's final setting (k1 0.3, k2 0.5,
 * a_ph 6500, lambda 2, eta 0.15, kappa 0.2, 150 iterations). */
typedef struct {
  float k1, k2, a_ph, lambda, eta, kappa;
  int iterations;
} tc_paper_params;

TC_API void tc_paper_default_params(tc_paper_params* p);

/* The paper's parameter presets (Sec. 4.2, parameter settings; Sec. 4.1 for
 * the fast preset), eta 0.15 and kappa 0.2 in all:
 *   TC_PRESET_FINAL      k1 0.3, k2 0.5, a_ph 6500, lambda 2, 150 iterations
 *                        (the setting of its results; = tc_paper_default_params)
 *   TC_PRESET_OBJECTIVE  k1 = k2 = 0.3, a_ph 10000, lambda 0.7, 150 iterations
 *                        (tuned for low warping error)
 *   TC_PRESET_FAST       the final setting with 50 iterations (the runtime
 *                        table's fast preset), paired with flow on
 *                        half-sized inputs (tc_flow_estimate_pair_half).
 * Returns TC_ERR_INVALID_ARG for a null `p` or an unknown preset. */
enum { TC_PRESET_FINAL = 0, TC_PRESET_OBJECTIVE = 1, TC_PRESET_FAST = 2 };
TC_API int tc_paper_preset_params(int preset, tc_paper_params* p);
TC_API size_t tc_paper_workspace_bytes(int n, int h, int w);

/* O_t of the paper's step.  Inputs n x 3 x h x w: I_{t-1}, I_t, I_{t+1},
 * P_{t-1}, P_t, P_{t+1}, O_{t-1}; flows n x 2 x h x w: flow_t_prev = flow from
 * frame t to t-1 and flow_t_next = from t to t+1, both on t's grid.  Per pixel
 * (warps are bilinear with border clamping):
 *   w_p = min(exp(-a_ph |I_t - warp(I_{t-1})|^2), k1), w_n likewise with k2 (Eq. 3)
 *   L_t = (1 - w_p - w_n) P_t + w_p warp(P_{t-1}) + w_n warp(P_{t+1})       (Eq. 2)
 *   A_t = w_p warp(O_{t-1}) + (1 - w_p) L_t                                  (Eq. 4, 5)
 *   w_c = lambda exp(-a_ph |I_t - A^I_t|^2), A^I_t as L_t over I             (Eq. 6, 7)
 * then `iterations` steps of O <- O - eta grad E(O) + kappa (O - O_old) with
 * grad E(O) = -Lap(O - P_t) + w_c (O - A_t) (Eq. 1 discretised with forward
 * differences and Neumann borders; Eq. 8), from O = O_old = A_t.  `out`
 * (n x 3 x h x w) must not alias an input. */
TC_API int tc_consistency_paper(const float* I_prev, const float* I, const float* I_next,
                                const float* P_prev, const float* P, const float* P_next,
                                const float* O_prev, const float* flow_t_prev,
                                const float* flow_t_next, const tc_paper_params* params, int n,
                                int h, int w, float* out, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---- measurement probe -------------------------------------------------- */

/* Forward-backward agreement of a flow pair: counts[i] (device, n
 * unsigned) = number of pixels of image i that pass the test of
 * tc_consistency_step's mask (target inside the frame and
 * |f_b + f~_f|^2 <= 0.01 (|f_b|^2 + |f~_f|^2) + 0.5).  Used to fall back from
 * a student network's flows to the teacher's when too few pixels agree. */
TC_API int tc_flow_agreement(const float* flow_fw, const float* flow_bw, int n, int h, int w,
                             unsigned* counts, hipStream_t stream);

/* ---- training of a student network on teacher flows --------------------
 *
 * Paper Sec. 3.2 ("Training") and the supplementary loss: the loss is a sum
 * over the flow estimators, weighted equally, of the robust loss of Eq. S2,
 * mean over the level's pixels of (|du| + |dv| + loss_eps)^loss_q, against
 * the teacher flow edge-padded to the network's grid, averaged over each
 * 2^l x 2^l block and divided by 2^l (level-l pixels).  The optimizer is
 * AdamW (decoupled weight decay): p <- p (1 - lr weight_decay), then the
 * bias-corrected Adam update with beta1, beta2, eps.  Everything is FP32;
 * weights, gradients and the two Adam moments are kept in the layout of the
 * weight blob (tc_weight_floats). */
typedef struct {
  float lr, beta1, beta2, eps, weight_decay;
  float loss_eps, loss_q;
} tc_train_params;
typedef struct tc_trainer tc_trainer; /* opaque */

/* lr 1e-4, beta1 0.9, beta2 0.99, eps 1e-8, weight_decay 4e-4, loss_eps
 * 0.01, loss_q 0.4. */
TC_API void tc_train_default_params(tc_train_params* p);

/* Trainer for batches of up to max_n frame pairs of h x w (any size; padded
 * to a multiple of 2^L like the inference path).  The network must have an
 * estimator at every level, no refinement, and ch[l] + 88 <= 128.  Copies
 * `host_weights` (the blob) as the initial weights; allocates all its device
 * memory here (nothing is allocated per step).  TC_ERR_SHAPE for an
 * unsupported descriptor or a wrong weight count. */
TC_API int tc_trainer_create(const tc_net_desc* desc, const float* host_weights, size_t n_floats,
                             const tc_train_params* params, int max_n, int h, int w,
                             tc_trainer** out);
TC_API void tc_trainer_destroy(tc_trainer* t);

/* Loss and gradient for n pairs: frames A (flow source) and B (n x 3 x h x
 * w, device), teacher flows A -> B (n x 2 x h x w, device, input pixels).
 * The gradient stays in the trainer; the loss (one float) is written to
 * device memory `loss_out` if not NULL.  Asynchronous on `stream`. */
TC_API int tc_trainer_grad(tc_trainer* t, const float* A, const float* B, const float* teacher,
                           int n, float* loss_out, hipStream_t stream);
/* tc_trainer_grad followed by one AdamW step. */
TC_API int tc_trainer_step(tc_trainer* t, const float* A, const float* B, const float* teacher,
                           int n, float* loss_out, hipStream_t stream);
/* Copies weights (which = 0), gradient (1), first (2) or second moment (3),
 * n_floats values in blob layout, to `dst` (host or device). */
TC_API int tc_trainer_copy(const tc_trainer* t, int which, float* dst, hipStream_t stream);
/* Number of AdamW steps taken. */
TC_API int tc_trainer_steps_done(const tc_trainer* t);

/* Stage ids: TC_STAGE(level, op) for the per-level ops, plus three
 * whole-frame stages. */
#define TC_STAGE(level, op) ((level) * 16 + (op))
enum {
  TC_OP_PYR_A = 0,       /* pyramid stride-2 conv of level l          */
  TC_OP_PYR_B = 1,       /* pyramid stride-1 conv of level l          */
  TC_OP_UP2 = 2,         /* U_l = 2 up2(flow_{l+1})                   */
  TC_OP_COST_VOLUME = 3, /* feature warp + cost volume of level l     */
  TC_OP_C1 = 4,          /* decoder convs of level l                  */
  TC_OP_C2 = 5,
  TC_OP_C3 = 6,
  TC_OP_HEAD = 7,
  TC_OP_REFINE = 8       /* all refinement layers (level = finest)    */
};
#define TC_STAGE_INPUT 1        /* frame staging (pad + relayout)       */
#define TC_STAGE_OUTPUT 2       /* final upsample + crop of the flow     */
#define TC_STAGE_CONSISTENCY 3  /* fused consistency step               */
#define TC_STAGE_PAPER 4        /* the paper's consistency step (all kernels) */

/* Bracket every launch of `stage` with a pair of hipEvents on its stream,
 * for up to `max_launches` launches (process-wide; a measurement aid, not
 * thread safe; events are created here, outside any call path). */
TC_API int tc_probe_enable(int stage, int max_launches);
/* Waits for the recorded events; *launches = number recorded, *total_ms =
 * summed device time between each pair.  Resets the count. */
TC_API int tc_probe_read(int* launches, float* total_ms);
TC_API void tc_probe_disable(void);

#ifdef __cplusplus
}
#endif
#endif /* TCFLOW_H */
