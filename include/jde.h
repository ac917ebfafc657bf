/*
 * jde.h -- C ABI of the MI355X (gfx950) JDE hot-path library (libjde.so).
 *
 * The library runs the joint detection-and-embedding (JDE) tracker's hot path
 * on one GPU: the model forward over a batch of frames (Sec. 3.1 and the
 * batch-wise inference of Sec. 4.2), then the post-processing of Appendix A up
 * to the cost matrix: confidence threshold (item 2), sort and IoU non-max
 * suppression (item 3), embedding normalisation, and the tracks x detections
 * cosine cost with Kalman-gated infinite entries (items 5-6).  The Kalman
 * filter (item 4, 7) and the Hungarian assignment (item 7) run on the host in
 * FP64 through the jde_kf_* and jde_assign calls.
 *
 * Conventions (every call):
 *  - Device memory is owned by the caller.  The library never allocates device
 *    memory: the caller allocates the weight buffer (jde_weights_bytes), the
 *    workspace (jde_workspace_bytes) and all inputs/outputs, and passes raw
 *    device pointers.  Host pointers are marked "host".
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Device calls only enqueue work on it; nothing synchronises implicitly.
 *    Device-side results (counts, overflow flags) are valid after the caller
 *    synchronises the stream.
 *  - Errors are returned as jde_status; jde_last_error() gives a thread-local
 *    message.  No exception crosses the ABI.  Argument checks happen before
 *    any work is enqueued, so a failing call enqueues nothing.
 *  - A context is used by one host thread at a time; contexts share nothing.
 *  - Layouts: activations NHWC; frames NCHW FP32; frames of one batch are
 *    packed back to back in submission order, each with its own size
 *    (jde_frame_desc), which may differ within a batch.
 */
#ifndef JDE_H
#define JDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct jde_ctx jde_ctx;

typedef enum {
    JDE_OK = 0,
    JDE_EINVAL = -1,        /* bad argument (shape, pointer, size, alignment)        */
    JDE_ENOMEM = -2,        /* caller buffer smaller than the size query returned    */
    JDE_EDEVICE = -3,       /* a HIP call failed                                     */
    JDE_ECAPACITY = -4,     /* batch exceeds the capacity given at jde_create        */
    JDE_EUNSUPPORTED = -5,  /* configuration the library does not implement          */
    JDE_ESTATE = -6,        /* call out of order (e.g. forward before load_weights)  */
    JDE_EBUDGET = -7        /* admission refused: the device-memory budget is spent  */
} jde_status;

/* Arithmetic of the convolutions (Sec. 4.1 runs the model in mixed precision).
 * Accumulation is FP32 in every mode; head outputs, decode and normalisation
 * stay FP32.  JDE_FP8 runs the backbone 3x3 convolutions in OCP FP8 e4m3 with
 * per-channel and per-32-k-block weight scales and per-32-channel activation
 * scales (see jde_fp8_block_scales), and the rest in BF16.  JDE_FP6 and JDE_FP4
 * do the same with OCP microscaling elements FP6 E2M3 (largest value 7.5) and
 * FP4 E2M1 (largest value 6), always with block scales (a precision study
 * beyond the paper). */
typedef enum { JDE_FP32 = 0, JDE_BF16 = 1, JDE_FP16 = 2, JDE_FP8 = 3, JDE_FP6 = 4, JDE_FP4 = 5 } jde_precision;

typedef struct {
    int base_ch;             /* stem width c0 (32 for Darknet-53)                       */
    int blocks[5];           /* residual blocks per stage (1,2,8,8,4 for Darknet-53)    */
    int emb_dim;             /* embedding length E (512 in Appendix A item 1); mult. of 64 */
    int num_anchors;         /* anchors per cell per scale, A (4)                       */
    float anchors[3][4][2];  /* (w, h) in pixels for strides 8, 16, 32                  */
    int precision;           /* jde_precision                                            */
    int max_frames;          /* largest batch (frames) any call will pass               */
    int max_h, max_w;        /* largest frame; every frame's h, w divisible by 32       */
    int max_candidates;      /* per-frame cap on candidates entering NMS (<= 8192)      */
    size_t max_pixels;       /* most pixels of one batch (sum of h*w over its frames); the
                                workspace is planned for it.  0 = max_frames*max_h*max_w.
                                Lets a batch hold many frames of mixed sizes without
                                reserving max_frames frames of the largest size.       */
} jde_config;

typedef struct { int h, w; } jde_frame_desc;

/* Model outputs (device, FP32, NHWC, frames packed back to back per scale).
 * Scale index 0, 1, 2 = stride 8, 16, 32.  det[s]: [sum_f H_f/st * W_f/st, 6A],
 * channel 6a + (dx, dy, dw, dh, c_bg, c_fg).  emb[s]: [sum_f ..., E]. */
typedef struct { float* det[3]; float* emb[3]; } jde_head_out;

/* Detections after threshold + NMS (device).  Frame f owns rows
 * [f*cap, f*cap + count[f]) of every array, in keep order (score descending,
 * canonical anchor index ascending on ties).  The canonical anchor index is
 * base_s + A*(i*W_s + j) + a with scales ordered 8, 16, 32. */
typedef struct {
    float* boxes;      /* [n*cap, 4] x1, y1, x2, y2 (pixels of the frame)        */
    float* scores;     /* [n*cap] foreground softmax score                      */
    float* margins;    /* [n*cap] c_fg - c_bg (the sort key)                    */
    float* emb;        /* [n*cap, E] L2-normalised embeddings                   */
    int* anchor_idx;   /* [n*cap] canonical anchor index                        */
    int* count;        /* [n] detections kept                                   */
    int* n_cand;       /* [n] candidates over the threshold before the cap      */
    int* overflow;     /* [n] 1 if n_cand > cap (the top-cap by key were kept)  */
    int cap;           /* rows per frame; must equal the context's max_candidates */
} jde_dets;

/* ---- context ----------------------------------------------------------- */

/* Validates cfg and builds the layer plan (Darknet-53 backbone, FPN, three
 * heads; Sec. 3.1) and the workspace plan.  Host-only.  *out receives a
 * context to free with jde_destroy.  JDE_EINVAL on bad sizes, JDE_EUNSUPPORTED
 * on an unknown precision or num_anchors != 4. */
jde_status jde_create(const jde_config* cfg, jde_ctx** out);
void jde_destroy(jde_ctx* ctx);
const char* jde_status_str(int status);
const char* jde_last_error(void);

/* Number of convolutions and their shapes, in weight-blob order:
 * stem; per stage: down, then (c1, c2) per block; per head at strides 32, 16,
 * 8: set0..set4, det3, det1, emb, and lat (strides 32, 16 only). */
int jde_num_layers(const jde_ctx* ctx);
jde_status jde_layer_info(const jde_ctx* ctx, int i, int* cout, int* k, int* cin, int* stride);

/* ---- weights ------------------------------------------------------------ */

/* Length in floats of the host FP32 weight blob: per layer in blob order,
 * w[Cout][k][k][Cin] then b[Cout] (batch norm already folded into w, b). */
size_t jde_blob_floats(const jde_ctx* ctx);
/* Bytes of the device weight buffer in the context's precision. */
size_t jde_weights_bytes(const jde_ctx* ctx);
/* Converts the host blob (host, FP32, jde_blob_floats floats) to the device
 * format of the context's precision and copies it into d_weights (device,
 * >= jde_weights_bytes, 256-byte aligned).  Blocks until the copy is done.
 * The context keeps d_weights; the caller keeps it alive until jde_destroy. */
jde_status jde_load_weights(jde_ctx* ctx, const float* host_blob, size_t n_floats,
                            void* d_weights, size_t weights_bytes, void* stream);

/* ---- workspace ---------------------------------------------------------- */

/* Bytes of device workspace that jde_forward, jde_decode and jde_nms need for
 * any batch within the context's capacity (total pixels of a batch <=
 * max_pixels, or max_frames * max_h * max_w when that is 0; frames <=
 * max_frames). */
size_t jde_workspace_bytes(const jde_ctx* ctx);
/* Float counts of each head output for a batch: det[s] and emb[s] lengths. */
jde_status jde_head_sizes(const jde_ctx* ctx, const jde_frame_desc* descs, int n,
                          size_t det_floats[3], size_t emb_floats[3]);

/* Device bytes one frame of h x w occupies while it is in flight through
 * jde_forward and jde_decode in this context: its FP32 pixels, its head outputs
 * (det and emb, FP32), its detection rows (cap rows of box, score, margin,
 * index and E-wide embedding) and its share, by pixels, of the workspace.
 * 0 when h, w are not positive multiples of 32 or exceed the context's frame
 * size.  Host-only. */
size_t jde_frame_bytes(const jde_ctx* ctx, int h, int w);
/* Admission of waiting frames by device-memory budget (the serving pipeline of
 * Sec. 4.3-4.4, with frames of many video streams in flight at once): the
 * longest prefix of descs[0..n) -- at most max_frames frames -- whose
 * jde_frame_bytes, added to in_flight_bytes, stay within budget_bytes.
 * *n_admit (host) receives its length.  JDE_OK when at least one frame fits,
 * JDE_EBUDGET with *n_admit = 0 when the first frame does not, JDE_EINVAL on a
 * frame the context cannot hold.  Host-only. */
jde_status jde_admit(const jde_ctx* ctx, const jde_frame_desc* descs, int n, size_t in_flight_bytes,
                     size_t budget_bytes, int* n_admit);

/* ---- hot path ------------------------------------------------------------ */

/* Frame ingest (the capture stage of Sec. 4.4 feeds the model FullHD video;
 * Sec. 5.1 resizes it to 1088x608): n 8-bit RGB frames of src_h x src_w
 * (d_src: device, [n][src_h][src_w][3] bytes, back to back) -> the model input
 * of jde_forward (d_dst: device FP32 NCHW in [0, 1], frames packed back to back
 * at the sizes descs[0..n) (host)).  Letterbox: scale r = min(h / src_h,
 * w / src_w), the resized image (round(src_w r) x round(src_h r)) centred at
 * column (w - new_w) / 2 and row (h - new_h) / 2 (integer division), border 0.5;
 * bilinear resampling with aligned pixel centres (output column u samples
 * (u + 1/2) src_w / new_w - 1/2, clamped to the image), then / 255.  One pass
 * over the source and the output; n <= 64. */
jde_status jde_ingest(const uint8_t* d_src, int n, int src_h, int src_w, const jde_frame_desc* descs,
                      float* d_dst, void* stream);

/* Model forward over a batch (Sec. 3.1, Sec. 4.2).  d_frames: device FP32
 * NCHW pixels, frames packed back to back (frame f: 3*h_f*w_f floats).  descs:
 * host, n entries.  d_ws: device workspace (>= jde_workspace_bytes).  out:
 * host struct of device pointers sized by jde_head_sizes.  The frames and
 * workspace must stay valid until the stream reaches the end of the call. */
jde_status jde_forward(jde_ctx* ctx, const float* d_frames, const jde_frame_desc* descs, int n,
                       void* d_ws, size_t ws_bytes, const jde_head_out* out, void* stream);

/* Tile autotuner of the convolutions (batch-wise inference, Sec. 4.2, is only
 * as fast as its kernels on the batch shape used).  Runs one forward, then
 * times every tile configuration that fits each convolution (reps launches
 * each, on the stream; blocks until done) and keeps the fastest per launch for
 * later forwards of any batch.  Arguments as for jde_forward; the buffers hold
 * meaningless values afterwards. */
jde_status jde_autotune(jde_ctx* ctx, const float* d_frames, const jde_frame_desc* descs, int n,
                        void* d_ws, size_t ws_bytes, const jde_head_out* out, int reps, void* stream);
/* Reads (set = 0) or writes (set = 1) the tile choice of every forward launch:
 * tiles[n_ops] host, n_ops = number of forward launches (jde_profile_collect's
 * *n_ops); -1 = the built-in default.  Entries of non-MFMA launches are ignored
 * on write; a tile that does not fit its launch falls back to the default.
 * Tile 37 is the persistent pointwise kernel (1x1 convs of 256 -> 128 and
 * 512 -> 256 channels, BF16 / FP16: weights held in registers, pixel tiles
 * streamed through LDS; same summation order as the implicit GEMM). */
jde_status jde_tiles(jde_ctx* ctx, int* tiles, int n_ops, int set);

/* FP8 scaling (mixed precision, Sec. 4.1, taken to the e4m3 format of gfx950).
 * In a JDE_FP8 context the backbone 3x3 convolutions whose Cin is a multiple of
 * 128 run on e4m3 operands, and every 32 consecutive k of a row carry a power-of-two
 * (E8M0) scale that the matrix core applies: weights have a per-output-channel
 * scale max|w_c| / 448 and, inside it, one exponent per 32-k block (set by
 * jde_load_weights).  Input activations (stored BF16) are converted when staged:
 * with on != 0 (the default) each pixel's 32-channel block gets the smallest
 * power of two 2^s with max|x| / 2^s <= 448; with on = 0 one static per-tensor
 * scale from jde_calibrate serves the whole tensor.  JDE_EUNSUPPORTED outside a
 * JDE_FP8 context. */
jde_status jde_fp8_block_scales(jde_ctx* ctx, int on);
/* FP8 calibration for per-tensor activation scales (jde_fp8_block_scales off).
 * Runs one BF16 forward of the given batch, records the largest |value| each
 * convolution writes, and sets every FP8 launch's input scale to that of its
 * producer / 448.  Arguments as for jde_forward; blocks until done.  With block
 * scales off and before this has run, jde_forward of a JDE_FP8 context returns
 * JDE_ESTATE; jde_load_weights resets it. */
jde_status jde_calibrate(jde_ctx* ctx, const float* d_frames, const jde_frame_desc* descs, int n,
                         void* d_ws, size_t ws_bytes, const jde_head_out* out, void* stream);
/* Input scale of every forward launch (0 for launches that do not run in FP8);
 * in_scales: host, n_ops = number of forward launches. */
jde_status jde_fp8_scales(const jde_ctx* ctx, float* in_scales, int n_ops);
/* With on != 0 (the default), 16-bit contexts run the stem (3 -> c0 = 32) and
 * the first downsample conv (3x3 stride 2, 32 -> 64) as one launch that keeps the
 * stem's output in on-chip memory (Sec. 3.1 backbone; the result is the same
 * network, rounded the same way); on = 0 runs them as two launches.  Other
 * configurations always run unfused.  In jde_profile_collect the fused launch is
 * kind 2 at op 0 and op 1 is kind 3 with no time or FLOPs of its own. */
jde_status jde_fuse_stem(jde_ctx* ctx, int on);
/* With on != 0 (the default), 16-bit contexts run each residual block of 64 or
 * 128 channels (Sec. 3.1 backbone: 1x1 C -> C/2, 3x3 C/2 -> C, leaky, + input)
 * as one launch that keeps the C/2-channel intermediate in on-chip memory and
 * reads the block input once; on = 0 runs the two convs as two launches.  Same
 * network, same roundings.  Blocks whose convs run in FP8, and calibration
 * forwards, always run unfused.  In jde_profile_collect the fused launch is kind
 * 4 at the block's first conv and the second conv is kind 5 with no time or
 * FLOPs of its own. */
jde_status jde_fuse_blocks(jde_ctx* ctx, int on);
/* With on != 0 (the default), 16-bit contexts run each head's det 1x1 (Sec. 3.1
 * heads: det 3x3 F -> 2F with leaky, then a linear 1x1 2F -> 6A, 6A <= 32) in the
 * det 3x3's launch, where that launch runs on a direct-to-LDS tile whose
 * activated output tile fits its pipeline stages (not the 4-wave tiles of 32 K
 * elements) and whose channel width divides 2F: the 2F-channel output never goes
 * to memory.  The 1x1 multiplies the same storage-rounded values; a 3x3 tile
 * covering part of the 2F channels writes its FP32 partial sums to a workspace
 * buffer, and the last of a pixel range's tiles sums them in channel order, so
 * the result is deterministic (the same in a graph for any batch) but rounds
 * differently from the unfused 1x1 (FP32 sums in another order).  FP8
 * launches and calibration forwards always run unfused; on = 0 runs the 1x1 as its
 * own launch.  In jde_profile_collect the 3x3 launch is then kind 7 (its FLOPs
 * include the 1x1's) and the 1x1 kind 8 with no time or FLOPs of its own. */
jde_status jde_fold_det(jde_ctx* ctx, int on);
/* With on != 0 (the default), 16-bit contexts run the backbone's 3x3 stride-2
 * downsample convs with Cin 64 (Sec. 3.1: into the stride-4 level) with a
 * persistent window kernel: each workgroup keeps 128 output
 * channels' weights in registers and loads each tile's input window once into
 * on-chip memory, instead of gathering every input pixel 2.25 times through the
 * implicit GEMM's short K loop.  Same sums in the same order: bitwise equal.
 * FP8 launches and calibration forwards always run the implicit GEMM; on = 0
 * runs it everywhere.  In jde_profile_collect such a launch is kind 9. */
jde_status jde_window_down(jde_ctx* ctx, int on);
/* With on != 0 (default off), 16-bit contexts run each 3x3 stride-1 conv with
 * Cin % 64 == 0 and Cout % 128 == 0 (Sec. 3.1: the residual blocks of the deep
 * stages and the head convs) from an LDS window loaded once per 32-channel input
 * slice for all nine taps, when every frame's width at that level is <= 190;
 * on = 0 runs them as implicit GEMMs.  Same network; the FP32 accumulation runs
 * in another order (slice-major instead of tap-major), so results agree to
 * rounding, not bitwise.  FP8 launches are unaffected.  Off by default: with its
 * 144 KB of LDS one workgroup fills a compute unit, and its per-step barrier then
 * idles the matrix cores; the implicit GEMM is faster on MI355X. */
jde_status jde_window_convs(jde_ctx* ctx, int on);
/* With on != 0 (default off), the embedding branch of each head (3x3 conv F -> E,
 * linear + bias, Sec. 3.1) runs only where it is used: jde_forward runs the det
 * 3x3 conv alone and leaves out->emb unwritten (those pointers may be NULL),
 * and jde_decode computes each kept detection's embedding from the head's
 * feature map (kept in the workspace since the forward) at its cell -- the
 * same conv, K summed in the dense conv's (tap, channel) order in FP32 -- then
 * L2-normalises it.  The detections are the same as with the dense head; the
 * forward saves the emb convs' 21.3 GFLOP and 27.8 MB of FP32 output per
 * 608x1088 frame (Appendix A item 1 needs an embedding per detection only).
 * The feature maps stay valid until the next jde_forward on the workspace. */
jde_status jde_sparse_emb(jde_ctx* ctx, int on);
/* Host helper: x (host, n floats) -> OCP e4m3 codes (host, n bytes), round to
 * nearest even, saturating at +-448, NaN -> 0x7f; the encoding of the weights. */
void jde_fp8_encode(const float* x, uint8_t* out, size_t n);
/* Host helper: x (host, n floats) -> codes of FP6 E2M3 (fmt 2) or FP4 E2M1
 * (fmt 4), one code per byte in its low 6 / 4 bits (sign in the top one), round
 * to nearest even, saturating at +-7.5 / +-6; the encoding of those weights.
 * Any other fmt leaves out unchanged. */
void jde_mx_encode(int fmt, const float* x, uint8_t* out, size_t n);

/* Post-processing of Appendix A items 1-3 plus embedding normalisation, for
 * every frame of the batch: anchor decode, keep iff score >= conf_thr
 * (evaluated as (c_fg + off_f) - c_bg >= ln(conf_thr / (1 - conf_thr)) in FP32,
 * off_f = d_logit_offset[f], or 0 when d_logit_offset is NULL), sort by
 * (margin desc, index asc), keep the top cap, greedy NMS (suppress iff IoU
 * with an earlier kept box > nms_iou, FP32 predicate inter > thr * union), and
 * gather + L2-normalise the embedding at each kept anchor's cell.  The margin
 * and score written out include the offset.  d_logit_offset: device [n] FP32 or
 * NULL (a per-frame confidence offset, e.g. to set a video stream's density of
 * candidates).  heads as written by jde_forward; out: host struct of device
 * pointers. */
jde_status jde_decode(jde_ctx* ctx, const jde_head_out* heads, const jde_frame_desc* descs, int n,
                      float conf_thr, float nms_iou, const float* d_logit_offset, void* d_ws,
                      size_t ws_bytes, const jde_dets* out, void* stream);

/* Greedy NMS alone (Appendix A item 3) on one list of K <= max_candidates
 * candidates (device): boxes [K,4], margins [K], idx [K] (distinct).  Writes
 * the positions (into the inputs) of the kept boxes, in keep order, to d_keep
 * [K] and their number to d_nkeep [1]. */
jde_status jde_nms(jde_ctx* ctx, const float* d_boxes, const float* d_margins, const int* d_idx,
                   int K, float nms_iou, void* d_ws, size_t ws_bytes, int* d_keep, int* d_nkeep,
                   void* stream);

/* jde_nms without a workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same inputs, outputs and keep list as jde_nms, no context.  Its
 * scratch (8.3 MiB: keys, positions, sorted boxes, keep list and the K x K/64
 * suppression mask) is a static device array that the library holds on each GPU
 * it runs on until the process ends; the call allocates nothing.  K <= 8192,
 * else JDE_ECAPACITY before any work is enqueued.  Runs on the current device;
 * `stream` must belong to it.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams, other host threads) race and
 * must be serialised by the caller. */
jde_status jde_nms_noalloc(const float* d_boxes, const float* d_margins, const int* d_idx, int K,
                           float nms_iou, int* d_keep, int* d_nkeep, void* stream);

/* Tracks x detections cost (Appendix A items 5-6).  All pointers device.
 * track_emb [T,E] FP32, mean [T,8] FP64 (cx, cy, a, h, vcx, vcy, va, vh),
 * cov [T,8,8] FP64 (predicted state), det_boxes [D,4] FP32 (x1, y1, x2, y2),
 * det_emb [D,E] FP32.  cost [T,D] FP32 row-major:
 *   cost = +inf if d2 > gate_chi2, else clamp(1 - <f_t, e_d>, 0, 2),
 * d2 = (z - Hx)^T S^-1 (z - Hx), S = H P H^T + R(h), z = (cx, cy, w/h, h),
 * R = diag((h/20)^2, (h/20)^2, 0.1^2, (h/20)^2) with h the track's height,
 * solved in FP64 by Cholesky.  T, D >= 0; E multiple of 4. */
jde_status jde_cost_matrix(const float* d_track_emb, const double* d_mean, const double* d_cov, int T,
                           const float* d_det_boxes, const float* d_det_emb, int D, int E,
                           double gate_chi2, float* d_cost, void* stream);

/* The same cost against one frame of a jde_decode result, with D read from
 * dets->count[frame] on the device (no host round trip).  d_cost [T, cap]
 * (row stride cap = dets->cap); columns >= count[frame] are left untouched. */
jde_status jde_cost_matrix_dets(const float* d_track_emb, const double* d_mean, const double* d_cov,
                                int T, const jde_dets* dets, int frame, int E, double gate_chi2,
                                float* d_cost, void* stream);

/* The cost for every frame of a jde_decode result in one launch.  Frame f
 * (0 <= f < n) is scored against tracks [track_begin[f], track_begin[f+1]) of
 * the track arrays (e.g. the tracks of the video stream the frame belongs to)
 * and its rows start at row track_begin[f] of d_cost [track_begin[n], cap]
 * (row stride cap).  track_begin: host, n+1 non-decreasing ints, n <= 64.
 * D of each frame is read from dets->count[f] on the device. */
jde_status jde_cost_matrix_batch(const float* d_track_emb, const double* d_mean, const double* d_cov,
                                 const int* track_begin, const jde_dets* dets, int n, int E,
                                 double gate_chi2, float* d_cost, void* stream);

/* jde_cost_matrix_batch with motion fused into the cost (an association
 * variant beyond Appendix A, which uses the embedding distance gated by the
 * Kalman distance): where the gate passes, cost = (1 - w) clamp(1 - <f, e>, 0, 2)
 * + w d2 (evaluated in FP64, stored FP32), +inf where d2 > gate_chi2;
 * motion_weight w in [0, 1] (0 = jde_cost_matrix_batch). */
jde_status jde_cost_matrix_batch_fused(const float* d_track_emb, const double* d_mean, const double* d_cov,
                                       const int* track_begin, const jde_dets* dets, int n, int E,
                                       double gate_chi2, float motion_weight, float* d_cost, void* stream);
/* Box-overlap cost for a second association stage on the tracks and detections
 * the first stage left unmatched: d_cost [track_begin[n], cap] (row stride cap)
 * = 1 - IoU(track box, detection box) in FP64, stored FP32, where the track box
 * comes from its Kalman state (cx, cy, a, h): width a*h.  Batched layout as
 * jde_cost_matrix_batch; D of frame f from dets->count[f] on the device;
 * columns >= count[f] are left untouched. */
jde_status jde_iou_cost_batch(const double* d_mean, const int* track_begin, const jde_dets* dets, int n,
                              float* d_cost, void* stream);

/* Track embedding smoothing for matched pairs: f_t <- normalise(m f_t + (1-m) e_d)
 * (the track's appearance state follows its matched detections).  d_pairs
 * [P,2] int (t, d) device, each t at most once; pairs with t outside [0, T) or
 * d outside [0, D) are skipped.  d_det_emb [D,E], d_track_emb [T,E] FP32. */
jde_status jde_track_emb_update(const int* d_pairs, int P, const float* d_det_emb, int D,
                                float* d_track_emb, int T, int E, float momentum, void* stream);

/* ---- device-side association (Appendix A items 4 and 7) ------------------
 * The same FP64 arithmetic as the host jde_kf_* and jde_assign calls (operation
 * for operation, no contraction: bit-identical states, the same assignment),
 * run on the device so that a batch's association needs no host round trip.
 * Batched layout as for jde_cost_matrix_batch: frame f (0 <= f < n <= 64) owns
 * tracks [track_begin[f], track_begin[f+1]) (track_begin: host, n+1
 * non-decreasing ints) and detection rows [f*cap, f*cap + count[f]) of dets. */

/* Predicts T track states in place (device mean [T,8], cov [T,8,8], FP64), as
 * jde_kf_predict. */
jde_status jde_kf_predict_dev(int T, double* d_mean, double* d_cov, void* stream);
/* Kalman update of every track t with det_of_track[t] >= 0 (device [T]) by the
 * measurement of box f*cap + det_of_track[t] of dets (z = (cx, cy, w/h, h) of
 * the FP32 box), as jde_kf_update; tracks with -1 are untouched.  d_status
 * (device [T] or NULL): 1 where S was not positive definite (track untouched),
 * else 0. */
jde_status jde_kf_update_dev(const int* track_begin, int n, const int* d_det_of_track, const jde_dets* dets,
                             double* d_mean, double* d_cov, int* d_status, void* stream);
/* Min-cost assignment of every frame, as jde_assign, on the cost written by
 * jde_cost_matrix_batch (d_cost [track_begin[n], cap], row stride cap; D of
 * frame f read from dets->count[f] on the device).  One workgroup per frame
 * runs the shortest-augmenting-path method (Kuhn-Munkres, Jonker-Volgenant
 * form) with its state in LDS: at most 2048 tracks and 2048 detections per
 * frame (JDE_ECAPACITY for more tracks; a frame whose count exceeds 2048 gets
 * d_status[f] = 1 and no pairs).  Outputs (device): d_det_of_track [T] (the
 * detection's row within its frame, or -1), d_track_of_det [n*cap] (the track's
 * index within its frame, or -1), d_kept [n] pairs kept, d_total [n] FP64 sum of
 * their costs, d_status [n]. */
jde_status jde_assign_dev(const float* d_cost, const int* track_begin, int n, const jde_dets* dets,
                          float max_cost, int* d_det_of_track, int* d_track_of_det, int* d_kept,
                          double* d_total, int* d_status, void* stream);

/* ---- HIP graph of one step (batch-wise inference replayed as one launch) ---- */

typedef struct jde_graph jde_graph;
/* Captures, on `stream` (a non-default stream), one jde_forward + jde_decode
 * and, when track_begin is not NULL, one jde_cost_matrix_batch for a fixed
 * batch shape into a HIP graph.  All pointers are captured: between replays the
 * caller may change the contents of d_frames and of the track arrays, not the
 * buffers themselves.  Nothing runs during capture.  The graph uses no memset
 * nodes.  Fails with JDE_ESTATE while per-launch profiling is on. */
jde_status jde_graph_capture(jde_ctx* ctx, const float* d_frames, const jde_frame_desc* descs, int n,
                             void* d_ws, size_t ws_bytes, const jde_head_out* heads, float conf_thr,
                             float nms_iou, const float* d_logit_offset, const jde_dets* dets,
                             const float* d_track_emb,
                             const double* d_mean, const double* d_cov, const int* track_begin,
                             float* d_cost, void* stream, jde_graph** out);
/* Replays the captured step on `stream` (graphs of jde_graph_capture). */
jde_status jde_graph_launch(jde_graph* g, void* stream);
/* One graph for any batch within the context's capacity (batch-wise inference
 * of frames of several sizes, Sec. 4.2): captures jde_forward + jde_decode once,
 * with every launch sized for the capacity (max_frames frames, max_pixels
 * pixels) and reading the batch it works on from a header in the workspace;
 * jde_graph_launch_batch writes that header and the frame table for the given
 * batch (one small kernel on the stream) and replays the graph, so any mix of
 * frame sizes and counts within the capacity replays the same graph.  BF16 and
 * FP16 contexts with the fused stem (JDE_EUNSUPPORTED otherwise).  d_frames
 * holds the batch's frames packed back to back (as for jde_forward); heads
 * must be sized for the capacity (jde_head_sizes of max_frames frames of
 * max_h x max_w, or of the largest batch) and dets for max_frames frames;
 * d_logit_offset: device [max_frames] or NULL.  Detection counts of frames past
 * the batch read 0.  The batched cost (whose tracks per frame vary) is launched
 * after the replay. */
jde_status jde_graph_capture_any(jde_ctx* ctx, const float* d_frames, void* d_ws, size_t ws_bytes,
                                 const jde_head_out* heads, float conf_thr, float nms_iou,
                                 const float* d_logit_offset, const jde_dets* dets, void* stream,
                                 jde_graph** out);
/* Writes the header of batch descs[0..n) (host) and replays a graph of
 * jde_graph_capture_any on `stream`.  The batch is validated as for jde_forward. */
jde_status jde_graph_launch_batch(jde_graph* g, const jde_frame_desc* descs, int n, void* stream);
void jde_graph_destroy(jde_graph* g);

/* ---- per-launch timing of the forward (Sec. 5.1 profiles where time goes) -- */

/* on = 1: every later jde_forward records a HIP event pair around each of its
 * launches, on the launch stream, into a ring of 8 forwards (a 9th forward
 * first waits for the oldest ring entry).  Resets the accumulators.  on = 0
 * stops recording.  Not for use inside graph capture. */
jde_status jde_profile_begin(jde_ctx* ctx, int on);
/* Waits for the recorded events and returns, per forward launch i < *n_ops
 * (launch order; at most max_ops entries written): summed duration in ms over
 * the profiled forwards (op_ms), FLOPs of one launch for the last batch
 * (op_flop: 2*M*N*K), kind (op_kind: 0 = stem, 1 = MFMA conv; 2-5 = fused
 * launches, see jde_fuse_stem and jde_fuse_blocks; 6 = MFMA conv run by the
 * persistent pointwise kernel, tile 37 of jde_tiles; 7-8 see jde_fold_det; 9
 * see jde_window_down).  *n_fwd gets
 * the number of forwards summed.  All arrays host. */
jde_status jde_profile_collect(jde_ctx* ctx, int max_ops, double* op_ms, double* op_flop, int* op_kind,
                               int* n_ops, int* n_fwd);

/* ---- host FP64 association (Appendix A items 4, 7-9) --------------------- */

/* Kalman filter on the state (cx, cy, a, h, vcx, vcy, va, vh) with constant
 * velocity, stds scaled by the height h (process: h/20 position, h/160
 * velocity, 1e-2 / 1e-5 for a / va; measurement: h/20, and 0.1 for a).
 * All arrays host, row-major. */
void jde_kf_initiate(const double z[4], double mean[8], double cov[64]);
/* jde_kf_initiate for n measurements z [n,4] -> mean [n,8], cov [n,8,8]. */
void jde_kf_initiate_n(int n, const double* z, double* mean, double* cov);
/* Predicts T states in place (mean [T,8], cov [T,8,8]). */
void jde_kf_predict(int T, double* mean, double* cov);
/* Update with measurement z; Joseph-form covariance, symmetrised.
 * JDE_EINVAL if S is not positive definite. */
jde_status jde_kf_update(double mean[8], double cov[64], const double z[4]);
/* jde_kf_update for n (track, detection) pairs: track track_idx[i] (a row of
 * mean [*,8] / cov [*,8,8], updated in place) takes measurement z[det_idx[i]]
 * (z [*,4]).  Indices are not range-checked (the caller owns the arrays); a
 * track listed twice is updated twice, in order.  Returns JDE_OK, or JDE_EINVAL
 * when some S was not positive definite (those tracks are left unchanged, every
 * other pair is still applied). */
jde_status jde_kf_update_n(int n, const int* track_idx, const int* det_idx, double* mean, double* cov,
                           const double* z);

/* Kalman measurement of each detection box (Appendix A item 4 tracks boxes
 * with a Kalman filter): z = (cx, cy, w / h, h) in FP64 from the FP32 box
 * x1, y1, x2, y2 (w = x2 - x1, h = y2 - y1).  boxes [n,4], z [n,4], host. */
void jde_box_to_z(int n, const float* boxes, double* z);

/* Min-cost assignment (Hungarian) on cost [T,D] (host, FP32, row-major):
 * entries > max_cost (and +inf) are forbidden; among complete matchings the
 * one with the most allowed pairs, then the least total cost, is chosen, and
 * forbidden pairs are dropped.  det_of_track [T] / track_of_det [D] (host)
 * receive the partner index or -1; *total (host, may be NULL) the kept cost.
 * Returns the number of kept pairs, or a negative jde_status. */
int jde_assign(const float* cost, int T, int D, float max_cost, int* det_of_track,
               int* track_of_det, double* total);

#ifdef __cplusplus
}
#endif
#endif /* JDE_H */
