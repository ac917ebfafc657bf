// Internal declarations of libjde (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "jde.h"

namespace jde {

typedef __bf16 bf16;
typedef _Float16 f16;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr int kMaxFrames = 64;     // frames per batch
constexpr int kLevels = 6;         // strides 1, 2, 4, 8, 16, 32
constexpr int kMaxCap = 8192;      // per-frame candidate cap entering NMS
constexpr int kSortLds = 4096;     // keys sorted in LDS; larger lists sort in global memory

// Per-frame geometry of a batch, stored in device memory (int32 each):
//   [0] h, [1] w of the frame (pixels),
//   [2 + l] first packed pixel of the frame at level l (stride 2^l), l = 0..5,
//   [8 + l] = [2 + l] of the next frame (so a frame's range is [2+l], [8+l]).
constexpr int kGeomInts = 14;

enum ElemType { kF32 = 0, kBF16 = 1, kF16 = 2, kFP8 = 3 };

// Batch header in device memory for launches that serve any batch within the
// capacity (a captured graph replayed for different mixes of frame sizes): the
// host writes it, with the geometry table, before each replay; grids are sized
// for the capacity and work past the batch exits.
constexpr int kDynN = 0;          // frames in the batch
constexpr int kDynUniform = 1;    // all frames the same size
constexpr int kDynM = 2;          // [2 + l]: pixels of the batch at level l (l = 0..5)
constexpr int kDynStemTiles = 8;  // tiles of the fused stem + first downsample
constexpr int kDynRb64 = 9;       // tiles of the fused 64-channel residual blocks
constexpr int kDynRb128 = 10;     // tiles of the fused 128-channel residual blocks
constexpr int kDynInts = 16;

inline size_t elem_bytes(int t) { return t == kF32 ? 4 : (t == kFP8 ? 1 : 2); }

// Arguments of one convolution launch (implicit GEMM: M = output pixels of the
// batch, N = output channels, K = k*k*Cin).
struct ConvArgs {
    const void* in;        // NHWC input, level lvl_in (for concat: the half-res source)
    const void* in2;       // concat: the skip source (same level as the output), else null
    const void* w;         // [Cout][k][k][Cin]
    const float* bias;     // [Cout]
    const float* wscale;   // FP8: per-output-channel weight dequantisation scale, else null
    const unsigned char* wbscale;  // FP8: E8M0 exponent per output channel and 32-k block [Cout][K/32]
    const void* res;       // residual [M][Cout] (same type as out0), or null
    void* out0;            // [M][ld0], columns [0, n_split)
    float* out1;           // [M][ld1] FP32, columns [n_split, Cout) (linear), or null
    const int* geom;       // [nframes][kGeomInts]
    int nframes;
    int uniform;           // all frames the same size (row -> frame by division)
    int lvl_in, lvl_out;
    int cin, cout, ksz, stride, pad;
    int cin1;              // concat: channels taken from `in` (upsampled x2); 0 = no concat
    int K;                 // ksz*ksz*cin
    int M;                 // output pixels of the batch
    int n_split;           // columns < n_split go to out0
    int ld0, ld1;
    int act;               // leaky ReLU 0.1 on out0 columns
    int out0_f32;          // out0 holds FP32 (head outputs) instead of the activation type
    float in_scale;        // FP8: per-tensor scale of the input activations (x ~= in_scale * q);
                           // 1 with act_blocks
    int act_blocks;        // FP8: input activations take an E8M0 scale per pixel and 32 channels
    int mx_fmt;            // element format of the block-scaled operands: 0 e4m3, 2 FP6 E2M3, 4 FP4 E2M1
    int in_bytes, in2_bytes, w_bytes;  // sizes of the in / in2 / w buffers (< 2^31): loads past them read 0
    int n_major;           // tile order per XCD: 1 = pixel tiles of a channel range (weights dominate)
    unsigned* amax;        // calibration: max |out0| folded in with atomicMax on the float bits, or null
    const int* dyn;        // batch header (kDyn*): M, nframes, uniform read from it; M above is then the
                           // capacity the grid was sized for; null = the values above
    // Det 1x1 folded into this conv's epilogue (conv_tile_folds_det tiles only), or
    // det_w null: the 1x1 (det_n x n_split, linear) runs on the activated, storage-
    // rounded columns [0, n_split) in place of storing them to out0.
    const void* det_w;     // [det_n][n_split], storage type
    const float* det_b;    // [det_n]
    float* det_out;        // [M][det_n] FP32 head output
    float* det_part;       // [M][n_split / BN][det_n] FP32 partial sums of the channel tiles
    unsigned* det_cnt;     // per pixel tile: channel tiles finished; 0 between launches
    int det_n;             // det_n % 4 == 0, <= 32
};

// Launchers (conv.hip).
hipError_t launch_stem(const float* frames, const int* geom, int nframes, int uniform, int rows, int max_w,
                       int M, const float* w, const float* bias, int cout, void* out, int out_type,
                       hipStream_t s);
hipError_t launch_conv(const ConvArgs& a, int elem_type, int tile_cfg, hipStream_t s);
// Tiles whose launches can take the det 1x1 in their epilogue (ConvArgs::det_w)
// for a det 3x3 of n_split det channels (whole channel tiles only), in eager
// launches and graphs for any batch alike.
bool conv_tile_folds_det(int tile_cfg, int elem_type, int n_split);
// Stem fused with the first 3x3 stride-2 conv (c0 = 32 -> 64, 16-bit storage):
// frames -> stride-2 level output; `tiles` = sum over frames of stem_down_tiles(h, w).
hipError_t launch_stem_down(const float* frames, const int* geom, int nframes, int tiles, const float* w0,
                            const float* b0, const void* w1, const float* b1, void* out, int out_type,
                            hipStream_t s, const int* dyn = nullptr);
int stem_down_tiles(int h, int w);
// Residual block (1x1 C -> C/2, 3x3 C/2 -> C, + x) as one launch, 16-bit storage,
// C = 64 or 128, all at level lvl; out must not alias x.  `tiles` = sum over
// frames of resblock_tiles(C, h, w) with the level's frame sizes.
hipError_t launch_resblock(const void* x, void* out, const void* w1, const float* b1, const void* w2,
                           const float* b2, const int* geom, int nframes, int lvl, int C, int tiles, size_t x_bytes,
                           int et, hipStream_t s, const int* dyn = nullptr);
int resblock_tiles(int C, int h, int w);
// 3x3 stride-1 convolution from an LDS window (16-bit storage): applies when
// conv3w_ok and every frame's level width is <= kW3MaxW; `pixel_tiles` = sum over
// frames of conv3w_tiles(h, w) at the level.
constexpr int kW3MaxW = 190;
bool conv3w_ok(const ConvArgs& a, int et);
int conv3w_tiles(int h, int w);
hipError_t launch_conv3w(const ConvArgs& a, int et, int pixel_tiles, hipStream_t s);
// 3x3 stride-2 convolution from an LDS window (16-bit storage, bias + leaky, no
// concat, no residual) where down_win_ok: level lvl_in -> lvl_in + 1 of every
// frame, bitwise equal to the implicit GEMM.
bool down_win_ok(int cin, int cout, int ksz, int stride, int et);
hipError_t launch_down_win(const void* in, void* out, const void* w, const float* bias, const int* geom, int nframes,
                           int lvl_in, int cin, int cout, int et, hipStream_t s, const int* dyn = nullptr);
// FP8 e4m3 convolution: BF16 activations quantised on load with in_scale, FP8
// weights with per-channel wscale; needs cin % 128 == 0 and no concat.
hipError_t launch_conv_fp8(const ConvArgs& a, int tile_cfg, hipStream_t s);
int conv_fp8_num_tiles();
bool conv_fp8_ok(const ConvArgs& a);
int conv_num_tile_cfgs();
bool conv_tile_ok(int tile_cfg, int elem_type, const ConvArgs& a);
int conv_default_tile(int elem_type, const ConvArgs& a);
void conv_tile_shape(int tile_cfg, int* bm, int* bn);
// Tile config that selects the persistent pointwise (1x1) kernel.
bool conv_tile_pw(int tile_cfg);

// Post-processing launchers (post.hip).
struct DecodeArgs {
    const float* det[3];
    const int* geom;
    int nframes;
    int A;
    float anchors[3][4][2];
    float lthr;              // ln(thr / (1 - thr)) in FP32
    const float* logit_offset;  // [nframes] added to every c_fg of the frame, or null
    const int* dyn;          // batch header: frames >= its kDynN exit; null = all nframes
    int keycap;              // key slots per frame
    unsigned long long* keys;  // [n][keycap]
    int* vals;               // [n][keycap]
    int* cand_count;         // [n]
};
hipError_t launch_decode(const DecodeArgs& a, int max_anchors, hipStream_t s);
// Writes the batch geometry table and zeroes `ncount` ints (graph-safe: a kernel, no memset).
struct GeomParams { int n; int hw[kMaxFrames][2]; };
hipError_t launch_setup(const GeomParams& p, int* geom, int* counters, int ncount, hipStream_t s);
// The same plus the batch header (host-computed, kDynInts ints) written to dyn,
// zeroing three counter ranges.
struct DynHeader { int v[kDynInts]; };
hipError_t launch_setup_dyn(const GeomParams& p, const DynHeader& h, int* geom, int* dyn, int* counters,
                            int ncount, int* counters2, int ncount2, int* counters3, int ncount3, hipStream_t s);
hipError_t launch_sort(unsigned long long* keys, int* vals, const int* counts, int keycap, int n,
                       hipStream_t s);
struct GatherArgs {
    const float* det[3];
    const int* geom;
    int A;
    float anchors[3][4][2];
    const unsigned long long* keys;
    const int* cand_count;
    int keycap;
    int cap;
    float* sboxes;           // [n][cap][4]
    int* kcount;             // [n] min(count, cap)
};
hipError_t launch_gather_boxes(const GatherArgs& a, int n, hipStream_t s);
hipError_t launch_nms(const float* sboxes, const int* kcount, int cap, float thr,
                      unsigned long long* mask, int* keep, int* nkeep, int n, hipStream_t s);
struct EmitArgs {
    const float* emb[3];
    const int* geom;
    int A, E;
    const unsigned long long* keys;  // sorted
    int keycap, cap;
    const float* sboxes;
    const int* keep;                 // [n][cap] positions in sorted order
    const int* nkeep;                // [n]
    const int* cand_count;           // [n]
    float* boxes; float* scores; float* margins; float* emb_out;
    int* anchor_idx; int* count; int* n_cand; int* overflow;
    int* work;                       // deferred embedding: [3][work_cap][3] (row, frame, cell), or null
    int* work_count;                 // [3]
    int work_cap;
};
// Deferred sparse embedding head (post.hip): the emb 3x3 conv at kept cells only.
struct SparseEmbArgs {
    const void* feat[3];             // head feature maps F[s] channels, NHWC at level 3 + s (storage type)
    const void* w[3];                // emb conv weights [E][9 F] (storage type), K = (tap, channel)
    const float* bias[3];            // [E]
    int F[3];
    int E;
    const int* geom;
    const int* work;                 // [3][work_cap][3]
    const int* count;                // [3]
    int work_cap;
    float* out;                      // dets emb rows [n * cap][E] (raw, then normalised)
};
hipError_t launch_sparse_emb(const SparseEmbArgs& a, int et, int n, int cap, const int* nkeep, hipStream_t s);
hipError_t launch_emit(const EmitArgs& a, int n, hipStream_t s);
hipError_t launch_nms_prepare(const float* boxes, const float* margins, const int* idx, int K,
                              unsigned long long* keys, int* vals, int* count, hipStream_t s);
hipError_t launch_nms_gather(const float* boxes, const unsigned long long* keys, const int* vals,
                             int K, float* sboxes, int* kcount, hipStream_t s);
hipError_t launch_nms_finish(const int* keep, const int* nkeep, const int* vals, int* out_keep,
                             int* out_nkeep, int K, hipStream_t s);
hipError_t launch_cost(const float* trk_emb, const double* mean, const double* cov, int T,
                       const float* det_boxes, const float* det_emb, int D, const int* dcount, int ldc,
                       int E, double gate, float* cost, hipStream_t s);
struct CostBatch { int n; int begin[kMaxFrames + 1]; };
hipError_t launch_cost_batch(const float* trk_emb, const double* mean, const double* cov, const CostBatch& b,
                             int max_t, const float* det_boxes, const float* det_emb, const int* dcount, int cap,
                             int E, double gate, float* cost, hipStream_t s, float motion_w = 0.f);
hipError_t launch_iou_cost(const double* mean, const CostBatch& b, int max_t, const float* boxes, const int* dcount,
                           int cap, float* cost, hipStream_t s);
// Frame ingest (ingest.hip): 8-bit RGB [n][src_h][src_w][3] -> packed NCHW FP32.
struct IngestFrame {
    int h, w;                // model input size of the frame
    int new_h, new_w;        // resized image inside it
    int top, left;           // its position (the rest is the 0.5 border)
    size_t dst_off;          // first float of the frame in the packed output
};
struct IngestArgs {
    const unsigned char* src;
    int n, src_h, src_w;
    float* dst;
    IngestFrame fr[kMaxFrames];
};
hipError_t launch_ingest(const IngestArgs& a, int max_pix, hipStream_t s);

// Device association (assoc.hip).  Frame f of a batch owns tracks [begin[f], begin[f+1]).
typedef CostBatch AssocBatch;
constexpr int kAssignMax = 2048;   // most rows / columns of one frame's assignment (LDS-resident)
hipError_t launch_kf_predict(int T, double* mean, double* cov, hipStream_t s);
hipError_t launch_kf_update(const AssocBatch& b, int max_t, const int* det_of_track, const float* boxes, int cap,
                            double* mean, double* cov, int* status, hipStream_t s);
size_t assign_lds_bytes(int max_dim);
hipError_t launch_assign(const float* cost, const AssocBatch& b, int max_dim, const int* dcount, int cap,
                         float max_cost, int* det_of_track, int* track_of_det, int* kept, double* total, int* status,
                         hipStream_t s);
hipError_t launch_emb_update(const int* pairs, int P, const float* det_emb, int D, float* trk_emb, int T,
                             int E, float momentum, hipStream_t s);

// Host-side weight conversion helpers (api.cpp).
uint16_t f32_to_bf16_rne(float x);
uint16_t f32_to_f16_rne(float x);
uint8_t f32_to_e4m3(float x);

}  // namespace jde
