// C ABI of libjde: context, layer plan, workspace planner, weight packing, and
// the orchestration of the forward, decode, NMS and cost launches.
#include <math.h>

#include <cmath>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "jde_internal.h"

using namespace jde;

namespace {

thread_local std::string g_err;

jde_status fail(jde_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
jde_status fail(jde_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return fail(JDE_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// One convolution of the weight blob.
struct Layer {
    int cout, k, cin, stride;
    size_t blob_w, blob_b;   // float offsets in the host blob
};

enum OpKind { OP_STEM = 0, OP_CONV = 1 };
enum { HEAD_NONE = -1 };

// One launch of the forward.
struct Op {
    int kind;
    int layer, layer2;       // weights (layer2: fused second GEMM sharing the input, or -1)
    int in_t, in2_t, res_t, out_t;
    int det_out;             // scale index if out0 is the det head output (FP32), else -1
    int emb_out;             // scale index if out1 is the emb head output (FP32), else -1
    int lvl_in, lvl_out, cin, cout, ksz, stride, cin1, n_split, act;
    size_t dev_w, dev_b;     // byte offsets in the device weight buffer
    int tile;                // tile configuration (-1: default)
    int fp8;                 // runs as an FP8 e4m3 convolution once calibrated
    size_t dev_w8, dev_ws;   // FP8 weights [Cout][K] and their per-channel scales
    size_t dev_wbs;          // FP8: E8M0 exponent per output channel and 32-k block [Cout][K/32]
    float in_scale;          // per-tensor scale of the input activations (calibrated)
    int producer;            // op whose output this op reads (-1: the stem or none)
    int tile8;               // FP8 tile configuration
};

struct Tensor {
    int lvl, ch;
    int first, last;         // op indices of definition and last use
    size_t off, bytes;
};

}  // namespace

struct jde_ctx {
    jde_config cfg;
    size_t cap_pix = 0;              // most pixels a batch may hold (max_pixels or frames x max size)
    int et;                          // element type of activations / conv operands
    std::vector<Layer> layers;
    std::vector<Op> ops;
    std::vector<Tensor> tens;
    size_t blob_floats = 0;
    size_t weights_bytes = 0;
    size_t arena_bytes = 0;
    // decode scratch layout (byte offsets in the workspace)
    size_t ws_geom = 0, ws_counts = 0, ws_keys = 0, ws_vals = 0, ws_sboxes = 0, ws_kcount = 0, ws_mask = 0,
           ws_keep = 0, ws_nkeep = 0, ws_total = 0;
    int keycap = 0, cap = 0, max_anchors = 0;
    char* d_weights = nullptr;
    bool loaded = false;
    int n_backbone_ops = 0;
    bool fp8 = false, fp8_ready = false, calibrating = false;
    bool fp8_blocks = true;   // FP8 activations with an E8M0 scale per pixel and 32 channels
    int mx_fmt = 0;           // element format of the FP8-class convs: 0 e4m3, 2 FP6 E2M3, 4 FP4 E2M1
    // The stem and the first downsample conv run as one launch (16-bit storage),
    // and so do the two convs of each 64- and 128-channel residual block.
    // launch_kind[i] records how op i ran in the latest forward: 0 = its own
    // launch, 2 / 4 = head of a fused stem / residual-block launch, 3 / 5 = run
    // inside the previous op's fused launch, 6 = its own launch of the persistent
    // pointwise kernel, 7 = a det 3x3 launch that also runs the det 1x1, 8 = that
    // det 1x1 (no launch of its own), 9 = a downsample conv run by the window
    // kernel (window_down).
    bool fuse_stem = true, fuse_blocks = true;
    // The det 1x1 of each head runs in its det 3x3's epilogue (16-bit storage, the
    // 3x3 on a conv_tile_folds_det tile); its partial sums and per-pixel-tile
    // counters live in the workspace.
    bool fold_det = true;
    // The 3x3 stride-2 downsample convs with Cin 64 (16-bit storage) run
    // from an LDS window (down_win_kernel) instead of the implicit GEMM.
    bool window_down = true;
    size_t ws_det_part = 0, ws_det_cnt = 0;
    int det_cnt_n = 0;
    // 3x3 stride-1 convs run from an LDS window (conv3_win) where they qualify;
    // off by default: measured slower than the implicit GEMM on MI355X.
    bool window_convs = false;
    // Deferred sparse embedding head: the emb 3x3 convs run in jde_decode at
    // kept cells only (jde_sparse_emb); their inputs stay live in the arena.
    bool sparse_emb = false;
    int emb_op[3] = {-1, -1, -1};    // per scale (stride 8, 16, 32): the det3+emb op
    size_t ws_work = 0, ws_work_count = 0;
    size_t ws_dyn = 0;               // batch header of graphs that serve any batch (kDyn*)
    std::vector<int> launch_kind;
    size_t ws_amax = 0;
    // Per-launch timing: a ring of event pairs, one entry per profiled forward.
    static constexpr int kRing = 8;
    bool prof = false;
    std::vector<hipEvent_t> ev;          // [kRing][ops][2]
    bool pending[kRing] = {};
    int ring_pos = 0;
    std::vector<double> op_ms, op_flop;
    int n_fwd = 0;
    ~jde_ctx() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

namespace {

int ilog2(int x) {
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

// Builds the layer list (blob order) and the op list (launch order).
void build_plan(jde_ctx* c) {
    const jde_config& g = c->cfg;
    auto add_layer = [&](int cout, int k, int cin, int stride) {
        Layer L{cout, k, cin, stride, 0, 0};
        L.blob_w = c->blob_floats;
        c->blob_floats += (size_t)cout * k * k * cin;
        L.blob_b = c->blob_floats;
        c->blob_floats += cout;
        c->layers.push_back(L);
        return (int)c->layers.size() - 1;
    };
    auto add_tensor = [&](int lvl, int ch) {
        c->tens.push_back(Tensor{lvl, ch, -1, -1, 0, 0});
        return (int)c->tens.size() - 1;
    };
    auto add_op = [&](int kind, int layer, int in_t, int out_t, int lvl_in, int lvl_out) {
        Op o{};
        o.kind = kind;
        o.layer = layer;
        o.layer2 = -1;
        o.in_t = in_t;
        o.in2_t = -1;
        o.res_t = -1;
        o.out_t = out_t;
        o.det_out = HEAD_NONE;
        o.emb_out = HEAD_NONE;
        o.lvl_in = lvl_in;
        o.lvl_out = lvl_out;
        const Layer& L = c->layers[layer];
        o.cin = L.cin;
        o.cout = L.cout;
        o.ksz = L.k;
        o.stride = L.stride;
        o.cin1 = 0;
        o.n_split = L.cout;
        o.act = 1;
        o.tile = -1;
        o.fp8 = 0;
        o.in_scale = 1.f;
        o.producer = -1;
        o.tile8 = 0;
        c->ops.push_back(o);
        return (int)c->ops.size() - 1;
    };

    int ch = g.base_ch;
    const int stem = add_layer(ch, 3, 3, 1);
    int x = add_tensor(0, ch);
    add_op(OP_STEM, stem, -1, x, 0, 0);
    int feat[6] = {-1, -1, -1, -1, -1, -1};
    for (int s = 1; s <= 5; ++s) {
        const int down = add_layer(2 * ch, 3, ch, 2);
        ch *= 2;
        const int t = add_tensor(s, ch);
        add_op(OP_CONV, down, x, t, s - 1, s);
        x = t;
        // Blocks of 64 and 128 channels write a new tensor (the fused block
        // launch reads a halo of x around each output tile); the others run in
        // place.  Either way out = leaky(conv) + x.
        const bool out_of_place = ch == 64 || ch == 128;
        for (int b = 0; b < g.blocks[s - 1]; ++b) {
            const int c1 = add_layer(ch / 2, 1, ch, 1);
            const int c2 = add_layer(ch, 3, ch / 2, 1);
            const int mid = add_tensor(s, ch / 2);
            add_op(OP_CONV, c1, x, mid, s, s);
            const int y = out_of_place ? add_tensor(s, ch) : x;
            const int o = add_op(OP_CONV, c2, mid, y, s, s);
            c->ops[o].res_t = x;
            x = y;
        }
        feat[s] = x;
    }
    c->n_backbone_ops = (int)c->ops.size();
    const int nout = 6 * g.num_anchors;
    int lat = -1, lat_c = 0;
    const int lv[3] = {5, 4, 3};
    for (int h = 0; h < 3; ++h) {
        const int L = lv[h];
        const int cl = c->tens[feat[L]].ch;
        const int F = cl / 2;
        const int cin0 = cl + lat_c;
        const int set0 = add_layer(F, 1, cin0, 1);
        const int set1 = add_layer(2 * F, 3, F, 1);
        const int set2 = add_layer(F, 1, 2 * F, 1);
        const int set3 = add_layer(2 * F, 3, F, 1);
        const int set4 = add_layer(F, 1, 2 * F, 1);
        const int det3 = add_layer(2 * F, 3, F, 1);
        const int det1 = add_layer(nout, 1, 2 * F, 1);
        const int emb = add_layer(g.emb_dim, 3, F, 1);
        int lat_layer = -1;
        if (L != 3) lat_layer = add_layer(F / 2, 1, F, 1);

        int t0 = add_tensor(L, F);
        int o = add_op(OP_CONV, set0, lat < 0 ? feat[L] : lat, t0, lat < 0 ? L : L + 1, L);
        if (lat >= 0) {
            c->ops[o].in2_t = feat[L];
            c->ops[o].cin1 = lat_c;
        }
        int t1 = add_tensor(L, 2 * F);
        add_op(OP_CONV, set1, t0, t1, L, L);
        int t2 = add_tensor(L, F);
        add_op(OP_CONV, set2, t1, t2, L, L);
        int t3 = add_tensor(L, 2 * F);
        add_op(OP_CONV, set3, t2, t3, L, L);
        int t4 = add_tensor(L, F);
        add_op(OP_CONV, set4, t3, t4, L, L);
        // det 3x3 (leaky, to a tensor) and emb 3x3 (linear, FP32 head output) as one GEMM
        int td = add_tensor(L, 2 * F);
        o = add_op(OP_CONV, det3, t4, td, L, L);
        c->ops[o].layer2 = emb;
        c->ops[o].cout = 2 * F + g.emb_dim;
        c->ops[o].n_split = 2 * F;
        c->ops[o].emb_out = L - 3;
        o = add_op(OP_CONV, det1, td, -1, L, L);
        c->ops[o].det_out = L - 3;
        c->ops[o].act = 0;
        if (lat_layer >= 0) {
            lat = add_tensor(L, F / 2);
            lat_c = F / 2;
            add_op(OP_CONV, lat_layer, t4, lat, L, L);
        }
    }
}

// Liveness-based first-fit arena over the op sequence, sized for the capacity.
void plan_arena(jde_ctx* c) {
    const size_t pix0 = c->cap_pix;
    const size_t eb = elem_bytes(c->et);
    for (auto& t : c->tens) {
        t.first = -1;
        t.last = -1;
        t.bytes = align256((pix0 >> (2 * t.lvl)) * t.ch * eb);
    }
    for (int i = 0; i < (int)c->ops.size(); ++i) {
        const Op& o = c->ops[i];
        const int reads[3] = {o.in_t, o.in2_t, o.res_t};
        for (int r : reads)
            if (r >= 0) c->tens[r].last = std::max(c->tens[r].last, i);
        if (o.out_t >= 0) {
            Tensor& t = c->tens[o.out_t];
            if (t.first < 0) t.first = i;
            t.last = std::max(t.last, i);
        }
        // the emb conv's input outlives the forward: the sparse emb head reads it in jde_decode
        if (o.emb_out >= 0) {
            c->tens[o.in_t].last = (int)c->ops.size();
            c->emb_op[o.emb_out] = i;
        }
    }
    struct Block { size_t off, bytes; int tensor; };
    std::vector<Block> live;
    size_t top = 0;
    for (int i = 0; i < (int)c->ops.size(); ++i) {
        live.erase(std::remove_if(live.begin(), live.end(),
                                  [&](const Block& b) { return c->tens[b.tensor].last < i; }),
                   live.end());
        const int ot = c->ops[i].out_t;
        if (ot < 0 || c->tens[ot].first != i) continue;
        Tensor& t = c->tens[ot];
        std::sort(live.begin(), live.end(), [](const Block& a, const Block& b) { return a.off < b.off; });
        size_t cur = 0;
        for (const Block& b : live) {
            if (b.off >= cur + t.bytes) break;
            cur = std::max(cur, b.off + b.bytes);
        }
        t.off = cur;
        live.push_back(Block{cur, t.bytes, ot});
        top = std::max(top, cur + t.bytes);
    }
    c->arena_bytes = align256(top);
}

// FP8 launches: backbone convolutions whose Cin is a multiple of 128 (every
// 128-wide K chunk then lies in one tap).  Each op also learns its producer.
void plan_fp8(jde_ctx* c) {
    for (int i = 0; i < (int)c->ops.size(); ++i) {
        Op& o = c->ops[i];
        for (int j = i - 1; j >= 0; --j)
            if (c->ops[j].out_t >= 0 && c->ops[j].out_t == o.in_t) {
                o.producer = j;
                break;
            }
        // FP8 where the matrix cores bound the conv: the backbone's 3x3 convs (the 1x1
        // convs move 2-3 FLOP per byte of BF16 activations, which FP8 operands do not cut)
        o.fp8 = c->fp8 && o.kind == OP_CONV && i < c->n_backbone_ops && o.ksz == 3 && o.cin % 128 == 0 &&
                o.cin1 == 0 && o.producer >= 0;
    }
}

void plan_weights(jde_ctx* c) {
    size_t off = 0;
    const size_t eb = elem_bytes(c->et);
    for (auto& o : c->ops) {
        const int K = o.ksz * o.ksz * o.cin;
        const size_t wb = (o.kind == OP_STEM) ? (size_t)o.cout * K * 4 : (size_t)o.cout * K * eb;
        o.dev_w = off;
        off = align256(off + wb);
        o.dev_b = off;
        off = align256(off + (size_t)o.cout * 4);
        if (o.fp8) {
            o.dev_w8 = off;
            off = align256(off + (size_t)o.cout * K);
            o.dev_ws = off;
            off = align256(off + (size_t)o.cout * 4);
            o.dev_wbs = off;
            off = align256(off + (size_t)o.cout * (K / 32));
        }
    }
    c->weights_bytes = off;
}

void plan_decode_scratch(jde_ctx* c) {
    const jde_config& g = c->cfg;
    const int H = g.max_h, W = g.max_w, A = g.num_anchors;
    c->max_anchors = ((H >> 3) * (W >> 3) + (H >> 4) * (W >> 4) + (H >> 5) * (W >> 5)) * A;
    int kc = 1;
    while (kc < c->max_anchors) kc <<= 1;
    int kcap = 1;
    while (kcap < g.max_candidates) kcap <<= 1;
    c->keycap = std::max(kc, kcap);
    c->cap = g.max_candidates;
    const size_t n = g.max_frames;
    size_t off = c->arena_bytes;
    c->ws_geom = off;   off = align256(off + n * kGeomInts * 4);
    c->ws_counts = off; off = align256(off + n * 4);
    c->ws_kcount = off; off = align256(off + n * 4);
    c->ws_nkeep = off;  off = align256(off + n * 4);
    c->ws_keys = off;   off = align256(off + n * c->keycap * 8);
    c->ws_vals = off;   off = align256(off + n * c->keycap * 4);
    c->ws_sboxes = off; off = align256(off + n * c->cap * 16);
    c->ws_mask = off;   off = align256(off + n * (size_t)c->cap * (c->cap / 64) * 8);
    c->ws_keep = off;   off = align256(off + n * c->cap * 4);
    c->ws_amax = off;   off = align256(off + c->ops.size() * 4);
    c->ws_work = off;   off = align256(off + (size_t)3 * n * c->cap * 3 * 4);
    c->ws_work_count = off; off = align256(off + 3 * 4);
    c->ws_dyn = off;    off = align256(off + kDynInts * 4);
    // det 1x1 folded into the det 3x3: partials [M][2F / 64][nout] of the largest
    // head, and a counter per 64-pixel tile
    size_t part = 0, tiles = 0;
    for (const Op& o : c->ops)
        if (o.det_out >= 0) {
            const size_t m = c->cap_pix >> (2 * o.lvl_out);
            part = std::max(part, m * (size_t)(o.cin / 64) * o.cout * 4);
            tiles = std::max(tiles, (m + 63) / 64);
        }
    c->det_cnt_n = (int)tiles;
    c->ws_det_part = off; off = align256(off + part);
    c->ws_det_cnt = off;  off = align256(off + tiles * 4);
    c->ws_total = off;
}

jde_status batch_ok(const jde_ctx* c, const jde_frame_desc* d, int n, bool* uniform) {
    if (!d || n <= 0) return fail(JDE_EINVAL, "empty batch");
    if (n > c->cfg.max_frames || n > kMaxFrames)
        return fail(JDE_ECAPACITY, "batch of %d frames exceeds capacity %d", n, c->cfg.max_frames);
    size_t pix = 0;
    *uniform = true;
    for (int i = 0; i < n; ++i) {
        if (d[i].h <= 0 || d[i].w <= 0 || d[i].h % 32 || d[i].w % 32)
            return fail(JDE_EINVAL, "frame %d: %dx%d not a positive multiple of 32", i, d[i].h, d[i].w);
        if (d[i].h > c->cfg.max_h || d[i].w > c->cfg.max_w)
            return fail(JDE_ECAPACITY, "frame %d: %dx%d exceeds max %dx%d", i, d[i].h, d[i].w, c->cfg.max_h,
                        c->cfg.max_w);
        pix += (size_t)d[i].h * d[i].w;
        if (d[i].h != d[0].h || d[i].w != d[0].w) *uniform = false;
    }
    if (pix > c->cap_pix)
        return fail(JDE_ECAPACITY, "batch of %zu pixels exceeds the capacity of %zu", pix, c->cap_pix);
    return JDE_OK;
}

size_t level_pixels(const jde_frame_desc* d, int n, int lvl) {
    size_t p = 0;
    for (int i = 0; i < n; ++i) p += (size_t)(d[i].h >> lvl) * (d[i].w >> lvl);
    return p;
}

GeomParams geom_params(const jde_frame_desc* d, int n) {
    GeomParams p{};
    p.n = n;
    for (int i = 0; i < n; ++i) {
        p.hw[i][0] = d[i].h;
        p.hw[i][1] = d[i].w;
    }
    return p;
}

// An FP8 op runs on e4m3 operands once its activation scales are known: always
// with per-block activation scales, after calibration with per-tensor ones.
bool runs_fp8(const jde_ctx* c, const Op& o) {
    return o.fp8 && !c->calibrating && (c->fp8_blocks || c->mx_fmt != 0 || c->fp8_ready);
}

// Bits per element of the block-scaled formats (mx_fmt 0 e4m3, 2 FP6 E2M3, 4 FP4 E2M1).
static int mx_bits(int fmt) { return fmt == 0 ? 8 : (fmt == 2 ? 6 : 4); }

// Arguments of conv op `o` for a batch (d, n) with workspace W and head outputs `out`.
ConvArgs conv_args(const jde_ctx* c, const Op& o, const jde_frame_desc* d, int n, bool uniform, char* W,
                   const int* geom, const jde_head_out* out, int op_index = -1) {
    auto tptr = [&](int t) -> void* { return t < 0 ? nullptr : (void*)(W + c->tens[t].off); };
    const char* wb = c->d_weights;
    ConvArgs a{};
    a.in = tptr(o.in_t);
    a.in2 = tptr(o.in2_t);
    a.w = wb + o.dev_w;
    a.bias = (const float*)(wb + o.dev_b);
    a.wscale = nullptr;
    a.res = tptr(o.res_t);
    a.geom = geom;
    a.nframes = n;
    a.uniform = uniform;
    a.lvl_in = o.lvl_in;
    a.lvl_out = o.lvl_out;
    a.cin = o.cin;
    a.cout = o.cout;
    a.ksz = o.ksz;
    a.stride = o.stride;
    a.pad = o.ksz / 2;
    a.cin1 = o.cin1;
    a.K = o.ksz * o.ksz * o.cin;
    a.M = (int)level_pixels(d, n, o.lvl_out);
    a.n_split = o.n_split;
    a.act = o.act;
    a.in_scale = 1.f;
    a.in_bytes = o.in_t >= 0 ? (int)c->tens[o.in_t].bytes : 0;
    a.in2_bytes = o.in2_t >= 0 ? (int)c->tens[o.in2_t].bytes : 0;
    a.w_bytes = (int)((size_t)o.cout * a.K * elem_bytes(c->et));
    // weights dominate when Cout*K exceeds the activation rows read (M * Cin)
    a.n_major = (double)o.cout * a.K > (double)a.M * o.cin ? 1 : 0;
    if (o.det_out >= 0) {
        a.out0 = out->det[o.det_out];
        a.ld0 = o.cout;
        a.out0_f32 = 1;
    } else {
        a.out0 = tptr(o.out_t);
        a.ld0 = o.n_split;
        a.out0_f32 = 0;
    }
    if (o.emb_out >= 0) {
        if (c->sparse_emb) {
            // det3 alone: the emb rows of the weight block run later, at kept cells only
            // (every launch of this op -- forward and autotuner -- must drop them: there
            // is no dense emb output to write)
            a.cout = o.n_split;
            a.n_major = (double)a.cout * a.K > (double)a.M * a.cin ? 1 : 0;
        } else {
            a.out1 = out->emb[o.emb_out];
            a.ld1 = o.cout - o.n_split;
        }
    }
    if (runs_fp8(c, o)) {
        a.w = wb + o.dev_w8;
        a.wscale = (const float*)(wb + o.dev_ws);
        a.wbscale = (const unsigned char*)(wb + o.dev_wbs);
        a.mx_fmt = c->mx_fmt;
        const bool blocks = c->fp8_blocks || c->mx_fmt != 0;
        a.act_blocks = blocks ? 1 : 0;
        a.in_scale = blocks ? 1.f : o.in_scale;
        a.w_bytes = o.cout * (a.K / 8 * mx_bits(c->mx_fmt));
    }
    if (c->calibrating && op_index >= 0) a.amax = (unsigned*)(W + c->ws_amax) + op_index;
    return a;
}



// The stem (3 -> 32) and the stage-1 downsample conv (3x3 stride 2, 32 -> 64) run
// fused for 16-bit storage, except while calibrating (the fused launch records
// no output range).
static bool stem_fusable(const jde_ctx* c, const Op& stem, const Op& o1) {
    return c->fuse_stem && !c->calibrating && c->et != kF32 && stem.cout == 32 && o1.kind == OP_CONV &&
           o1.in_t == stem.out_t && o1.cin == 32 && o1.cout == 64 && o1.ksz == 3 && o1.stride == 2 && o1.cin1 == 0 &&
           o1.res_t < 0 && o1.act && o1.n_split == o1.cout && !runs_fp8(c, o1);
}

// A 64- or 128-channel residual block (1x1 C -> C/2, then 3x3 C/2 -> C + x,
// written out of place) runs as one launch for 16-bit storage, except while
// calibrating and when either conv runs in FP8.
static bool block_fusable(const jde_ctx* c, const Op& o1, const Op& o2) {
    return c->fuse_blocks && !c->calibrating && c->et != kF32 && o1.kind == OP_CONV && o2.kind == OP_CONV &&
           (o1.cin == 64 || o1.cin == 128) && o1.ksz == 1 && o1.stride == 1 && 2 * o1.cout == o1.cin &&
           o1.cin1 == 0 && o1.in2_t < 0 && o1.res_t < 0 && o1.act && o1.n_split == o1.cout && o1.layer2 < 0 &&
           o1.lvl_in == o1.lvl_out && o2.ksz == 3 && o2.stride == 1 && o2.cin == o1.cout && o2.cout == o1.cin &&
           o2.in_t == o1.out_t && o2.res_t == o1.in_t && o2.out_t >= 0 && o2.out_t != o1.in_t && o2.cin1 == 0 &&
           o2.in2_t < 0 && o2.act && o2.n_split == o2.cout && o2.layer2 < 0 && o2.lvl_in == o1.lvl_out &&
           o2.lvl_out == o1.lvl_out && !runs_fp8(c, o1) && !runs_fp8(c, o2);
}

}  // namespace

// ---- setup kernel: geometry table + counter reset ---------------------------
namespace jde {
__device__ __forceinline__ void setup_kernel_body(const GeomParams& p, int* geom, int* counters, int ncount) {
    const int t = threadIdx.x;
    if (t < p.n) {
        int pre[kLevels], nxt[kLevels];
        for (int l = 0; l < kLevels; ++l) pre[l] = 0;
        for (int i = 0; i < t; ++i)
            for (int l = 0; l < kLevels; ++l) pre[l] += (p.hw[i][0] >> l) * (p.hw[i][1] >> l);
        for (int l = 0; l < kLevels; ++l) nxt[l] = pre[l] + (p.hw[t][0] >> l) * (p.hw[t][1] >> l);
        int* g = geom + t * kGeomInts;
        g[0] = p.hw[t][0];
        g[1] = p.hw[t][1];
        for (int l = 0; l < kLevels; ++l) {
            g[2 + l] = pre[l];
            g[8 + l] = nxt[l];
        }
    }
    for (int i = t; i < ncount; i += blockDim.x) counters[i] = 0;
}
__global__ void setup_kernel(GeomParams p, int* geom, int* counters, int ncount) {
    setup_kernel_body(p, geom, counters, ncount);
}
hipError_t launch_setup(const GeomParams& p, int* geom, int* counters, int ncount, hipStream_t s) {
    setup_kernel<<<1, 256, 0, s>>>(p, geom, counters, ncount);
    return hipGetLastError();
}

__global__ void setup_dyn_kernel(GeomParams p, DynHeader h, int* geom, int* dyn, int* counters, int ncount,
                                 int* counters2, int ncount2, int* counters3, int ncount3) {
    setup_kernel_body(p, geom, counters, ncount);
    const int t = threadIdx.x;
    if (t < kDynInts) dyn[t] = h.v[t];
    for (int i = t; i < ncount2; i += blockDim.x) counters2[i] = 0;
    for (int i = t; i < ncount3; i += blockDim.x) counters3[i] = 0;
}
hipError_t launch_setup_dyn(const GeomParams& p, const DynHeader& h, int* geom, int* dyn, int* counters, int ncount,
                            int* counters2, int ncount2, int* counters3, int ncount3, hipStream_t s) {
    setup_dyn_kernel<<<1, 256, 0, s>>>(p, h, geom, dyn, counters, ncount, counters2, ncount2, counters3, ncount3);
    return hipGetLastError();
}

uint16_t f32_to_bf16_rne(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}
// OCP FP8 e4m3 (bias 7, 3 mantissa bits, no infinities, max 448), round to
// nearest even, saturating at +-448; NaN -> 0x7f.
// Largest value of the element format (mx_fmt 0 e4m3, 2 FP6 E2M3, 4 FP4 E2M1).
static float mx_top(int fmt) { return fmt == 0 ? 448.f : (fmt == 2 ? 7.5f : 6.f); }

// E8M0 exponent byte (127 + s) of the smallest 2^s with m / 2^s <= top (m >= 0,
// 127 for m = 0); the device conversion of activation blocks computes the same.
int e8m0_for_amax_host(float m, float top) {
    if (!(m > 0.f)) return 127;
    int E, Et;
    const float f = 2.f * frexpf(m, &E);     // m = f * 2^(E - 1), f in [1, 2)
    const float ft = 2.f * frexpf(top, &Et);  // top = ft * 2^(Et - 1)
    const int e = 127 + (E - 1) - (Et - 1) + (f > ft ? 1 : 0);
    return e < 0 ? 0 : (e > 254 ? 254 : e);
}

// FP6 E2M3 (fmt 2) / FP4 E2M1 (fmt 4) code of the value nearest x, ties to even,
// saturating: in binade e >= emin = 0 the spacing is 2^(e - M), below 1 it stays
// 2^-M (subnormals); n = the significand in units of the spacing.
unsigned mx_code_host(int fmt, float x) {
    const int M = fmt == 2 ? 3 : 1, bits = fmt == 2 ? 6 : 4;
    const unsigned sign = std::signbit(x) ? 1u : 0u;
    const float a = std::min(fabsf(x), mx_top(fmt));
    if (!(a > 0.f)) return sign << (bits - 1);
    int E;
    frexpf(a, &E);                         // a in [2^(E-1), 2^E)
    const int e = std::max(E - 1, 0);
    const int n = (int)nearbyintf(ldexpf(a, M - e));   // the default rounding mode is to nearest even
    unsigned code;
    if (n < (1 << M)) {
        code = (unsigned)n;
    } else {
        const int up = n >> (M + 1);
        code = ((unsigned)(e + up + 1) << M) | (up ? 0u : (unsigned)(n - (1 << M)));
    }
    return code | (sign << (bits - 1));
}

uint8_t f32_to_e4m3(float x) {
    if (x != x) return 0x7f;
    const uint8_t sign = std::signbit(x) ? 0x80 : 0x00;
    float a = fabsf(x);
    if (a >= 448.f) return sign | 0x7e;
    if (a == 0.f) return sign;
    int e;
    frexpf(a, &e);
    int E = e - 1 < -6 ? -6 : e - 1;          // binade; below 2^-6 the spacing stays 2^-9
    const float q = ldexpf(1.f, E - 3);
    const float v = nearbyintf(a / q) * q;     // the default rounding mode is to nearest even
    if (v >= 448.f) return sign | 0x7e;
    if (v == 0.f) return sign;
    frexpf(v, &e);
    E = e - 1;
    if (E < -6) return sign | (uint8_t)(v / ldexpf(1.f, -9));
    const int m = (int)((v / ldexpf(1.f, E) - 1.f) * 8.f);
    return sign | (uint8_t)(((E + 7) << 3) | m);
}

uint16_t f32_to_f16_rne(float x) {
    _Float16 h = (_Float16)x;   // host conversion is IEEE round-to-nearest-even
    uint16_t r;
    memcpy(&r, &h, 2);
    return r;
}
}  // namespace jde

// ---- NMS without caller-provided device memory -----------------------------
// jde_nms_noalloc runs jde_nms's kernels on a file-scope device array instead of
// a workspace.  Layout (byte offsets): sort keys u64[kNoallocK], positions
// int[kNoallocK], three counters in 256-byte slots, sorted boxes float4[kNoallocK],
// keep positions int[kNoallocK], suppression mask u64[kNoallocK][kNoallocK / 64].
namespace {
constexpr int kNoallocK = 8192;
constexpr size_t kNaKeys = 0;
constexpr size_t kNaVals = kNaKeys + (size_t)kNoallocK * 8;
constexpr size_t kNaCount = kNaVals + (size_t)kNoallocK * 4;
constexpr size_t kNaKcount = kNaCount + 256;
constexpr size_t kNaNkeep = kNaKcount + 256;
constexpr size_t kNaBoxes = kNaNkeep + 256;
constexpr size_t kNaKeep = kNaBoxes + (size_t)kNoallocK * 16;
constexpr size_t kNaMask = kNaKeep + (size_t)kNoallocK * 4;
constexpr size_t kNaBytes = kNaMask + (size_t)kNoallocK * (kNoallocK / 64) * 8;
constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
char* g_na_ptr[kNaMaxDevices] = {};
}  // namespace

// One copy per GPU, held until the process ends.  Host code never passes this
// name to a kernel: it is a host-side stand-in; the device address of each GPU's
// copy comes from hipGetSymbolAddress (noalloc_scratch below).
static __device__ __align__(256) unsigned char scratch[kNaBytes];

// Device address of the current device's copy of `scratch`, looked up once per
// device with that device current.
static jde_status noalloc_scratch(char** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaMaxDevices) return fail(JDE_EDEVICE, "device %d outside [0, %d)", dev, kNaMaxDevices);
    std::lock_guard<std::mutex> lock(g_na_mu);
    if (!g_na_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(JDE_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_na_ptr[dev] = (char*)p;
    }
    *out = g_na_ptr[dev];
    return JDE_OK;
}

// ---- C ABI -----------------------------------------------------------------
extern "C" {

const char* jde_status_str(int s) {
    switch (s) {
        case JDE_OK: return "ok";
        case JDE_EINVAL: return "invalid argument";
        case JDE_ENOMEM: return "buffer too small";
        case JDE_EDEVICE: return "device error";
        case JDE_ECAPACITY: return "capacity exceeded";
        case JDE_EUNSUPPORTED: return "unsupported";
        case JDE_ESTATE: return "bad call order";
        case JDE_EBUDGET: return "device-memory budget spent";
    }
    return "unknown status";
}

const char* jde_last_error(void) { return g_err.c_str(); }

jde_status jde_create(const jde_config* cfg, jde_ctx** out) {
    if (!cfg || !out) return fail(JDE_EINVAL, "null argument");
    *out = nullptr;
    const jde_config& g = *cfg;
    if (g.base_ch != 16 && g.base_ch != 32) return fail(JDE_EUNSUPPORTED, "base_ch must be 16 or 32");
    for (int i = 0; i < 5; ++i)
        if (g.blocks[i] < 0 || g.blocks[i] > 64) return fail(JDE_EINVAL, "blocks[%d] out of range", i);
    if (g.num_anchors != 4) return fail(JDE_EUNSUPPORTED, "num_anchors must be 4");
    if (g.emb_dim <= 0 || g.emb_dim % 64) return fail(JDE_EINVAL, "emb_dim must be a positive multiple of 64");
    if (g.precision < JDE_FP32 || g.precision > JDE_FP4)
        return fail(JDE_EUNSUPPORTED, "precision %d not implemented", g.precision);
    if (g.max_frames <= 0 || g.max_frames > kMaxFrames) return fail(JDE_EINVAL, "max_frames must be 1..%d", kMaxFrames);
    if (g.max_h <= 0 || g.max_w <= 0 || g.max_h % 32 || g.max_w % 32)
        return fail(JDE_EINVAL, "max_h, max_w must be positive multiples of 32");
    // Kernels index activations with 32-bit element offsets; the stem output
    // (max pixels x c0) is the largest tensor, the upsample/halo rows need 16-bit y, x.
    // (max pixels x c0) is the largest tensor, its bytes must stay below 2^31 (buffer
    // loads use 32-bit byte offsets with 2^31 as the out-of-range marker); the
    // upsample/halo rows need 16-bit y, x.
    const size_t full_pix = (size_t)g.max_frames * g.max_h * g.max_w;
    if (g.max_pixels > 0 && g.max_pixels < (size_t)g.max_h * g.max_w)
        return fail(JDE_EINVAL, "max_pixels must hold at least one frame of max_h x max_w");
    const size_t cap_pix = g.max_pixels > 0 && g.max_pixels < full_pix ? g.max_pixels : full_pix;
    {
        const size_t eb = g.precision == JDE_FP32 ? 4 : 2;
        if (cap_pix * g.base_ch * eb >= ((size_t)1 << 31) - 4096 ||
            g.max_h >= 32768 || g.max_w >= 32768)
            return fail(JDE_EINVAL, "capacity too large: the largest activation must stay below 2 GiB");
    }
    if (g.max_candidates < 64 || g.max_candidates > kMaxCap || g.max_candidates % 64)
        return fail(JDE_EINVAL, "max_candidates must be a multiple of 64 in [64, %d]", kMaxCap);
    jde_ctx* c = new jde_ctx();
    c->cfg = g;
    c->cap_pix = cap_pix;
    c->et = g.precision == JDE_FP32 ? kF32 : (g.precision == JDE_FP16 ? kF16 : kBF16);
    c->fp8 = g.precision == JDE_FP8 || g.precision == JDE_FP6 || g.precision == JDE_FP4;
    c->mx_fmt = g.precision == JDE_FP6 ? 2 : (g.precision == JDE_FP4 ? 4 : 0);
    build_plan(c);
    plan_fp8(c);
    plan_arena(c);
    plan_weights(c);
    plan_decode_scratch(c);
    *out = c;
    return JDE_OK;
}

void jde_destroy(jde_ctx* c) { delete c; }

static jde_status prof_harvest(jde_ctx* c, int slot) {
    if (!c->pending[slot]) return JDE_OK;
    const size_t nops = c->ops.size();
    hipEvent_t* e = c->ev.data() + (size_t)slot * nops * 2;
    HIP_TRY(hipEventSynchronize(e[nops * 2 - 1]));
    for (size_t i = 0; i < nops; ++i) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e[2 * i], e[2 * i + 1]));
        c->op_ms[i] += ms;
    }
    c->pending[slot] = false;
    c->n_fwd += 1;
    return JDE_OK;
}

jde_status jde_profile_begin(jde_ctx* c, int on) {
    if (!c) return fail(JDE_EINVAL, "null context");
    for (int k = 0; k < jde_ctx::kRing; ++k) c->pending[k] = false;
    c->ring_pos = 0;
    c->n_fwd = 0;
    c->op_ms.assign(c->ops.size(), 0.0);
    c->op_flop.assign(c->ops.size(), 0.0);
    if (on && c->ev.empty()) {
        c->ev.resize((size_t)jde_ctx::kRing * c->ops.size() * 2);
        for (auto& e : c->ev) HIP_TRY(hipEventCreate(&e));
    }
    c->prof = on != 0;
    return JDE_OK;
}

jde_status jde_profile_collect(jde_ctx* c, int max_ops, double* op_ms, double* op_flop, int* op_kind, int* n_ops,
                               int* n_fwd) {
    if (!c) return fail(JDE_EINVAL, "null context");
    if (c->prof)
        for (int k = 0; k < jde_ctx::kRing; ++k)
            if (jde_status st = prof_harvest(c, k)) return st;
    const int n = (int)c->ops.size();
    for (int i = 0; i < n && i < max_ops; ++i) {
        if (op_ms) op_ms[i] = i < (int)c->op_ms.size() ? c->op_ms[i] : 0.0;
        if (op_flop) op_flop[i] = i < (int)c->op_flop.size() ? c->op_flop[i] : 0.0;
        if (op_kind) {
            const int lk = i < (int)c->launch_kind.size() ? c->launch_kind[i] : 0;
            op_kind[i] = lk ? lk : c->ops[i].kind;
        }
    }
    if (n_ops) *n_ops = n;
    if (n_fwd) *n_fwd = c->n_fwd;
    return JDE_OK;
}

int jde_num_layers(const jde_ctx* c) { return c ? (int)c->layers.size() : 0; }

jde_status jde_layer_info(const jde_ctx* c, int i, int* cout, int* k, int* cin, int* stride) {
    if (!c || i < 0 || i >= (int)c->layers.size()) return fail(JDE_EINVAL, "layer index out of range");
    const Layer& L = c->layers[i];
    if (cout) *cout = L.cout;
    if (k) *k = L.k;
    if (cin) *cin = L.cin;
    if (stride) *stride = L.stride;
    return JDE_OK;
}

size_t jde_blob_floats(const jde_ctx* c) { return c ? c->blob_floats : 0; }
size_t jde_weights_bytes(const jde_ctx* c) { return c ? c->weights_bytes : 0; }
size_t jde_workspace_bytes(const jde_ctx* c) { return c ? c->ws_total : 0; }

jde_status jde_head_sizes(const jde_ctx* c, const jde_frame_desc* d, int n, size_t det[3], size_t emb[3]) {
    if (!c || !det || !emb) return fail(JDE_EINVAL, "null argument");
    bool uni;
    if (jde_status st = batch_ok(c, d, n, &uni)) return st;
    for (int s = 0; s < 3; ++s) {
        const size_t p = level_pixels(d, n, 3 + s);
        det[s] = p * 6 * c->cfg.num_anchors;
        emb[s] = p * c->cfg.emb_dim;
    }
    return JDE_OK;
}

size_t jde_frame_bytes(const jde_ctx* c, int h, int w) {
    if (!c || h <= 0 || w <= 0 || h % 32 || w % 32 || h > c->cfg.max_h || w > c->cfg.max_w) return 0;
    const jde_config& g = c->cfg;
    size_t b = (size_t)3 * h * w * 4;
    for (int s = 0; s < 3; ++s)
        b += (size_t)(h >> (3 + s)) * (w >> (3 + s)) * (6 * g.num_anchors + g.emb_dim) * 4;
    b += (size_t)c->cap * (4 + 1 + 1 + 1 + g.emb_dim) * 4 + 3 * 4;
    b += (size_t)ceil((double)c->ws_total * ((double)h * w / (double)c->cap_pix));
    return b;
}

jde_status jde_admit(const jde_ctx* c, const jde_frame_desc* d, int n, size_t in_flight, size_t budget,
                     int* n_admit) {
    if (!c || !n_admit || (n > 0 && !d) || n < 0) return fail(JDE_EINVAL, "bad arguments");
    *n_admit = 0;
    size_t used = in_flight;
    int k = 0;
    for (; k < n && k < c->cfg.max_frames; ++k) {
        const size_t fb = jde_frame_bytes(c, d[k].h, d[k].w);
        if (fb == 0) return fail(JDE_EINVAL, "frame %d: %dx%d does not fit the context", k, d[k].h, d[k].w);
        if (used > budget || fb > budget - used) break;
        used += fb;
    }
    *n_admit = k;
    if (k == 0 && n > 0)
        return fail(JDE_EBUDGET, "%zu bytes in flight + %zu for the next frame exceed the budget of %zu", in_flight,
                    jde_frame_bytes(c, d[0].h, d[0].w), budget);
    return JDE_OK;
}

jde_status jde_load_weights(jde_ctx* c, const float* blob, size_t nf, void* d_weights, size_t wbytes, void* stream) {
    if (!c || !blob || !d_weights) return fail(JDE_EINVAL, "null argument");
    if (nf != c->blob_floats) return fail(JDE_EINVAL, "blob has %zu floats, expected %zu", nf, c->blob_floats);
    if (wbytes < c->weights_bytes) return fail(JDE_ENOMEM, "weight buffer %zu < %zu bytes", wbytes, c->weights_bytes);
    if ((uintptr_t)d_weights % 256) return fail(JDE_EINVAL, "weight buffer not 256-byte aligned");
    std::vector<unsigned char> host(c->weights_bytes, 0);
    const size_t eb = elem_bytes(c->et);
    for (const Op& o : c->ops) {
        const int K = o.ksz * o.ksz * o.cin;
        const int nl = o.layer2 >= 0 ? 2 : 1;
        size_t row = 0;
        for (int q = 0; q < nl; ++q) {
            const Layer& L = c->layers[q == 0 ? o.layer : o.layer2];
            const float* w = blob + L.blob_w;
            const float* b = blob + L.blob_b;
            for (int co = 0; co < L.cout; ++co, ++row) {
                for (int k = 0; k < K; ++k) {
                    const float v = w[(size_t)co * K + k];
                    unsigned char* dst = host.data() + o.dev_w;
                    if (o.kind == OP_STEM || c->et == kF32) {
                        memcpy(dst + (row * K + k) * 4, &v, 4);
                    } else {
                        const uint16_t h = c->et == kBF16 ? f32_to_bf16_rne(v) : f32_to_f16_rne(v);
                        memcpy(dst + (row * K + k) * eb, &h, 2);
                    }
                }
                memcpy(host.data() + o.dev_b + row * 4, &b[co], 4);
                if (o.fp8) {
                    // w = sc * 2^(e_b - 127) * q: sc = max |w_c| / 448 per channel, then per
                    // 32-k block b the E8M0 exponent e_b that brings the block's max |w / sc|
                    // to at most 448 (e_b <= 127: blocks below the channel's range are
                    // scaled up into e4m3's normal range).
                    // FP6 / FP4: the same with the format's largest value, codes packed
                    // EB bits each, value k of the row at bit EB k (little-endian).
                    const int fmt = c->mx_fmt, eb_bits = mx_bits(fmt);
                    const float top = mx_top(fmt);
                    float amax = 0.f;
                    for (int k = 0; k < K; ++k) amax = std::max(amax, fabsf(w[(size_t)co * K + k]));
                    const float sc = amax > 0.f ? amax / top : 1.f;
                    memcpy(host.data() + o.dev_ws + row * 4, &sc, 4);
                    unsigned char* wrow = host.data() + o.dev_w8 + row * (size_t)(K / 8 * eb_bits);
                    for (int kb = 0; kb < K / 32; ++kb) {
                        float bm = 0.f;
                        for (int k = 32 * kb; k < 32 * kb + 32; ++k)
                            bm = std::max(bm, fabsf(w[(size_t)co * K + k] / sc));
                        const int e = e8m0_for_amax_host(bm, top);
                        host[o.dev_wbs + row * (K / 32) + kb] = (unsigned char)e;
                        for (int k = 32 * kb; k < 32 * kb + 32; ++k) {
                            const float v = ldexpf(w[(size_t)co * K + k] / sc, 127 - e);
                            if (fmt == 0) {
                                wrow[k] = f32_to_e4m3(v);
                            } else {
                                const unsigned code = mx_code_host(fmt, v);
                                for (int bb = 0; bb < eb_bits; ++bb)
                                    if ((code >> bb) & 1) {
                                        const size_t bit = (size_t)k * eb_bits + bb;
                                        wrow[bit / 8] |= (unsigned char)(1u << (bit % 8));
                                    }
                            }
                        }
                    }
                }
            }
        }
    }
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(d_weights, host.data(), c->weights_bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    c->d_weights = (char*)d_weights;
    c->loaded = true;
    c->fp8_ready = false;
    return JDE_OK;
}

// A backbone downsample conv that the window kernel runs: 3x3 stride 2 into the
// next level, Cin 64, nothing but bias + leaky in the epilogue (no concat, no
// residual, no head output), 16-bit storage, not in FP8 and not in a calibration
// pass (which records conv output ranges through the implicit GEMM's epilogue).
static bool window_down_op(const jde_ctx* c, const Op& o) {
    return c->window_down && !c->calibrating && down_win_ok(o.cin, o.cout, o.ksz, o.stride, c->et) &&
           o.lvl_out == o.lvl_in + 1 && o.cin1 == 0 && o.in2_t < 0 && o.res_t < 0 && o.act && o.n_split == o.cout &&
           o.det_out < 0 && o.emb_out < 0 && o.layer2 < 0 && !runs_fp8(c, o);
}

// Op i is a head's det 3x3 whose det 1x1 (op i + 1) can run in its epilogue:
// 16-bit storage, neither in FP8, no calibration pass (which records the 3x3's
// output range), a 1x1 over exactly the 3x3's det channels with at most 32
// outputs.  The 3x3's tile decides the rest (conv_tile_folds_det).
static bool det_foldable(const jde_ctx* c, size_t i) {
    if (!c->fold_det || c->calibrating || (c->et != kBF16 && c->et != kF16) || i + 1 >= c->ops.size()) return false;
    const Op& o = c->ops[i];
    const Op& o1 = c->ops[i + 1];
    return o.kind == OP_CONV && o.emb_out >= 0 && o1.kind == OP_CONV && o1.det_out >= 0 && o1.in_t == o.out_t &&
           o1.ksz == 1 && o1.cin == o.n_split && o1.cin % 64 == 0 && o1.cout % 4 == 0 && o1.cout <= 32 &&
           o1.cin1 == 0 && o1.in2_t < 0 && o1.res_t < 0 && !o1.act && !runs_fp8(c, o) && !runs_fp8(c, o1);
}
static void set_det_fold(const jde_ctx* c, const Op& o1, char* W, const jde_head_out* out, ConvArgs& a) {
    a.det_w = c->d_weights + o1.dev_w;
    a.det_b = (const float*)(c->d_weights + o1.dev_b);
    a.det_out = out->det[o1.det_out];
    a.det_part = (float*)(W + c->ws_det_part);
    a.det_cnt = (unsigned*)(W + c->ws_det_cnt);
    a.det_n = o1.cout;
}

// The forward's launches.  dynamic: for a batch described by the header in the
// workspace (written before each replay of a graph, see jde_graph_capture_any):
// grids are sized for the capacity and every launch reads the batch's pixels,
// frames and tile counts from the header; d, n are then ignored.
static jde_status forward_impl(jde_ctx* c, const float* frames, const jde_frame_desc* d, int n, void* ws,
                               size_t wsb, const jde_head_out* out, void* stream, bool dynamic) {
    if (!c || !frames || !ws || !out) return fail(JDE_EINVAL, "null argument");
    if (!c->loaded) return fail(JDE_ESTATE, "weights not loaded");
    if (c->fp8 && !c->fp8_blocks && !c->fp8_ready && !c->calibrating)
        return fail(JDE_ESTATE, "FP8 context with per-tensor activation scales not calibrated");
    if (wsb < c->ws_total) return fail(JDE_ENOMEM, "workspace %zu < %zu bytes", wsb, c->ws_total);
    for (int s = 0; s < 3; ++s)
        if (!out->det[s] || (!c->sparse_emb && !out->emb[s])) return fail(JDE_EINVAL, "null head output %d", s);
    bool uniform = false;
    if (!dynamic) {
        if (jde_status st = batch_ok(c, d, n, &uniform)) return st;
    } else {
        n = c->cfg.max_frames;
    }
    hipStream_t s = (hipStream_t)stream;
    char* W = (char*)ws;
    int* geom = (int*)(W + c->ws_geom);
    const int* dynp = dynamic ? (const int*)(W + c->ws_dyn) : nullptr;
    auto cap_m = [&](int lvl) { return c->cap_pix >> (2 * lvl); };
    // (the det 1x1 counters start at 0; every launch that uses them leaves them at 0)
    if (!dynamic) HIP_TRY(launch_setup(geom_params(d, n), geom, (int*)(W + c->ws_det_cnt), c->det_cnt_n, s));
    auto tptr = [&](int t) -> void* { return t < 0 ? nullptr : (void*)(W + c->tens[t].off); };
    hipEvent_t* pev = nullptr;
    if (c->prof) {
        const int slot = c->ring_pos;
        if (jde_status st = prof_harvest(c, slot)) return st;
        pev = c->ev.data() + (size_t)slot * c->ops.size() * 2;
        c->pending[slot] = true;
        c->ring_pos = (slot + 1) % jde_ctx::kRing;
    }
    c->launch_kind.assign(c->ops.size(), 0);
    for (size_t oi = 0; oi < c->ops.size(); ++oi) {
        const Op& o = c->ops[oi];
        const char* wb = c->d_weights;
        if (pev) HIP_TRY(hipEventRecord(pev[2 * oi], s));
        if (o.kind == OP_STEM && oi + 1 < c->ops.size() && stem_fusable(c, o, c->ops[oi + 1])) {
            const Op& o1 = c->ops[oi + 1];
            int tiles = dynamic ? (1 << 30) : 0;  // dynamic: the grid is the persistent maximum
            for (int f = 0; f < (dynamic ? 0 : n); ++f) tiles += stem_down_tiles(d[f].h, d[f].w);
            HIP_TRY(launch_stem_down(frames, geom, n, tiles, (const float*)(wb + o.dev_w), (const float*)(wb + o.dev_b),
                                     wb + o1.dev_w, (const float*)(wb + o1.dev_b), tptr(o1.out_t), c->et, s, dynp));
            if (pev) {
                HIP_TRY(hipEventRecord(pev[2 * oi + 1], s));
                HIP_TRY(hipEventRecord(pev[2 * oi + 2], s));
                HIP_TRY(hipEventRecord(pev[2 * oi + 3], s));
                const double M0 = (double)level_pixels(d, n, 0), M1 = (double)level_pixels(d, n, 1);
                c->op_flop[oi] = 2.0 * M0 * o.cout * 27 + 2.0 * M1 * o1.cout * o1.ksz * o1.ksz * o1.cin;
                c->op_flop[oi + 1] = 0.0;
            }
            c->launch_kind[oi] = 2;
            c->launch_kind[oi + 1] = 3;
            ++oi;
            continue;
        }
        if (o.kind == OP_CONV && oi + 1 < c->ops.size() && block_fusable(c, o, c->ops[oi + 1])) {
            const Op& o2 = c->ops[oi + 1];
            const int C = o.cin, lvl = o.lvl_in;
            int tiles = dynamic ? (1 << 30) : 0;
            for (int f = 0; f < (dynamic ? 0 : n); ++f) tiles += resblock_tiles(C, d[f].h >> lvl, d[f].w >> lvl);
            const size_t M = dynamic ? cap_m(lvl) : level_pixels(d, n, lvl);
            HIP_TRY(launch_resblock(tptr(o.in_t), tptr(o2.out_t), wb + o.dev_w, (const float*)(wb + o.dev_b),
                                    wb + o2.dev_w, (const float*)(wb + o2.dev_b), geom, n, lvl, C, tiles,
                                    M * C * elem_bytes(c->et), c->et, s, dynp));
            if (pev) {
                HIP_TRY(hipEventRecord(pev[2 * oi + 1], s));
                HIP_TRY(hipEventRecord(pev[2 * oi + 2], s));
                HIP_TRY(hipEventRecord(pev[2 * oi + 3], s));
                c->op_flop[oi] = 2.0 * M * o.cout * o.cin + 2.0 * M * o2.cout * 9.0 * o2.cin;
                c->op_flop[oi + 1] = 0.0;
            }
            c->launch_kind[oi] = 4;
            c->launch_kind[oi + 1] = 5;
            ++oi;
            continue;
        }
        if (o.kind == OP_STEM) {
            if (dynamic) return fail(JDE_EUNSUPPORTED, "a graph for any batch needs the fused 16-bit stem");
            const int M = (int)level_pixels(d, n, 0);
            int rows = 0, max_w = 0;
            for (int f = 0; f < n; ++f) {
                rows += d[f].h;
                max_w = d[f].w > max_w ? d[f].w : max_w;
            }
            HIP_TRY(launch_stem(frames, geom, n, uniform, rows, max_w, M, (const float*)(wb + o.dev_w),
                                (const float*)(wb + o.dev_b), o.cout, tptr(o.out_t), c->et, s));
            if (pev) {
                HIP_TRY(hipEventRecord(pev[2 * oi + 1], s));
                c->op_flop[oi] = 2.0 * M * o.cout * 27;
            }
            continue;
        }
        if (o.kind == OP_CONV && window_down_op(c, o)) {
            HIP_TRY(launch_down_win(tptr(o.in_t), tptr(o.out_t), wb + o.dev_w, (const float*)(wb + o.dev_b), geom, n,
                                    o.lvl_in, o.cin, o.cout, c->et, s, dynp));
            if (pev) {
                HIP_TRY(hipEventRecord(pev[2 * oi + 1], s));
                const double M = dynamic ? (double)cap_m(o.lvl_out) : (double)level_pixels(d, n, o.lvl_out);
                c->op_flop[oi] = 2.0 * M * o.cout * 9.0 * o.cin;
            }
            c->launch_kind[oi] = 9;
            continue;
        }
        ConvArgs a = conv_args(c, o, d, dynamic ? 0 : n, uniform, W, geom, out, (int)oi);
        if (dynamic) {
            // the capacity sizes the grid; the kernels read this batch's M, frames and layout from the header
            a.M = (int)cap_m(o.lvl_out);
            a.nframes = n;
            a.uniform = 0;
            a.dyn = dynp;
            a.n_major = (double)a.cout * a.K > (double)a.M * o.cin ? 1 : 0;
            if (runs_fp8(c, o)) return fail(JDE_EUNSUPPORTED, "a graph for any batch does not run FP8 convs");
        }
        int w3 = 0;  // pixel tiles of the window kernel, 0 = implicit GEMM
        if (c->window_convs && !dynamic && !runs_fp8(c, o) && conv3w_ok(a, c->et)) {
            for (int f = 0; f < n; ++f) {
                const int t = conv3w_tiles(d[f].h >> o.lvl_out, d[f].w >> o.lvl_out);
                if (t == 0) {
                    w3 = 0;
                    break;
                }
                w3 += t;
            }
        }
        bool folded = false;
        if (w3 > 0) {
            HIP_TRY(launch_conv3w(a, c->et, w3, s));
        } else if (runs_fp8(c, o)) {
            HIP_TRY(launch_conv_fp8(a, o.tile8, s));
        } else {
            const int tile = (o.tile >= 0 && conv_tile_ok(o.tile, c->et, a)) ? o.tile : conv_default_tile(c->et, a);
            folded = det_foldable(c, oi) && conv_tile_folds_det(tile, c->et, a.n_split);
            if (folded) set_det_fold(c, c->ops[oi + 1], W, out, a);
            HIP_TRY(launch_conv(a, c->et, tile, s));
            if (conv_tile_pw(tile)) c->launch_kind[oi] = 6;
        }
        if (pev) {
            HIP_TRY(hipEventRecord(pev[2 * oi + 1], s));
            c->op_flop[oi] = 2.0 * a.M * (double)a.cout * a.K;
        }
        if (folded) {
            const Op& o1 = c->ops[oi + 1];
            if (pev) {
                HIP_TRY(hipEventRecord(pev[2 * oi + 2], s));
                HIP_TRY(hipEventRecord(pev[2 * oi + 3], s));
                c->op_flop[oi] += 2.0 * a.M * (double)o1.cout * o1.cin;
                c->op_flop[oi + 1] = 0.0;
            }
            c->launch_kind[oi] = 7;
            c->launch_kind[oi + 1] = 8;
            ++oi;
        }
    }
    return JDE_OK;
}

jde_status jde_forward(jde_ctx* c, const float* frames, const jde_frame_desc* d, int n, void* ws, size_t wsb,
                       const jde_head_out* out, void* stream) {
    return forward_impl(c, frames, d, n, ws, wsb, out, stream, false);
}

jde_status jde_autotune(jde_ctx* c, const float* frames, const jde_frame_desc* d, int n, void* ws, size_t wsb,
                        const jde_head_out* out, int reps, void* stream) {
    if (reps <= 0) return fail(JDE_EINVAL, "reps must be positive");
    if (c && c->prof) return fail(JDE_ESTATE, "autotune while profiling");
    // A plain forward validates the arguments and fills every buffer.
    if (jde_status st = jde_forward(c, frames, d, n, ws, wsb, out, stream)) return st;
    bool uniform;
    (void)batch_ok(c, d, n, &uniform);
    hipStream_t s = (hipStream_t)stream;
    char* W = (char*)ws;
    const int* geom = (const int*)(W + c->ws_geom);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    jde_status st = JDE_OK;
    for (size_t oi = 0; oi < c->ops.size(); ++oi) {
        Op& o = c->ops[oi];
        if (o.kind != OP_CONV) continue;
        const ConvArgs a = conv_args(c, o, d, n, uniform, W, geom, out);
        const bool f8 = runs_fp8(c, o);
        float best = 1e30f;
        int best_t = -1;
        const int nt = f8 ? conv_fp8_num_tiles() : conv_num_tile_cfgs();
        // a det 3x3 whose det 1x1 can fold: a tile that folds is timed with the 1x1 in
        // its epilogue, any other followed by the 1x1's own launch (what the forward runs)
        const bool fold = det_foldable(c, oi);
        ConvArgs af = a, a1{};
        int tile1 = -1;
        if (fold) {
            set_det_fold(c, c->ops[oi + 1], W, out, af);
            a1 = conv_args(c, c->ops[oi + 1], d, n, uniform, W, geom, out);
            const Op& o1 = c->ops[oi + 1];
            tile1 = (o1.tile >= 0 && conv_tile_ok(o1.tile, c->et, a1)) ? o1.tile : conv_default_tile(c->et, a1);
        }
        auto go = [&](int t) {
            if (f8) return launch_conv_fp8(a, t, s);
            if (!fold) return launch_conv(a, c->et, t, s);
            if (conv_tile_folds_det(t, c->et, a.n_split)) return launch_conv(af, c->et, t, s);
            const hipError_t e = launch_conv(a, c->et, t, s);
            return e != hipSuccess ? e : launch_conv(a1, c->et, tile1, s);
        };
        for (int t = 0; t < nt && st == JDE_OK; ++t) {
            if (!f8 && !conv_tile_ok(t, c->et, a)) continue;
            hipError_t e = go(t);
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = go(t);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                st = fail(JDE_EDEVICE, "autotune launch: %s", hipGetErrorString(e));
                break;
            }
            if (ms < best) {
                best = ms;
                best_t = t;
            }
        }
        if (st != JDE_OK) break;
        if (f8)
            o.tile8 = best_t;
        else
            o.tile = best_t;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

jde_status jde_tiles(jde_ctx* c, int* tiles, int n_ops, int set) {
    if (!c || !tiles) return fail(JDE_EINVAL, "null argument");
    if (n_ops != (int)c->ops.size()) return fail(JDE_EINVAL, "expected %zu entries", c->ops.size());
    for (int i = 0; i < n_ops; ++i) {
        if (set) {
            if (tiles[i] < -1 || tiles[i] >= conv_num_tile_cfgs())
                return fail(JDE_EINVAL, "tile %d out of range", tiles[i]);
            c->ops[i].tile = c->ops[i].kind == OP_CONV ? tiles[i] : -1;
        } else {
            tiles[i] = c->ops[i].tile;
        }
    }
    return JDE_OK;
}

// dynamic: as in forward_impl, for the batch described by the header; the header
// write (setup_dyn) has zeroed the candidate and work-list counters.
static jde_status decode_impl(jde_ctx* c, const jde_head_out* heads, const jde_frame_desc* d, int n, float conf_thr,
                              float nms_iou, const float* logit_offset, void* ws, size_t wsb, const jde_dets* out,
                              void* stream, bool dynamic) {
    if (!c || !heads || !ws || !out) return fail(JDE_EINVAL, "null argument");
    if (wsb < c->ws_total) return fail(JDE_ENOMEM, "workspace %zu < %zu bytes", wsb, c->ws_total);
    if (out->cap != c->cap) return fail(JDE_EINVAL, "dets.cap %d != max_candidates %d", out->cap, c->cap);
    if (!out->boxes || !out->scores || !out->margins || !out->emb || !out->anchor_idx || !out->count ||
        !out->n_cand || !out->overflow)
        return fail(JDE_EINVAL, "null detection output");
    if (!(conf_thr >= 0.f && conf_thr <= 1.f)) return fail(JDE_EINVAL, "conf_thr outside [0, 1]");
    if (!(nms_iou >= 0.f)) return fail(JDE_EINVAL, "nms_iou must be >= 0");
    bool uniform;
    if (!dynamic) {
        if (jde_status st = batch_ok(c, d, n, &uniform)) return st;
    } else {
        n = c->cfg.max_frames;
    }
    hipStream_t s = (hipStream_t)stream;
    char* W = (char*)ws;
    int* geom = (int*)(W + c->ws_geom);
    int* counts = (int*)(W + c->ws_counts);
    if (!dynamic) HIP_TRY(launch_setup(geom_params(d, n), geom, counts, n, s));
    float lthr;
    if (conf_thr <= 0.f) lthr = -INFINITY;
    else if (conf_thr >= 1.f) lthr = INFINITY;
    else lthr = (float)log((double)conf_thr / (1.0 - (double)conf_thr));
    int max_anchors = dynamic ? c->max_anchors : 0;
    for (int i = 0; i < (dynamic ? 0 : n); ++i) {
        const int h = d[i].h, w = d[i].w;
        max_anchors = std::max(max_anchors, ((h >> 3) * (w >> 3) + (h >> 4) * (w >> 4) + (h >> 5) * (w >> 5)) * 4);
    }
    DecodeArgs da{};
    da.dyn = dynamic ? (const int*)(W + c->ws_dyn) : nullptr;
    GatherArgs ga{};
    EmitArgs ea{};
    for (int q = 0; q < 3; ++q) {
        da.det[q] = heads->det[q];
        ga.det[q] = heads->det[q];
        ea.emb[q] = heads->emb[q];
    }
    memcpy(da.anchors, c->cfg.anchors, sizeof da.anchors);
    memcpy(ga.anchors, c->cfg.anchors, sizeof ga.anchors);
    unsigned long long* keys = (unsigned long long*)(W + c->ws_keys);
    da.geom = geom;
    da.nframes = n;
    da.A = c->cfg.num_anchors;
    da.lthr = lthr;
    da.logit_offset = logit_offset;
    da.keycap = c->keycap;
    da.keys = keys;
    da.vals = nullptr;
    da.cand_count = counts;
    HIP_TRY(launch_decode(da, max_anchors, s));
    HIP_TRY(launch_sort(keys, nullptr, counts, c->keycap, n, s));
    float* sboxes = (float*)(W + c->ws_sboxes);
    int* kcount = (int*)(W + c->ws_kcount);
    ga.geom = geom;
    ga.A = c->cfg.num_anchors;
    ga.keys = keys;
    ga.cand_count = counts;
    ga.keycap = c->keycap;
    ga.cap = c->cap;
    ga.sboxes = sboxes;
    ga.kcount = kcount;
    HIP_TRY(launch_gather_boxes(ga, n, s));
    int* keep = (int*)(W + c->ws_keep);
    int* nkeep = (int*)(W + c->ws_nkeep);
    HIP_TRY(launch_nms(sboxes, kcount, c->cap, nms_iou, (unsigned long long*)(W + c->ws_mask), keep, nkeep, n, s));
    ea.geom = geom;
    ea.A = c->cfg.num_anchors;
    ea.E = c->cfg.emb_dim;
    ea.keys = keys;
    ea.keycap = c->keycap;
    ea.cap = c->cap;
    ea.sboxes = sboxes;
    ea.keep = keep;
    ea.nkeep = nkeep;
    ea.cand_count = counts;
    ea.boxes = out->boxes;
    ea.scores = out->scores;
    ea.margins = out->margins;
    ea.emb_out = out->emb;
    ea.anchor_idx = out->anchor_idx;
    ea.count = out->count;
    ea.n_cand = out->n_cand;
    ea.overflow = out->overflow;
    ea.work = nullptr;
    ea.work_count = nullptr;
    ea.work_cap = n * c->cap;
    if (c->sparse_emb) {
        if (!c->loaded) return fail(JDE_ESTATE, "sparse embedding head needs loaded weights");
        ea.work = (int*)(W + c->ws_work);
        ea.work_count = (int*)(W + c->ws_work_count);
        if (!dynamic) HIP_TRY(launch_setup(geom_params(d, n), geom, ea.work_count, 3, s));
    }
    HIP_TRY(launch_emit(ea, n, s));
    if (c->sparse_emb) {
        SparseEmbArgs sa{};
        for (int q = 0; q < 3; ++q) {
            const Op& o = c->ops[c->emb_op[q]];
            sa.feat[q] = W + c->tens[o.in_t].off;
            // the emb rows of the det3+emb weight block: rows n_split .. cout of [cout][K]
            sa.w[q] = c->d_weights + o.dev_w + (size_t)o.n_split * o.ksz * o.ksz * o.cin * elem_bytes(c->et);
            sa.bias[q] = (const float*)(c->d_weights + o.dev_b) + o.n_split;
            sa.F[q] = o.cin;
        }
        sa.E = c->cfg.emb_dim;
        sa.geom = geom;
        sa.work = ea.work;
        sa.count = ea.work_count;
        sa.work_cap = ea.work_cap;
        sa.out = out->emb;
        HIP_TRY(launch_sparse_emb(sa, c->et, n, c->cap, nkeep, s));
    }
    return JDE_OK;
}

jde_status jde_decode(jde_ctx* c, const jde_head_out* heads, const jde_frame_desc* d, int n, float conf_thr,
                      float nms_iou, const float* logit_offset, void* ws, size_t wsb, const jde_dets* out,
                      void* stream) {
    return decode_impl(c, heads, d, n, conf_thr, nms_iou, logit_offset, ws, wsb, out, stream, false);
}

jde_status jde_nms(jde_ctx* c, const float* boxes, const float* margins, const int* idx, int K, float iou, void* ws,
                   size_t wsb, int* keep_out, int* nkeep_out, void* stream) {
    if (!c || !ws || !keep_out || !nkeep_out) return fail(JDE_EINVAL, "null argument");
    if (K < 0 || K > c->cap) return fail(JDE_ECAPACITY, "K=%d outside [0, %d]", K, c->cap);
    if (K > 0 && (!boxes || !margins || !idx)) return fail(JDE_EINVAL, "null candidate arrays");
    if (wsb < c->ws_total) return fail(JDE_ENOMEM, "workspace %zu < %zu bytes", wsb, c->ws_total);
    if (!(iou >= 0.f)) return fail(JDE_EINVAL, "nms_iou must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    char* W = (char*)ws;
    unsigned long long* keys = (unsigned long long*)(W + c->ws_keys);
    int* vals = (int*)(W + c->ws_vals);
    int* counts = (int*)(W + c->ws_counts);
    float* sboxes = (float*)(W + c->ws_sboxes);
    int* kcount = (int*)(W + c->ws_kcount);
    int* keep = (int*)(W + c->ws_keep);
    int* nkeep = (int*)(W + c->ws_nkeep);
    HIP_TRY(launch_nms_prepare(boxes, margins, idx, K, keys, vals, counts, s));
    HIP_TRY(launch_sort(keys, vals, counts, c->keycap, 1, s));
    HIP_TRY(launch_nms_gather(boxes, keys, vals, K, sboxes, kcount, s));
    HIP_TRY(launch_nms(sboxes, kcount, c->cap, iou, (unsigned long long*)(W + c->ws_mask), keep, nkeep, 1, s));
    HIP_TRY(launch_nms_finish(keep, nkeep, vals, keep_out, nkeep_out, K, s));
    return JDE_OK;
}

jde_status jde_nms_noalloc(const float* boxes, const float* margins, const int* idx, int K, float iou, int* keep_out,
                           int* nkeep_out, void* stream) {
    if (!keep_out || !nkeep_out) return fail(JDE_EINVAL, "null argument");
    if (K < 0) return fail(JDE_EINVAL, "K=%d is negative", K);
    if (K > kNoallocK)
        return fail(JDE_ECAPACITY, "K=%d exceeds the %d candidates the static scratch array holds", K, kNoallocK);
    if (K > 0 && (!boxes || !margins || !idx)) return fail(JDE_EINVAL, "null candidate arrays");
    if (!(iou >= 0.f)) return fail(JDE_EINVAL, "nms_iou must be >= 0");
    char* S = nullptr;
    if (jde_status st = noalloc_scratch(&S)) return st;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* keys = (unsigned long long*)(S + kNaKeys);
    int* vals = (int*)(S + kNaVals);
    int* counts = (int*)(S + kNaCount);
    float* sboxes = (float*)(S + kNaBoxes);
    int* kcount = (int*)(S + kNaKcount);
    int* keep = (int*)(S + kNaKeep);
    int* nkeep = (int*)(S + kNaNkeep);
    // Every scratch word a kernel reads is written earlier in this sequence (the
    // counters by prepare / gather / scan, the mask words of rows < K by the mask
    // kernel), so nothing needs clearing between calls.
    HIP_TRY(launch_nms_prepare(boxes, margins, idx, K, keys, vals, counts, s));
    HIP_TRY(launch_sort(keys, vals, counts, kNoallocK, 1, s));
    HIP_TRY(launch_nms_gather(boxes, keys, vals, K, sboxes, kcount, s));
    HIP_TRY(launch_nms(sboxes, kcount, kNoallocK, iou, (unsigned long long*)(S + kNaMask), keep, nkeep, 1, s));
    HIP_TRY(launch_nms_finish(keep, nkeep, vals, keep_out, nkeep_out, K, s));
    return JDE_OK;
}

jde_status jde_cost_matrix(const float* fe, const double* mean, const double* cov, int T, const float* boxes,
                           const float* de, int D, int E, double gate, float* cost, void* stream) {
    if (T < 0 || D < 0 || E <= 0 || E % 4) return fail(JDE_EINVAL, "bad sizes T=%d D=%d E=%d", T, D, E);
    if (T > 0 && D > 0 && (!fe || !mean || !cov || !boxes || !de || !cost)) return fail(JDE_EINVAL, "null argument");
    if (!(gate >= 0.0)) return fail(JDE_EINVAL, "gate must be >= 0");
    HIP_TRY(launch_cost(fe, mean, cov, T, boxes, de, D, nullptr, D, E, gate, cost, (hipStream_t)stream));
    return JDE_OK;
}

static jde_status assoc_batch(const int* tb, int n, AssocBatch* b, int* max_t) {
    if (!tb || n < 0 || n > kMaxFrames) return fail(JDE_EINVAL, "bad batch: n=%d", n);
    *b = AssocBatch{};
    b->n = n;
    *max_t = 0;
    for (int f = 0; f <= n; ++f) {
        if (tb[f] < 0 || (f > 0 && tb[f] < tb[f - 1])) return fail(JDE_EINVAL, "track_begin must be non-decreasing");
        b->begin[f] = tb[f];
        if (f > 0) *max_t = std::max(*max_t, tb[f] - tb[f - 1]);
    }
    return JDE_OK;
}

jde_status jde_cost_matrix_batch(const float* fe, const double* mean, const double* cov, const int* tb,
                                 const jde_dets* dets, int n, int E, double gate, float* cost, void* stream) {
    return jde_cost_matrix_batch_fused(fe, mean, cov, tb, dets, n, E, gate, 0.f, cost, stream);
}

jde_status jde_iou_cost_batch(const double* mean, const int* tb, const jde_dets* dets, int n, float* cost,
                              void* stream) {
    AssocBatch b;
    int max_t;
    if (jde_status st = assoc_batch(tb, n, &b, &max_t)) return st;
    if (max_t > 0 && (!mean || !cost || !dets || !dets->boxes || !dets->count || dets->cap <= 0))
        return fail(JDE_EINVAL, "null argument");
    HIP_TRY(launch_iou_cost(mean, b, max_t, max_t ? dets->boxes : nullptr, max_t ? dets->count : nullptr,
                            max_t ? dets->cap : 0, cost, (hipStream_t)stream));
    return JDE_OK;
}

jde_status jde_cost_matrix_batch_fused(const float* fe, const double* mean, const double* cov, const int* tb,
                                       const jde_dets* dets, int n, int E, double gate, float motion_w, float* cost,
                                       void* stream) {
    if (!(motion_w >= 0.f && motion_w <= 1.f)) return fail(JDE_EINVAL, "motion weight outside [0, 1]");
    if (!dets || !tb || n < 0 || n > kMaxFrames || E <= 0 || E % 4 || dets->cap <= 0)
        return fail(JDE_EINVAL, "bad arguments n=%d E=%d", n, E);
    CostBatch b{};
    b.n = n;
    int max_t = 0;
    for (int f = 0; f <= n; ++f) {
        if (tb[f] < 0 || (f > 0 && tb[f] < tb[f - 1])) return fail(JDE_EINVAL, "track_begin must be non-decreasing");
        b.begin[f] = tb[f];
        if (f > 0) max_t = std::max(max_t, tb[f] - tb[f - 1]);
    }
    if (max_t > 0 && (!fe || !mean || !cov || !cost || !dets->boxes || !dets->emb || !dets->count))
        return fail(JDE_EINVAL, "null argument");
    if (!(gate >= 0.0)) return fail(JDE_EINVAL, "gate must be >= 0");
    HIP_TRY(launch_cost_batch(fe, mean, cov, b, max_t, dets->boxes, dets->emb, dets->count, dets->cap, E, gate, cost,
                              (hipStream_t)stream, motion_w));
    return JDE_OK;
}

jde_status jde_cost_matrix_dets(const float* fe, const double* mean, const double* cov, int T, const jde_dets* dets,
                                int frame, int E, double gate, float* cost, void* stream) {
    if (!dets || T < 0 || frame < 0 || E <= 0 || E % 4 || dets->cap <= 0)
        return fail(JDE_EINVAL, "bad arguments T=%d frame=%d E=%d", T, frame, E);
    if (T > 0 && (!fe || !mean || !cov || !cost || !dets->boxes || !dets->emb || !dets->count))
        return fail(JDE_EINVAL, "null argument");
    if (!(gate >= 0.0)) return fail(JDE_EINVAL, "gate must be >= 0");
    const size_t row = (size_t)frame * dets->cap;
    HIP_TRY(launch_cost(fe, mean, cov, T, dets->boxes + row * 4, dets->emb + row * E, dets->cap,
                        dets->count + frame, dets->cap, E, gate, cost, (hipStream_t)stream));
    return JDE_OK;
}

jde_status jde_track_emb_update(const int* pairs, int P, const float* de, int D, float* fe, int T, int E, float mom,
                                void* stream) {
    if (P < 0 || E <= 0 || T < 0 || D < 0) return fail(JDE_EINVAL, "bad sizes P=%d T=%d D=%d E=%d", P, T, D, E);
    if (P > 0 && (!pairs || !de || !fe)) return fail(JDE_EINVAL, "null argument");
    HIP_TRY(launch_emb_update(pairs, P, de, D, fe, T, E, mom, (hipStream_t)stream));
    return JDE_OK;
}


jde_status jde_ingest(const uint8_t* src, int n, int src_h, int src_w, const jde_frame_desc* d, float* dst,
                      void* stream) {
    if (n < 0 || n > kMaxFrames) return fail(JDE_EINVAL, "n=%d outside [0, %d]", n, kMaxFrames);
    if (n == 0) return JDE_OK;
    if (!src || !dst || !d) return fail(JDE_EINVAL, "null argument");
    if (src_h <= 0 || src_w <= 0 || (size_t)src_h * src_w * 3 >= ((size_t)1 << 31))
        return fail(JDE_EINVAL, "bad source size %dx%d", src_h, src_w);
    IngestArgs a{};
    a.src = src;
    a.n = n;
    a.src_h = src_h;
    a.src_w = src_w;
    a.dst = dst;
    size_t off = 0;
    int max_pix = 0;
    for (int f = 0; f < n; ++f) {
        const int h = d[f].h, w = d[f].w;
        if (h <= 0 || w <= 0) return fail(JDE_EINVAL, "frame %d: bad size %dx%d", f, h, w);
        const double r = std::min((double)h / src_h, (double)w / src_w);
        IngestFrame& g = a.fr[f];
        g.h = h;
        g.w = w;
        g.new_w = std::min((int)std::lround(src_w * r), w);
        g.new_h = std::min((int)std::lround(src_h * r), h);
        g.new_w = std::max(g.new_w, 1);
        g.new_h = std::max(g.new_h, 1);
        g.top = (h - g.new_h) / 2;
        g.left = (w - g.new_w) / 2;
        g.dst_off = off;
        off += (size_t)3 * h * w;
        max_pix = std::max(max_pix, h * w);
    }
    HIP_TRY(launch_ingest(a, max_pix, (hipStream_t)stream));
    return JDE_OK;
}

jde_status jde_kf_predict_dev(int T, double* mean, double* cov, void* stream) {
    if (T < 0 || (T > 0 && (!mean || !cov))) return fail(JDE_EINVAL, "bad arguments T=%d", T);
    HIP_TRY(launch_kf_predict(T, mean, cov, (hipStream_t)stream));
    return JDE_OK;
}

jde_status jde_kf_update_dev(const int* tb, int n, const int* det_of_track, const jde_dets* dets, double* mean,
                             double* cov, int* status, void* stream) {
    AssocBatch b;
    int max_t;
    if (jde_status st = assoc_batch(tb, n, &b, &max_t)) return st;
    if (max_t > 0 && (!det_of_track || !dets || !dets->boxes || !mean || !cov || dets->cap <= 0))
        return fail(JDE_EINVAL, "null argument");
    HIP_TRY(launch_kf_update(b, max_t, det_of_track, max_t ? dets->boxes : nullptr, max_t ? dets->cap : 0, mean, cov,
                             status, (hipStream_t)stream));
    return JDE_OK;
}

jde_status jde_assign_dev(const float* cost, const int* tb, int n, const jde_dets* dets, float max_cost,
                          int* det_of_track, int* track_of_det, int* kept, double* total, int* status,
                          void* stream) {
    AssocBatch b;
    int max_t;
    if (jde_status st = assoc_batch(tb, n, &b, &max_t)) return st;
    if (n == 0) return JDE_OK;
    if (!dets || !dets->count || dets->cap <= 0 || !track_of_det || !kept || !total || !status ||
        (max_t > 0 && (!cost || !det_of_track)))
        return fail(JDE_EINVAL, "null argument");
    if (max_t > kAssignMax) return fail(JDE_ECAPACITY, "%d tracks in one frame exceed %d", max_t, kAssignMax);
    if (!(max_cost >= 0.f)) return fail(JDE_EINVAL, "max_cost must be >= 0");
    const int max_dim = std::min(std::max(max_t, dets->cap), kAssignMax);
    HIP_TRY(launch_assign(cost, b, max_dim, dets->count, dets->cap, max_cost, det_of_track, track_of_det, kept, total,
                          status, (hipStream_t)stream));
    return JDE_OK;
}

jde_status jde_calibrate(jde_ctx* c, const float* frames, const jde_frame_desc* d, int n, void* ws, size_t wsb,
                         const jde_head_out* out, void* stream) {
    if (!c || !ws) return fail(JDE_EINVAL, "null argument");
    if (!c->fp8) return fail(JDE_EUNSUPPORTED, "calibration applies to FP8 contexts");
    if (!c->loaded) return fail(JDE_ESTATE, "weights not loaded");
    if (c->prof) return fail(JDE_ESTATE, "calibration while profiling");
    if (wsb < c->ws_total) return fail(JDE_ENOMEM, "workspace %zu < %zu bytes", wsb, c->ws_total);
    bool uniform;
    if (jde_status st = batch_ok(c, d, n, &uniform)) return st;
    hipStream_t s = (hipStream_t)stream;
    char* W = (char*)ws;
    unsigned* amax = (unsigned*)(W + c->ws_amax);
    HIP_TRY(launch_setup(geom_params(d, n), (int*)(W + c->ws_geom), (int*)amax, (int)c->ops.size(), s));
    c->calibrating = true;
    const jde_status st = jde_forward(c, frames, d, n, ws, wsb, out, stream);
    c->calibrating = false;
    if (st != JDE_OK) return st;
    std::vector<unsigned> h(c->ops.size());
    HIP_TRY(hipMemcpyAsync(h.data(), amax, h.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (Op& o : c->ops) {
        if (!o.fp8) continue;
        float m;
        memcpy(&m, &h[o.producer], 4);
        o.in_scale = m > 0.f ? m / 448.f : 1.f;
    }
    c->fp8_ready = true;
    return JDE_OK;
}

jde_status jde_fp8_block_scales(jde_ctx* c, int on) {
    if (!c) return fail(JDE_EINVAL, "null context");
    if (!c->fp8) return fail(JDE_EUNSUPPORTED, "block scales apply to FP8 contexts");
    if (c->mx_fmt != 0 && !on) return fail(JDE_EUNSUPPORTED, "FP6 / FP4 activations always take block scales");
    c->fp8_blocks = on != 0;
    return JDE_OK;
}

jde_status jde_fuse_stem(jde_ctx* c, int on) {
    if (!c) return fail(JDE_EINVAL, "null context");
    c->fuse_stem = on != 0;
    return JDE_OK;
}

jde_status jde_fuse_blocks(jde_ctx* c, int on) {
    if (!c) return fail(JDE_EINVAL, "null context");
    c->fuse_blocks = on != 0;
    return JDE_OK;
}

jde_status jde_sparse_emb(jde_ctx* c, int on) {
    if (!c) return fail(JDE_EINVAL, "null context");
    c->sparse_emb = on != 0;
    return JDE_OK;
}

jde_status jde_window_down(jde_ctx* c, int on) {
    if (!c) return fail(JDE_EINVAL, "null context");
    c->window_down = on != 0;
    return JDE_OK;
}

jde_status jde_fold_det(jde_ctx* c, int on) {
    if (!c) return fail(JDE_EINVAL, "null context");
    c->fold_det = on != 0;
    return JDE_OK;
}

jde_status jde_window_convs(jde_ctx* c, int on) {
    if (!c) return fail(JDE_EINVAL, "null context");
    c->window_convs = on != 0;
    return JDE_OK;
}

jde_status jde_fp8_scales(const jde_ctx* c, float* in_scales, int n_ops) {
    if (!c || !in_scales) return fail(JDE_EINVAL, "null argument");
    if (n_ops != (int)c->ops.size()) return fail(JDE_EINVAL, "expected %zu entries", c->ops.size());
    for (int i = 0; i < n_ops; ++i) in_scales[i] = c->ops[i].fp8 ? c->ops[i].in_scale : 0.f;
    return JDE_OK;
}

void jde_fp8_encode(const float* x, uint8_t* out, size_t n) {
    for (size_t i = 0; i < n; ++i) out[i] = f32_to_e4m3(x[i]);
}

void jde_mx_encode(int fmt, const float* x, uint8_t* out, size_t n) {
    if (fmt != 2 && fmt != 4) return;
    for (size_t i = 0; i < n; ++i) out[i] = (uint8_t)mx_code_host(fmt, x[i]);
}

struct jde_graph {
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    jde_ctx* ctx = nullptr;          // graphs for any batch: their context and workspace
    char* ws = nullptr;
};

jde_status jde_graph_capture(jde_ctx* c, const float* frames, const jde_frame_desc* d, int n, void* ws, size_t wsb,
                             const jde_head_out* heads, float conf, float iou, const float* logit_offset,
                             const jde_dets* dets, const float* fe, const double* mean, const double* cov,
                             const int* tb, float* cost, void* stream, jde_graph** out) {
    if (!c || !out) return fail(JDE_EINVAL, "null argument");
    *out = nullptr;
    if (c->prof) return fail(JDE_ESTATE, "graph capture while profiling");
    if (!stream) return fail(JDE_EINVAL, "capture needs a non-default stream");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    jde_status st = jde_forward(c, frames, d, n, ws, wsb, heads, stream);
    if (st == JDE_OK) st = jde_decode(c, heads, d, n, conf, iou, logit_offset, ws, wsb, dets, stream);
    if (st == JDE_OK && tb) st = jde_cost_matrix_batch(fe, mean, cov, tb, dets, n, c->cfg.emb_dim, 9.4877, cost, stream);
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(s, &g);
    if (st != JDE_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (ee != hipSuccess) return fail(JDE_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ee));
    jde_graph* G = new jde_graph();
    G->g = g;
    const hipError_t ie = hipGraphInstantiate(&G->e, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(g);
        delete G;
        return fail(JDE_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ie));
    }
    *out = G;
    return JDE_OK;
}

jde_status jde_graph_capture_any(jde_ctx* c, const float* frames, void* ws, size_t wsb, const jde_head_out* heads,
                                 float conf, float iou, const float* logit_offset, const jde_dets* dets, void* stream,
                                 jde_graph** out) {
    if (!c || !out) return fail(JDE_EINVAL, "null argument");
    *out = nullptr;
    if (c->prof) return fail(JDE_ESTATE, "graph capture while profiling");
    if (!stream) return fail(JDE_EINVAL, "capture needs a non-default stream");
    if (c->et == kF32 || c->fp8) return fail(JDE_EUNSUPPORTED, "a graph for any batch runs BF16 or FP16 contexts");
    if (!c->fuse_stem) return fail(JDE_EUNSUPPORTED, "a graph for any batch needs the fused stem");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    jde_status st = forward_impl(c, frames, nullptr, 0, ws, wsb, heads, stream, true);
    if (st == JDE_OK) st = decode_impl(c, heads, nullptr, 0, conf, iou, logit_offset, ws, wsb, dets, stream, true);
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(s, &g);
    if (st != JDE_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (ee != hipSuccess) return fail(JDE_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ee));
    jde_graph* G = new jde_graph();
    G->g = g;
    G->ctx = c;
    G->ws = (char*)ws;
    const hipError_t ie = hipGraphInstantiate(&G->e, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(g);
        delete G;
        return fail(JDE_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ie));
    }
    *out = G;
    return JDE_OK;
}

jde_status jde_graph_launch_batch(jde_graph* g, const jde_frame_desc* d, int n, void* stream) {
    if (!g || !g->e || !g->ctx) return fail(JDE_EINVAL, "not a graph for any batch");
    jde_ctx* c = g->ctx;
    bool uniform;
    if (jde_status st = batch_ok(c, d, n, &uniform)) return st;
    DynHeader h{};
    h.v[kDynN] = n;
    h.v[kDynUniform] = uniform ? 1 : 0;
    for (int l = 0; l < kLevels; ++l) h.v[kDynM + l] = (int)level_pixels(d, n, l);
    for (int f = 0; f < n; ++f) {
        h.v[kDynStemTiles] += stem_down_tiles(d[f].h, d[f].w);
        h.v[kDynRb64] += resblock_tiles(64, d[f].h >> 1, d[f].w >> 1);
        h.v[kDynRb128] += resblock_tiles(128, d[f].h >> 2, d[f].w >> 2);
    }
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_setup_dyn(geom_params(d, n), h, (int*)(g->ws + c->ws_geom), (int*)(g->ws + c->ws_dyn),
                             (int*)(g->ws + c->ws_counts), c->cfg.max_frames, (int*)(g->ws + c->ws_work_count), 3,
                             (int*)(g->ws + c->ws_det_cnt), c->det_cnt_n, s));
    HIP_TRY(hipGraphLaunch(g->e, s));
    return JDE_OK;
}

jde_status jde_graph_launch(jde_graph* g, void* stream) {
    if (!g || !g->e) return fail(JDE_EINVAL, "null graph");
    if (g->ctx) return fail(JDE_EINVAL, "a graph for any batch is launched with jde_graph_launch_batch");
    HIP_TRY(hipGraphLaunch(g->e, (hipStream_t)stream));
    return JDE_OK;
}

void jde_graph_destroy(jde_graph* g) {
    if (!g) return;
    if (g->e) (void)hipGraphExecDestroy(g->e);
    if (g->g) (void)hipGraphDestroy(g->g);
    delete g;
}

}  // extern "C"
