// Convolutions of the JDE forward (Darknet-53 backbone, FPN, heads; Sec. 3.1)
// for gfx950.
//
// * stem: frame ingest (NCHW FP32 pixels) fused with the 3x3 3->c0 conv, folded
//   BN bias and leaky ReLU.  It is HBM-bound (12 bytes in, 2*c0 out per pixel);
//   with 16-bit storage it runs on MFMA from an LDS-staged input window, in
//   FP32 on the vector ALUs (one output pixel per thread).
// * conv_igemm: every other conv as an implicit GEMM on MFMA.  Rows of the MFMA
//   A operand are output channels (weights [Cout][k][k][Cin] are K-contiguous),
//   rows of the B operand are output pixels gathered from NHWC activations
//   (im2col on the fly with zero halo).  Both tiles are staged through LDS,
//   double-buffered, one barrier per K chunk.  The epilogue is fused: folded-BN
//   bias, leaky ReLU 0.1, residual add (after the activation), cast, and an
//   optional split of the output columns into a second, linear FP32 output (the
//   det 3x3 and emb 3x3 of a head share their input and run as one GEMM).
//   The FPN's nearest x2 upsample + concat is fused into the B-tile loader: the
//   first conv of the stride-16 and stride-8 heads reads channels [0, cin1)
//   from the half-resolution lateral map at (y/2, x/2) and the rest from the
//   skip map at (y, x), so the concatenated tensor is never materialised.
#include <type_traits>

#include "jde_internal.h"

namespace jde {

// f(integral_constant<int, I>) for I = B .. E - 1, in order
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// leaky ReLU 0.1: max(x, 0.1 x) equals (x > 0 ? x : 0.1 x) for every x (signed
// zeros included).  Written as the median of (x, 0.1 x, FLT_MAX), the same value
// for every finite x: the median instruction takes its operands as they are,
// where fmax first quiets a possible signalling NaN in x with an extra
// instruction whenever x comes from a matrix-core accumulator (two instructions,
// not three; with +inf as the bound the compiler turns the median back into fmax).
__device__ __forceinline__ float leaky01(float x) {
    return __builtin_amdgcn_fmed3f(x, 0.1f * x, 3.40282347e38f);
}

template <typename T> struct V16;
template <> struct V16<float> { typedef f32x4 type; };
template <> struct V16<bf16> { typedef bf16x8 type; };
template <> struct V16<f16> { typedef f16x8 type; };

template <typename T> __device__ __forceinline__ T cvt_out(float x) { return (T)x; }

// Word 3 of a raw buffer resource on gfx9-class GPUs (32-bit dword format);
// kOOB is a byte offset past every buffer (all are < 2^31 bytes).
constexpr int kBufFlags = 0x00020000;
constexpr int kXCDs = 8;     // accelerator complex dies of an MI355X, each with its own L2
constexpr int kOOB = 0x80000000;
// s_waitcnt immediate (gfx9 encoding): vmcnt vm, lgkmcnt lgkm, expcnt not waited
constexpr int waitcnt_imm(int vm, int lgkm) { return (vm & 15) | ((vm >> 4) << 14) | (7 << 4) | (lgkm << 8); }

// Row m of a level-`lvl` packed tensor -> (frame, y, x).
__device__ __forceinline__ void map_pixel(const int* __restrict__ geom, int nframes, int uniform, int lvl,
                                          int m, int& f, int& y, int& x) {
    if (uniform) {
        const int h = geom[0] >> lvl, w = geom[1] >> lvl;
        const int hw = h * w;
        f = m / hw;
        const int p = m - f * hw;
        y = p / w;
        x = p - y * w;
    } else {
        f = 0;
        while (f + 1 < nframes && m >= geom[(f + 1) * kGeomInts + 2 + lvl]) ++f;
        const int p = m - geom[f * kGeomInts + 2 + lvl];
        const int w = geom[f * kGeomInts + 1] >> lvl;
        y = p / w;
        x = p - y * w;
    }
}

// ---------------------------------------------------------------------------
// Stem: out[m][co] = leaky(b[co] + sum_{r,s,c} frame[c][y+r-1][x+s-1] w[co][r][s][c]).
// ---------------------------------------------------------------------------
template <typename TO, int COUT>
__global__ __launch_bounds__(256) void stem_kernel(const float* __restrict__ frames,
                                                   const int* __restrict__ geom, int nframes,
                                                   int uniform, int M,
                                                   const float* __restrict__ w,
                                                   const float* __restrict__ bias,
                                                   TO* __restrict__ out) {
    const int m = blockIdx.x * 256 + threadIdx.x;
    if (m >= M) return;
    int f, y, x;
    map_pixel(geom, nframes, uniform, 0, m, f, y, x);
    const int h = geom[f * kGeomInts + 0], wd = geom[f * kGeomInts + 1];
    const float* fr = frames + (size_t)geom[f * kGeomInts + 2] * 3;
    float in[27];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int iy = y + r - 1, ix = x + s - 1;
            const bool ok = (unsigned)iy < (unsigned)h && (unsigned)ix < (unsigned)wd;
#pragma unroll
            for (int c = 0; c < 3; ++c)
                in[(r * 3 + s) * 3 + c] = ok ? fr[((size_t)c * h + iy) * wd + ix] : 0.f;
        }
    TO* o = out + (size_t)m * COUT;
#pragma unroll
    for (int c0 = 0; c0 < COUT; c0 += 8) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float* wc = w + (c0 + j) * 27;
            float acc = bias[c0 + j];
#pragma unroll
            for (int t = 0; t < 27; ++t) acc = __builtin_fmaf(in[t], wc[t], acc);
            v[j] = leaky01(acc);
        }
        if constexpr (sizeof(TO) == 4) {
            *(f32x4*)(o + c0) = f32x4{v[0], v[1], v[2], v[3]};
            *(f32x4*)(o + c0 + 4) = f32x4{v[4], v[5], v[6], v[7]};
        } else {
            typedef TO T8 __attribute__((ext_vector_type(8)));
            T8 pk;
#pragma unroll
            for (int j = 0; j < 8; ++j) pk[j] = (TO)v[j];
            *(T8*)(o + c0) = pk;
        }
    }
}

// Workgroup L of W runs on XCD L % 8; returns the logical index that gives every
// XCD a contiguous range of [0, W) (a bijection), so that neighbouring work items
// share one XCD's L2.
__device__ __forceinline__ int xcd_remap(int L, int W) {
    const int xcd = L % kXCDs, local = L / kXCDs;
    const int base = W / kXCDs, extra = W % kXCDs;
    return xcd < extra ? xcd * (base + 1) + local : extra * (base + 1) + (xcd - extra) * base + local;
}

// ---------------------------------------------------------------------------
// Stem operands on the matrix cores.  The 3 x 3 x 3 receptive field of a stem
// output is laid out over two 32-wide k-steps as k = 16 r + 4 s + c (row r and
// column s of the 3x3, channel c; the s = 3 and c = 3 slots and k >= 48 carry
// zero weights).  The input window sits in LDS as FP16 positions of 4 channel
// slots (8 bytes: c0, c1, c2, 0), so a lane's eight k-values of a k-step -- two
// horizontally adjacent positions x 4 slots -- are 16 contiguous bytes: one LDS
// read per k-step instead of eight reads and eight conversions.  FP16 storage
// also keeps a window of the low parts x - fp16(x).
// ---------------------------------------------------------------------------
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

// Marks registers as read here (an empty asm statement taking them as inputs),
// so that the waits for the loads that wrote them are placed here rather than
// inside a later loop.
template <typename X>
__device__ __forceinline__ void touch_regs1(const X& x) {
    if constexpr (sizeof(X) <= 16 && !__is_array(X)) {
        asm volatile("" ::"v"(x));
    } else {
#pragma unroll
        for (int i = 0; i < (int)(sizeof(x) / sizeof(x[0])); ++i) touch_regs1(x[i]);
    }
}
template <typename... X>
__device__ __forceinline__ void touch_regs(const X&... x) {
    (touch_regs1(x), ...);
}

// A operand of output channel co, k-step m, lane group kg: FP16 hi and lo parts
__device__ __forceinline__ void stem_wfrag(const float* __restrict__ w, int co, int m, int kg, f16x8& hi,
                                           f16x8& lo) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = 32 * m + 8 * kg + j, r = k >> 4, s = (k >> 2) & 3, c = k & 3;
        const float v = (r < 3 && s < 3 && c < 3) ? w[co * 27 + (r * 3 + s) * 3 + c] : 0.f;
        hi[j] = (f16)v;
        lo[j] = (f16)(v - (float)hi[j]);
    }
}

// B operand of k-step m for a pixel whose 3x3 window starts at position `pos`
// (row 0, column 0 of the receptive field) in a window of row stride `ws`.  The
// lane groups of kernel row 3 (k-step 1, kg >= 2) meet zero weights (stem_wfrag):
// they read row 2 again -- finite frame values, so the products are zeros --
// rather than branch, which would keep the compiler from overlapping one
// block's LDS reads with another's matrix-core work.
__device__ __forceinline__ f16x8 stem_bfrag(const f16x4* __restrict__ win, int pos, int ws, int m, int kg) {
    const int r = 2 * m + (kg >> 1);
    const f16x4* q = win + pos + (r > 2 ? 2 : r) * ws + 2 * (kg & 1);
    const f16x4 a = q[0], b = q[1];
    return f16x8{a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
}

// One 16-pixel block of stem outputs for channel groups 0..NG-1: FP32
// accumulation started at the bias (bv: this lane's 4 channels per group); with
// split, lo x hi + hi x lo + hi x hi per k-step.
template <int NG, bool split>
__device__ __forceinline__ void stem_block(const f16x4* __restrict__ wh, const f16x4* __restrict__ wlo, int pos,
                                           int ws, int kg, const f16x8 (&wa)[NG][2], const f16x8 (&wl)[NG][2],
                                           const float (&bv)[NG][4], f32x4 (&acc)[NG]) {
#pragma unroll
    for (int cg = 0; cg < NG; ++cg) acc[cg] = f32x4{bv[cg][0], bv[cg][1], bv[cg][2], bv[cg][3]};
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const f16x8 b = stem_bfrag(wh, pos, ws, m, kg);
        f16x8 bl{};
        if constexpr (split) bl = stem_bfrag(wlo, pos, ws, m, kg);
#pragma unroll
        for (int cg = 0; cg < NG; ++cg) {
            if constexpr (split) {
                acc[cg] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wl[cg][m], b, acc[cg], 0, 0, 0);
                acc[cg] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wa[cg][m], bl, acc[cg], 0, 0, 0);
            }
            acc[cg] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wa[cg][m], b, acc[cg], 0, 0, 0);
        }
    }
}

// ---------------------------------------------------------------------------
// Stem on the matrix cores (16-bit activation storage).  Work items are
// segments of up to kStemSeg output pixels of one image row, walked by
// persistent workgroups.  For each item the input window it
// needs (3 channels x 3 rows x kStemSeg + 2 columns, zero outside the frame) is
// read with coalesced loads -- the next item's window is loaded into registers
// while the current one is computed -- and parked in LDS (double-buffered).
// Items are split into 8 contiguous bands, one per XCD, and the workgroups of
// an XCD walk their band together, so neighbouring rows -- whose windows
// overlap -- are fetched once into that XCD's L2.
// Each wave then runs 16-pixel blocks from LDS (stem_block: two k-steps of
// v_mfma_f32_16x16x32_f16 per 16 output channels; A = folded weights, rows =
// channels; B = pixels), FP32 accumulation.  For FP16 storage each operand is
// split into FP16 parts
// x = hi + lo (hi = fp16(x), lo = fp16(x - hi)) and the product is formed as
// lo*hi + hi*lo + hi*hi (the lo*lo term is below FP32 rounding): about 22
// significant bits, as the FP32 stem keeps.  For BF16 storage (8 significant
// bits) the FP16 operands alone (11 bits) suffice.  The output is written with
// streaming (non-temporal) 16-byte stores: it is far larger than the caches and
// is next read by the following layer, so keeping it out of L2 leaves the L2 to
// the frames.  Image widths are multiples of 32, so a 16-pixel block never
// crosses a row.
// ---------------------------------------------------------------------------
constexpr int kStemSeg = 256;

template <typename TO, int COUT>
__global__ __launch_bounds__(256) void stem_mfma_kernel(const float* __restrict__ frames,
                                                        const int* __restrict__ geom, int nframes, int uniform,
                                                        const float* __restrict__ w,
                                                        const float* __restrict__ bias, TO* __restrict__ out,
                                                        int nseg, int total) {
    // window: 3 rows x WS positions, position j <-> x = x0 + j - 1 (the last one
    // only feeds zero-weight slots)
    constexpr int WS = kStemSeg + 3, NP = 3 * WS, NG = COUT / 16;
    constexpr bool split = __is_same(TO, f16);
    __shared__ f16x4 wh[2][NP];
    __shared__ f16x4 wlo[split ? 2 : 1][split ? NP : 1];
    // item P -> frame f, row y, first column x0 (x0 >= width: nothing to do)
    auto locate = [&](int P, int& f, int& y, int& x0) {
        x0 = (P % nseg) * kStemSeg;
        y = P / nseg;
        f = 0;
        if (uniform) {
            f = y / geom[0];
            y -= f * geom[0];
        } else {
            while (f + 1 < nframes && y >= geom[f * kGeomInts]) {
                y -= geom[f * kGeomInts];
                ++f;
            }
        }
    };
    constexpr int NLD = (NP + 255) / 256;
    float wv[NLD][3];
    auto load = [&](int P) {  // every load of the window in flight at once
        int f, y, x0;
        locate(P, f, y, x0);
        const int* g = geom + f * kGeomInts;
        const int h = g[0], wd = g[1];
        const float* fr = frames + (size_t)g[2] * 3;
#pragma unroll
        for (int it = 0; it < NLD; ++it) {
            const int i = threadIdx.x + it * 256;
            const int r = i / WS, j = i - r * WS;
            const int iy = y + r - 1, ix = x0 + j - 1;
            const bool ok = i < NP && j < WS - 1 && (unsigned)iy < (unsigned)h && (unsigned)ix < (unsigned)wd;
#pragma unroll
            for (int c = 0; c < 3; ++c) wv[it][c] = ok ? fr[((size_t)c * h + iy) * wd + ix] : 0.f;
        }
    };
    auto park = [&](int buf) {
#pragma unroll
        for (int it = 0; it < NLD; ++it) {
            const int i = threadIdx.x + it * 256;
            if (i < NP) {
                f16x4 hv, lv;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    hv[c] = (f16)wv[it][c];
                    lv[c] = (f16)(wv[it][c] - (float)hv[c]);
                }
                hv[3] = lv[3] = (f16)0.f;
                wh[buf][i] = hv;
                if constexpr (split) wlo[buf][i] = lv;
            }
        }
    };
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int p = lane & 15, kg = lane >> 4;
    f16x8 wa[NG][2], wl[NG][2];
    float bv[NG][4];
#pragma unroll
    for (int cg = 0; cg < NG; ++cg) {
#pragma unroll
        for (int m = 0; m < 2; ++m) stem_wfrag(w, cg * 16 + p, m, kg, wa[cg][m], wl[cg][m]);
#pragma unroll
        for (int i = 0; i < 4; ++i) bv[cg][i] = bias[cg * 16 + kg * 4 + i];
    }
    touch_regs(wa, wl, bv);  // weights landed before the loop (see stem_down_kernel)
    // band of this workgroup's XCD (gridDim.x is a multiple of 8): items
    // [lo, hi), walked with stride per = gridDim.x / 8 from lo + blockIdx.x / 8
    const int per = gridDim.x / kXCDs, xcd = blockIdx.x % kXCDs;
    const int band = (total + kXCDs - 1) / kXCDs;
    const int lo = xcd * band, hi = lo + band < total ? lo + band : total;
    int P = lo + (int)blockIdx.x / kXCDs;
    if (P >= hi) return;  // uniform over the workgroup
    load(P);
    park(0);
    __syncthreads();
    for (int t = 0; P < hi; ++t, P += per) {
        const int buf = t & 1;
        const int Pn = P + per;
        if (Pn < hi) load(Pn);
        int f, y, x0;
        locate(P, f, y, x0);
        const int* g = geom + f * kGeomInts;
        const int wd = g[1];
        const size_t row_m = (size_t)g[2] + (size_t)y * wd;
        for (int blk = wave; blk < kStemSeg / 16; blk += 4) {
            const int xb = x0 + blk * 16;
            if (xb >= wd) break;
            f32x4 acc[NG];
            stem_block<NG, split>(wh[buf], wlo[split ? buf : 0], blk * 16 + p, WS, kg, wa, wl, bv, acc);
            typedef TO T4 __attribute__((ext_vector_type(4)));
            T4 pk[NG];
#pragma unroll
            for (int cg = 0; cg < NG; ++cg)
#pragma unroll
                for (int i = 0; i < 4; ++i) pk[cg][i] = (TO)leaky01(acc[cg][i]);
            TO* o = out + (row_m + xb + p) * COUT;
            if constexpr (NG == 1) {
                // 16 pixels x 32 bytes: one contiguous 512-byte store
                typedef unsigned U2 __attribute__((ext_vector_type(2)));
                U2 u2;
                __builtin_memcpy(&u2, &pk[0], 8);
                __builtin_nontemporal_store(u2, (U2*)(o + kg * 4));
            } else {
                // Lanes l and l ^ 16 (kg and kg ^ 1) trade halves so that each holds 8
                // consecutive channels: the even lane channels 4 kg .. 4 kg + 7 of group
                // 0, the odd lane 16 + 4 (kg - 1) .. + 7 of group 1.  Each lane then
                // stores 16 bytes and one store covers 16 pixels x 64 bytes contiguously.
                const bool odd = kg & 1;
                const T4 give = odd ? pk[0] : pk[1];
                unsigned g2[2], r2[2];
                __builtin_memcpy(g2, &give, 8);
                r2[0] = __shfl_xor(g2[0], 16);
                r2[1] = __shfl_xor(g2[1], 16);
                T4 got;
                __builtin_memcpy(&got, r2, 8);
                const T4 lo = odd ? got : pk[0], hi = odd ? pk[1] : got;
                typedef unsigned U4 __attribute__((ext_vector_type(4)));
                U4 u4;
                __builtin_memcpy(&u4, &lo, 8);
                __builtin_memcpy((char*)&u4 + 8, &hi, 8);
                __builtin_nontemporal_store(u4, (U4*)(o + (odd ? 16 + 4 * (kg - 1) : 4 * kg)));
            }
        }
        if (Pn < hi) park(buf ^ 1);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Stem fused with the first downsample conv (16-bit storage, c0 = 32): the
// stem's output -- the largest tensor of the network -- never goes to HBM.
// Work items are 2 x 64 tiles of the stride-2 level output (all 64 channels),
// walked by persistent workgroups.  Per tile: the frame window it needs (3
// channels x 7 rows x 131 columns, zero outside the frame; loaded into
// registers while the previous tile is computed) is parked in LDS; the 5 x 129
// stem outputs the 3x3 stride-2 conv reads are computed on MFMA (as in
// stem_mfma_kernel; a stem position outside the image is the conv's zero
// padding, not a stem value) and kept in LDS in the storage type -- the same
// rounding as a stored stem output -- with even and odd columns in separate
// planes (80-byte pixel slots), so that the conv's stride-2 reads are unit-
// stride and bank-conflict-free; the conv then runs from LDS with K = 9 taps x
// 32 channels, one MFMA k-step per tap in the same order as the unfused GEMM.
// Wave w computes output channels 16 w .. 16 w + 15 for the whole tile, so its
// weights (9 taps x 16 channels x 32) stay in registers for the workgroup's life.
// ---------------------------------------------------------------------------
constexpr int kSdTY = 2, kSdTX = 64;  // output tile (stride-2 level)

// (two waves per SIMD: two workgroups per CU, as the persistent grid assumes;
// the FP16 form, which also holds the low parts, spills 10 registers for it --
// 488 -> 372 us measured -- the BF16 form fits in 226)
template <typename TO>
__global__ __launch_bounds__(256, 2) void stem_down_kernel(const float* __restrict__ frames,
                                                        const int* __restrict__ geom, int nframes, int total,
                                                        const float* __restrict__ w0, const float* __restrict__ b0,
                                                        const TO* __restrict__ w1, const float* __restrict__ b1,
                                                        TO* __restrict__ out, const int* __restrict__ dyn) {
    if (dyn) {  // batch header: frames and tiles of this batch (the grid covers the capacity)
        nframes = dyn[kDynN];
        total = dyn[kDynStemTiles];
    }
    constexpr int C0 = 32, C1 = 64;
    constexpr int WR = 2 * kSdTY + 1, WC = 2 * kSdTX + 1;  // stem window: 5 x 129
    constexpr int FR = WR + 2, FC = WC + 2;                  // frame window: 7 x 131
    constexpr int FS = FC + 1;                               // positions per window row (+1: zero-weight slots)
    constexpr int NE = kSdTX + 1;                            // pixels per parity plane (even: 65, odd: 64)
    constexpr int PS = 40;                                   // elements per pixel slot (32 + 8 padding)
    constexpr int NPF = FR * FS;
    constexpr int NSB = (WR * WC + 15) / 16;                 // 16-pixel stem blocks (41)
    constexpr bool split = __is_same(TO, f16);
    typedef typename V16<TO>::type V;
    __shared__ f16x4 fwh[NPF];                               // FP16 positions x 4 channel slots
    __shared__ f16x4 fwl[split ? NPF : 1];                   // low parts (FP16 storage)
    __shared__ __attribute__((aligned(16))) TO sw[WR * 2 * NE * PS];

    // item -> frame, output tile origin (ty0, tx0) on the stride-2 level
    struct Tile { int f, ty0, tx0, h1, w1; };
    auto locate = [&](int item) {
        Tile t{0, 0, 0, 0, 0};
        for (;; ++t.f) {
            t.h1 = geom[t.f * kGeomInts] >> 1;
            t.w1 = geom[t.f * kGeomInts + 1] >> 1;
            const int n = ((t.h1 + kSdTY - 1) / kSdTY) * ((t.w1 + kSdTX - 1) / kSdTX);
            if (item < n || t.f + 1 >= nframes) break;
            item -= n;
        }
        const int tw = (t.w1 + kSdTX - 1) / kSdTX;
        t.ty0 = (item / tw) * kSdTY;
        t.tx0 = (item % tw) * kSdTX;
        return t;
    };
    // The frame window is loaded as 16-byte groups of 4 columns from x = 2 tx0 - 4
    // (16-byte aligned: widths are multiples of 32), so a group lies wholly inside
    // or wholly outside the frame; thread i < 7 x 34 loads group i % 34 of row i / 34
    // for the 3 channels.
    constexpr int NGR = (FS + 2 + 3) / 4;  // groups per row: positions -2 .. 4 NGR - 3
    static_assert(FR * NGR <= 256, "one group per thread");
    typedef float f32x4v __attribute__((ext_vector_type(4)));
    f32x4v fv[3];
    const int gr = threadIdx.x / NGR, gq = threadIdx.x - gr * NGR;
    auto load = [&](const Tile& t) {
        const int* g = geom + t.f * kGeomInts;
        const int h = g[0], wd = g[1];
        const float* fr = frames + (size_t)g[2] * 3;
        const int iy = 2 * t.ty0 - 2 + gr, x = 2 * t.tx0 - 4 + 4 * gq;
        const bool ok = gr < FR && (unsigned)iy < (unsigned)h && x >= 0 && x + 4 <= wd;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            fv[c] = ok ? *(const f32x4v*)(fr + ((size_t)c * h + iy) * wd + x) : f32x4v{0.f, 0.f, 0.f, 0.f};
    };
    auto park = [&]() {
        if (gr < FR) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int j = 4 * gq - 2 + k;  // window position of column x + k
                if (j >= 0 && j < FS) {
                    f16x4 hv, lv;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        hv[c] = (f16)fv[c][k];
                        lv[c] = (f16)(fv[c][k] - (float)hv[c]);
                    }
                    hv[3] = lv[3] = (f16)0.f;
                    fwh[gr * FS + j] = hv;
                    if constexpr (split) fwl[gr * FS + j] = lv;
                }
            }
        }
    };

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int p = lane & 15, kg = lane >> 4;
    // stem weights of this lane as FP16 hi (+ lo), two k-steps per channel group
    f16x8 wa[2][2], wl[2][2];
    float bv[2][4];
#pragma unroll
    for (int cg = 0; cg < 2; ++cg) {
#pragma unroll
        for (int m = 0; m < 2; ++m) stem_wfrag(w0, cg * 16 + p, m, kg, wa[cg][m], wl[cg][m]);
#pragma unroll
        for (int i = 0; i < 4; ++i) bv[cg][i] = b0[cg * 16 + kg * 4 + i];
    }
    // conv weights of this wave's channel block, all 9 taps: lane = (channel p, k-slot kg)
    V af[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) af[t] = *(const V*)(w1 + (size_t)(wave * 16 + p) * (9 * C0) + t * C0 + kg * 8);
    float cb1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) cb1[q] = b1[wave * 16 + kg * 4 + q];
    // Use the weights once here: otherwise the compiler, merging loop entry and
    // back edge, counts their loads as outstanding inside the loop and waits for
    // the next tile's frame loads (issued later) before the conv's MFMAs and the
    // epilogue.
    touch_regs(af, cb1, wa, bv);
    // output buffer: every level-1 pixel of the batch x 64 channels
    const int out_bytes = geom[(nframes - 1) * kGeomInts + 8 + 1] * C1 * (int)sizeof(TO);
    const __amdgpu_buffer_rsrc_t r_out = __builtin_amdgcn_make_buffer_rsrc((void*)out, 0, out_bytes, kBufFlags);

    int P = blockIdx.x;
    if (P >= total) return;  // uniform over the workgroup
    Tile t = locate(P);
    load(t);
    park();
    __syncthreads();
    for (; P < total; P += gridDim.x) {
        const int* g = geom + t.f * kGeomInts;
        const int h = g[0], wd = g[1];
        // the next tile's frame window: in flight during this tile's stem and conv
        const int Pn = P + gridDim.x;
        Tile tn = t;
        if (Pn < total) {
            tn = locate(Pn);
            load(tn);
        }
        // stem window: flat 16-pixel blocks over the 5 x 129 positions; in an
        // interior tile every stem position lies inside the frame
        const bool interior = 2 * t.ty0 - 1 >= 0 && 2 * t.tx0 - 1 >= 0 && 2 * t.ty0 - 1 + WR <= h &&
                              2 * t.tx0 - 1 + WC <= wd;
        // batches of SB blocks per wave, unrolled so that the blocks' LDS reads,
        // MFMAs and epilogues overlap; slots past the last block recompute it
        // without storing
        // (all SB blocks' operand reads first, then their MFMAs -- per accumulator in
        // stem_block's order -- then their epilogues)
        constexpr int SB = 4;
        for (int b0 = 0; b0 < (NSB + 3) / 4; b0 += SB) {
            f16x8 fbh[SB][2], fbl[SB][2];
            f32x4 accs[SB][2];
#pragma unroll
            for (int b = 0; b < SB; ++b) {
                const int bi = wave + 4 * (b0 + b);
                const int q = (bi < NSB ? bi : NSB - 1) * 16 + p;
                const int R = q / WC, C = q - R * WC;
                const int pos = q < WR * WC ? R * FS + C : 0;
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    fbh[b][m] = stem_bfrag(fwh, pos, FS, m, kg);
                    fbl[b][m] = split ? stem_bfrag(fwl, pos, FS, m, kg) : f16x8{};
                }
            }
#pragma unroll
            for (int b = 0; b < SB; ++b) {
#pragma unroll
                for (int cg = 0; cg < 2; ++cg) accs[b][cg] = f32x4{bv[cg][0], bv[cg][1], bv[cg][2], bv[cg][3]};
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int cg = 0; cg < 2; ++cg) {
                        if constexpr (split) {
                            accs[b][cg] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wl[cg][m], fbh[b][m], accs[b][cg], 0,
                                                                                 0, 0);
                            accs[b][cg] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wa[cg][m], fbl[b][m], accs[b][cg], 0,
                                                                                 0, 0);
                        }
                        accs[b][cg] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wa[cg][m], fbh[b][m], accs[b][cg], 0, 0,
                                                                             0);
                    }
            }
#pragma unroll
            for (int b = 0; b < SB; ++b) {
                const int bi = wave + 4 * (b0 + b);
                const bool live = bi < NSB;  // wave-uniform
                const int q = (live ? bi : NSB - 1) * 16 + p;
                const int R = q / WC, C = q - R * WC;
                const bool valid = live && q < WR * WC;
                const f32x4 (&acc)[2] = accs[b];
                const int sy = 2 * t.ty0 - 1 + R, sx = 2 * t.tx0 - 1 + C;
                const bool inside = (unsigned)sy < (unsigned)h && (unsigned)sx < (unsigned)wd;
#pragma unroll
                for (int cg = 0; cg < 2; ++cg) {
                    typedef TO T4 __attribute__((ext_vector_type(4)));
                    T4 pk;
#pragma unroll
                    for (int i = 0; i < 4; ++i) pk[i] = (TO)leaky01(acc[cg][i]);
                    if (!interior && !inside) pk = T4{};  // the conv's zero padding
                    if (valid) *(T4*)(&sw[((R * 2 + (C & 1)) * NE + (C >> 1)) * PS + cg * 16 + kg * 4]) = pk;
                }
            }
        }
        __syncthreads();  // stem window complete; the frame window is free
        // the next tile's frame window into LDS now (its loads were issued before the
        // stem), so that one barrier per tile -- the one below -- covers both buffers
        if (Pn < total) park();
        const int obase1 = g[2 + 1];  // first level-1 pixel of the frame
        // the 3x3 stride-2 conv from LDS: 8 blocks of 16 pixels (2 rows x 64 columns)
        f32x4 acc[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int tp = 0; tp < 9; ++tp) {
            const int r = tp / 3, s = tp % 3;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int ty = i >> 2, tx = (i & 3) * 16 + p;  // output row, column within the tile
                const V bf = *(const V*)(&sw[(((2 * ty + r) * 2 + (s & 1)) * NE + tx + (s >> 1)) * PS + kg * 8]);
                if constexpr (__is_same(TO, bf16))
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[tp], bf, acc[i], 0, 0, 0);
                else
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_f16(af[tp], bf, acc[i], 0, 0, 0);
            }
        }
        // epilogue: bias, leaky, store this wave's 16 channels (32 bytes of each
        // 128-byte pixel row); the frame's base pixel is read before the stores (a
        // scalar load after vector stores to memory it may alias waits for them)
        // Buffer stores, issued by every lane (outside the frame: an out-of-range
        // offset, dropped): a fixed count per wave, which the compiler's wait for
        // the next tile's window loads counts exactly.
        typedef TO T4 __attribute__((ext_vector_type(4)));
        typedef unsigned U2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int oy = t.ty0 + (i >> 2), ox = t.tx0 + (i & 3) * 16 + p;
            T4 pk;
#pragma unroll
            for (int q = 0; q < 4; ++q) pk[q] = (TO)leaky01(acc[i][q] + cb1[q]);
            U2 u2;
            __builtin_memcpy(&u2, &pk, 8);
            const int off = (oy < t.h1 && ox < t.w1)
                                ? ((obase1 + oy * t.w1 + ox) * C1 + wave * 16 + kg * 4) * (int)sizeof(TO)
                                : kOOB;
            __builtin_amdgcn_raw_buffer_store_b64(u2, r_out, off, 0, 0);
        }
        __syncthreads();  // every wave is done with the stem window; the next frame window is parked
        t = tn;
    }
}

hipError_t launch_stem_down(const float* frames, const int* geom, int nframes, int tiles, const float* w0,
                            const float* b0, const void* w1, const float* b1, void* out, int out_type,
                            hipStream_t s, const int* dyn) {
    // persistent: 2 workgroups per compute unit (63 KB of LDS each), all resident
    // (with a batch header, `tiles` is the capacity's)
    dim3 grid(tiles < 512 ? tiles : 512), block(256);
    if (out_type == kBF16)
        stem_down_kernel<bf16><<<grid, block, 0, s>>>(frames, geom, nframes, tiles, w0, b0, (const bf16*)w1, b1,
                                                      (bf16*)out, dyn);
    else if (out_type == kF16)
        stem_down_kernel<f16><<<grid, block, 0, s>>>(frames, geom, nframes, tiles, w0, b0, (const f16*)w1, b1,
                                                     (f16*)out, dyn);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}
int stem_down_tiles(int h, int w) { return ((h / 2 + kSdTY - 1) / kSdTY) * ((w / 2 + kSdTX - 1) / kSdTX); }

// ---------------------------------------------------------------------------
// 3x3 stride-2 convolution from an LDS window (16-bit storage; Cin = 64, Cout a
// multiple of 128, bias + leaky, no concat input, no residual): the backbone's
// downsample conv into the stride-4 level (Sec. 3.1).  Its K (576) is short, so
// the implicit GEMM pays a pipeline fill and drain per tile and gathers each
// input pixel 2.25 times through the load path.
// Here a persistent workgroup (8 waves) owns 128 output channels -- wave w's 16
// channels' weights for all nine taps stay in registers for the workgroup's life
// -- and walks output tiles of one row x kDwTX pixels.  A tile's input window (3
// rows x 2 kDwTX + 1 columns x Cin) is loaded once, into registers during the
// previous tile's MFMAs, then parked in the second of two LDS windows (one
// barrier per tile) with even and odd columns in separate
// planes and 16-byte-padded pixel slots (Cin + 16 elements: 160 bytes, full-rate
// operand reads), so the stride-2 reads are unit-stride.  Per pixel
// block and channel block the MFMAs run tap-major, 32 channels per k-step: the
// implicit GEMM's order, so the result is bitwise the same.
// ---------------------------------------------------------------------------
constexpr int kDwTX = 64;

template <typename T, int CIN>
__global__ __launch_bounds__(512) void down_win_kernel(const T* __restrict__ in, const T* __restrict__ w,
                                                       const float* __restrict__ bias, T* __restrict__ out,
                                                       const int* __restrict__ geom, int nframes, int lvl_in,
                                                       int cout, const int* __restrict__ dyn) {
    if (dyn) nframes = dyn[kDynN];
    constexpr int TX = kDwTX, WC = 2 * TX + 1, NE = TX + 1;
    constexpr int PS = CIN + 16;              // elements per pixel slot
    constexpr int KS = CIN / 32;              // MFMA k-steps per tap
    constexpr int CH = CIN / 8;               // 16-byte chunks per input pixel
    constexpr int NCHUNK = 3 * WC * CH;       // chunks of a window
    constexpr int LPT = (NCHUNK + 511) / 512; // window loads per thread
    typedef typename V16<T>::type V;
    typedef T T4 __attribute__((ext_vector_type(4)));
    constexpr int WE = 3 * 2 * NE * PS;       // elements of one window
    __shared__ __attribute__((aligned(16))) T win2[2 * WE];  // two windows: this tile's, the next one's

    const int lvl_out = lvl_in + 1;
    const int ncg = cout / 128;                       // channel groups of 128
    const int cg = blockIdx.x % ncg, walker = blockIdx.x / ncg, stride = gridDim.x / ncg;
    // output tiles of the batch: per frame, ho rows x ceil(wo / TX) column tiles
    int total = 0;
    for (int f = 0; f < nframes; ++f)
        total += (geom[f * kGeomInts] >> lvl_out) * (((geom[f * kGeomInts + 1] >> lvl_out) + TX - 1) / TX);
    struct Tile { int f, oy, ox0; };
    auto locate = [&](int item) {
        Tile t{0, 0, 0};
        for (;; ++t.f) {
            const int n = (geom[t.f * kGeomInts] >> lvl_out) * (((geom[t.f * kGeomInts + 1] >> lvl_out) + TX - 1) / TX);
            if (item < n || t.f + 1 >= nframes) break;
            item -= n;
        }
        const int tw = ((geom[t.f * kGeomInts + 1] >> lvl_out) + TX - 1) / TX;
        t.oy = item / tw;
        t.ox0 = (item - t.oy * tw) * TX;
        return t;
    };
    // window chunks of this thread: chunk e = tid + 512 j -> row r, window column c, 16-byte slot k
    V fv[LPT];
    auto load = [&](const Tile& t) {
        const int* g = geom + t.f * kGeomInts;
        const int hi = g[0] >> lvl_in, wi = g[1] >> lvl_in;
        const T* src = in + (size_t)g[2 + lvl_in] * CIN;
#pragma unroll
        for (int j = 0; j < LPT; ++j) {
            const int e = threadIdx.x + 512 * j;
            const int r = e / (WC * CH), rem = e - r * (WC * CH), c = rem / CH, k = rem - c * CH;
            const int iy = 2 * t.oy - 1 + r, ix = 2 * t.ox0 - 1 + c;
            const bool ok = e < NCHUNK && (unsigned)iy < (unsigned)hi && (unsigned)ix < (unsigned)wi;
            fv[j] = ok ? *(const V*)(src + ((size_t)iy * wi + ix) * CIN + 8 * k) : V{};
        }
    };
    auto park = [&](T* win) {
#pragma unroll
        for (int j = 0; j < LPT; ++j) {
            const int e = threadIdx.x + 512 * j;
            if (e < NCHUNK) {
                const int r = e / (WC * CH), rem = e - r * (WC * CH), c = rem / CH, k = rem - c * CH;
                *(V*)&win[((r * 2 + (c & 1)) * NE + (c >> 1)) * PS + 8 * k] = fv[j];
            }
        }
    };

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int p = lane & 15, kg = lane >> 4;
    const int cbase = cg * 128 + wave * 16;
    // this wave's weights, all taps and k-steps: lane = (channel p, k-slot kg)
    V af[9][KS];
#pragma unroll
    for (int tp = 0; tp < 9; ++tp)
#pragma unroll
        for (int h = 0; h < KS; ++h)
            af[tp][h] = *(const V*)(w + (size_t)(cbase + p) * (9 * CIN) + tp * CIN + h * 32 + kg * 8);
    f32x4 bv = *(const f32x4*)(bias + cbase + kg * 4);
    touch_regs(af, bv);  // the weight loads complete here, not inside the tile loop

    if (walker >= total) return;  // uniform over the workgroup
    Tile t = locate(walker);
    load(t);
    park(win2);
    __syncthreads();
    int cur = 0;
    for (int P = walker; P < total; P += stride) {
        const T* win = win2 + cur * WE;
        const int Pn = P + stride;
        Tile tn = t;
        if (Pn < total) {
            tn = locate(Pn);
            load(tn);  // in flight during this tile's MFMAs
        }
        f32x4 acc[TX / 16];
#pragma unroll
        for (int i = 0; i < TX / 16; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
        // pixel operands of a tap, read one tap ahead into a second register set so
        // that the LDS latency hides behind the previous tap's MFMAs
        V bfr[2][KS][TX / 16];
        auto rd = [&](auto tp_c, auto set_c) {
            constexpr int tp = decltype(tp_c)::value, st = decltype(set_c)::value;
            constexpr int r = tp / 3, s = tp % 3;
#pragma unroll
            for (int h = 0; h < KS; ++h)
#pragma unroll
                for (int i = 0; i < TX / 16; ++i)
                    bfr[st][h][i] = *(const V*)&win[((r * 2 + (s & 1)) * NE + i * 16 + p + (s >> 1)) * PS + h * 32 + kg * 8];
        };
        rd(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{});
        static_for<0, 9>([&](auto tp_c) {
            constexpr int tp = decltype(tp_c)::value;
            if constexpr (tp + 1 < 9) rd(std::integral_constant<int, tp + 1>{}, std::integral_constant<int, (tp + 1) & 1>{});
            __builtin_amdgcn_sched_barrier(0);  // (the scheduler would otherwise pull them just in time)
#pragma unroll
            for (int h = 0; h < KS; ++h)
#pragma unroll
                for (int i = 0; i < TX / 16; ++i) {
                    if constexpr (__is_same(T, bf16))
                        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[tp][h], bfr[tp & 1][h][i], acc[i], 0, 0, 0);
                    else
                        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_f16(af[tp][h], bfr[tp & 1][h][i], acc[i], 0, 0, 0);
                }
        });
        // the next window into the other buffer (whose last reader, the previous
        // tile, every wave finished before the barrier that ended it)
        if (Pn < total) park(win2 + (cur ^ 1) * WE);
        // epilogue: bias, leaky, this wave's 16 channels (8 bytes per lane and pixel)
        const int* g = geom + t.f * kGeomInts;
        const int wo = g[1] >> lvl_out;
        const size_t orow = (size_t)g[2 + lvl_out] + (size_t)t.oy * wo;
#pragma unroll
        for (int i = 0; i < TX / 16; ++i) {
            const int ox = t.ox0 + i * 16 + p;
            T4 pk;
#pragma unroll
            for (int q = 0; q < 4; ++q) pk[q] = cvt_out<T>(leaky01(acc[i][q] + bv[q]));
            if (ox < wo) *(T4*)(out + (orow + ox) * cout + cbase + kg * 4) = pk;
        }
        __syncthreads();  // the next window is parked; every wave is done with this one
        cur ^= 1;
        t = tn;
    }
}

// Cin 64 only: with Cin 128 the weights (144 VGPRs) and the window prefetch do not
// fit a wave's 256 registers.
bool down_win_ok(int cin, int cout, int ksz, int stride, int et) {
    return (et == kBF16 || et == kF16) && ksz == 3 && stride == 2 && cin == 64 && cout % 128 == 0;
}

static int resident_grid(const void* fn, int threads);

hipError_t launch_down_win(const void* in, void* out, const void* w, const float* bias, const int* geom, int nframes,
                           int lvl_in, int cin, int cout, int et, hipStream_t s, const int* dyn) {
    if (!down_win_ok(cin, cout, 3, 2, et)) return hipErrorInvalidValue;
    auto go = [&](auto kern, auto tag) {
        typedef decltype(tag) T;
        // persistent: the workgroups the device holds at once, a multiple of the
        // channel groups and of the 8 XCDs
        const int ncg = cout / 128;
        int g = resident_grid(reinterpret_cast<const void*>(kern), 512);
        g -= g % (8 * ncg);
        if (g < 8 * ncg) g = 8 * ncg;
        kern<<<dim3(g), dim3(512), 0, s>>>((const T*)in, (const T*)w, bias, (T*)out, geom, nframes, lvl_in, cout,
                                           dyn);
        return hipGetLastError();
    };
    if (et == kBF16) return go(down_win_kernel<bf16, 64>, bf16{});
    return go(down_win_kernel<f16, 64>, f16{});
}

hipError_t launch_stem(const float* frames, const int* geom, int nframes, int uniform, int rows, int max_w,
                       int M, const float* w, const float* bias, int cout, void* out, int out_type,
                       hipStream_t s) {
    if (out_type != kF32) {
        // 16-bit storage: the matrix-core stem, one workgroup per kStemSeg-pixel row segment
        // persistent: 4 workgroups per compute unit (256 of them), all resident at
        // once; a multiple of 8 workgroups (one band per XCD)
        const int nseg = (max_w + kStemSeg - 1) / kStemSeg;
        const int total = rows * nseg;
        const int g = total < 1024 ? ((total + 7) / 8) * 8 : 1024;
        dim3 grid2(g), block2(256);
        if (cout == 32) {
            if (out_type == kF16)
                stem_mfma_kernel<f16, 32><<<grid2, block2, 0, s>>>(frames, geom, nframes, uniform, w, bias, (f16*)out,
                                                                   nseg, total);
            else
                stem_mfma_kernel<bf16, 32><<<grid2, block2, 0, s>>>(frames, geom, nframes, uniform, w, bias,
                                                                    (bf16*)out, nseg, total);
        } else if (cout == 16) {
            if (out_type == kF16)
                stem_mfma_kernel<f16, 16><<<grid2, block2, 0, s>>>(frames, geom, nframes, uniform, w, bias, (f16*)out,
                                                                   nseg, total);
            else
                stem_mfma_kernel<bf16, 16><<<grid2, block2, 0, s>>>(frames, geom, nframes, uniform, w, bias,
                                                                    (bf16*)out, nseg, total);
        } else {
            return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    dim3 grid((M + 255) / 256), block(256);
    if (cout == 32) {
        if (out_type == kF32)
            stem_kernel<float, 32><<<grid, block, 0, s>>>(frames, geom, nframes, uniform, M, w, bias, (float*)out);
        else if (out_type == kF16)
            stem_kernel<f16, 32><<<grid, block, 0, s>>>(frames, geom, nframes, uniform, M, w, bias, (f16*)out);
        else
            stem_kernel<bf16, 32><<<grid, block, 0, s>>>(frames, geom, nframes, uniform, M, w, bias, (bf16*)out);
    } else if (cout == 16) {
        if (out_type == kF32)
            stem_kernel<float, 16><<<grid, block, 0, s>>>(frames, geom, nframes, uniform, M, w, bias, (float*)out);
        else if (out_type == kF16)
            stem_kernel<f16, 16><<<grid, block, 0, s>>>(frames, geom, nframes, uniform, M, w, bias, (f16*)out);
        else
            stem_kernel<bf16, 16><<<grid, block, 0, s>>>(frames, geom, nframes, uniform, M, w, bias, (bf16*)out);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused epilogue of one wave's tile (rows m_base.., channels n_base..): + bias
// (after an optional per-channel dequantisation scale), leaky ReLU 0.1, residual
// add, cast and store; columns >= n_split go linear to the FP32 output out1.
// Every group of 4 channels lies entirely below or at/above n_split and below
// Cout (both are multiples of 4).  With a.amax set, the largest |value| stored
// to out0 is folded into *a.amax (float bits as unsigned, non-negative).
// ---------------------------------------------------------------------------
// Residual tile of a conv_dma tile staged in LDS (see conv_dma): the first half of
// the tile's pixels in h0, the second in h1, row_bytes (2 x the tile's channels,
// 256 or 512) per pixel row, 16-byte slot c of row r at slot c ^ (r % 16) (16
// rows of a column read by 16 lanes hit 16 different slots).  m_tile, n_tile: the
// tile's origin; half_rows: pixels per half.
struct ResLds { const char* h0; const char* h1; int m_tile, n_tile, half_rows, row_bytes; };

template <typename T, int TM, int TN, int WTM, int WTN, bool NT = false>
__device__ __forceinline__ void store_tile(const ConvArgs& a, const f32x4 (&acc)[TM][TN], int m_base, int n_base,
                                           int lane, const float* __restrict__ dq, const ResLds* rl = nullptr) {
    typedef T T4 __attribute__((ext_vector_type(4)));
    // Every load of the epilogue (bias, scales, residual) is issued before the
    // first store, so a tile pays one memory latency rather than one per 16x16
    // block.  With the in-place residual (res == out0) each element is read and
    // then overwritten by this same lane only, so reading them all first is exact.
    f32x4 bv[TN], sv[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const int cb = n_base + j * 16 + (lane >> 4) * 4;
        const bool ok = cb < a.cout;
        bv[j] = ok ? *(const f32x4*)(a.bias + cb) : f32x4{0.f, 0.f, 0.f, 0.f};
        sv[j] = (ok && dq) ? *(const f32x4*)(dq + cb) * a.in_scale : f32x4{1.f, 1.f, 1.f, 1.f};
    }
    const bool res_t = a.res && !a.out0_f32;  // residual of the storage type (every model's case)
    T4 rv[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int m = m_base + i * 16 + (lane & 15);
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int cb = n_base + j * 16 + (lane >> 4) * 4;
            rv[i][j] = T4{};
            if (res_t && rl) {
                const int p = m - rl->m_tile, cl = cb - rl->n_tile;
                const bool second = p >= rl->half_rows;
                const int r = second ? p - rl->half_rows : p;
                const char* base = second ? rl->h1 : rl->h0;
                rv[i][j] = *(const T4*)(base + r * rl->row_bytes + (((cl >> 3) ^ (r & 15)) << 4) + (cl & 7) * 2);
            } else if (res_t && m < a.M && cb < a.n_split) {
                rv[i][j] = *(const T4*)((const T*)a.res + (size_t)m * a.ld0 + cb);
            }
        }
    }
    float amax = 0.f;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int m = m_base + i * 16 + (lane & 15);
        if (m >= a.M) continue;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int cb = n_base + j * 16 + (lane >> 4) * 4;
            if (cb >= a.cout) continue;
            float v[4];
            if (dq) {
#pragma unroll
                for (int t = 0; t < 4; ++t) v[t] = acc[i][j][t] * sv[j][t] + bv[j][t];
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) v[t] = acc[i][j][t] + bv[j][t];
            }
            if (cb < a.n_split) {
                if (a.act) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) v[t] = leaky01(v[t]);
                }
                const size_t o = (size_t)m * a.ld0 + cb;
                if (a.out0_f32) {
                    float* op = (float*)a.out0 + o;
                    if (a.res) {
                        const f32x4 r = *(const f32x4*)((const float*)a.res + o);
#pragma unroll
                        for (int t = 0; t < 4; ++t) v[t] += r[t];
                    }
                    *(f32x4*)op = f32x4{v[0], v[1], v[2], v[3]};
                } else {
                    if (res_t) {
#pragma unroll
                        for (int t = 0; t < 4; ++t) v[t] += (float)rv[i][j][t];
                    }
                    T4 pk;
#pragma unroll
                    for (int t = 0; t < 4; ++t) pk[t] = cvt_out<T>(v[t]);
                    if constexpr (NT && sizeof(T) == 2) {  // streaming store (not kept in L2)
                        typedef unsigned U2 __attribute__((ext_vector_type(2)));
                        U2 u;
                        __builtin_memcpy(&u, &pk, 8);
                        __builtin_nontemporal_store(u, (U2*)((T*)a.out0 + o));
                    } else {
                        *(T4*)((T*)a.out0 + o) = pk;
                    }
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) amax = fmaxf(amax, fabsf(v[t]));
            } else {
                *(f32x4*)(a.out1 + (size_t)m * a.ld1 + (cb - a.n_split)) = f32x4{v[0], v[1], v[2], v[3]};
            }
        }
    }
    if (a.amax) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o));
        if (lane == 0) atomicMax(a.amax, __float_as_uint(amax));
    }
}

// ---------------------------------------------------------------------------
// Where the det fold (below) keeps a conv_dma tile in LDS: rows of 2 BN bytes,
// `rows` pixel rows (a multiple of 16, as many as fit) per pipeline stage of
// `stage` bytes, `parts` stages in use, and the 4-byte last-tile flag at byte
// `flag` of stage `flag_stage` (after the rows of the last part, or in the next
// stage).  ok: the tile fits the S stages.
struct FoldLayout { bool ok; int rows, parts, flag_stage, flag; };
constexpr FoldLayout fold_layout(int bm, int bn, int bk, int st) {
    const int stage = (bm + bn) * bk * 2, row = bn * 2;
    const int rows = (stage / row) / 16 * 16 < bm ? (stage / row) / 16 * 16 : bm;
    if (rows < 16 || st < 1) return {false, 0, 0, 0, 0};
    const int parts = (bm + rows - 1) / rows;
    const int used = (bm - (parts - 1) * rows) * row;
    if (used + 4 <= stage) return {parts <= st, rows, parts, parts - 1, used};
    return {parts + 1 <= st, rows, parts, parts, 0};
}

// conv_dma tiles that carry the det fold: the tile fits the stages; not the
// 4-wave tiles of 32 K elements, whose walking form (graphs for any batch) the
// fold pushes past 256 registers (one workgroup per CU instead of two) -- and a
// tile folds in every form or in none, so that a graph for any batch computes
// what the eager forward computes, bit for bit.
constexpr bool fold_det_tile(int bm, int bn, int bk, int st, int nw) {
    return fold_layout(bm, bn, bk, st).ok && !(nw == 4 && bm * bn >= 32768);
}

// ---------------------------------------------------------------------------
// Det head's 1x1 folded into the det 3x3's epilogue (Sec. 3.1 heads: the det 3x3
// F -> 2F with leaky ReLU, then a linear 1x1 2F -> 6A).  The 3x3 tile (BM pixels
// x BN of the 2F channels) never goes to memory: after bias and leaky each wave
// rounds its values to the storage type -- what the unfused conv stores -- into
// LDS (fold_layout: pixel p in stage p / rows, row p % rows, 2 BN bytes per row,
// 16-byte slot c of row r at c ^ (r % min(16, BN / 8))), and the workgroup
// multiplies the tile by the 1x1 weights of its BN channels on MFMA, wave w
// taking pixel rows w BM/NW ...  A tile that covers all 2F channels writes the
// head output (+ the 1x1 bias).  Otherwise each channel tile writes its FP32
// partial sums to det_part[m][tile][o], and the last of the nN channel tiles of
// a pixel range to finish (a per-range counter, incremented after the partials
// are visible device-wide, reset to 0 by that last tile) adds them in channel-
// tile order, then the bias: the sum does not depend on which tile finished last.
// All threads of the workgroup call this (it has barriers); st0 .. st3: the
// pipeline stages.
// ---------------------------------------------------------------------------
template <typename T, int BM, int BN, int NW, int TM, int TN, int WTM, int WTN, int BK, int S>
__device__ __forceinline__ void det_fold(const ConvArgs& a, const f32x4 (&acc)[TM][TN], int m0, int n0, int wm,
                                         int wn, int wave, int lane, int tid, char* st0, char* st1, char* st2,
                                         char* st3) {
    typedef T T4 __attribute__((ext_vector_type(4)));
    typedef typename V16<T>::type V;
    constexpr FoldLayout L = fold_layout(BM, BN, BK, S);
    constexpr int RROW = BN * 2, SW = (BN / 8 < 16 ? BN / 8 : 16) - 1;
    constexpr int RW = BM / NW, MB = RW / 16, KS = BN / 32;
    static_assert(L.ok && RW % 16 == 0 && BN % 32 == 0 && L.rows % 16 == 0, "det fold");
    auto stage = [&](int q) { return q == 0 ? st0 : q == 1 ? st1 : q == 2 ? st2 : st3; };
    // LDS address of channel cl of tile pixel p (a 16-pixel group never straddles stages)
    auto at = [&](int p, int cl) {
        const int r = p % L.rows;
        return stage(p / L.rows) + r * RROW + (((cl >> 3) ^ (r & SW)) << 4) + (cl & 7) * 2;
    };
    int* flag = (int*)(stage(L.flag_stage) + L.flag);
    __syncthreads();  // every wave is done reading the stages the tile overlays
#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const int cl = wn * WTN + j * 16 + (lane >> 4) * 4;
        const f32x4 bv = *(const f32x4*)(a.bias + n0 + cl);
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int p = wm * WTM + i * 16 + (lane & 15);
            T4 pk;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                float v = acc[i][j][t] + bv[t];
                if (a.act) v = leaky01(v);
                pk[t] = cvt_out<T>(v);
            }
            *(T4*)at(p, cl) = pk;
        }
    }
    // 1x1 weights of this tile's channels: operand rows o = 16 ob + lane % 16 (zero past det_n)
    V wa[KS][2];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int ob = 0; ob < 2; ++ob) {
            const int o = ob * 16 + (lane & 15);
            wa[ks][ob] = o < a.det_n
                             ? *(const V*)((const T*)a.det_w + (size_t)o * a.n_split + n0 + ks * 32 + (lane >> 4) * 8)
                             : V{};
        }
    __syncthreads();
    f32x4 d[MB][2];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int ob = 0; ob < 2; ++ob) d[mb][ob] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int p = wave * RW + mb * 16 + (lane & 15);
            const V xb = *(const V*)at(p, ks * 32 + (lane >> 4) * 8);
#pragma unroll
            for (int ob = 0; ob < 2; ++ob) {
                if constexpr (__is_same(T, bf16))
                    d[mb][ob] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[ks][ob], xb, d[mb][ob], 0, 0, 0);
                else
                    d[mb][ob] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wa[ks][ob], xb, d[mb][ob], 0, 0, 0);
            }
        }
    // lane holds outputs o = 16 ob + 4 (lane / 16) + t of pixel m0 + wave RW + 16 mb + lane % 16
    const int nN = a.n_split / BN;
    if (nN == 1) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int m = m0 + wave * RW + mb * 16 + (lane & 15);
#pragma unroll
            for (int ob = 0; ob < 2; ++ob) {
                const int o = ob * 16 + (lane >> 4) * 4;
                if (m < a.M && o < a.det_n)
                    *(f32x4*)(a.det_out + (size_t)m * a.det_n + o) = d[mb][ob] + *(const f32x4*)(a.det_b + o);
            }
        }
        return;
    }
    // The partials travel through device-coherent accesses (16-byte stores and
    // agent-scope atomic loads with the device-coherence bit, which the compute
    // unit's caches and this XCD's L2 neither hold back nor serve stale): a partial
    // is at the coherence point once its store has completed, which the wait below
    // ensures before the barrier and the count.  A release fence does the same with
    // a write-back of this XCD's whole L2 per workgroup (measured: the stride-8 det
    // 3x3 launch 3.4x slower), an acquire fence with an invalidation of it, and
    // per-float coherent stores add three times what the 16-byte ones add.
    const int nt = n0 / BN;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        const int m = m0 + wave * RW + mb * 16 + (lane & 15);
#pragma unroll
        for (int ob = 0; ob < 2; ++ob) {
            const int o = ob * 16 + (lane >> 4) * 4;
            if (m < a.M && o < a.det_n) {
                float* pp = a.det_part + ((size_t)m * nN + nt) * a.det_n + o;
                asm volatile("global_store_dwordx4 %0, %1, off sc1" : : "v"(pp), "v"(d[mb][ob]) : "memory");
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 15));  // this wave's partials have landed
    __syncthreads();
    unsigned* cnt = a.det_cnt + m0 / BM;
    if (tid == 0) *flag = atomicAdd(cnt, 1u) == (unsigned)(nN - 1);
    __syncthreads();
    if (*flag) {
        const int q4 = a.det_n / 4;
        for (int e = tid; e < BM * q4; e += 64 * NW) {
            const int m = m0 + e / q4, o = (e % q4) * 4;
            if (m >= a.M) continue;
            const float* pp = a.det_part + (size_t)m * nN * a.det_n + o;
            f32x4 sum;
            for (int t = 0; t < nN; ++t)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float v = __hip_atomic_load(pp + (size_t)t * a.det_n + c, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                    sum[c] = t == 0 ? v : sum[c] + v;
                }
            *(f32x4*)(a.det_out + (size_t)m * a.det_n + o) = sum + *(const f32x4*)(a.det_b + o);
        }
        if (tid == 0) atomicExch(cnt, 0u);
    }
}

// XCD-aware tile order: workgroup L runs on XCD L % 8.  Every XCD gets a
// contiguous range of logical tiles (a bijection on [0, tiles)), ordered so that
// the tiles of one XCD share the larger operand in its L2: all channel tiles of
// a pixel range (activations dominate) or all pixel tiles of a channel range
// (weights dominate).
__device__ __forceinline__ void tile_origin(const ConvArgs& a, int BM, int BN, int& m0, int& n0) {
    const int gm = (a.M + BM - 1) / BM, gn = (a.cout + BN - 1) / BN;
    const int P = xcd_remap(blockIdx.x, gm * gn);
    if (a.n_major) {
        m0 = (P % gm) * BM;
        n0 = (P / gm) * BN;
    } else {
        n0 = (P % gn) * BN;
        m0 = (P / gn) * BM;
    }
}

// The batch a conv launch covers: this launch's grid (one tile per workgroup), or,
// in a graph for any batch (DYN), the pixels, frames and layout of the batch the
// header describes, whose tiles the workgroups walk.
struct DynBatch { int tiles, M, nframes, uniform; };

template <bool DYN>
__device__ __forceinline__ DynBatch dyn_batch(const ConvArgs& a, int BM, int BN) {
    if constexpr (!DYN) {
        return {(int)gridDim.x, a.M, a.nframes, a.uniform};
    } else {
        const int M = a.dyn[kDynM + a.lvl_out];
        return {((M + BM - 1) / BM) * ((a.cout + BN - 1) / BN), M, a.dyn[kDynN], a.dyn[kDynUniform]};
    }
}

// The arguments of one tile.  DYN: re-read from the kernel-argument segment at each
// tile through an offset the compiler cannot see is zero, so that they are not
// hoisted out of the walk and held in registers across it (which spills and costs
// the kernels a wave per SIMD of occupancy); the explicit arguments start at offset 0.
template <bool DYN>
__device__ __forceinline__ ConvArgs tile_args(const ConvArgs& a0, const DynBatch& db) {
    if constexpr (!DYN) {
        return a0;
    } else {
#if defined(__HIP_DEVICE_COMPILE__)
        typedef const __attribute__((address_space(4))) char KChar;
        typedef const __attribute__((address_space(4))) ConvArgs KArgs;
        int off = 0;
        asm volatile("" : "+s"(off));
        ConvArgs a = *(KArgs*)((KChar*)__builtin_amdgcn_kernarg_segment_ptr() + off);
#else
        ConvArgs a = a0;  // the host pass only parses device code
#endif
        a.M = db.M;
        a.nframes = db.nframes;
        a.uniform = db.uniform;
        return a;
    }
}

// The thread's index; DYN: made opaque at each tile for the same reason (values
// that depend only on the lane would otherwise be computed once and held in vector
// registers through every tile's K loop).
// NT: the workgroup's threads (a power of two; masking with it restores the range
// the opaque copy hides from the compiler).
template <bool DYN, int NT>
__device__ __forceinline__ int tile_tid() {
    int tid = threadIdx.x;
    if constexpr (DYN) {
        asm volatile("" : "+v"(tid));
        tid &= NT - 1;
    }
    return tid;
}

// The same for logical tile L of W = gm * gn tiles (a workgroup walking tiles
// L = blockIdx.x, + gridDim.x, ... with gridDim.x a multiple of 8 keeps each tile
// on the XCD the one-tile-per-workgroup order gives it).
__device__ __forceinline__ void tile_origin_at(const ConvArgs& a, int BM, int BN, int L, int W, int& m0, int& n0) {
    const int gm = (a.M + BM - 1) / BM, gn = (a.cout + BN - 1) / BN;
    const int P = xcd_remap(L, W);
    if (a.n_major) {
        m0 = (P % gm) * BM;
        n0 = (P / gm) * BN;
    } else {
        n0 = (P % gn) * BN;
        m0 = (P / gn) * BM;
    }
}

// ---------------------------------------------------------------------------
// MFMA implicit GEMM.
//   BM pixels x BN channels per workgroup of 4 waves (WGM x WGN), K chunks of BK.
//   Each wave owns a (BM/WGM) x (BN/WGN) tile of 16x16 MFMA blocks.
//   bf16/f16: v_mfma_f32_16x16x32 -- each lane feeds 8 consecutive k of one
//   row of A (a channel) and of B (a pixel), one 16-byte LDS read each.
//   fp32: v_mfma_f32_16x16x4 -- each lane reads 4 consecutive k (16 bytes)
//   and issues 4 MFMAs; lane group g = lane/16 covers k = 4g + t at step t,
//   the same assignment on both operands, so the contraction is unchanged.
//   Output: lane l holds channels 4(l/16) .. +3 of pixel l%16 of each block.
// ---------------------------------------------------------------------------
template <typename T, int BM, int BN, int WGM, int WGN, int BK, bool ALIGNED, bool DYN = false>
__global__ __launch_bounds__(256) void conv_igemm(ConvArgs a0) {
    constexpr int VEC = 16 / sizeof(T);
    constexpr int VR = BK / VEC;
    // Padded LDS row, in elements.  16-bit types: 32 bytes of padding make the
    // row stride an odd multiple of 32 bytes (96 or 160), so the 16 rows x 2
    // k-slots one ds_read_b128 serves at a time hit distinct 16-byte units
    // modulo 512 bytes.  FP32 (the checking path) keeps 16 bytes.
    constexpr int LDR = BK + (sizeof(T) == 4 ? VEC : 2 * VEC);
    constexpr int WTM = BM / WGM, WTN = BN / WGN;
    constexpr int TM = WTM / 16, TN = WTN / 16;
    constexpr int BVEC = BM * VR, AVEC = BN * VR;
    constexpr int BPT = (BVEC + 255) / 256, APT = (AVEC + 255) / 256;
    constexpr int SZ = sizeof(T);
    static_assert(WGM * WGN == 4, "4 waves");
    static_assert(TM >= 1 && TN >= 1, "wave tile");
    typedef typename V16<T>::type V;

    __shared__ __attribute__((aligned(16))) T sA[2][BN * LDR];
    __shared__ __attribute__((aligned(16))) T sB[2][BM * LDR];

    // One tile per workgroup; DYN (a graph serving any batch): this batch's pixels,
    // frames and layout come from the header, and the resident workgroups walk this
    // batch's tiles.
    const DynBatch db = dyn_batch<DYN>(a0, BM, BN);
    for (int tl = blockIdx.x; tl < db.tiles; tl += gridDim.x) {
    const ConvArgs a = tile_args<DYN>(a0, db);
    const int W = db.tiles;
    const int tid = tile_tid<DYN, 256>();
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WGM, wn = wave / WGM;
    int m0, n0;
    tile_origin_at(a, BM, BN, tl, W, m0, n0);
    const bool concat = a.cin1 > 0;
    // Buffer resources: a load whose byte offset is out of range returns zeros,
    // which is how the zero halo, rows past M and channels past Cout are read.
    const __amdgpu_buffer_rsrc_t r_in = __builtin_amdgcn_make_buffer_rsrc((void*)a.in, 0, a.in_bytes, kBufFlags);
    const __amdgpu_buffer_rsrc_t r_in2 =
        __builtin_amdgcn_make_buffer_rsrc((void*)(concat ? a.in2 : a.in), 0, concat ? a.in2_bytes : a.in_bytes,
                                          kBufFlags);
    const __amdgpu_buffer_rsrc_t r_w = __builtin_amdgcn_make_buffer_rsrc((void*)a.w, 0, a.w_bytes, kBufFlags);

    // ---- pixel-side rows owned by this thread (fixed over the K loop) ----
    // Three 32-bit registers per row (every element offset of a tensor is < 2^31):
    //   b_off: offset of the row's window origin, frame base + (iy0 w + ix0) Cin + its
    //          16-byte slot (concat: offset in the upsampled source);
    //   b_yx:  iy0 << 16 | (ix0 & 0xffff), the window origin (concat: skip-source offset);
    //   b_hw:  h << 16 | w of the input level, 0 for a row outside the batch.
    int b_off[BPT], b_yx[BPT], b_hw[BPT];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int v = tid + i * 256;
        const int row = v / VR, kv = v % VR;
        const int m = m0 + row;
        b_off[i] = 0;
        b_yx[i] = 0;
        b_hw[i] = 0;
        if (v < BVEC && m < a.M) {
            int f, y, x;
            map_pixel(a.geom, a.nframes, a.uniform, a.lvl_out, m, f, y, x);
            const int* g = a.geom + f * kGeomInts;
            if (concat) {
                const int l1 = a.lvl_out + 1;
                b_off[i] = (g[2 + l1] + (y >> 1) * (g[1] >> l1) + (x >> 1)) * a.cin1 + kv * VEC;
                b_yx[i] = (g[2 + a.lvl_out] + y * (g[1] >> a.lvl_out) + x) * (a.cin - a.cin1) + kv * VEC;
                b_hw[i] = 1;
            } else {
                const int iy0 = y * a.stride - a.pad, ix0 = x * a.stride - a.pad;
                const int h = g[0] >> a.lvl_in, w = g[1] >> a.lvl_in;
                b_off[i] = (g[2 + a.lvl_in] + iy0 * w + ix0) * a.cin + kv * VEC;
                b_yx[i] = (iy0 << 16) | (ix0 & 0xffff);
                b_hw[i] = (h << 16) | w;
            }
        }
    }
    int a_off[APT];
#pragma unroll
    for (int i = 0; i < APT; ++i) {
        const int v = tid + i * 256;
        const int row = v / VR, kv = v % VR;
        a_off[i] = (v < AVEC && n0 + row < a.cout) ? (n0 + row) * a.K + kv * VEC : -1;
    }
    auto kslot = [&](int i) { return ((tid + i * 256) % VR) * VEC; };

    // Position (tap r, s and channel ci) of the next chunk to load; advanced
    // without branches.  Past the last chunk it keeps moving: those loads are
    // never consumed, and out-of-range offsets only read zeros.
    int ld_ci = 0, ld_r = 0, ld_s = 0;
    // Two register sets: chunk c is loaded into set c & 1 three iterations before
    // it is computed and stored to LDS one iteration before, so every global load
    // has two iterations of MFMA work to arrive in.
    V ra2[2][APT], rb2[2][BPT];

    auto load_chunk = [&](int kc, V (&ra)[APT], V (&rb)[BPT]) {
        const int k0 = kc * BK;
#pragma unroll
        for (int i = 0; i < APT; ++i) {
            const bool ok = a_off[i] >= 0 && (ALIGNED || k0 + kslot(i) < a.K);
            const int off = ok ? (a_off[i] + k0) * SZ : kOOB;
            ra[i] = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r_w, off, 0, 0));
        }
        if constexpr (ALIGNED) {
            if (concat) {
                const bool first = k0 < a.cin1;
#pragma unroll
                for (int i = 0; i < BPT; ++i) {
                    const int off = b_hw[i] == 0 ? kOOB : (first ? b_off[i] + k0 : b_yx[i] + (k0 - a.cin1)) * SZ;
                    rb[i] = __builtin_bit_cast(
                        V, __builtin_amdgcn_raw_buffer_load_b128(first ? r_in : r_in2, off, 0, 0));
                }
            } else {
#pragma unroll
                for (int i = 0; i < BPT; ++i) {
                    const int iy = (b_yx[i] >> 16) + ld_r, ix = (int)(short)(b_yx[i] & 0xffff) + ld_s;
                    const int h = b_hw[i] >> 16, w = b_hw[i] & 0xffff;
                    const bool ok = (unsigned)iy < (unsigned)h && (unsigned)ix < (unsigned)w;
                    const int off = ok ? (b_off[i] + (ld_r * w + ld_s) * a.cin + ld_ci) * SZ : kOOB;
                    rb[i] = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r_in, off, 0, 0));
                }
            }
            ld_ci += BK;
            const int wrap = ld_ci >= a.cin;
            ld_ci = wrap ? 0 : ld_ci;
            ld_s += wrap;
            const int wrap2 = ld_s >= a.ksz;
            ld_s = wrap2 ? 0 : ld_s;
            ld_r += wrap2;
        } else {
#pragma unroll
            for (int i = 0; i < BPT; ++i) {
                const int kv = kslot(i);
                const int k = k0 + kv;
                const int tap = k / a.cin, ci = k - tap * a.cin;
                const int r = tap / a.ksz, s = tap - r * a.ksz;
                const int iy = (b_yx[i] >> 16) + r, ix = (int)(short)(b_yx[i] & 0xffff) + s;
                const int h = b_hw[i] >> 16, w = b_hw[i] & 0xffff;
                const bool ok = k < a.K && (unsigned)iy < (unsigned)h && (unsigned)ix < (unsigned)w;
                const int off = ok ? (b_off[i] - kv + (r * w + s) * a.cin + ci) * SZ : kOOB;
                rb[i] = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r_in, off, 0, 0));
            }
        }
    };
    auto lds_slot = [&](int i) {
        const int v = tid + i * 256;
        return (v / VR) * LDR + (v % VR) * VEC;
    };
    auto store_chunk = [&](int buf, const V (&ra)[APT], const V (&rb)[BPT]) {
#pragma unroll
        for (int i = 0; i < APT; ++i)
            if (AVEC % 256 == 0 || tid + i * 256 < AVEC) *(V*)(&sA[buf][lds_slot(i)]) = ra[i];
#pragma unroll
        for (int i = 0; i < BPT; ++i)
            if (BVEC % 256 == 0 || tid + i * 256 < BVEC) *(V*)(&sB[buf][lds_slot(i)]) = rb[i];
    };

    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int arow = wn * WTN + (lane & 15), brow = wm * WTM + (lane & 15);
    const int kofs = (lane >> 4) * VEC;
    auto compute = [&](int buf) {
        const T* A = sA[buf];
        const T* B = sB[buf];
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4 * VEC) {
            V af[TN], bfr[TM];
#pragma unroll
            for (int j = 0; j < TN; ++j) af[j] = *(const V*)(A + (arow + j * 16) * LDR + kk + kofs);
#pragma unroll
            for (int i = 0; i < TM; ++i) bfr[i] = *(const V*)(B + (brow + i * 16) * LDR + kk + kofs);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    if constexpr (sizeof(T) == 4) {
#pragma unroll
                        for (int t = 0; t < 4; ++t)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[j][t], bfr[i][t], acc[i][j], 0, 0, 0);
                    } else if constexpr (__is_same(T, bf16)) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[j], bfr[i], acc[i][j], 0, 0, 0);
                    } else {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(af[j], bfr[i], acc[i][j], 0, 0, 0);
                    }
                }
        }
    };

    const int nk = (a.K + BK - 1) / BK;
    load_chunk(0, ra2[0], rb2[0]);
    load_chunk(1, ra2[1], rb2[1]);
    store_chunk(0, ra2[0], rb2[0]);
    load_chunk(2, ra2[0], rb2[0]);
    __syncthreads();
    // Iteration kc: store chunk kc+1 (set (kc+1)&1) to LDS buffer (kc+1)&1, load
    // chunk kc+3 into the same set, compute chunk kc from LDS buffer kc&1.
    auto iter = [&](int kc, auto cur_c) {
        constexpr int cur = decltype(cur_c)::value;
        store_chunk(cur ^ 1, ra2[cur ^ 1], rb2[cur ^ 1]);
        load_chunk(kc + 3, ra2[cur ^ 1], rb2[cur ^ 1]);
        compute(cur);
        __syncthreads();
    };
    int kc = 0;
    for (; kc + 1 < nk; kc += 2) {
        iter(kc, std::integral_constant<int, 0>{});
        iter(kc + 1, std::integral_constant<int, 1>{});
    }
    if (kc < nk) iter(kc, std::integral_constant<int, 0>{});

    store_tile<T, TM, TN, WTM, WTN>(a, acc, m0 + wm * WTM, n0 + wn * WTN, lane, nullptr);
    if constexpr (!DYN) break;
    __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// MFMA implicit GEMM with direct-to-LDS loads (16-bit types, Cin % 32 == 0, no
// concat input).  The same GEMM as conv_igemm, but the K chunks (32 elements =
// 64 bytes per row) go from global memory straight into LDS with
// buffer_load_dwordx4 ... lds: no staging registers and no LDS stores, so S
// stages can be in flight at once (S - 1 chunks loading while one is computed).
//
// A stage holds BN weight rows then BM pixel rows, 64 bytes each.  One DMA
// instruction fills 16 rows (1 KB, lane L -> bytes 16 L): lane L carries row
// L / 4 of its group and 16-byte slot L % 4, into which it loads k-slot
// (L % 4) ^ sw(row).  A reader wanting k-slot c of row r reads slot
// c ^ sw(r & 15); with sw as below, the 16 rows of an MFMA operand read land on
// distinct banks for 32- and 64-bank LDS alike.  Weight rows and pixel rows
// share one offset formula: offset = base + (r * w + s) * Cin + ci for tap
// (r, s) and channel ci, where w is the image width for a pixel row and the
// kernel width for a weight row (so that (r * k + s) * Cin + ci = k index),
// and a zero halo / out-of-range row gets an out-of-range offset (zeros).
//
// Stage k % S holds chunk k.  S chunks are in flight while a chunk is computed:
// its MFMA operands are read from LDS into registers one step ahead (two
// register sets), so its stage is refilled as soon as every wave has read it.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void* lds_ptr_t;

// One 16-byte-per-lane DMA: lane L's dwordx4 at buffer offset voff lands in LDS
// at lds + 16 L (lds is wave-uniform, passed in M0).  Issued as inline assembly
// so that the compiler adds no waits of its own for it: the loop below waits
// explicitly, and a vmcnt the compiler computes for any other load stays
// correct (vector memory operations complete in order; extra ones in flight
// only make such a wait stronger).
__device__ __forceinline__ void dma16(__amdgpu_buffer_rsrc_t r, const void* lds, int voff) {
    const unsigned addr = (unsigned)(unsigned long)(lds_ptr_t)lds;
    asm volatile("s_mov_b32 m0, %0\n\tbuffer_load_dwordx4 %1, %2, 0 offen lds"
                 :
                 : "s"(addr), "v"(voff), "s"(r)
                 : "memory", "m0");
}


// 16-byte slot swizzle of the 64-byte LDS rows.  A wave's ds_read_b128 is served
// 32 lanes at a time and runs at full rate (256 B/clk per CU) only if those 32
// lanes -- 16 consecutive rows x 2 k-slots here -- touch distinct 16-byte units
// modulo 512 bytes.  Rows r and r + 8 share units modulo 512, so row bit 3 flips
// slot bit 1 (their slot pairs {0,1} and {2,3} become disjoint).  Measured on
// gfx950: the unswizzled layout and an XOR of row bits 1-3 into both slot bits
// both run at half rate.
__device__ __forceinline__ int dma_swizzle(int r) { return ((r >> 3) & 1) << 1; }
// For 128-byte rows (8 slots): slot bit 2 ^= row bit 1, slot bit 1 ^= row bit 2 --
// one of the linear XOR swizzles a lane-pattern probe found to keep the 16 rows x
// 4 slots of an MFMA operand read at full rate (unswizzled: quarter rate).
template <int RB>
__device__ __forceinline__ int lds_swizzle(int r) {
    if constexpr (RB == 64) return dma_swizzle(r);
    else return (((r >> 1) & 1) << 2) | (((r >> 2) & 1) << 1);
}

template <typename T, int BM, int BN, int WGM, int WGN, int S, bool NT, int BK, bool DYN = false, bool RL = false>
__global__ __launch_bounds__(64 * WGM * WGN) void conv_dma(ConvArgs a0) {
    constexpr int NW = WGM * WGN;                  // waves (4 or 8)
    constexpr int WTM = BM / WGM, WTN = BN / WGN;
    constexpr int TM = WTM / 16, TN = WTN / 16;
    constexpr int RB = BK * 2;                     // bytes per LDS row (one K chunk of a row)
    constexpr int KK = BK / 32;                    // MFMA k-steps per chunk
    constexpr int RPI = 1024 / RB;                 // rows per DMA instruction
    constexpr int ROWS = BM + BN, SB = ROWS * RB;  // bytes per stage
    constexpr int NPW = ROWS / (RPI * NW);         // DMA instructions per wave per chunk
    static_assert((NW == 4 || NW == 8) && TM >= 1 && TN >= 1 && (BK == 32 || BK == 64), "tile");
    static_assert(BM % (RPI * NW) == 0 && BN % (RPI * NW) == 0 && S >= 3 && S <= 4, "tile");
    typedef typename V16<T>::type V;

    __shared__ __attribute__((aligned(1024))) char st0[SB];
    __shared__ __attribute__((aligned(1024))) char st1[SB];
    __shared__ __attribute__((aligned(1024))) char st2[SB];
    __shared__ __attribute__((aligned(1024))) char st3[S > 3 ? SB : 16];

    // One tile per workgroup; DYN: as in conv_igemm, workgroups walk this batch's tiles.
    const DynBatch db = dyn_batch<DYN>(a0, BM, BN);
    for (int tl = blockIdx.x; tl < db.tiles; tl += gridDim.x) {
    const ConvArgs a = tile_args<DYN>(a0, db);
    const int W = db.tiles;
    const int tid = tile_tid<DYN, 64 * NW>();
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % WGM, wn = wave / WGM;
    int m0, n0;
    tile_origin_at(a, BM, BN, tl, W, m0, n0);
    const __amdgpu_buffer_rsrc_t r_in = __builtin_amdgcn_make_buffer_rsrc((void*)a.in, 0, a.in_bytes, kBufFlags);
    const __amdgpu_buffer_rsrc_t r_w = __builtin_amdgcn_make_buffer_rsrc((void*)a.w, 0, a.w_bytes, kBufFlags);
    // FPN concat (1x1 convs only): channels [0, cin1) from `in` at the next level
    // (nearest x2 upsample: pixel (y / 2, x / 2)), the rest from in2 at this level
    // (never in the residual form: no concat conv has a residual)
    const bool concat = !RL && a.cin1 > 0;
    const __amdgpu_buffer_rsrc_t r_in2 =
        concat ? __builtin_amdgcn_make_buffer_rsrc((void*)a.in2, 0, a.in2_bytes, kBufFlags) : r_in;

    // Row descriptors of this lane's DMA instructions (instruction i of this
    // wave fills rows RPI q .. RPI q + RPI - 1 of a stage, q = NW i + wave):
    //   d_off:  element offset of the row's origin (+ its k-slot);
    //   d_wc:   elements between kernel rows (image width x Cin for a pixel row,
    //           k x Cin for a weight row);
    //   d_mask: bit r * k + s set iff tap (r, s) lies inside the image (every tap of
    //           a weight row; none for a row past M or Cout).
    // With concat a pixel row's d_off addresses `in` and d_wc (unused by a 1x1)
    // the row's origin in in2.
    int d_off[NPW], d_wc[NPW], d_mask[NPW];
    const int rloc = lane / (RB / 16);
    // (rows of a 128-byte-row instruction start at multiples of 8: rloc carries
    // the row bits 1 and 2 the swizzle uses)
    const int kslot = ((lane % (RB / 16)) ^ lds_swizzle<RB>(rloc)) * 8;
    const int taps = a.ksz * a.ksz;
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
        const int q = NW * i + wave;
        const int row = RPI * q + rloc;
        d_off[i] = 0;
        d_wc[i] = 0;
        d_mask[i] = 0;
        if (RPI * NW * i < BN) {  // weight row: channel n0 + row (BN % (RPI NW) == 0: static per i)
            const int n = n0 + row;
            if (n < a.cout) {
                d_off[i] = n * a.K + kslot;
                d_wc[i] = a.ksz * a.cin;
                d_mask[i] = (1 << taps) - 1;
            }
        } else {  // pixel row: output pixel m0 + row - BN
            const int m = m0 + row - BN;
            if (m < a.M) {
                int f, y, x;
                map_pixel(a.geom, a.nframes, a.uniform, a.lvl_out, m, f, y, x);
                const int* g = a.geom + f * kGeomInts;
                const int iy0 = y * a.stride - a.pad, ix0 = x * a.stride - a.pad;
                const int h = g[0] >> a.lvl_in, w = g[1] >> a.lvl_in;
                d_off[i] = (g[2 + a.lvl_in] + iy0 * w + ix0) * a.cin + kslot;
                d_wc[i] = w * a.cin;
                if (concat) {
                    const int l1 = a.lvl_out + 1;
                    d_off[i] = (g[2 + l1] + (y >> 1) * (g[1] >> l1) + (x >> 1)) * a.cin1 + kslot;
                    d_wc[i] = (g[2 + a.lvl_out] + y * (g[1] >> a.lvl_out) + x) * (a.cin - a.cin1) + kslot;
                }
                int mk = 0;
                for (int r = 0; r < a.ksz; ++r)
                    for (int t = 0; t < a.ksz; ++t)
                        if ((unsigned)(iy0 + r) < (unsigned)h && (unsigned)(ix0 + t) < (unsigned)w)
                            mk |= 1 << (r * a.ksz + t);
                d_mask[i] = concat ? 1 : mk;  // concat: its one tap, every pixel of the level
            }
        }
    }

    // Tap (r, s) and channel ci of the next chunk to issue, advanced without
    // branches; chunks past the end read nothing (out-of-range offsets).
    int ld_ci = 0, ld_r = 0, ld_s = 0, issued = 0;
    const int nk = a.K / BK;
    auto issue = [&](auto u_c) {
        constexpr int u = decltype(u_c)::value;
        const int tap = issued < nk ? ld_r * a.ksz + ld_s : 31;  // bit 31 is never set
        const int sc = ld_s * a.cin + ld_ci;
        const bool first = !concat || ld_ci < a.cin1;  // concat: this chunk's source
#pragma unroll
        for (int i = 0; i < NPW; ++i) {
            const int q = NW * i + wave;
            const bool ok = (d_mask[i] >> tap) & 1;
            const bool wrow = RPI * NW * i < BN;  // weight row (static per i)
            const int e = (wrow || !concat) ? d_off[i] + ld_r * d_wc[i] + sc
                                            : (first ? d_off[i] + ld_ci : d_wc[i] + (ld_ci - a.cin1));
            const int off = ok ? e * (int)sizeof(T) : kOOB;
            const char* sp = u == 0 ? st0 : u == 1 ? st1 : u == 2 ? st2 : st3;
            dma16(wrow ? r_w : (first ? r_in : r_in2), sp + q * 1024, off);
        }
        ++issued;
        ld_ci += BK;
        const int wrap = ld_ci >= a.cin;
        ld_ci = wrap ? 0 : ld_ci;
        ld_s += wrap;
        const int wrap2 = ld_s >= a.ksz;
        ld_s = wrap2 ? 0 : ld_s;
        ld_r += wrap2;
    };

    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // lane-constant LDS read offsets (per k-step kk of a chunk): row lane % 16 of a
    // 16-row group, k-slot 4 kk + lane / 16
    int rd[KK];
#pragma unroll
    for (int kk = 0; kk < KK; ++kk)
        rd[kk] = (lane & 15) * RB + (((4 * kk + (lane >> 4)) ^ lds_swizzle<RB>(lane & 15)) << 4);
    const int a_rd = (wn * WTN) * RB, b_rd = (BN + wm * WTM) * RB;
    // MFMA operands of a chunk are read from LDS into one of two register sets
    // one step ahead, so that the LDS latency hides behind the previous chunk's MFMAs.
    V fa[2][KK][TN], fb[2][KK][TM];
    if constexpr (DYN) {
        // The second set is written only when a chunk follows; left undefined at the
        // first tile, the compiler carries it from tile to tile in registers that stay
        // live through every epilogue and prologue (an occupancy step on 128 x 128).
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) {
#pragma unroll
            for (int j = 0; j < TN; ++j) fa[1][kk][j] = V{};
#pragma unroll
            for (int i = 0; i < TM; ++i) fb[1][kk][i] = V{};
        }
    }
    auto read = [&](auto st_c, auto fr_c) {
        constexpr int st = decltype(st_c)::value, fr = decltype(fr_c)::value;
        const char* sp = st == 0 ? st0 : st == 1 ? st1 : st == 2 ? st2 : st3;
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) {
#pragma unroll
            for (int j = 0; j < TN; ++j) fa[fr][kk][j] = *(const V*)(sp + a_rd + rd[kk] + j * 16 * RB);
#pragma unroll
            for (int i = 0; i < TM; ++i) fb[fr][kk][i] = *(const V*)(sp + b_rd + rd[kk] + i * 16 * RB);
        }
    };
    auto mma = [&](auto fr_c) {
        constexpr int fr = decltype(fr_c)::value;
#pragma unroll
        for (int kk = 0; kk < KK; ++kk)
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    if constexpr (__is_same(T, bf16))
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[fr][kk][j], fb[fr][kk][i], acc[i][j],
                                                                            0, 0, 0);
                    else
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(fa[fr][kk][j], fb[fr][kk][i], acc[i][j],
                                                                           0, 0, 0);
                }
    };

    // Prologue: chunks 0 .. S-2 in flight; once chunk 0 has landed everywhere its
    // operands are read and chunk S-1 is issued into the last stage.
    issue(std::integral_constant<int, 0>{});
    issue(std::integral_constant<int, 1>{});
    if constexpr (S > 3) issue(std::integral_constant<int, 2>{});
    __builtin_amdgcn_s_waitcnt(waitcnt_imm((S - 2) * NPW, 0));
    __builtin_amdgcn_s_barrier();
    read(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{});
    issue(std::integral_constant<int, S - 1>{});
    // Step k (chunks k+1 .. k+S-1 in flight, chunk k's operands in registers):
    // wait until chunk k+1 has landed (at most (S-2) NPW younger DMAs of this wave
    // outstanding) and this wave's operand reads of chunk k are done; barrier (so
    // for every wave; chunk k's stage is then free); issue chunk k+S into it; read
    // chunk k+1's operands; run chunk k's MFMAs.
    // RL: the tile's residual (BM x BN of the storage type, two halves of BM / 2
    // pixels, each no larger than a stage) comes into LDS by DMA during the last
    // steps, in place of the loads of chunks past the end that those steps would
    // issue; a wave still issues NPW instructions per step (the half's
    // instructions, then out-of-range ones into the rest of the stage), so every
    // wait count stays as it is.  The epilogue then reads the residual from LDS
    // instead of waiting on TM x TN global loads per lane.  Step nk - S writes the
    // first half into chunk nk - S's stage, step nk - S + 1 the second into the
    // next one: both stages' operands are in registers by then.  The launcher
    // picks this form for convs with a residual only.
    constexpr int RROW = BN * 2;                      // bytes per pixel row of the residual
    constexpr int RIPR = 1024 / RROW;                  // pixel rows per 1-KB instruction
    constexpr int RINS = BM * BN / 1024 / NW;          // a wave's instructions per half
    static_assert(!RL || (sizeof(T) == 2 && (BN == 128 || BN == 256) && BM * BN <= SB &&
                          (BM * BN / 1024) % NW == 0 && RINS <= NPW), "residual in LDS");
    const bool res_lds = RL && a.res && !a.out0_f32 && nk >= S + 1;
    // det 1x1 in the epilogue: the activated tile (BM x BN of the storage type) over
    // the stages (not in the residual form: a det 3x3 has no residual)
    constexpr bool kFoldDet = !RL && sizeof(T) == 2 && fold_det_tile(BM, BN, BK, S, NW);
    int res_st0 = 0, res_st1 = 1;   // stage of each half
    auto res_issue = [&](auto st_c, auto h_c) {
        constexpr int st = decltype(st_c)::value, h = decltype(h_c)::value;
        const char* sp = st == 0 ? st0 : st == 1 ? st1 : st == 2 ? st2 : st3;
        const __amdgpu_buffer_rsrc_t r_res = __builtin_amdgcn_make_buffer_rsrc(
            (void*)a.res, 0, (int)((size_t)a.M * a.ld0 * sizeof(T) < 0x7fffffff ? (size_t)a.M * a.ld0 * sizeof(T)
                                                                                    : 0x7fffffff), kBufFlags);
#pragma unroll
        for (int i = 0; i < NPW; ++i) {
            const int q = NW * i + wave;                 // 1-KB instruction: pixel rows RIPR q .. of the half
            const int r = RIPR * q + lane / (RROW / 16), c = (lane % (RROW / 16)) ^ (r & 15);
            const int m = m0 + (BM / 2) * h + r, ch = n0 + 8 * c;
            const bool ok = i < RINS && m < a.M && ch < a.n_split;
            dma16(r_res, sp + q * 1024, ok ? (int)(((size_t)m * a.ld0 + ch) * sizeof(T)) : kOOB);
        }
        if constexpr (h == 0) res_st0 = st; else res_st1 = st;
    };
    auto step = [&](auto u_c, int k) {
        constexpr int u = decltype(u_c)::value;
        __builtin_amdgcn_s_waitcnt(waitcnt_imm((S - 2) * NPW, 0));
        __builtin_amdgcn_s_barrier();
        if (res_lds && k == nk - S)
            res_issue(std::integral_constant<int, u % S>{}, std::integral_constant<int, 0>{});
        else if (res_lds && k == nk - S + 1)
            res_issue(std::integral_constant<int, u % S>{}, std::integral_constant<int, 1>{});
        else
            issue(std::integral_constant<int, u % S>{});
        if (k + 1 < nk) read(std::integral_constant<int, (u + 1) % S>{}, std::integral_constant<int, (u + 1) & 1>{});
        mma(std::integral_constant<int, u & 1>{});
    };
    constexpr int L = S == 3 ? 6 : 4;  // steps per loop trip: stage and register set repeat
    for (int kc = 0;; kc += L) {
        step(std::integral_constant<int, 0>{}, kc);
        if (kc + 1 >= nk) break;
        step(std::integral_constant<int, 1>{}, kc + 1);
        if (kc + 2 >= nk) break;
        step(std::integral_constant<int, 2>{}, kc + 2);
        if (kc + 3 >= nk) break;
        step(std::integral_constant<int, 3>{}, kc + 3);
        if constexpr (L > 4) {
            if (kc + 4 >= nk) break;
            step(std::integral_constant<int, 4>{}, kc + 4);
            if (kc + 5 >= nk) break;
            step(std::integral_constant<int, 5>{}, kc + 5);
        }
        if (kc + L >= nk) break;
    }
    // no DMA may still be writing LDS when the workgroup ends (or starts its next tile)
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 15));

    if (res_lds) {
        __syncthreads();   // every wave's share of the residual has landed
        auto stp = [&](int st) -> const char* { return st == 0 ? st0 : st == 1 ? st1 : st == 2 ? st2 : st3; };
        const ResLds rl{stp(res_st0), stp(res_st1), m0, n0, BM / 2, RROW};
        store_tile<T, TM, TN, WTM, WTN, NT>(a, acc, m0 + wm * WTM, n0 + wn * WTN, lane, nullptr, &rl);
    } else if (kFoldDet && a.det_w && n0 < a.n_split) {
        if constexpr (kFoldDet) {
            // the arguments read afresh here, so that the walking form holds none of the
            // fold's through the K loop
            const ConvArgs af = tile_args<DYN>(a0, db);
            det_fold<T, BM, BN, NW, TM, TN, WTM, WTN, BK, S>(af, acc, m0, n0, wm, wn, wave, lane, tid, st0, st1,
                                                              st2, st3);
        }
    } else {
        store_tile<T, TM, TN, WTM, WTN, NT>(a, acc, m0 + wm * WTM, n0 + wn * WTN, lane, nullptr);
    }
    if constexpr (!DYN) break;
    // every wave is done reading this tile's stages before the next tile's DMAs refill them
    __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// 3x3 stride-1 convolution from an LDS window (16-bit storage; Cin % 64 == 0,
// Cout % 128 == 0, no concat input, level width <= 190).
//
// The implicit GEMM above gathers every input pixel once per tap: nine loads of
// each activation per K slice, which keeps a compute unit's texture-address path
// ~80 % busy on the deep 3x3 layers (hardware counters) -- the load path, not the
// matrix cores, bounds them.  Here a workgroup owns a tile of whole output rows
// of one frame (TY rows x W, at most 272 pixels) and 128 output channels.  Per
// 32-channel input slice it loads the (TY + 2) x (W + 2) window once into LDS
// and runs all nine taps from it, the pixel operand of tap (r, s) being the
// window shifted by (r - 1, s - 1); only the 128 x 32 weight slice is loaded per
// tap.  K order: slice-major, tap-minor (a different FP32 summation order from
// the implicit GEMM's tap-major order).
//
// Pipeline (8 waves: 2 pixel halves x 4 groups of 32 channels; one workgroup
// per compute unit): weight slices of steps k + 1 .. k + 3 are in flight in four
// LDS stages while step k computes, the next slice's window streams into the
// second window buffer over the first seven taps, and a step's MFMA operands are
// read from LDS one step ahead into the other register set.  Every wave issues
// the same DMAs in the same order at every step (past the end: out-of-range
// offsets, which load zeros into free buffers), so the wait before each step's
// barrier is a static vmcnt per tap position.  The epilogue is store_tile's
// (bias, leaky, residual, split FP32 output) with the tile's pixel range as M.
// ---------------------------------------------------------------------------
constexpr int kW3Px = 272;   // output pixels per tile at most (17 blocks of 16)
constexpr int kW3Win = 576;  // window pixels at most

// Tile height for a level of width w (1 <= w <= kW3MaxW).
__host__ __device__ inline int w3_rows(int w) {
    const int a = kW3Px / w, b = kW3Win / (w + 2) - 2;
    return a < b ? a : b;
}

template <typename T, bool NT>
__global__ __launch_bounds__(512) void conv3_win(ConvArgs a, int ntc, int total) {
    constexpr int NW = 8, BN = 128, TM = 9, TN = 2, PS = 96;       // PS: LDS bytes per window pixel
    constexpr int NWD = (kW3Win * (PS / 16) + 64 * NW - 1) / (64 * NW);  // window DMAs per wave per slice
    constexpr int WB = NWD * NW * 1024, WS = BN * 64;              // window buffer, weight stage bytes
    static_assert(NWD <= 7, "window DMAs must finish by tap 6");
    typedef typename V16<T>::type V;

    __shared__ __attribute__((aligned(1024))) char win[2][WB];
    __shared__ __attribute__((aligned(1024))) char wst[4][WS];

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave & 1, wn = wave >> 1;
    const int p = lane & 15, kg = lane >> 4;

    // tile: pixel tile pt (channel tiles innermost, XCD-aware), frame f, rows y0..
    const int Lt = xcd_remap(blockIdx.x, total);
    int pt = Lt / ntc;
    const int n0 = (Lt - pt * ntc) * BN;
    int f = 0, H = 0, W = 1, TY = 1;
    for (;;) {
        H = a.geom[f * kGeomInts] >> a.lvl_out;
        W = a.geom[f * kGeomInts + 1] >> a.lvl_out;
        TY = w3_rows(W);
        const int n = (H + TY - 1) / TY;
        if (pt < n || f + 1 >= a.nframes) break;
        pt -= n;
        ++f;
    }
    const int y0 = pt * TY, rows = H - y0 < TY ? H - y0 : TY, P = rows * W;
    const int fbase = a.geom[f * kGeomInts + 2 + a.lvl_out];
    const int mt0 = fbase + y0 * W;
    const int WX = W + 2, npx = (rows + 2) * WX;
    const int nc = a.cin / 32, nk = 9 * nc;

    const __amdgpu_buffer_rsrc_t r_in = __builtin_amdgcn_make_buffer_rsrc((void*)a.in, 0, a.in_bytes, kBufFlags);
    const __amdgpu_buffer_rsrc_t r_w = __builtin_amdgcn_make_buffer_rsrc((void*)a.w, 0, a.w_bytes, kBufFlags);

    // window DMA i of this wave: lane -> (window pixel, 16-byte unit); element
    // offset of the slice-0 data, or -1 (padding unit, outside the window/frame)
    int dgeo[NWD];
#pragma unroll
    for (int i = 0; i < NWD; ++i) {
        const int L = (wave + NW * i) * 64 + lane;
        const int px = L / (PS / 16), u = L - px * (PS / 16);
        const int wy = px / WX, wx = px - wy * WX;
        const int iy = y0 - 1 + wy, ix = wx - 1;
        const bool ok = u < 4 && px < npx && (unsigned)iy < (unsigned)H && (unsigned)ix < (unsigned)W;
        dgeo[i] = ok ? ((fbase + iy * W + ix) * a.cin + u * 8) : -1;
    }
    auto win_dma = [&](int c, int i) {  // slice c into window buffer c & 1
        const int off = (dgeo[i] >= 0 && c < nc) ? (dgeo[i] + c * 32) * (int)sizeof(T) : kOOB;
        dma16(r_in, &win[c & 1][(wave + NW * i) * 1024], off);
    };
    // weight DMA of step k (slice k / 9, tap k % 9): rows n0 + 16 wave .., 64 bytes each
    const int wrow = n0 + 16 * wave + (lane >> 2);
    const int wslot = ((lane & 3) ^ dma_swizzle(lane >> 2)) * 8;
    auto w_dma = [&](int k) {
        const int c = k / 9, t = k - 9 * c;
        const int off = k < nk ? (wrow * a.K + t * a.cin + c * 32 + wslot) * (int)sizeof(T) : kOOB;
        dma16(r_w, &wst[k & 3][wave * 1024], off);
    };

    // B operand bases: window centre of this lane's pixel in block i (+ its k-slot)
    int cb[TM];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int q = (wm * TM + i) * 16 + p;
        int ctr = WX + 1;  // past the tile: any window pixel (not stored)
        if (q < P) {
            const int ty = q / W, tx = q - ty * W;
            ctr = (ty + 1) * WX + tx + 1;
        }
        cb[i] = ctr * PS + kg * 16;
    }
    const int a_rd = (wn * 32 + p) * 64 + ((kg ^ dma_swizzle(p)) << 4);

    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    V fa[2][TN], fb[2][TM];
    auto read = [&](int k, int set) {
        const int c = k / 9, t = k - 9 * c;
        const char* ws = wst[k & 3];
#pragma unroll
        for (int j = 0; j < TN; ++j) fa[set][j] = *(const V*)(ws + a_rd + j * 16 * 64);
        const int toff = ((t / 3 - 1) * WX + (t % 3 - 1)) * PS;
        const char* wb = win[c & 1] + toff;
#pragma unroll
        for (int i = 0; i < TM; ++i) fb[set][i] = *(const V*)(wb + cb[i]);
    };
    auto mma = [&](int set) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                if constexpr (__is_same(T, bf16))
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[set][j], fb[set][i], acc[i][j], 0, 0, 0);
                else
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(fa[set][j], fb[set][i], acc[i][j], 0, 0, 0);
            }
    };

    // prologue: slice 0's window and the weights of steps 0..2
#pragma unroll
    for (int i = 0; i < NWD; ++i) win_dma(0, i);
    w_dma(0);
    w_dma(1);
    w_dma(2);
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 15));
    __syncthreads();
    read(0, 0);
    // Step k = 9 c + t.  Issue order per step: weights of k + 3, then (t < NWD)
    // window DMA t of slice c + 1.  Before the barrier of step k the weights of
    // k + 1 must have landed (issued at step k - 2) and, at t = 8, slice c + 1's
    // whole window: the ops issued after those are what vmcnt may leave.
    auto step = [&](auto u_c, int k) {
        constexpr int u = decltype(u_c)::value, t = u % 9;
        constexpr int wprev2 = ((t + 7) % 9) < NWD, wprev1 = ((t + 8) % 9) < NWD;
        constexpr int vm = t == 8 ? 1 : wprev2 + 1 + wprev1;
        __builtin_amdgcn_s_waitcnt(waitcnt_imm(vm, 0));
        __builtin_amdgcn_s_barrier();
        w_dma(k + 3);
        if constexpr (t < NWD) win_dma(k / 9 + 1, t);
        if (k + 1 < nk) read(k + 1, (u + 1) & 1);
        mma(u & 1);
        __builtin_amdgcn_sched_barrier(0);  // keeps the register sets bounded
    };
    for (int kc = 0; kc < nk; kc += 18) {
        static_for<0, 18>([&](auto u_c) { step(u_c, kc + decltype(u_c)::value); });
    }
    // no DMA may still be writing LDS when the workgroup ends
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 15));

    ConvArgs at = a;
    at.M = mt0 + P;  // the tile's pixels end here (rows past the frame are not computed)
    store_tile<T, TM, TN, TM * 16, TN * 16, NT>(at, acc, mt0 + wm * TM * 16, n0 + wn * 32, lane, nullptr);
}

// Tiles of one frame level (h x w) for conv3_win, 0 if the width does not fit.
int conv3w_tiles(int h, int w) {
    if (w < 1 || w > kW3MaxW || h < 1) return 0;
    const int ty = w3_rows(w);
    return (h + ty - 1) / ty;
}

bool conv3w_ok(const ConvArgs& a, int et) {
    return (et == kBF16 || et == kF16) && a.ksz == 3 && a.stride == 1 && a.pad == 1 && a.cin % 64 == 0 &&
           a.cout % 128 == 0 && a.cin1 == 0 && a.lvl_in == a.lvl_out && !a.wscale;
}

// Output columns at or past n_split go to out1: refuse a launch that would write
// them through a null pointer (and outputs that are missing altogether).
static bool conv_outputs_ok(const ConvArgs& a) {
    return a.out0 && (a.n_split >= a.cout || a.out1);
}

hipError_t launch_conv3w(const ConvArgs& a, int et, int pixel_tiles, hipStream_t s) {
    if (!conv_outputs_ok(a) || !conv3w_ok(a, et) || pixel_tiles <= 0) return hipErrorInvalidValue;
    const int ntc = a.cout / 128, total = pixel_tiles * ntc;
    dim3 grid(total), block(512);
    if (et == kBF16)
        conv3_win<bf16, false><<<grid, block, 0, s>>>(a, ntc, total);
    else
        conv3_win<f16, false><<<grid, block, 0, s>>>(a, ntc, total);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP8 (OCP e4m3) implicit GEMM for the deep backbone convolutions.
//   K chunks of 128 = one v_mfma_scale_f32_16x16x128_f8f6f4 per 16x16 output
//   block; each lane feeds 32 k of its row (two 16-byte LDS reads per operand,
//   placed so that every 32 consecutive k of the chunk fall in the block whose
//   E8M0 exponent one lane group passes; the matrix core applies it to the
//   products).
//   Weights are e4m3 in HBM with a per-output-channel FP32 scale (max |w_c| / 448)
//   and, within it, an E8M0 exponent per 32-k block ([Cout][K/32] bytes), staged
//   through LDS beside the chunk.  Activations stay BF16 in HBM: the B loader
//   fetches 8 channels (16 bytes) per buffer load and, when staging to LDS,
//   converts them to e4m3.  BLK (the default): the four lanes that hold a
//   pixel's 32 channels of the chunk take their max |x| (a DPP exchange within
//   the quad), set the block's exponent to the smallest s with max |x| / 2^s
//   <= 448 and store x / 2^s (exact) rounded to e4m3; the exponent goes to LDS
//   beside the pixel row.  !BLK: a static per-tensor scale from calibration,
//   round(clamp(x / in_scale, +-448)), and unit activation exponents.  The
//   epilogue multiplies the FP32 accumulator by wscale[co] * in_scale (in_scale
//   is 1 with block scales).  Requires Cin % 128 == 0 (every chunk lies within
//   one tap) and no concat input.
// ---------------------------------------------------------------------------
// Element formats of the block-scaled MFMA operands (the instruction's format code):
// 0 = e4m3 (8 bits), 2 = FP6 E2M3 (6 bits), 4 = FP4 E2M1 (4 bits).
template <int FMT> struct MxFmt;
template <> struct MxFmt<0> { static constexpr int bits = 8, mant = 3, emin = -6, top_e = 8; static constexpr unsigned top_m = 0x600000; };
template <> struct MxFmt<2> { static constexpr int bits = 6, mant = 3, emin = 0, top_e = 2; static constexpr unsigned top_m = 0x700000; };
template <> struct MxFmt<4> { static constexpr int bits = 4, mant = 1, emin = 0, top_e = 2; static constexpr unsigned top_m = 0x400000; };

// E8M0 exponent byte (127 + s) of the smallest power of two 2^s with m / 2^s <= top,
// the format's largest value f_t * 2^top_e (e4m3: 1.75 * 2^8, E2M3: 1.875 * 2^2,
// E2M1: 1.5 * 2^2), for m = max |x| >= 0 of a block: with m = f * 2^E, f in [1, 2),
// s = E - top_e when f <= f_t, else E - top_e + 1.  127 (s = 0) for m = 0.
template <int FMT>
__device__ __forceinline__ int e8m0_for_amax(float m) {
    const unsigned b = __float_as_uint(m);
    if (m == 0.f) return 127;
    const int eb = (int)(b >> 23) & 0xff;   // biased exponent (m is finite and >= 0)
    const unsigned mant = b & 0x7fffff;
    const int e = eb - MxFmt<FMT>::top_e + (mant > MxFmt<FMT>::top_m ? 1 : 0);
    return e < 0 ? 0 : (e > 254 ? 254 : e);
}

// Code of the FP6 E2M3 / FP4 E2M1 value nearest x (ties to even), x already within
// the format's range: in binade e >= emin the spacing is 2^(e - M), below 2^emin it
// stays 2^(emin - M); n = rint(|x| / spacing) is the significand in units of the
// spacing (2^M <= n <= 2^(M+1) for a normal result, n < 2^M for a subnormal one).
template <int FMT>
__device__ __forceinline__ unsigned mx_code(float x) {
    constexpr int M = MxFmt<FMT>::mant, EMIN = MxFmt<FMT>::emin, BITS = MxFmt<FMT>::bits;
    const unsigned sign = __float_as_uint(x) >> 31;
    const float a = fabsf(x);
    int e = (int)((__float_as_uint(a) >> 23) & 0xff) - 127;
    e = e < EMIN ? EMIN : e;
    const int n = (int)rintf(__builtin_amdgcn_ldexpf(a, M - e));
    unsigned code;
    if (n < (1 << M)) {                      // subnormal (e == EMIN) or zero
        code = (unsigned)n;
    } else {
        const int up = n >> (M + 1);          // rounded up into the next binade
        const unsigned mm = up ? 0u : (unsigned)(n - (1 << M));
        code = ((unsigned)(e + up - EMIN + 1) << M) | mm;
    }
    return code | (sign << (BITS - 1));
}

template <int BM, int BN, int WGM, int WGN, bool BLK, int FMT = 0>
__global__ __launch_bounds__(256) void conv_igemm_f8(ConvArgs a) {
    constexpr int BK = 128;                  // elements per chunk (one MFMA's K)
    constexpr int EB = MxFmt<FMT>::bits;     // bits per element
    constexpr int RB = BK * EB / 8;          // bytes of a row's chunk: 128 / 96 / 64
    constexpr int LDR = RB + 16;             // padded LDS row, bytes
    constexpr int WTM = BM / WGM, WTN = BN / WGN;
    constexpr int TM = WTM / 16, TN = WTN / 16;
    constexpr int VRB = BK / 8;              // 16-byte BF16 loads per pixel row and chunk
    constexpr int VRA = RB / 16;             // 16-byte loads per weight row and chunk
    constexpr float TOP = FMT == 0 ? 448.f : (FMT == 2 ? 7.5f : 6.f);   // largest element value
    static_assert(FMT == 0 || BLK, "FP6 / FP4 operands take block scales");
    constexpr int BVEC = BM * VRB, AVEC = BN * VRA;
    constexpr int BPT = (BVEC + 255) / 256, APT = (AVEC + 255) / 256;
    static_assert(WGM * WGN == 4 && TM >= 1 && TN >= 1, "tile");
    typedef int i32x4 __attribute__((ext_vector_type(4)));
    typedef int i32x2 __attribute__((ext_vector_type(2)));

    __shared__ __attribute__((aligned(16))) unsigned char sA[2][BN * LDR];
    __shared__ __attribute__((aligned(16))) unsigned char sB[2][BM * LDR];
    // E8M0 exponents of the chunk: 4 bytes (the chunk's four 32-k blocks) per row
    __shared__ __attribute__((aligned(16))) unsigned sAs[2][BN];
    __shared__ __attribute__((aligned(16))) unsigned sBs[2][BLK ? BM : 1];
    static_assert(BN <= 256, "one weight-scale dword per thread");

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WGM, wn = wave / WGM;
    int m0, n0;
    {
        const int gm = (a.M + BM - 1) / BM, gn = (a.cout + BN - 1) / BN;
        const int W = gm * gn, L = blockIdx.x;
        const int xcd = L % kXCDs, local = L / kXCDs;
        const int base = W / kXCDs, extra = W % kXCDs;
        const int P = xcd < extra ? xcd * (base + 1) + local : extra * (base + 1) + (xcd - extra) * base + local;
        if (a.n_major) {
            m0 = (P % gm) * BM;
            n0 = (P / gm) * BN;
        } else {
            n0 = (P % gn) * BN;
            m0 = (P / gn) * BM;
        }
    }
    const __amdgpu_buffer_rsrc_t r_in = __builtin_amdgcn_make_buffer_rsrc((void*)a.in, 0, a.in_bytes, kBufFlags);
    const __amdgpu_buffer_rsrc_t r_w = __builtin_amdgcn_make_buffer_rsrc((void*)a.w, 0, a.w_bytes, kBufFlags);
    const int kb_row = a.K / 32;   // weight-scale bytes per output channel
    const __amdgpu_buffer_rsrc_t r_ws =
        __builtin_amdgcn_make_buffer_rsrc((void*)a.wbscale, 0, a.cout * kb_row, kBufFlags);
    const float inv_scale = 1.0f / a.in_scale;
    // this thread's weight-scale row (thread t < BN stages row n0 + t's 4 bytes per chunk)
    const int ws_off = (tid < BN && n0 + tid < a.cout) ? (n0 + tid) * kb_row : -1;

    int b_off[BPT], b_yx[BPT], b_hw[BPT];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int v = tid + i * 256;
        const int row = v / VRB, kv = v % VRB;
        const int m = m0 + row;
        b_off[i] = 0;
        b_yx[i] = 0;
        b_hw[i] = 0;
        if (v < BVEC && m < a.M) {
            int f, y, x;
            map_pixel(a.geom, a.nframes, a.uniform, a.lvl_out, m, f, y, x);
            const int* g = a.geom + f * kGeomInts;
            const int iy0 = y * a.stride - a.pad, ix0 = x * a.stride - a.pad;
            const int h = g[0] >> a.lvl_in, w = g[1] >> a.lvl_in;
            b_off[i] = (g[2 + a.lvl_in] + iy0 * w + ix0) * a.cin + kv * 8;
            b_yx[i] = (iy0 << 16) | (ix0 & 0xffff);
            b_hw[i] = (h << 16) | w;
        }
    }
    int a_off[APT];   // byte offsets into the packed weight rows (K EB / 8 bytes per row)
#pragma unroll
    for (int i = 0; i < APT; ++i) {
        const int v = tid + i * 256;
        const int row = v / VRA, kv = v % VRA;
        a_off[i] = (v < AVEC && n0 + row < a.cout) ? (n0 + row) * (a.K / 8 * EB) + kv * 16 : -1;
    }

    int ld_ci = 0, ld_r = 0, ld_s = 0;
    i32x4 ra2[2][APT], rb2[2][BPT];
    unsigned rs2[2];
    auto load_chunk = [&](int kc, i32x4 (&ra)[APT], i32x4 (&rb)[BPT], unsigned& rs) __attribute__((always_inline)) {
        const int k0 = kc * RB;
#pragma unroll
        for (int i = 0; i < APT; ++i)
            ra[i] = __builtin_amdgcn_raw_buffer_load_b128(r_w, a_off[i] >= 0 ? a_off[i] + k0 : kOOB, 0, 0);
        rs = (unsigned)__builtin_amdgcn_raw_buffer_load_b32(r_ws, ws_off >= 0 ? ws_off + kc * 4 : kOOB, 0, 0);
#pragma unroll
        for (int i = 0; i < BPT; ++i) {
            const int iy = (b_yx[i] >> 16) + ld_r, ix = (int)(short)(b_yx[i] & 0xffff) + ld_s;
            const int h = b_hw[i] >> 16, w = b_hw[i] & 0xffff;
            const bool ok = (unsigned)iy < (unsigned)h && (unsigned)ix < (unsigned)w;
            const int off = ok ? (b_off[i] + (ld_r * w + ld_s) * a.cin + ld_ci) * 2 : kOOB;
            rb[i] = __builtin_amdgcn_raw_buffer_load_b128(r_in, off, 0, 0);
        }
        ld_ci += BK;
        const int wrap = ld_ci >= a.cin;
        ld_ci = wrap ? 0 : ld_ci;
        ld_s += wrap;
        const int wrap2 = ld_s >= a.ksz;
        ld_s = wrap2 ? 0 : ld_s;
        ld_r += wrap2;
    };
    // 8 BF16 values -> 8 elements (e4m3: two dwords; E2M3: 48 bits, low dword then
    // the high 16 bits; E2M1: one dword), scaled and saturated; element q of the 8
    // sits at bits EB q.  BLK: every lane of the quad that holds one pixel's
    // 32-channel block computes the block's exponent (returned in *e8) and scales by
    // it exactly.
    auto to_fp8 = [&](i32x4 v, int* e8) __attribute__((always_inline)) {
        float f[8];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            f[2 * q] = __uint_as_float(((unsigned)v[q]) << 16);
            f[2 * q + 1] = __uint_as_float(((unsigned)v[q]) & 0xffff0000u);
        }
        if constexpr (BLK) {
            float m = 0.f;
#pragma unroll
            for (int q = 0; q < 8; ++q) m = fmaxf(m, fabsf(f[q]));
            // max over the quad (lanes 4j .. 4j+3 of the wave hold one block)
            m = fmaxf(m, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(m), 0xB1, 0xF, 0xF, true)));
            m = fmaxf(m, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(m), 0x4E, 0xF, 0xF, true)));
            const int e = e8m0_for_amax<FMT>(m);
            *e8 = e;
#pragma unroll
            for (int q = 0; q < 8; ++q) f[q] = fminf(fmaxf(__builtin_amdgcn_ldexpf(f[q], 127 - e), -TOP), TOP);
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) f[q] = fminf(fmaxf(f[q] * inv_scale, -TOP), TOP);
        }
        if constexpr (FMT == 0) {
            int lo = 0, hi = 0;
            lo = __builtin_amdgcn_cvt_pk_fp8_f32(f[0], f[1], lo, false);
            lo = __builtin_amdgcn_cvt_pk_fp8_f32(f[2], f[3], lo, true);
            hi = __builtin_amdgcn_cvt_pk_fp8_f32(f[4], f[5], hi, false);
            hi = __builtin_amdgcn_cvt_pk_fp8_f32(f[6], f[7], hi, true);
            return i32x2{lo, hi};
        } else {
            unsigned long long bits = 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) bits |= (unsigned long long)mx_code<FMT>(f[q]) << (EB * q);
            return i32x2{(int)(unsigned)bits, (int)(unsigned)(bits >> 32)};
        }
    };
    static_assert(BVEC % 256 == 0, "every lane converts: the quad exchange needs all four lanes");
    auto store_chunk = [&](int buf, const i32x4 (&ra)[APT], const i32x4 (&rb)[BPT], unsigned rs) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < APT; ++i) {
            const int v = tid + i * 256;
            if (AVEC % 256 == 0 || v < AVEC) *(i32x4*)(&sA[buf][(v / VRA) * LDR + (v % VRA) * 16]) = ra[i];
        }
        if (tid < BN) sAs[buf][tid] = rs;
#pragma unroll
        for (int i = 0; i < BPT; ++i) {
            const int v = tid + i * 256;
            int e8 = 127;
            const i32x2 q = to_fp8(rb[i], &e8);
            unsigned char* dst = &sB[buf][(v / VRB) * LDR + (v % VRB) * EB];
            if constexpr (FMT == 0) {
                *(i32x2*)dst = q;
            } else if constexpr (FMT == 4) {
                *(int*)dst = q[0];
            } else {  // 6 bytes at a 2-byte-aligned offset
                ((unsigned short*)dst)[0] = (unsigned short)((unsigned)q[0] & 0xffff);
                ((unsigned short*)dst)[1] = (unsigned short)((unsigned)q[0] >> 16);
                ((unsigned short*)dst)[2] = (unsigned short)((unsigned)q[1] & 0xffff);
            }
            if constexpr (BLK) {
                // lane 4j of the quad writes the block's exponent: row v / VRB, block (v % VRB) / 4
                if ((v & 3) == 0) ((unsigned char*)sBs[buf])[(v / VRB) * 4 + (v % VRB) / 4] = (unsigned char)e8;
            }
        }
    };

    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int arow = wn * WTN + (lane & 15), brow = wm * WTM + (lane & 15);
    // e4m3: the matrix core takes a lane's 32 bytes as two 16-value halves: lane
    // group g (lane / 16) supplies k = 16 g .. 16 g + 15 in bytes 0-15 and k = 64 +
    // 16 g .. in bytes 16-31, and the block scale of lane group b covers k = 32 b ..
    // 32 b + 31 (groups 2 (b % 2) and 2 (b % 2) + 1, half b / 2).  Reading the
    // chunk's bytes 16 g and 64 + 16 g puts chunk k = 32 b .. 32 b + 31 -- one weight
    // or activation scale block -- exactly where lane group b's scale applies.
    // FP6 / FP4: lane group g's 32 packed values (24 / 16 bytes) are all of block g,
    // so it reads the chunk's values 32 g .. 32 g + 31 as they lie.
    const int kofs = (lane >> 4) * (FMT == 0 ? 16 : 32 * EB / 8);
    const int kblk = lane >> 4;   // the 32-k block this lane feeds
    auto operand = [&](const unsigned char* p) __attribute__((always_inline)) -> i32x8 {
        if constexpr (FMT == 0) {
            const i32x4 x0 = *(const i32x4*)p, x1 = *(const i32x4*)(p + 64);
            return i32x8{x0[0], x0[1], x0[2], x0[3], x1[0], x1[1], x1[2], x1[3]};
        } else if constexpr (FMT == 4) {
            const i32x4 x0 = *(const i32x4*)p;
            return i32x8{x0[0], x0[1], x0[2], x0[3], 0, 0, 0, 0};
        } else {  // 24 bytes at an 8-byte-aligned offset
            const i32x2 x0 = *(const i32x2*)p, x1 = *(const i32x2*)(p + 8), x2 = *(const i32x2*)(p + 16);
            return i32x8{x0[0], x0[1], x1[0], x1[1], x2[0], x2[1], 0, 0};
        }
    };
    auto compute = [&](int buf) __attribute__((always_inline)) {
        const unsigned char* A = sA[buf];
        const unsigned char* B = sB[buf];
        i32x8 af[TN], bfr[TM];
        int sa[TN], sb[TM];
#pragma unroll
        for (int j = 0; j < TN; ++j) sa[j] = ((const unsigned char*)sAs[buf])[(arow + j * 16) * 4 + kblk];
#pragma unroll
        for (int i = 0; i < TM; ++i)
            sb[i] = BLK ? ((const unsigned char*)sBs[buf])[(brow + i * 16) * 4 + kblk] : 127;
#pragma unroll
        for (int j = 0; j < TN; ++j) af[j] = operand(A + (arow + j * 16) * LDR + kofs);
#pragma unroll
        for (int i = 0; i < TM; ++i) bfr[i] = operand(B + (brow + i * 16) * LDR + kofs);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(af[j], bfr[i], acc[i][j], FMT, FMT,
                                                                             0, sa[j], 0, sb[i]);
    };

    const int nk = a.K / BK;
    load_chunk(0, ra2[0], rb2[0], rs2[0]);
    load_chunk(1, ra2[1], rb2[1], rs2[1]);
    store_chunk(0, ra2[0], rb2[0], rs2[0]);
    load_chunk(2, ra2[0], rb2[0], rs2[0]);
    __syncthreads();
    auto iter = [&](int kc, auto cur_c) __attribute__((always_inline)) {
        constexpr int cur = decltype(cur_c)::value;
        store_chunk(cur ^ 1, ra2[cur ^ 1], rb2[cur ^ 1], rs2[cur ^ 1]);
        load_chunk(kc + 3, ra2[cur ^ 1], rb2[cur ^ 1], rs2[cur ^ 1]);
        compute(cur);
        __syncthreads();
    };
    int kc = 0;
    for (; kc + 1 < nk; kc += 2) {
        iter(kc, std::integral_constant<int, 0>{});
        iter(kc + 1, std::integral_constant<int, 1>{});
    }
    if (kc < nk) iter(kc, std::integral_constant<int, 0>{});
    store_tile<bf16, TM, TN, WTM, WTN>(a, acc, m0 + wm * WTM, n0 + wn * WTN, lane, a.wscale);
}

struct TileCfg8 { int bm, bn, wgm, wgn; };
static constexpr TileCfg8 kTiles8[] = {
    {128, 128, 2, 2},
    {128, 64, 2, 2},
    {64, 128, 2, 2},
    {64, 64, 2, 2},
};
int conv_fp8_num_tiles() { return sizeof(kTiles8) / sizeof(kTiles8[0]); }
bool conv_fp8_ok(const ConvArgs& a) { return a.cin % 128 == 0 && a.cin1 == 0 && a.K % 128 == 0; }

template <int C>
static hipError_t launch_f8(const ConvArgs& a, hipStream_t s) {
    constexpr TileCfg8 t = kTiles8[C];
    dim3 grid(((a.M + t.bm - 1) / t.bm) * ((a.cout + t.bn - 1) / t.bn));
    if (a.mx_fmt == 4 && a.act_blocks)
        conv_igemm_f8<t.bm, t.bn, t.wgm, t.wgn, true, 4><<<grid, 256, 0, s>>>(a);
    else if (a.mx_fmt == 2 && a.act_blocks)
        conv_igemm_f8<t.bm, t.bn, t.wgm, t.wgn, true, 2><<<grid, 256, 0, s>>>(a);
    else if (a.mx_fmt != 0)
        return hipErrorInvalidValue;   // FP6 / FP4 activations take block scales
    else if (a.act_blocks)
        conv_igemm_f8<t.bm, t.bn, t.wgm, t.wgn, true><<<grid, 256, 0, s>>>(a);
    else
        conv_igemm_f8<t.bm, t.bn, t.wgm, t.wgn, false><<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_conv_fp8(const ConvArgs& a, int c, hipStream_t s) {
    if (!conv_outputs_ok(a) || !conv_fp8_ok(a) || !a.wscale || !a.wbscale || !(a.in_scale > 0.f))
        return hipErrorInvalidValue;
    switch (c) {
        case 0: return launch_f8<0>(a, s);
        case 1: return launch_f8<1>(a, s);
        case 2: return launch_f8<2>(a, s);
        case 3: return launch_f8<3>(a, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Residual block fused into one launch (16-bit storage, C = 64 or 128):
//   out = leaky(b2 + W2 (*) y) + x,   y = leaky(b1 + W1 x)  (1x1 C -> C/2, then
// 3x3 C/2 -> C; Sec. 3.1's Darknet-53 blocks).  The C/2-channel intermediate y
// never goes to HBM, and x is read once (as the 1x1's input and as the
// residual).  Work items are TY x TX tiles of output pixels (all C channels),
// walked by persistent workgroups (8 waves, one per compute unit); the items
// are split into 8 contiguous bands, one per XCD, so that tiles whose windows
// overlap are fetched into the same L2.  Per tile:
//   * the (TY + 2) x (TX + 2)-pixel window of x (zero outside the frame) is in
//     LDS, brought in by direct-to-LDS loads while the previous tile computes
//     (two window buffers);
//   * y over the whole window, on MFMA (A = W1 rows, B = window pixels), stored
//     in LDS in the storage type -- the rounding of a stored y -- with the
//     conv's zero padding at window positions outside the frame;
//   * the 3x3 conv from LDS, K = 9 taps x C/2 in the unfused GEMM's order (tap-
//     major, then 32-channel k-steps), bias, leaky, + x (from the window),
//     stored to `out` (not x: neighbouring tiles still read x's halo).
// Wave roles (8 waves, two per SIMD): in the 1x1, a wave owns GA groups of 16 y
// channels (weights in registers) over a strided set of 16-pixel blocks; in the
// 3x3 a wave owns JB groups of 16 output channels (JB MFMA blocks share each
// pixel operand; weights of all 9 taps in registers: 36 JB registers per
// 32-channel k-step) over a part of the tile's pixels.  C = 128 takes JB = 1 so
// that the weights fit beside the accumulators.
// Pixel rows in LDS are padded by 32 bytes (x: 2C + 32, y: C + 32 bytes per
// pixel: 6, 10 or 18 16-byte units, twice an odd number), so that 16 consecutive
// pixels at two k-slots -- the 32 lanes a ds_read_b128 serves at once -- hit
// distinct 16-byte units modulo 512 bytes (full LDS rate), and every operand
// address is a per-lane base plus an immediate offset.
// ---------------------------------------------------------------------------
template <int C> struct RbCfg;
// DA: window DMAs per wave issued during the 1x1 (the rest go one per 3x3
// step); measured fastest with all of them in the 1x1.
template <> struct RbCfg<64> { static constexpr int TY = 8, TX = 32, GA = 2, JB = 2, NW = 8, DA = 7; };
template <> struct RbCfg<128> { static constexpr int TY = 8, TX = 16, GA = 1, JB = 1, NW = 8, DA = 7; };

template <typename T, int C>
__global__ __launch_bounds__(64 * RbCfg<C>::NW) void resblock_kernel(const T* __restrict__ x, T* __restrict__ out,
                                                       const T* __restrict__ w1, const float* __restrict__ b1,
                                                       const T* __restrict__ w2, const float* __restrict__ b2,
                                                       const int* __restrict__ geom, int nframes, int lvl,
                                                       int total, int x_bytes, const int* __restrict__ dyn) {
    if (dyn) {  // batch header: frames and tiles of this batch (the grid covers the capacity)
        nframes = dyn[kDynN];
        total = dyn[C == 64 ? kDynRb64 : kDynRb128];
    }
    constexpr int C2 = C / 2, NW = RbCfg<C>::NW;
    constexpr int TY = RbCfg<C>::TY, TX = RbCfg<C>::TX, GA = RbCfg<C>::GA, JB = RbCfg<C>::JB;
    constexpr int WY = TY + 2, WX = TX + 2, NPX = WY * WX;
    constexpr int NBA = (NPX + 15) / 16, NPXP = NBA * 16;        // 1x1 blocks over the window
    constexpr int XS = C * 2 + 32, YS = C2 * 2 + 32;              // LDS bytes per pixel (padded)
    constexpr int XSL = C / 8;                                    // 16-byte slots of x per pixel
    constexpr int NDMA = (NPXP * XS + 1023) / 1024, DPW = (NDMA + NW - 1) / NW;  // 1-KB DMAs per window
    constexpr int XB = NDMA * 1024;                               // bytes per window buffer
    constexpr int NGA = C2 / 16, GSETS = NGA / GA;                // 1x1: y-channel group sets
    constexpr int NGB = C / (16 * JB), PG = NW / NGB;             // 3x3: channel groups, pixel groups
    constexpr int BPR = TX / 16, NBB = TY * BPR, BPW = NBB / PG;   // 3x3: 16-pixel blocks
    constexpr int KA = C / 32, KB = C2 / 32;                      // k-steps per tap
    constexpr int NBW = (NBA + NW / GSETS - 1) / (NW / GSETS);    // 1x1 blocks per wave (at most)
    constexpr int AB = NBW < 3 ? NBW : 3, NBAT = (NBW + AB - 1) / AB;  // 1x1 batches of AB blocks
    // The next window's DMAs: the first DA are issued over the 1x1 batches, the
    // rest one per 3x3 step.  A compute unit's vector memory path moves 32-64
    // B/clk, so a wave issuing DMAs stalls wherever it issues them.
    constexpr int DA = RbCfg<C>::DA, DPB = (DA + NBAT - 1) / NBAT;
    static_assert(DA <= DPW && DPW - DA <= 9 * KB, "DMA steps");
    static_assert(NGA % GA == 0 && NW % NGB == 0 && NBB % PG == 0 && BPW % BPR == 0, "tile");
    static_assert(2 * XB + NPXP * YS <= 160 * 1024, "LDS");
    typedef typename V16<T>::type V;
    typedef T T4 __attribute__((ext_vector_type(4)));

    __shared__ __attribute__((aligned(1024))) char xw[2][XB];
    __shared__ __attribute__((aligned(1024))) char yw[NPXP * YS];

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int p = lane & 15, kg = lane >> 4;
    const __amdgpu_buffer_rsrc_t r_x = __builtin_amdgcn_make_buffer_rsrc((void*)x, 0, x_bytes, kBufFlags);

    // weights of this wave, for the workgroup's life
    const int gset = wave % GSETS;
    V a1[GA][KA];
    float bb1[GA][4];
#pragma unroll
    for (int g = 0; g < GA; ++g) {
        const int ch = (gset * GA + g) * 16;
#pragma unroll
        for (int kk = 0; kk < KA; ++kk) a1[g][kk] = *(const V*)(w1 + (size_t)(ch + p) * C + kk * 32 + kg * 8);
#pragma unroll
        for (int q = 0; q < 4; ++q) bb1[g][q] = b1[ch + kg * 4 + q];
    }
    const int cg = wave % NGB, pg = wave / NGB;
    V a2[JB][9][KB];
    float bb2[JB][4];
#pragma unroll
    for (int j = 0; j < JB; ++j) {
        const int ch = (cg * JB + j) * 16;
#pragma unroll
        for (int tp = 0; tp < 9; ++tp)
#pragma unroll
            for (int kk = 0; kk < KB; ++kk)
                a2[j][tp][kk] = *(const V*)(w2 + (size_t)(ch + p) * (9 * C2) + tp * C2 + kk * 32 + kg * 8);
#pragma unroll
        for (int q = 0; q < 4; ++q) bb2[j][q] = b2[ch + kg * 4 + q];
    }

    // Work items are visited in increasing order, so the frame of the next item
    // is found by advancing a cursor (frame f: items [first, first + n)).
    struct Tile { int ty0, tx0, h, w, base; };
    int cf = 0, cfirst = 0, cn = 0, ctw = 1, ch_ = 0, cw_ = 0, cbase = 0;
    auto load_frame = [&]() {
        ch_ = geom[cf * kGeomInts] >> lvl;
        cw_ = geom[cf * kGeomInts + 1] >> lvl;
        cbase = geom[cf * kGeomInts + 2 + lvl];
        ctw = (cw_ + TX - 1) / TX;
        cn = ((ch_ + TY - 1) / TY) * ctw;
    };
    auto locate = [&](int item) {
        while (item >= cfirst + cn && cf + 1 < nframes) {
            cfirst += cn;
            ++cf;
            load_frame();
        }
        const int r = item - cfirst, ty = r / ctw;
        return Tile{ty * TY, (r - ty * ctw) * TX, ch_, cw_, cbase};
    };
    // Window DMA: lane i of instruction q fills the 16-byte LDS slot 64 q + i,
    // i.e. slot s of window pixel (wy, wx) (s >= XSL is the padding: zeros).
    // The lane's (wy, wx, s) per instruction is fixed: packed once, -1 = padding.
    // For a window inside the frame the offset is the window origin's plus a
    // per-lane term that depends only on the frame width (drel, for width drw).
    int dgeo[DPW], drel[DPW], drw = -1;
#pragma unroll
    for (int i = 0; i < DPW; ++i) {
        const int L = (wave + NW * i) * 64 + lane;
        const int px = L / (XSL + 2), sl = L - px * (XSL + 2);
        const int wy = px / WX, wx = px - wy * WX;
        dgeo[i] = (sl < XSL && px < NPX) ? (wy << 16) | (wx << 8) | sl : -1;
    }
    auto issue_one = [&](const Tile& t, int buf, int i) {
        const int q = wave + NW * i;
        if (q < NDMA) {  // wave-uniform
            const int g = dgeo[i];
            const bool interior = t.ty0 >= 1 && t.tx0 >= 1 && t.ty0 + TY < t.h && t.tx0 + TX < t.w;  // uniform
            int off;
            if (interior) {
                if (t.w != drw) {  // uniform; once per frame width
                    drw = t.w;
#pragma unroll
                    for (int k = 0; k < DPW; ++k)
                        drel[k] = (((dgeo[k] >> 16) * drw + ((dgeo[k] >> 8) & 255)) * C + (dgeo[k] & 255) * 8) *
                                  (int)sizeof(T);
                }
                off = g >= 0 ? ((t.base + (t.ty0 - 1) * t.w + t.tx0 - 1) * C) * (int)sizeof(T) + drel[i] : kOOB;
            } else {
                const int iy = t.ty0 - 1 + (g >> 16), ix = t.tx0 - 1 + ((g >> 8) & 255);
                const bool ok = g >= 0 && (unsigned)iy < (unsigned)t.h && (unsigned)ix < (unsigned)t.w;
                off = ok ? ((t.base + iy * t.w + ix) * C + (g & 255) * 8) * (int)sizeof(T) : kOOB;
            }
            // the LDS address is wave-uniform; buf lives in a vector register
            const unsigned la = __builtin_amdgcn_readfirstlane(
                (unsigned)(unsigned long)(lds_ptr_t)&xw[0][0] + (unsigned)(buf * XB + q * 1024));
            asm volatile("s_mov_b32 m0, %0\n\tbuffer_load_dwordx4 %1, %2, 0 offen lds"
                         :
                         : "s"(la), "v"(off), "s"(r_x)
                         : "memory", "m0");
        }
    };
    const __amdgpu_buffer_rsrc_t r_out = __builtin_amdgcn_make_buffer_rsrc((void*)out, 0, x_bytes, kBufFlags);

    const int per = gridDim.x / kXCDs, xcd = blockIdx.x % kXCDs;
    const int band = (total + kXCDs - 1) / kXCDs;
    const int lo = xcd * band, hi = lo + band < total ? lo + band : total;
    int P = lo + (int)blockIdx.x / kXCDs;
    if (P >= hi) return;  // uniform over the workgroup
    load_frame();
    Tile t = locate(P);
#pragma unroll
    for (int i = 0; i < DPW; ++i) issue_one(t, 0, i);
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 15));
    // Per tile: barrier (every wave's share of this tile's window has landed, and
    // every wave is done with the previous tile: its window buffer and y are
    // free); 1x1 -> y, issuing the next tile's window into the other buffer;
    // barrier; 3x3 + epilogue; wait for this wave's share of the next window.
    // Vector memory operations complete in order, and each wave issues exactly
    // BPW JB stores after its window loads, so vmcnt(BPW JB) waits for the loads
    // only.
    for (int it = 0; P < hi; ++it, P += per) {
        const int buf = it & 1;
        __syncthreads();
        const int Pn = P + per;
        const bool more = Pn < hi;
        const Tile tn = more ? locate(Pn) : t;
        const char* xb = xw[buf];
        // 1x1 over the window -> y (LDS), in batches of AB blocks per wave (operand
        // reads, then MFMAs, then epilogues); the next tile's window DMAs are
        // issued between batches.
        static_for<0, NBAT>([&](auto bt_c) {
            constexpr int bt = decltype(bt_c)::value;
            if (more) {
#pragma unroll
                for (int i = bt * DPB; i < (bt + 1) * DPB && i < DA; ++i) issue_one(tn, buf ^ 1, i);
            }
            V bfa[AB][KA];
            int pxs[AB];
#pragma unroll
            for (int b = 0; b < AB; ++b) {
                const int blk = wave / GSETS + (bt * AB + b) * (NW / GSETS);
                pxs[b] = (blk < NBA ? blk : NBA - 1) * 16 + p;  // past the window: recomputed, not stored
#pragma unroll
                for (int kk = 0; kk < KA; ++kk) bfa[b][kk] = *(const V*)(xb + pxs[b] * XS + (kk * 4 + kg) * 16);
            }
            f32x4 acc[AB][GA];
#pragma unroll
            for (int b = 0; b < AB; ++b)
#pragma unroll
                for (int g = 0; g < GA; ++g) {
                    acc[b][g] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kk = 0; kk < KA; ++kk) {
                        if constexpr (__is_same(T, bf16))
                            acc[b][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[g][kk], bfa[b][kk], acc[b][g], 0, 0, 0);
                        else
                            acc[b][g] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1[g][kk], bfa[b][kk], acc[b][g], 0, 0, 0);
                    }
                }
#pragma unroll
            for (int b = 0; b < AB; ++b) {
                const int blk = wave / GSETS + (bt * AB + b) * (NW / GSETS);
                if (blk < NBA) {  // wave-uniform
                    const int px = pxs[b];
                    const int wy = px / WX, wx = px - wy * WX;
                    const int iy = t.ty0 - 1 + wy, ix = t.tx0 - 1 + wx;
                    const bool inside = px < NPX && (unsigned)iy < (unsigned)t.h && (unsigned)ix < (unsigned)t.w;
#pragma unroll
                    for (int g = 0; g < GA; ++g) {
                        const int yc = (gset * GA + g) * 16 + kg * 4;  // first of this lane's 4 y channels
                        T4 pk;
#pragma unroll
                        for (int q = 0; q < 4; ++q) pk[q] = (T)leaky01(acc[b][g][q] + bb1[g][q]);
                        *(T4*)(yw + px * YS + yc * 2) = inside ? pk : T4{};
                    }
                }
            }
        });
        __syncthreads();  // y complete
        // 3x3 from y, this wave's BPW blocks x 16 JB channels.  Steps are (tap,
        // k-step) pairs in the unfused GEMM's K order; a step's pixel operands are
        // read from LDS one step ahead into the other register set, and nothing is
        // scheduled across steps (this bounds the registers the reads hold).
        f32x4 acc[BPW][JB];
#pragma unroll
        for (int i = 0; i < BPW; ++i)
#pragma unroll
            for (int j = 0; j < JB; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        V bfr[2][BPW];
        auto rd_b = [&](auto st_c) {
            constexpr int st = decltype(st_c)::value, tp = st / KB, kk = st % KB;
            constexpr int r = tp / 3, s = tp % 3;
#pragma unroll
            for (int i = 0; i < BPW; ++i) {
                const int blk = pg * BPW + i;
                const int ty = blk / BPR, tx = (blk % BPR) * 16 + p;
                const int wpx = (ty + r) * WX + tx + s;
                bfr[st & 1][i] = *(const V*)(yw + wpx * YS + (kk * 4 + kg) * 16);
            }
        };
        auto mm_b = [&](auto st_c) {
            constexpr int st = decltype(st_c)::value, tp = st / KB, kk = st % KB;
#pragma unroll
            for (int i = 0; i < BPW; ++i)
#pragma unroll
                for (int j = 0; j < JB; ++j) {
                    if constexpr (__is_same(T, bf16))
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[j][tp][kk], bfr[st & 1][i], acc[i][j], 0, 0, 0);
                    else
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a2[j][tp][kk], bfr[st & 1][i], acc[i][j], 0, 0, 0);
                }
        };
        rd_b(std::integral_constant<int, 0>{});
        static_for<0, 9 * KB>([&](auto st_c) {
            constexpr int st = decltype(st_c)::value;
            if constexpr (st + 1 < 9 * KB) rd_b(std::integral_constant<int, st + 1>{});
            if constexpr (DA + st < DPW) {
                if (more) issue_one(tn, buf ^ 1, DA + st);
            }
            mm_b(st_c);
            __builtin_amdgcn_sched_barrier(0);
        });
        // epilogue: bias, leaky, + x, store
#pragma unroll
        for (int i = 0; i < BPW; ++i) {
            const int blk = pg * BPW + i;
            const int ty = blk / BPR, tx = (blk % BPR) * 16 + p;
            const int cpx = (ty + 1) * WX + tx + 1;  // window pixel of this output pixel
            T4 pk[JB];
#pragma unroll
            for (int j = 0; j < JB; ++j) {
                const int c = (cg * JB + j) * 16 + kg * 4;
                const T4 rv = *(const T4*)(xb + cpx * XS + c * 2);
#pragma unroll
                for (int q = 0; q < 4; ++q) pk[j][q] = (T)(leaky01(acc[i][j][q] + bb2[j][q]) + (float)rv[q]);
            }
            const int oy = t.ty0 + ty, ox = t.tx0 + tx;
            const bool in = oy < t.h && ox < t.w;
            // 8 bytes per lane and channel block; pixels outside the frame get an
            // out-of-range offset (the store is dropped but still issued)
            const int ob = ((t.base + oy * t.w + ox) * C + cg * JB * 16 + kg * 4) * (int)sizeof(T);
            typedef unsigned U2 __attribute__((ext_vector_type(2)));
#pragma unroll
            for (int j = 0; j < JB; ++j) {
                U2 u2;
                __builtin_memcpy(&u2, &pk[j], 8);
                __builtin_amdgcn_raw_buffer_store_b64(u2, r_out, in ? ob + j * 16 * (int)sizeof(T) : kOOB, 0, 0);
            }
        }
        __builtin_amdgcn_s_waitcnt(waitcnt_imm(BPW * JB, 15));
        t = tn;
    }
    // no DMA may still be writing LDS when the workgroup ends
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 15));
}

int resblock_tiles(int C, int h, int w) {
    if (C == 64) return ((h + RbCfg<64>::TY - 1) / RbCfg<64>::TY) * ((w + RbCfg<64>::TX - 1) / RbCfg<64>::TX);
    if (C == 128) return ((h + RbCfg<128>::TY - 1) / RbCfg<128>::TY) * ((w + RbCfg<128>::TX - 1) / RbCfg<128>::TX);
    return 0;
}

hipError_t launch_resblock(const void* x, void* out, const void* w1, const float* b1, const void* w2,
                           const float* b2, const int* geom, int nframes, int lvl, int C, int tiles, size_t x_bytes,
                           int et, hipStream_t s, const int* dyn) {
    if ((C != 64 && C != 128) || (et != kBF16 && et != kF16) || tiles <= 0 || x_bytes >= (size_t)1 << 31 ||
        x == out)
        return hipErrorInvalidValue;
    // persistent: one workgroup per compute unit, a multiple of 8 (one band per XCD)
    const int g = tiles < 256 ? ((tiles + 7) / 8) * 8 : 256;
    dim3 grid(g), block(64 * (C == 64 ? RbCfg<64>::NW : RbCfg<128>::NW));
#define JDE_RB(TT, CC)                                                                                          \
    resblock_kernel<TT, CC><<<grid, block, 0, s>>>((const TT*)x, (TT*)out, (const TT*)w1, b1, (const TT*)w2, b2, \
                                                   geom, nframes, lvl, tiles, (int)x_bytes, dyn)
    if (et == kBF16) {
        if (C == 64) JDE_RB(bf16, 64); else JDE_RB(bf16, 128);
    } else {
        if (C == 64) JDE_RB(f16, 64); else JDE_RB(f16, 128);
    }
#undef JDE_RB
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pointwise (1x1, stride 1) conv as a persistent streaming GEMM, 16-bit storage:
// out[m][:] = act(b + W x[m][:]) for the batch's M pixels (the 1x1 halves of
// the Darknet-53 residual blocks of Sec. 3.1 and the FPN's 1x1 convs with no
// concatenated input).  With K = Cin <= 512 the work per pixel is small (2 Cout
// FLOP per input byte), so the launch is bound by moving x in and out to HBM;
// the implicit GEMM pays a pipeline fill per short K loop instead.  Here every
// wave keeps its 16 G output channels' weights for all of K in registers for the
// workgroup's life, and one workgroup per compute unit walks BN-pixel tiles
// of x, brought into a ring of NBUF LDS buffers by direct-to-LDS loads NBUF - 1
// tiles ahead of the one computing.  Workgroup g takes the pixels [g M / grid,
// (g + 1) M / grid) in tiles from the range's start (the last one partial), so
// that every workgroup moves the same bytes (equal tiles dealt round robin
// would leave up to a whole tile's imbalance: 16 % at 5 tiles per workgroup).
//   * tile layout in LDS: pixel rows of 2 Cin + 32 bytes (16-byte slots, the two
//     last are padding, loaded as zeros), so that the 16 pixels x 2 k-slots a
//     ds_read_b128 serves at once hit distinct 16-byte units modulo 512 bytes;
//   * each wave issues a fixed number of 1-KB loads per tile (DPW or DPW - 1;
//     loads past the range read zeros), so the wait for the next tile is one of
//     two fixed vmcnts;
//   * K is summed in the implicit GEMM's order (32-channel k-steps from 0, the
//     bias after the last), so the outputs equal its outputs bit for bit.
// ---------------------------------------------------------------------------
// BN pixels per tile, G 16-channel groups per wave, NBUF ring buffers; on MI355X
// 32 / 16 pixels with four buffers measured about 6 % faster than 64 / 32 with
// three, and 128 / 64 with two about 12 % slower.
template <int CIN, int COUT> struct PwCfg;
template <> struct PwCfg<256, 128> { static constexpr int BN = 32, G = 1, NBUF = 4; };
template <> struct PwCfg<512, 256> { static constexpr int BN = 16, G = 2, NBUF = 4; };
// 1024 -> 512 in four workgroups of 128 output channels (ngroups = 4)
template <> struct PwCfg<1024, 128> { static constexpr int BN = 16, G = 1, NBUF = 4; };

template <typename T, int CIN, int COUT>
__global__ __launch_bounds__(512) void conv_pw_stream(const T* __restrict__ x, T* __restrict__ out,
                                                      const T* __restrict__ w, const float* __restrict__ bias, int M,
                                                      int ld, int act, int x_bytes, int out_bytes,
                                                      const int* __restrict__ dyn_m, int ngroups) {
    constexpr int NW = 8, BN = PwCfg<CIN, COUT>::BN, G = PwCfg<CIN, COUT>::G;
    static_assert(NW * G * 16 == COUT, "one wave per 16 G output channels");
    constexpr int KA = CIN / 32, NB = BN / 16;
    constexpr int XSL = CIN / 8, XS = (XSL + 2) * 16;              // slots of x per pixel, bytes per LDS row
    constexpr int NSL = BN * (XSL + 2);                             // 16-byte slots per tile
    constexpr int NDMA = (NSL + 63) / 64, DPW = (NDMA + NW - 1) / NW;  // 1-KB loads per tile, per wave (at most)
    constexpr int XB = NDMA * 1024, NBUF = PwCfg<CIN, COUT>::NBUF;  // bytes per buffer, buffers
    constexpr int NST = NB * G;                                     // stores per wave per tile
    static_assert(NBUF >= 2 && NBUF * XB <= 160 * 1024 && (NBUF - 2) * DPW + NB * G <= 63, "LDS, vmcnt");
    typedef typename V16<T>::type V;
    typedef T T4 __attribute__((ext_vector_type(4)));

    __shared__ __attribute__((aligned(1024))) char xw[NBUF * XB];

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int p = lane & 15, kg = lane >> 4;
    const __amdgpu_buffer_rsrc_t r_x = __builtin_amdgcn_make_buffer_rsrc((void*)x, 0, x_bytes, kBufFlags);
    const __amdgpu_buffer_rsrc_t r_out = __builtin_amdgcn_make_buffer_rsrc((void*)out, 0, out_bytes, kBufFlags);

    // ngroups > 1: output channels c0 .. c0 + COUT of ngroups x COUT; the ngroups
    // workgroups of one pixel range run on one XCD (workgroup b on XCD b % 8; the
    // grid is a multiple of 8 ngroups), so that its L2 fetches the range once
    const int ng = ngroups > 1 ? (int)(blockIdx.x / 8) % ngroups : 0;
    const int walker = ngroups > 1 ? (int)(blockIdx.x % 8) + 8 * (int)(blockIdx.x / (8 * ngroups)) : (int)blockIdx.x;
    const int nwalk = (int)gridDim.x / ngroups;
    const int c0 = ng * COUT;
    // Weights: the MFMA operand of k-step kk wants lane (p, kg) to hold W[ch + p]
    // [32 kk + 8 kg, +8): loaded that way, an instruction reads 16 rows x 64 bytes,
    // at half the load path's rate.  Instead two instructions read rows ch .. ch + 7
    // and ch + 8 .. ch + 15 in 128-byte segments (lane L: row L / 8, 16-byte unit
    // L % 8 of k-steps 2 kp and 2 kp + 1), and a cross-lane permute hands each lane
    // its 16 bytes: unit 4 h + kg of row p, from lane 8 (p % 8) + 4 h + kg of
    // instruction p / 8.
    V a[G][KA];
    float bb[G][4];
    static_assert(KA % 2 == 0, "k-steps in pairs");
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int ch = c0 + (wave * G + g) * 16;
#pragma unroll
        for (int kp = 0; kp < KA / 2; ++kp) {
            int src[2][4];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const V v = *(const V*)(w + (size_t)(ch + 8 * i + (lane >> 3)) * CIN + kp * 64 + (lane & 7) * 8);
                __builtin_memcpy(src[i], &v, 16);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int from = ((p & 7) * 8 + 4 * h + kg) * 4;  // source lane, as a byte address
                int dst[4];
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const int lo8 = __builtin_amdgcn_ds_bpermute(from, src[0][d]);
                    const int hi8 = __builtin_amdgcn_ds_bpermute(from, src[1][d]);
                    dst[d] = p < 8 ? lo8 : hi8;
                }
                __builtin_memcpy(&a[g][2 * kp + h], dst, 16);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) bb[g][q] = bias[ch + kg * 4 + q];
    }
    touch_regs(a, bb);  // the weights have landed before the loop's first wait

    // Load i of this wave fills tile slots (wave + NW i) 64 + lane: pixel px,
    // slot sl of that pixel's row; rel = its byte offset from the tile's first
    // pixel, -1 for padding slots and slots past the tile.
    int rel[DPW], pxi[DPW];
#pragma unroll
    for (int i = 0; i < DPW; ++i) {
        const int L = (wave + NW * i) * 64 + lane;
        const int px = L / (XSL + 2), sl = L - px * (XSL + 2);
        pxi[i] = px;
        rel[i] = (L < NSL && sl < XSL) ? (px * CIN + sl * 8) * (int)sizeof(T) : -1;
    }
    const unsigned lbase = __builtin_amdgcn_readfirstlane((unsigned)(unsigned long)(lds_ptr_t)&xw[0]);
    // this workgroup's pixels [lo, hi) and tiles (with a batch header, M is this
    // batch's and the grid the capacity's: a workgroup may get no pixels)
    if (dyn_m) M = *dyn_m;
    const int lo = (int)((long long)walker * M / nwalk);
    const int hi = (int)((long long)(walker + 1) * M / nwalk);
    if (hi <= lo) return;  // uniform over the workgroup, before any load or barrier
    const int nt = (hi - lo + BN - 1) / BN;
    // Load i of tile j into ring slot buf (tile j >= nt: zeros, so that the count
    // per wave stays fixed); waves whose last load index is past the tile's NDMA
    // loads issue DPW - 1 per tile (`full` is false for them).
    auto issue_one = [&](int j, int buf, int i) {
        if (wave + NW * i < NDMA) {  // wave-uniform
            const int p0 = lo + (j < nt ? j : 0) * BN;
            const int off = (j < nt && rel[i] >= 0 && p0 + pxi[i] < hi)
                                ? (int)((unsigned)p0 * (unsigned)(CIN * sizeof(T)) + (unsigned)rel[i])
                                : kOOB;
            const unsigned la = lbase + (unsigned)(buf * XB + (wave + NW * i) * 1024);
            asm volatile("s_mov_b32 m0, %0\n\tbuffer_load_dwordx4 %1, %2, 0 offen lds"
                         :
                         : "s"(la), "v"(off), "s"(r_x)
                         : "memory", "m0");
        }
    };
    const bool full = wave + NW * (DPW - 1) < NDMA;

    // nwalk <= ceil(M / BN): every pixel range has at least one pixel
    static_for<0, NBUF - 1>([&](auto j_c) {
#pragma unroll
        for (int i = 0; i < DPW; ++i) issue_one(decltype(j_c)::value, decltype(j_c)::value, i);
    });
    // this wave's loads of the first tile
    if (full)
        __builtin_amdgcn_s_waitcnt(waitcnt_imm((NBUF - 2) * DPW, 15));
    else
        __builtin_amdgcn_s_waitcnt(waitcnt_imm((NBUF - 2) * (DPW - 1), 15));
    // Per tile (ring slot it % NBUF): barrier (every wave's loads of this tile
    // have landed; every wave is done with the previous tile, whose slot is
    // refilled with the tile NBUF - 1 ahead, its loads spread over the k-steps so
    // that the compute unit's load path works while the matrix cores do); MFMAs
    // from LDS; epilogue stores; wait for this wave's loads of the next tile: in
    // issue order they are followed by the loads of the NBUF - 2 tiles after it
    // and by this tile's NST stores (and possibly earlier tiles' stores, which only
    // waits longer), and vector memory operations complete in order.
    for (int it = 0; it < nt; ++it) {
        const int buf = it % NBUF;
        __builtin_amdgcn_s_barrier();
        const int jn = it + NBUF - 1, bn = jn % NBUF;
        const char* xb = xw + buf * XB;
        f32x4 acc[NB][G];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int g = 0; g < G; ++g) acc[b][g] = f32x4{0.f, 0.f, 0.f, 0.f};
        V bf[2][NB];
        auto rd = [&](auto kk_c) {
            constexpr int kk = decltype(kk_c)::value;
#pragma unroll
            for (int b = 0; b < NB; ++b) bf[kk & 1][b] = *(const V*)(xb + (b * 16 + p) * XS + (kk * 4 + kg) * 16);
        };
        rd(std::integral_constant<int, 0>{});
        static_for<0, KA>([&](auto kk_c) {
            constexpr int kk = decltype(kk_c)::value;
            static_for<0, DPW>([&](auto i_c) {  // load i at k-step i KA / DPW
                if constexpr ((decltype(i_c)::value * KA) / DPW == kk) issue_one(jn, bn, decltype(i_c)::value);
            });
            if constexpr (kk + 1 < KA) rd(std::integral_constant<int, kk + 1>{});
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    if constexpr (__is_same(T, bf16))
                        acc[b][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[g][kk], bf[kk & 1][b], acc[b][g], 0, 0, 0);
                    else
                        acc[b][g] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[g][kk], bf[kk & 1][b], acc[b][g], 0, 0, 0);
                }
            __builtin_amdgcn_sched_barrier(0);
        });
        // epilogue: + bias, leaky (act), cast; 8 bytes per lane and 16-channel
        // group; pixels past the range get an out-of-range offset (dropped, issued)
        typedef unsigned U2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int m = lo + it * BN + b * 16 + p;
            const int mo = m < hi ? m : lo;  // offsets computed for in-range pixels only
#pragma unroll
            for (int g = 0; g < G; ++g) {
                T4 pk;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float v = acc[b][g][q] + bb[g][q];
                    if (act) v = leaky01(v);
                    pk[q] = cvt_out<T>(v);
                }
                U2 u2;
                __builtin_memcpy(&u2, &pk, 8);
                const int ob = (mo * ld + c0 + (wave * G + g) * 16 + kg * 4) * (int)sizeof(T);
                __builtin_amdgcn_raw_buffer_store_b64(u2, r_out, m < hi ? ob : kOOB, 0, 0);
            }
        }
        if (full)
            __builtin_amdgcn_s_waitcnt(waitcnt_imm((NBUF - 2) * DPW + NST, 15));
        else
            __builtin_amdgcn_s_waitcnt(waitcnt_imm((NBUF - 2) * (DPW - 1) + NST, 15));
    }
    // no load may still be writing LDS when the workgroup ends
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 15));
}

static bool conv_pw_ok(const ConvArgs& a, int et) {
    if (et != kBF16 && et != kF16) return false;
    if (a.ksz != 1 || a.stride != 1 || a.pad != 0 || a.cin1 != 0 || a.lvl_in != a.lvl_out) return false;
    if (a.res || a.out1 || a.n_split != a.cout || a.out0_f32 || a.wscale || a.amax) return false;
    if (!((a.cin == 256 && a.cout == 128) || (a.cin == 512 && a.cout == 256) || (a.cin == 1024 && a.cout == 512)))
        return false;
    if (a.ld0 < a.cout || a.ld0 % 4 || a.M <= 0) return false;
    return (size_t)a.M * a.cin * 2 <= (size_t)a.in_bytes && (size_t)a.M * a.ld0 * 2 < ((size_t)1 << 31);
}

template <typename T, int CIN, int COUT>
static hipError_t launch_pw_t(const ConvArgs& a, hipStream_t s, int ngroups = 1) {
    constexpr int BN = PwCfg<CIN, COUT>::BN;
    const int ntiles = (a.M + BN - 1) / BN;
    // one workgroup per compute unit (68-132 KB of LDS); with channel groups, a
    // multiple of 8 ngroups of them (pixel ranges in whole XCD rounds)
    int walkers = ntiles < 256 / ngroups ? ntiles : 256 / ngroups;
    if (ngroups > 1) walkers = walkers >= 8 ? walkers - walkers % 8 : 8;
    conv_pw_stream<T, CIN, COUT><<<dim3(walkers * ngroups), dim3(512), 0, s>>>(
        (const T*)a.in, (T*)a.out0, (const T*)a.w, a.bias, a.M, a.ld0, a.act, a.in_bytes, a.M * a.ld0 * 2,
        a.dyn ? a.dyn + kDynM + a.lvl_out : nullptr, ngroups);
    return hipGetLastError();
}

static hipError_t launch_pw(const ConvArgs& a, int et, hipStream_t s) {
    if (!conv_pw_ok(a, et)) return hipErrorInvalidValue;
    if (et == kBF16)
        return a.cin == 256   ? launch_pw_t<bf16, 256, 128>(a, s)
               : a.cin == 512 ? launch_pw_t<bf16, 512, 256>(a, s)
                              : launch_pw_t<bf16, 1024, 128>(a, s, 4);
    return a.cin == 256   ? launch_pw_t<f16, 256, 128>(a, s)
           : a.cin == 512 ? launch_pw_t<f16, 512, 256>(a, s)
                          : launch_pw_t<f16, 1024, 128>(a, s, 4);
}

// ---------------------------------------------------------------------------
// Tile configurations and dispatch.
// ---------------------------------------------------------------------------
// st = 0: register-staged conv_igemm; st = S >= 3: conv_dma with S stages;
// nt = 1: streaming (non-temporal) output stores.
// pw = 1: the persistent pointwise kernel (conv_pw_stream; 1x1 convs of 256 -> 128,
// 512 -> 256 and 1024 -> 512 channels only, the other fields unused).
struct TileCfg { int bm, bn, wgm, wgn, bk, st, nt, pw = 0; };
constexpr int kDynConvGrid = 1024;  // fallback grid of a conv launch in a graph for any batch

// Workgroups of kernel `fn` (of `threads` threads) that the device holds at once.
// A graph for any batch launches exactly that many (never more: a workgroup that
// only starts after the resident ones finished their whole walk doubles the
// launch) and lets each walk the batch's tiles.  A multiple of the 8 XCDs, so that
// a walk keeps each tile on the XCD the one-tile-per-workgroup order gives it.
static int resident_grid(const void* fn, int threads) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0) != hipSuccess || per_cu < 1 ||
        cus < 1)
        return kDynConvGrid;
    const int n = per_cu * cus;
    return n >= kXCDs ? n - n % kXCDs : n;
}
static constexpr TileCfg kTiles[] = {
    {128, 128, 2, 2, 32, 0, 0},  // 0: 64x64 per wave
    {256, 64, 4, 1, 32, 0, 0},   // 1: 64x64 per wave (Cout 64)
    {128, 64, 2, 2, 32, 0, 0},   // 2: 64x32 per wave
    {64, 128, 2, 2, 32, 0, 0},   // 3: 32x64 per wave
    {256, 32, 4, 1, 32, 0, 0},   // 4: 64x32 per wave (Cout <= 32)
    {64, 64, 2, 2, 32, 0, 0},    // 5: 32x32 per wave (also the unaligned-Cin path)
    {128, 32, 4, 1, 32, 0, 0},   // 6: 32x32 per wave
    {32, 128, 2, 2, 32, 0, 0},   // 7: 16x64 per wave
    {128, 128, 2, 2, 64, 0, 0},  // 8: as 0, K chunks of 64 (16-bit types)
    {256, 64, 4, 1, 64, 0, 0},   // 9: as 1, K chunks of 64
    {128, 64, 2, 2, 64, 0, 0},   // 10: as 2, K chunks of 64
    {64, 128, 2, 2, 64, 0, 0},   // 11: as 3, K chunks of 64
    {256, 128, 2, 2, 32, 0, 0},  // 12: 128x64 per wave
    {128, 256, 2, 2, 32, 0, 0},  // 13: 64x128 per wave
    {256, 128, 2, 2, 64, 0, 0},  // 14: 128x64 per wave, K chunks of 64
    {128, 128, 2, 2, 32, 4, 0},  // 15: direct-to-LDS, 4 stages (64 KB)
    {128, 128, 2, 2, 32, 3, 0},  // 16: direct-to-LDS, 3 stages (48 KB)
    {256, 128, 2, 2, 32, 3, 0},  // 17: direct-to-LDS, 128x64 per wave (72 KB)
    {128, 256, 2, 2, 32, 3, 0},  // 18: direct-to-LDS, 64x128 per wave (72 KB)
    {256, 64, 4, 1, 32, 4, 0},   // 19: direct-to-LDS, Cout 64 (80 KB)
    {128, 64, 2, 2, 32, 4, 0},   // 20: direct-to-LDS, 64x32 per wave (48 KB)
    {64, 128, 2, 2, 32, 4, 0},   // 21: direct-to-LDS, 32x64 per wave (48 KB)
    {128, 128, 2, 2, 32, 3, 1},  // 22: as 16, streaming stores
    {256, 128, 2, 2, 32, 3, 1},  // 23: as 17, streaming stores
    {128, 64, 2, 2, 32, 4, 1},   // 24: as 20, streaming stores
    {64, 128, 2, 2, 32, 4, 1},   // 25: as 21, streaming stores
    {128, 64, 2, 2, 32, 3, 0},   // 26: direct-to-LDS, 3 stages (36 KB: 4 workgroups per CU)
    {64, 64, 2, 2, 32, 4, 0},    // 27: direct-to-LDS, 32x32 per wave (32 KB: 5 per CU)
    {64, 64, 2, 2, 32, 3, 0},    // 28: direct-to-LDS, 3 stages (24 KB: 6 per CU)
    {256, 128, 4, 2, 32, 3, 0},  // 29: direct-to-LDS, 8 waves of 64x64 (72 KB)
    {128, 256, 2, 4, 32, 3, 0},  // 30: direct-to-LDS, 8 waves of 64x64 (72 KB)
    {256, 128, 4, 2, 32, 3, 1},  // 31: as 29, streaming stores
    {256, 256, 2, 4, 32, 3, 0},  // 32: direct-to-LDS, 8 waves of 128x64 (96 KB: half the loads per FLOP of 29/30)
    {256, 256, 4, 2, 32, 3, 0},  // 33: direct-to-LDS, 8 waves of 64x128 (96 KB)
    {256, 128, 4, 2, 64, 3, 0},  // 34: direct-to-LDS, 64-channel K chunks (128-byte rows), 8 waves (144 KB)
    {128, 256, 2, 4, 64, 3, 0},  // 35: as 34, 8 waves (144 KB)
    {128, 128, 2, 2, 64, 3, 0},  // 36: as 34, 4 waves (96 KB)
    {64, 128, 1, 1, 32, 0, 0, 1},  // 37: persistent pointwise stream (68 KB)
};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

template <typename T>
constexpr int lds_bytes(const TileCfg& t) {
    if (t.st) return t.st * (t.bm + t.bn) * t.bk * 2;
    return 2 * (t.bm + t.bn) * (t.bk + (sizeof(T) == 4 ? 4 : 16)) * (int)sizeof(T);
}
// 16-bit types may use every tile; FP32 only the register-staged K-32 tiles
// whose LDS fits.
template <typename T>
constexpr bool tile_built(int c) {
    if (kTiles[c].pw) return sizeof(T) == 2;
    if (kTiles[c].st) return sizeof(T) == 2 && lds_bytes<T>(kTiles[c]) <= 160 * 1024;
    return (sizeof(T) == 2 || kTiles[c].bk == 32) && lds_bytes<T>(kTiles[c]) <= 96 * 1024;
}

int conv_num_tile_cfgs() { return kNumTiles; }
bool conv_tile_folds_det(int c, int et, int n_split) {
    if (c < 0 || c >= kNumTiles || (et != kBF16 && et != kF16)) return false;
    const TileCfg& t = kTiles[c];
    return t.st > 0 && !t.pw && fold_det_tile(t.bm, t.bn, t.bk, t.st, t.wgm * t.wgn) && n_split > 0 &&
           n_split % t.bn == 0;
}
bool conv_tile_pw(int c) { return c >= 0 && c < kNumTiles && kTiles[c].pw; }
void conv_tile_shape(int c, int* bm, int* bn) {
    *bm = kTiles[c].bm;
    *bn = kTiles[c].bn;
}

static bool aligned_cin(const ConvArgs& a, int bk) {
    if (a.cin % bk) return false;
    if (a.cin1 > 0 && (a.cin1 % bk || a.ksz != 1 || a.stride != 1)) return false;
    return true;
}

static bool built(int c, int et) {
    if (et == kF32) return tile_built<float>(c);
    return tile_built<bf16>(c);
}

bool conv_tile_ok(int c, int et, const ConvArgs& a) {
    if (c < 0 || c >= kNumTiles) return false;
    if (et != kF32 && et != kBF16 && et != kF16) return false;
    if (!built(c, et)) return false;
    if (kTiles[c].pw) return conv_pw_ok(a, et);
    if (kTiles[c].st) {
        const int bk = kTiles[c].bk;
        if (a.cin1 > 0)  // concat: 1x1 stride 1, both sources in whole K chunks
            return a.ksz == 1 && a.stride == 1 && a.cin1 % bk == 0 && (a.cin - a.cin1) % bk == 0;
        return a.cin % bk == 0;
    }
    if (!aligned_cin(a, kTiles[c].bk)) return c == 5 && a.cin1 == 0 && a.cin % (et == kF32 ? 4 : 8) == 0;
    return true;
}

int conv_default_tile(int et, const ConvArgs& a) {
    // the persistent pointwise kernel wherever it fits (same sums, faster)
    for (int t = 0; t < kNumTiles; ++t)
        if (kTiles[t].pw && conv_tile_ok(t, et, a)) return t;
    if (!aligned_cin(a, 32)) return 5;
    // Prefer the largest tile that still gives at least ~2 workgroups per CU.
    static const int pref_wide[] = {0, 2, 3, 5, 7};
    static const int pref_64[] = {1, 2, 5};
    static const int pref_32[] = {4, 6};
    const int* pref;
    int np;
    if (a.cout <= 32) { pref = pref_32; np = 2; }
    else if (a.cout <= 64) { pref = pref_64; np = 3; }
    else { pref = pref_wide; np = 5; }
    int best = pref[np - 1];
    for (int i = 0; i < np; ++i) {
        if (!built(pref[i], et)) continue;
        const TileCfg& t = kTiles[pref[i]];
        const long wgs = (long)((a.M + t.bm - 1) / t.bm) * ((a.cout + t.bn - 1) / t.bn);
        if (wgs >= 512) { best = pref[i]; break; }
    }
    return best;
}

// conv_dma tiles that take a residual through LDS: a half tile (BM / 2 pixels x BN
// channels) fits one stage, its 1-KB instructions split evenly over the waves, no
// more of them than a chunk's, and 128 or 256 channels (rows of 256 or 512 bytes)
template <typename T, int C>
constexpr bool res_lds_tile() {
    constexpr TileCfg t = kTiles[C];
    constexpr int nw = t.wgm * t.wgn, npw = (t.bm + t.bn) / ((1024 / (t.bk * 2)) * (nw > 0 ? nw : 1));
    return t.st > 0 && sizeof(T) == 2 && (t.bn == 128 || t.bn == 256) && t.bm * t.bn <= (t.bm + t.bn) * t.bk * 2 &&
           (t.bm * t.bn / 1024) % nw == 0 && t.bm * t.bn / 1024 / nw <= npw;
}
template <typename T, int C>
static bool res_lds_launch(const ConvArgs& a) {
    return res_lds_tile<T, C>() && a.res && !a.out0_f32;
}

template <typename T, int C>
static hipError_t launch_t(const ConvArgs& a, bool aligned, hipStream_t s) {
    if constexpr (!tile_built<T>(C) || kTiles[C].pw) {  // pointwise tiles: launch_pw
        return hipErrorInvalidValue;
    } else {
        constexpr TileCfg t = kTiles[C];
        const int tiles = ((a.M + t.bm - 1) / t.bm) * ((a.cout + t.bn - 1) / t.bn);
        dim3 block(64 * t.wgm * t.wgn);
        if (a.dyn) {
            // a graph for any batch: a.M is the capacity's; the resident workgroups (at most
            // one per tile) walk the batch's tiles (the header's M), so a small batch pays no
            // empty workgroups
            if constexpr (sizeof(T) == 2) {
                auto go = [&](auto kern) {
                    const int cap = resident_grid(reinterpret_cast<const void*>(kern), (int)block.x);
                    kern<<<dim3(tiles < cap ? tiles : cap), block, 0, s>>>(a);
                    return hipGetLastError();
                };
                if constexpr (t.st > 0)
                    return res_lds_launch<T, C>(a) ? go(conv_dma<T, t.bm, t.bn, t.wgm, t.wgn, t.st, t.nt != 0, t.bk, true,
                                                              res_lds_tile<T, C>()>)
                                                   : go(conv_dma<T, t.bm, t.bn, t.wgm, t.wgn, t.st, t.nt != 0, t.bk, true>);
                else if (aligned)
                    return go(conv_igemm<T, t.bm, t.bn, t.wgm, t.wgn, t.bk, true, true>);
                else if constexpr (C == 5)
                    return go(conv_igemm<T, t.bm, t.bn, t.wgm, t.wgn, t.bk, false, true>);
                else
                    return hipErrorInvalidValue;
            } else {
                return hipErrorInvalidValue;  // FP32 contexts do not build graphs for any batch
            }
        }
        dim3 grid(tiles);
        if constexpr (t.st > 0)
            if (res_lds_launch<T, C>(a))
                conv_dma<T, t.bm, t.bn, t.wgm, t.wgn, t.st, t.nt != 0, t.bk, false, res_lds_tile<T, C>()>
                    <<<grid, block, 0, s>>>(a);
            else
                conv_dma<T, t.bm, t.bn, t.wgm, t.wgn, t.st, t.nt != 0, t.bk><<<grid, block, 0, s>>>(a);
        else if (aligned)
            conv_igemm<T, t.bm, t.bn, t.wgm, t.wgn, t.bk, true><<<grid, block, 0, s>>>(a);
        else if constexpr (C == 5)
            conv_igemm<T, t.bm, t.bn, t.wgm, t.wgn, t.bk, false><<<grid, block, 0, s>>>(a);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
}

template <typename T>
static hipError_t launch_type(const ConvArgs& a, int c, bool aligned, hipStream_t s) {
    switch (c) {
        case 0: return launch_t<T, 0>(a, aligned, s);
        case 1: return launch_t<T, 1>(a, aligned, s);
        case 2: return launch_t<T, 2>(a, aligned, s);
        case 3: return launch_t<T, 3>(a, aligned, s);
        case 4: return launch_t<T, 4>(a, aligned, s);
        case 5: return launch_t<T, 5>(a, aligned, s);
        case 6: return launch_t<T, 6>(a, aligned, s);
        case 7: return launch_t<T, 7>(a, aligned, s);
        case 8: return launch_t<T, 8>(a, aligned, s);
        case 9: return launch_t<T, 9>(a, aligned, s);
        case 10: return launch_t<T, 10>(a, aligned, s);
        case 11: return launch_t<T, 11>(a, aligned, s);
        case 12: return launch_t<T, 12>(a, aligned, s);
        case 13: return launch_t<T, 13>(a, aligned, s);
        case 14: return launch_t<T, 14>(a, aligned, s);
        case 15: return launch_t<T, 15>(a, aligned, s);
        case 16: return launch_t<T, 16>(a, aligned, s);
        case 17: return launch_t<T, 17>(a, aligned, s);
        case 18: return launch_t<T, 18>(a, aligned, s);
        case 19: return launch_t<T, 19>(a, aligned, s);
        case 20: return launch_t<T, 20>(a, aligned, s);
        case 21: return launch_t<T, 21>(a, aligned, s);
        case 22: return launch_t<T, 22>(a, aligned, s);
        case 23: return launch_t<T, 23>(a, aligned, s);
        case 24: return launch_t<T, 24>(a, aligned, s);
        case 25: return launch_t<T, 25>(a, aligned, s);
        case 26: return launch_t<T, 26>(a, aligned, s);
        case 27: return launch_t<T, 27>(a, aligned, s);
        case 28: return launch_t<T, 28>(a, aligned, s);
        case 29: return launch_t<T, 29>(a, aligned, s);
        case 30: return launch_t<T, 30>(a, aligned, s);
        case 31: return launch_t<T, 31>(a, aligned, s);
        case 32: return launch_t<T, 32>(a, aligned, s);
        case 33: return launch_t<T, 33>(a, aligned, s);
        case 34: return launch_t<T, 34>(a, aligned, s);
        case 35: return launch_t<T, 35>(a, aligned, s);
        case 36: return launch_t<T, 36>(a, aligned, s);
        case 37: return launch_t<T, 37>(a, aligned, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_conv(const ConvArgs& a, int et, int c, hipStream_t s) {
    if (!conv_outputs_ok(a) || !conv_tile_ok(c, et, a)) return hipErrorInvalidValue;
    if (kTiles[c].pw) return launch_pw(a, et, s);
    const bool aligned = aligned_cin(a, kTiles[c].bk);
    if (et == kF32) return launch_type<float>(a, c, aligned, s);
    if (et == kBF16) return launch_type<bf16>(a, c, aligned, s);
    return launch_type<f16>(a, c, aligned, s);
}

}  // namespace jde
