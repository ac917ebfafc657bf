// Post-processing of the JDE detections (Appendix A items 1-3, 5-6) for gfx950:
// decode + confidence threshold, sort, greedy IoU NMS, embedding gather and L2
// normalisation, the tracks x detections cost with Mahalanobis gating, and the
// track embedding update.  All per-frame work of a batch runs in one launch
// per step, with the frame on the grid's y axis.
#include <type_traits>

#include "jde_internal.h"

namespace jde {

typedef unsigned long long u64;

// Order-preserving map of FP32 bits to uint32 (larger float -> larger uint).
__device__ __forceinline__ unsigned ord_f32(float x) {
    unsigned u = __float_as_uint(x);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord_f32(unsigned o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}
// Ascending order of the key = margin descending, then index ascending.
__device__ __forceinline__ u64 make_key(float margin, unsigned idx) {
    return ((u64)(~ord_f32(margin)) << 32) | idx;
}
__device__ __forceinline__ float key_margin(u64 k) { return unord_f32(~(unsigned)(k >> 32)); }

__device__ __forceinline__ u64 shfl64(u64 v, int src) {
    const unsigned lo = __shfl((int)(unsigned)v, src), hi = __shfl((int)(unsigned)(v >> 32), src);
    return ((u64)hi << 32) | lo;
}

// Anchor decode of candidate `idx` (canonical order: scales 8, 16, 32; cell; anchor).
struct AnchorLoc { int s, cell, an; };
__device__ __forceinline__ AnchorLoc locate(unsigned idx, const int* g, int A) {
    const int h = g[0], w = g[1];
    const unsigned n8 = (unsigned)((h >> 3) * (w >> 3)) * A, n16 = (unsigned)((h >> 4) * (w >> 4)) * A;
    AnchorLoc L;
    unsigned t = idx;
    if (t < n8) L.s = 0;
    else if (t < n8 + n16) { L.s = 1; t -= n8; }
    else { L.s = 2; t -= n8 + n16; }
    L.cell = t / A;
    L.an = t - L.cell * A;
    return L;
}

// ---------------------------------------------------------------------------
// Decode + threshold: one thread per anchor; kept anchors are appended to the
// frame's key list by a wave ballot and one atomic per wave.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void decode_kernel(DecodeArgs a) {
    const int f = blockIdx.y;
    if (a.dyn && f >= a.dyn[kDynN]) return;  // grid covers the capacity; frame past this batch
    const int* g = a.geom + f * kGeomInts;
    const int h = g[0], w = g[1];
    const int A = a.A;
    const int total = ((h >> 3) * (w >> 3) + (h >> 4) * (w >> 4) + (h >> 5) * (w >> 5)) * A;
    const int t = blockIdx.x * 256 + threadIdx.x;
    bool keep = false;
    u64 key = 0;
    if (t < total) {
        const AnchorLoc L = locate((unsigned)t, g, A);
        const float* d = a.det[L.s] + ((size_t)g[2 + 3 + L.s] + L.cell) * (6 * A) + 6 * L.an;
        // per-frame offset added to the foreground logit (FP32 add, then the margin)
        const float cfg = a.logit_offset ? d[5] + a.logit_offset[f] : d[5];
        const float margin = (cfg - d[4]) + 0.0f;   // +0.0 folds -0 into +0
        keep = margin >= a.lthr;
        key = make_key(margin, (unsigned)t);
    }
    const u64 bal = __ballot(keep);
    if (bal == 0) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)bal) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(a.cand_count + f, __popcll(bal));
    base = __shfl(base, leader);
    if (keep) {
        const int pos = base + __popcll(bal & ((1ull << lane) - 1ull));
        if (pos < a.keycap) {
            a.keys[(size_t)f * a.keycap + pos] = key;
            if (a.vals) a.vals[(size_t)f * a.keycap + pos] = t;
        }
    }
}

hipError_t launch_decode(const DecodeArgs& a, int max_anchors, hipStream_t s) {
    dim3 grid((max_anchors + 255) / 256, a.nframes), block(256);
    decode_kernel<<<grid, block, 0, s>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sort each frame's keys ascending (bitonic); values follow when given.
// Lists up to kSortLds sort in LDS; longer ones sort in place in global memory
// (the key buffer has a power-of-two capacity per frame).
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 1024;
constexpr int kSortLdsKV = kSortLds;

__global__ __launch_bounds__(kSortThreads) void sort_kernel(u64* keys, int* vals, const int* counts, int keycap) {
    __shared__ u64 sk[kSortLdsKV];
    __shared__ int sv[kSortLdsKV];
    const int f = blockIdx.x;
    const int tid = threadIdx.x;
    int n = counts[f];
    if (n > keycap) n = keycap;
    if (n <= 1) return;
    int n2 = 1;
    while (n2 < n) n2 <<= 1;
    u64* K = keys + (size_t)f * keycap;
    int* Vv = vals ? vals + (size_t)f * keycap : nullptr;
    if (n2 <= kSortLdsKV) {
        for (int i = tid; i < n2; i += kSortThreads) {
            sk[i] = i < n ? K[i] : ~0ull;
            if (Vv) sv[i] = i < n ? Vv[i] : 0;
        }
        __syncthreads();
        for (int k = 2; k <= n2; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = tid; i < n2; i += kSortThreads) {
                    const int ixj = i ^ j;
                    if (ixj > i) {
                        const bool up = (i & k) == 0;
                        const u64 x = sk[i], y = sk[ixj];
                        if ((x > y) == up) {
                            sk[i] = y;
                            sk[ixj] = x;
                            if (Vv) {
                                const int t = sv[i];
                                sv[i] = sv[ixj];
                                sv[ixj] = t;
                            }
                        }
                    }
                }
                __syncthreads();
            }
        for (int i = tid; i < n; i += kSortThreads) {
            K[i] = sk[i];
            if (Vv) Vv[i] = sv[i];
        }
    } else {
        for (int i = n + tid; i < n2; i += kSortThreads) {
            K[i] = ~0ull;
            if (Vv) Vv[i] = 0;
        }
        __syncthreads();
        for (int k = 2; k <= n2; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = tid; i < n2; i += kSortThreads) {
                    const int ixj = i ^ j;
                    if (ixj > i) {
                        const bool up = (i & k) == 0;
                        const u64 x = K[i], y = K[ixj];
                        if ((x > y) == up) {
                            K[i] = y;
                            K[ixj] = x;
                            if (Vv) {
                                const int t = Vv[i];
                                Vv[i] = Vv[ixj];
                                Vv[ixj] = t;
                            }
                        }
                    }
                }
                __syncthreads();
            }
    }
}

hipError_t launch_sort(u64* keys, int* vals, const int* counts, int keycap, int n, hipStream_t s) {
    sort_kernel<<<n, kSortThreads, 0, s>>>(keys, vals, counts, keycap);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Boxes of the top-cap sorted candidates, decoded from the head outputs.
// ---------------------------------------------------------------------------
__constant__ float kClipLog64 = 4.15888308335967186f;  // ln 64

__global__ __launch_bounds__(256) void gather_boxes_kernel(GatherArgs a) {
    const int f = blockIdx.y;
    const int p = blockIdx.x * 256 + threadIdx.x;
    int n = a.cand_count[f];
    if (n > a.cap) n = a.cap;
    if (p == 0) a.kcount[f] = n;
    if (p >= n) return;
    const int* g = a.geom + f * kGeomInts;
    const u64 key = a.keys[(size_t)f * a.keycap + p];
    const unsigned idx = (unsigned)key;
    const AnchorLoc L = locate(idx, g, a.A);
    const int ws = g[1] >> (3 + L.s);
    const int i = L.cell / ws, j = L.cell - (L.cell / ws) * ws;
    const float st = (float)(8 << L.s);
    const float* d = a.det[L.s] + ((size_t)g[2 + 3 + L.s] + L.cell) * (6 * a.A) + 6 * L.an;
    const float aw = a.anchors[L.s][L.an][0], ah = a.anchors[L.s][L.an][1];
    const float cx = ((float)j + 0.5f) * st + d[0] * aw;
    const float cy = ((float)i + 0.5f) * st + d[1] * ah;
    const float bw = aw * __expf(fminf(d[2], kClipLog64));
    const float bh = ah * __expf(fminf(d[3], kClipLog64));
    *(float4*)(a.sboxes + ((size_t)f * a.cap + p) * 4) =
        make_float4(cx - 0.5f * bw, cy - 0.5f * bh, cx + 0.5f * bw, cy + 0.5f * bh);
}

hipError_t launch_gather_boxes(const GatherArgs& a, int n, hipStream_t s) {
    dim3 grid((a.cap + 255) / 256, n), block(256);
    gather_boxes_kernel<<<grid, block, 0, s>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Greedy NMS in two kernels.
//   mask: bit c of mask[row][cb] is set iff column cb*64+c comes after `row`
//         in sorted order and IoU(row, col) > thr (FP32, no contraction).
//   scan: one wave walks the sorted rows 64 at a time; the diagonal word of a
//         block is resolved lane-serially in registers, the kept rows' mask
//         words are OR-ed into the removed set of the later blocks.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool iou_exceeds(float4 a, float4 b, float thr) {
#pragma clang fp contract(off)
    const float iw = fmaxf(0.f, fminf(a.z, b.z) - fmaxf(a.x, b.x));
    const float ih = fmaxf(0.f, fminf(a.w, b.w) - fmaxf(a.y, b.y));
    const float inter = iw * ih;
    const float area_a = (a.z - a.x) * (a.w - a.y);
    const float area_b = (b.z - b.x) * (b.w - b.y);
    const float uni = (area_a + area_b) - inter;
    return inter > thr * uni;
}

__global__ __launch_bounds__(256) void nms_mask_kernel(const float* sboxes, const int* kcount, int cap, float thr,
                                                       u64* mask) {
    __shared__ float4 scol[4][64];
    const int f = blockIdx.y;
    const int K = kcount[f];
    const int nb = (K + 63) / 64;
    const int words = cap / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float4* B = (const float4*)(sboxes + (size_t)f * cap * 4);
    for (int rb = blockIdx.x; rb < nb; rb += gridDim.x) {
        const int row = rb * 64 + lane;
        const float4 rbox = row < K ? B[row] : make_float4(0.f, 0.f, 0.f, 0.f);
        for (int cb = rb + wave; cb < nb; cb += 4) {
            const int col0 = cb * 64;
            scol[wave][lane] = (col0 + lane < K) ? B[col0 + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
            __builtin_amdgcn_wave_barrier();
            u64 bits = 0;
            if (row < K) {
                const int cmax = min(64, K - col0);
                for (int c = 0; c < cmax; ++c) {
                    const int col = col0 + c;
                    if (col > row && iou_exceeds(rbox, scol[wave][c], thr)) bits |= 1ull << c;
                }
                mask[((size_t)f * cap + row) * words + cb] = bits;
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
}

__global__ __launch_bounds__(64) void nms_scan_kernel(const u64* mask, const int* kcount, int cap, int* keep,
                                                      int* nkeep) {
    const int f = blockIdx.x;
    const int lane = threadIdx.x;
    const int K = kcount[f];
    const int nb = (K + 63) / 64;
    const int words = cap / 64;
    const u64* Mf = mask + (size_t)f * cap * words;
    u64 rem0 = 0, rem1 = 0;  // removed bits of word `lane` and `lane + 64`
    int nk = 0;
    for (int b = 0; b < nb; ++b) {
        const int row = b * 64 + lane;
        const u64 diag = row < K ? Mf[(size_t)row * words + b] : 0ull;
        u64 remb = shfl64(b < 64 ? rem0 : rem1, b & 63);
        u64 kept = 0;
        const int lim = min(64, K - b * 64);
        for (int i = 0; i < lim; ++i) {
            const u64 di = shfl64(diag, i);
            if (!((remb >> i) & 1ull)) {
                kept |= 1ull << i;
                remb |= di;
            }
        }
        if ((kept >> lane) & 1ull) keep[(size_t)f * cap + nk + __popcll(kept & ((1ull << lane) - 1ull))] = row;
        nk += __popcll(kept);
        u64 k2 = kept;
        while (k2) {
            const int i = __ffsll((long long)k2) - 1;
            k2 &= k2 - 1;
            const u64* mr = Mf + (size_t)(b * 64 + i) * words;
            if (lane > b && lane < nb) rem0 |= mr[lane];
            if (lane + 64 > b && lane + 64 < nb) rem1 |= mr[lane + 64];
        }
    }
    if (lane == 0) nkeep[f] = nk;
}

hipError_t launch_nms(const float* sboxes, const int* kcount, int cap, float thr, u64* mask, int* keep, int* nkeep,
                      int n, hipStream_t s) {
    const int gx = (cap + 63) / 64 < 32 ? (cap + 63) / 64 : 32;
    nms_mask_kernel<<<dim3(gx, n), 256, 0, s>>>(sboxes, kcount, cap, thr, mask);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    nms_scan_kernel<<<n, 64, 0, s>>>(mask, kcount, cap, keep, nkeep);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Emit the kept detections: box, margin, score, index, and the L2-normalised
// embedding at the anchor's cell (one wave per detection).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void emit_kernel(EmitArgs a) {
    const int f = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int nk = a.nkeep[f];
    const int* g = a.geom + f * kGeomInts;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.count[f] = nk;
        a.n_cand[f] = a.cand_count[f];
        a.overflow[f] = a.cand_count[f] > a.cap ? 1 : 0;
    }
    for (int k = blockIdx.x * 4 + (threadIdx.x >> 6); k < nk; k += gridDim.x * 4) {
        const int p = a.keep[(size_t)f * a.cap + k];
        const u64 key = a.keys[(size_t)f * a.keycap + p];
        const unsigned idx = (unsigned)key;
        const size_t r = (size_t)f * a.cap + k;
        const AnchorLoc L = locate(idx, g, a.A);
        if (a.work) {
            // deferred embedding: queue (row, frame, cell) for the sparse emb conv
            if (lane == 0) {
                const int q = atomicAdd(a.work_count + L.s, 1);
                int* w = a.work + ((size_t)L.s * a.work_cap + q) * 3;
                w[0] = (int)r;
                w[1] = f;
                w[2] = L.cell;
            }
        } else {
            const float* e = a.emb[L.s] + ((size_t)g[2 + 3 + L.s] + L.cell) * a.E;
            float ss = 0.f;
            for (int c = lane; c < a.E; c += 64) {
                const float v = e[c];
                ss = __builtin_fmaf(v, v, ss);
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
            const float inv = 1.0f / fmaxf(sqrtf(ss), 1e-12f);
            float* eo = a.emb_out + r * a.E;
            for (int c = lane; c < a.E; c += 64) eo[c] = e[c] * inv;
        }
        if (lane == 0) {
            const float m = key_margin(key);
            *(float4*)(a.boxes + r * 4) = *(const float4*)(a.sboxes + ((size_t)f * a.cap + p) * 4);
            a.margins[r] = m;
            a.scores[r] = 1.0f / (1.0f + __expf(-m));
            a.anchor_idx[r] = (int)idx;
        }
    }
}

hipError_t launch_emit(const EmitArgs& a, int n, hipStream_t s) {
    const int gx = (a.cap + 3) / 4 < 64 ? (a.cap + 3) / 4 : 64;
    emit_kernel<<<dim3(gx, n), 256, 0, s>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Deferred sparse embedding head: the emb 3x3 conv (F -> E, linear + bias) of a
// head runs only at the cells of kept detections, after NMS, on the head's
// feature map (kept in the workspace since the forward).
//   emit (sparse mode) appends each kept detection to its scale's work list:
//     (output row f * cap + k, frame f, cell);
//   sparse_emb_kernel: a GEMM on the matrix cores per scale, D = detections x
//     E outputs, K = 9F in the dense conv's (tap, channel) order: one workgroup
//     (4 waves) per 32 detections x 64 outputs; each 128-wide K chunk of the
//     detections' 3x3 neighbourhoods (gathered from the NHWC map, zero outside
//     the frame) and of the conv's own weight rows [E][K] goes through LDS,
//     the next two chunks loading into registers while one is computed (the
//     loop is latency-bound: a handful of workgroups per scale walk K); the
//     MFMAs run in the dense conv's k order, so the rows equal the dense map's
//     bitwise; FP32 accumulation, bias added, raw rows written;
//   emb_normalize_kernel: L2-normalises each row in place (one wave per row).
// ---------------------------------------------------------------------------
template <typename T> struct EmbV;
template <> struct EmbV<float> { typedef f32x4 type; };
template <> struct EmbV<bf16> { typedef bf16x8 type; };
template <> struct EmbV<f16> { typedef f16x8 type; };

constexpr int kEmbDets = 32, kEmbOuts = 64, kEmbBK = 128;

template <typename T>
__global__ __launch_bounds__(256) void sparse_emb_kernel(SparseEmbArgs a) {
    typedef typename EmbV<T>::type V;
    constexpr int VEC = 16 / sizeof(T);                       // elements per 16-byte load
    constexpr int LDR = kEmbBK + (sizeof(T) == 4 ? VEC : 2 * VEC);  // padded LDS row (elements)
    constexpr int SEG = kEmbBK / VEC;                         // 16-byte segments per row and chunk
    constexpr int AV = kEmbOuts * SEG / 256;                  // weight loads per thread per chunk
    constexpr int BVT = kEmbDets * SEG / 256;                 // gather loads per thread per chunk
    static_assert(AV >= 1 && BVT >= 1, "tile");
    __shared__ __align__(16) T sA[2][kEmbOuts * LDR];
    __shared__ __align__(16) T sB[2][kEmbDets * LDR];
    __shared__ int s_row[kEmbDets], s_pix[kEmbDets], s_i[kEmbDets], s_j[kEmbDets], s_h[kEmbDets], s_w[kEmbDets];
    const int sc = blockIdx.z;
    const int cnt = a.count[sc];
    const int F = a.F[sc], E = a.E;
    const int K = 9 * F;
    const int o0 = blockIdx.y * kEmbOuts;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const T* X = (const T*)a.feat[sc];
    const T* W = (const T*)a.w[sc];
    const int* wl = a.work + (size_t)sc * a.work_cap * 3;
    const int nk = (K + kEmbBK - 1) / kEmbBK;
    for (int tile = blockIdx.x; tile * kEmbDets < cnt; tile += gridDim.x) {
        __syncthreads();
        if (tid < kEmbDets) {
            const int q = tile * kEmbDets + tid;
            if (q < cnt) {
                const int f = wl[3 * q + 1], cell = wl[3 * q + 2];
                const int* gm = a.geom + f * kGeomInts;
                const int lvl = 3 + sc;
                const int w = gm[1] >> lvl;
                s_row[tid] = wl[3 * q];
                s_pix[tid] = gm[2 + lvl];
                s_i[tid] = cell / w;
                s_j[tid] = cell - (cell / w) * w;
                s_h[tid] = gm[0] >> lvl;
                s_w[tid] = w;
            } else {
                s_row[tid] = -1;
            }
        }
        __syncthreads();
        // chunk kc: weight rows o0 .. o0+63 and the 32 detections' gathered rows, k in [kc*128, +128)
        auto load = [&](int kc, V* ar, V* br) {
            const int k0 = kc * kEmbBK;
#pragma unroll
            for (int q = 0; q < AV; ++q) {
                const int v = tid + q * 256;
                const int r = v / SEG, sg = v % SEG;
                const int k = k0 + sg * VEC;
                ar[q] = (o0 + r < E && k < K) ? *(const V*)(W + (size_t)(o0 + r) * K + k) : V{};
            }
#pragma unroll
            for (int q = 0; q < BVT; ++q) {
                const int v = tid + q * 256;
                const int d = v / SEG, sg = v % SEG;
                const int k = k0 + sg * VEC;
                V x{};
                if (s_row[d] >= 0 && k < K) {
                    const int tap = k / F, c = k - tap * F;     // a 16-byte segment never straddles a tap
                    const int y = s_i[d] + tap / 3 - 1, xx = s_j[d] + (tap - (tap / 3) * 3) - 1;
                    if (y >= 0 && y < s_h[d] && xx >= 0 && xx < s_w[d])
                        x = *(const V*)(X + ((size_t)s_pix[d] + (size_t)y * s_w[d] + xx) * F + c);
                }
                br[q] = x;
            }
        };
        auto store = [&](int buf, const V* ar, const V* br) {
#pragma unroll
            for (int q = 0; q < AV; ++q) {
                const int v = tid + q * 256;
                *(V*)(&sA[buf][(v / SEG) * LDR + (v % SEG) * VEC]) = ar[q];
            }
#pragma unroll
            for (int q = 0; q < BVT; ++q) {
                const int v = tid + q * 256;
                *(V*)(&sB[buf][(v / SEG) * LDR + (v % SEG) * VEC]) = br[q];
            }
        };
        // each wave: outputs o0 + 16 wave .. +15 x the 32 detections (2 blocks of 16)
        f32x4 acc[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
        const int arow = wave * 16 + (lane & 15), brow = lane & 15;
        const int kofs = (lane >> 4) * VEC;
        auto compute = [&](int buf, int kc) {
            const int kend = K - kc * kEmbBK < kEmbBK ? K - kc * kEmbBK : kEmbBK;
#pragma unroll
            for (int kk = 0; kk < kEmbBK; kk += 4 * VEC) {
                if (kk >= kend) break;
                const V af = *(const V*)(&sA[buf][arow * LDR + kk + kofs]);
                V bf_[2];
#pragma unroll
                for (int j = 0; j < 2; ++j) bf_[j] = *(const V*)(&sB[buf][(brow + 16 * j) * LDR + kk + kofs]);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    if constexpr (sizeof(T) == 4) {
#pragma unroll
                        for (int t = 0; t < 4; ++t)
                            acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[t], bf_[j][t], acc[j], 0, 0, 0);
                    } else if constexpr (__is_same(T, bf16)) {
                        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf_[j], acc[j], 0, 0, 0);
                    } else {
                        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(af, bf_[j], acc[j], 0, 0, 0);
                    }
                }
            }
        };
        // two register sets: chunks kc + 1 and kc + 2 are in flight while kc is computed
        V ra[2][AV], rb[2][BVT];
        load(0, ra[0], rb[0]);
        if (nk > 1) load(1, ra[1], rb[1]);
        store(0, ra[0], rb[0]);
        if (nk > 2) load(2, ra[0], rb[0]);
        __syncthreads();
        auto iter = [&](int kc, auto cur_c) {
            constexpr int cur = decltype(cur_c)::value;
            if (kc + 1 < nk) store(cur ^ 1, ra[cur ^ 1], rb[cur ^ 1]);
            if (kc + 3 < nk) load(kc + 3, ra[cur ^ 1], rb[cur ^ 1]);
            compute(cur, kc);
            __syncthreads();
        };
        int kc = 0;
        for (; kc + 1 < nk; kc += 2) {
            iter(kc, std::integral_constant<int, 0>{});
            iter(kc + 1, std::integral_constant<int, 1>{});
        }
        if (kc < nk) iter(kc, std::integral_constant<int, 0>{});
        // lane l of detection block j: outputs 4 (l / 16) + e of the wave's 16, detection l % 16 of block j
        const int o = o0 + wave * 16 + 4 * (lane >> 4);
        if (o < E) {                    // E is a multiple of 64: a lane's 4 outputs are all in or all out
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int r = s_row[16 * j + (lane & 15)];
                if (r < 0) continue;
                float4 v;
                v.x = acc[j][0] + a.bias[sc][o];
                v.y = acc[j][1] + a.bias[sc][o + 1];
                v.z = acc[j][2] + a.bias[sc][o + 2];
                v.w = acc[j][3] + a.bias[sc][o + 3];
                *(float4*)(a.out + (size_t)r * E + o) = v;
            }
        }
    }
}

__global__ __launch_bounds__(256) void emb_normalize_kernel(float* emb, const int* nkeep, int cap, int E) {
    const int f = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int nk = nkeep[f];
    for (int k = blockIdx.x * 4 + (threadIdx.x >> 6); k < nk; k += gridDim.x * 4) {
        float* e = emb + ((size_t)f * cap + k) * E;
        float ss = 0.f;
        for (int c = lane; c < E; c += 64) ss = __builtin_fmaf(e[c], e[c], ss);
#pragma unroll
        for (int q = 32; q > 0; q >>= 1) ss += __shfl_xor(ss, q);
        const float inv = 1.0f / fmaxf(sqrtf(ss), 1e-12f);
        for (int c = lane; c < E; c += 64) e[c] = e[c] * inv;
    }
}

hipError_t launch_sparse_emb(const SparseEmbArgs& a, int et, int n, int cap, const int* nkeep, hipStream_t s) {
    const int max_tiles = (n * cap + kEmbDets - 1) / kEmbDets;
    dim3 grid(max_tiles < 64 ? max_tiles : 64, (a.E + kEmbOuts - 1) / kEmbOuts, 3);
    if (et == kF32) sparse_emb_kernel<float><<<grid, 256, 0, s>>>(a);
    else if (et == kF16) sparse_emb_kernel<f16><<<grid, 256, 0, s>>>(a);
    else sparse_emb_kernel<bf16><<<grid, 256, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int gx = (cap + 3) / 4 < 64 ? (cap + 3) / 4 : 64;
    emb_normalize_kernel<<<dim3(gx, n), 256, 0, s>>>(a.out, nkeep, cap, a.E);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Standalone NMS (one list): keys/values from the inputs, gather, unmap.
// ---------------------------------------------------------------------------
__global__ void nms_prepare_kernel(const float* margins, const int* idx, int K, u64* keys, int* vals, int* count) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) *count = K;
    if (p < K) {
        keys[p] = make_key(margins[p] + 0.0f, (unsigned)idx[p]);
        vals[p] = p;
    }
}
hipError_t launch_nms_prepare(const float* boxes, const float* margins, const int* idx, int K, u64* keys, int* vals,
                              int* count, hipStream_t s) {
    (void)boxes;
    nms_prepare_kernel<<<(K + 255) / 256 + (K == 0), 256, 0, s>>>(margins, idx, K, keys, vals, count);
    return hipGetLastError();
}

__global__ void nms_gather_kernel(const float* boxes, const int* vals, int K, float* sboxes, int* kcount) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) *kcount = K;
    if (q < K) *(float4*)(sboxes + (size_t)q * 4) = *(const float4*)(boxes + (size_t)vals[q] * 4);
}
hipError_t launch_nms_gather(const float* boxes, const u64* keys, const int* vals, int K, float* sboxes, int* kcount,
                             hipStream_t s) {
    (void)keys;
    nms_gather_kernel<<<(K + 255) / 256 + (K == 0), 256, 0, s>>>(boxes, vals, K, sboxes, kcount);
    return hipGetLastError();
}

__global__ void nms_finish_kernel(const int* keep, const int* nkeep, const int* vals, int* out_keep, int* out_nkeep) {
    const int n = *nkeep;
    for (int k = threadIdx.x; k < n; k += blockDim.x) out_keep[k] = vals[keep[k]];
    if (threadIdx.x == 0) *out_nkeep = n;
}
hipError_t launch_nms_finish(const int* keep, const int* nkeep, const int* vals, int* out_keep, int* out_nkeep, int K,
                             hipStream_t s) {
    (void)K;
    nms_finish_kernel<<<1, 256, 0, s>>>(keep, nkeep, vals, out_keep, out_nkeep);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cost matrix: 32 tracks x 32 detections per workgroup.  The FP32 dot products
// of the embeddings are staged through LDS in 64-wide chunks; each track's
// innovation covariance S = P[0:4,0:4] + R(h) is factored once per workgroup
// in FP64 (Cholesky), each pair's gate distance is an FP64 forward solve.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void cost_kernel(const float* __restrict__ fe, const double* __restrict__ mean,
                                                   const double* __restrict__ cov, int T,
                                                   const float* __restrict__ boxes, const float* __restrict__ de,
                                                   int D, const int* __restrict__ dcount, int ldc, int E,
                                                   double gate, float* __restrict__ cost,
                                                   CostBatch batch, float motion_w) {
    __shared__ float sf[32][65], se[32][65];
    __shared__ double sL[32][10], sHx[32][4], sZ[32][4];
    __shared__ int sPD[32];
    const int tid = threadIdx.x;
    const int t0 = blockIdx.y * 32, d0 = blockIdx.x * 32;
    if (batch.n) {
        // frame blockIdx.z: tracks [tb[z], tb[z+1]), detections at rows z*ldc of the dets, cost rows from tb[z]
        const int z = blockIdx.z;
        const int tb = batch.begin[z];
        T = batch.begin[z + 1] - tb;
        fe += (size_t)tb * E;
        mean += (size_t)tb * 8;
        cov += (size_t)tb * 64;
        cost += (size_t)tb * ldc;
        boxes += (size_t)z * ldc * 4;
        de += (size_t)z * ldc * E;
        dcount += z;
        if (t0 >= T) return;
    }
    if (dcount) {
        const int dn = *dcount;
        D = dn < D ? dn : D;
    }
    if (d0 >= D) return;
    if (tid < 32) {
        const int t = t0 + tid;
        if (t < T) {
            const double* m = mean + (size_t)t * 8;
            const double* P = cov + (size_t)t * 64;
            const double h = m[3];
            const double sp = h / 20.0;
            const double r[4] = {sp * sp, sp * sp, 0.1 * 0.1, sp * sp};
            double S[4][4];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) S[i][j] = P[i * 8 + j] + (i == j ? r[i] : 0.0);
            // Cholesky S = L L^T (lower), packed row-wise: L00, L10, L11, L20, L21, L22, L30..L33.
            double L[4][4] = {};
            int pd = 1;
            for (int i = 0; i < 4; ++i) {
                for (int j = 0; j <= i; ++j) {
                    double acc = S[i][j];
                    for (int k = 0; k < j; ++k) acc -= L[i][k] * L[j][k];
                    if (i == j) {
                        if (!(acc > 0.0)) pd = 0;
                        L[i][i] = sqrt(acc > 0.0 ? acc : 1.0);
                    } else {
                        L[i][j] = acc / L[j][j];
                    }
                }
            }
            int q = 0;
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j <= i; ++j) sL[tid][q++] = L[i][j];
            for (int i = 0; i < 4; ++i) sHx[tid][i] = m[i];
            sPD[tid] = pd;
        }
    } else if (tid < 64) {
        const int d = d0 + tid - 32;
        if (d < D) {
            const float* b = boxes + (size_t)d * 4;
            const double x1 = b[0], y1 = b[1], x2 = b[2], y2 = b[3];
            const double w = x2 - x1, h = y2 - y1;
            sZ[tid - 32][0] = (x1 + x2) / 2.0;
            sZ[tid - 32][1] = (y1 + y2) / 2.0;
            sZ[tid - 32][2] = w / h;
            sZ[tid - 32][3] = h;
        }
    }
    const int ty = tid >> 4, tx = tid & 15;  // rows ty*2 + {0,1}, cols tx*2 + {0,1}
    float acc[2][2] = {{0.f, 0.f}, {0.f, 0.f}};
    // 64-wide slices of the embeddings: all loads of a slice in flight at once, the
    // next slice loading while the current one is reduced
    float rf[8], re[8];
    auto fetch = [&](int e0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int v = tid + k * 256;
            const int r = v >> 6, c = v & 63;
            const int t = t0 + r, d = d0 + r, e = e0 + c;
            rf[k] = (t < T && e < E) ? fe[(size_t)t * E + e] : 0.f;
            re[k] = (d < D && e < E) ? de[(size_t)d * E + e] : 0.f;
        }
    };
    fetch(0);
    for (int e0 = 0; e0 < E; e0 += 64) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int v = tid + k * 256;
            sf[v >> 6][v & 63] = rf[k];
            se[v >> 6][v & 63] = re[k];
        }
        __syncthreads();
        if (e0 + 64 < E) fetch(e0 + 64);
#pragma unroll 8
        for (int c = 0; c < 64; ++c) {
            const float f0 = sf[ty * 2][c], f1 = sf[ty * 2 + 1][c];
            const float g0 = se[tx * 2][c], g1 = se[tx * 2 + 1][c];
            acc[0][0] = __builtin_fmaf(f0, g0, acc[0][0]);
            acc[0][1] = __builtin_fmaf(f0, g1, acc[0][1]);
            acc[1][0] = __builtin_fmaf(f1, g0, acc[1][0]);
            acc[1][1] = __builtin_fmaf(f1, g1, acc[1][1]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int tl = ty * 2 + i, dl = tx * 2 + j;
            const int t = t0 + tl, d = d0 + dl;
            if (t >= T || d >= D) continue;
            const double* L = sL[tl];
            const double y0 = sZ[dl][0] - sHx[tl][0], y1 = sZ[dl][1] - sHx[tl][1];
            const double y2 = sZ[dl][2] - sHx[tl][2], y3 = sZ[dl][3] - sHx[tl][3];
            const double u0 = y0 / L[0];
            const double u1 = (y1 - L[1] * u0) / L[2];
            const double u2 = (y2 - L[3] * u0 - L[4] * u1) / L[5];
            const double u3 = (y3 - L[6] * u0 - L[7] * u1 - L[8] * u2) / L[9];
            const double d2 = u0 * u0 + u1 * u1 + u2 * u2 + u3 * u3;
            float c = fminf(fmaxf(1.0f - acc[i][j], 0.f), 2.f);
            // motion-fused variant: (1 - w) cos + w d2, in FP64
            if (motion_w != 0.f) c = (float)((1.0 - (double)motion_w) * (double)c + (double)motion_w * d2);
            if (!sPD[tl] || !(d2 <= gate)) c = __builtin_inff();
            cost[(size_t)t * ldc + d] = c;
        }
}

hipError_t launch_cost(const float* trk_emb, const double* mean, const double* cov, int T, const float* det_boxes,
                       const float* det_emb, int D, const int* dcount, int ldc, int E, double gate, float* cost,
                       hipStream_t s) {
    if (T == 0 || D == 0) return hipSuccess;
    dim3 grid((D + 31) / 32, (T + 31) / 32);
    CostBatch none{};
    cost_kernel<<<grid, 256, 0, s>>>(trk_emb, mean, cov, T, det_boxes, det_emb, D, dcount, ldc, E, gate, cost, none,
                                     0.f);
    return hipGetLastError();
}

hipError_t launch_cost_batch(const float* trk_emb, const double* mean, const double* cov, const CostBatch& b,
                             int max_t, const float* det_boxes, const float* det_emb, const int* dcount, int cap,
                             int E, double gate, float* cost, hipStream_t s, float motion_w) {
    if (b.n == 0 || max_t == 0) return hipSuccess;
    dim3 grid((cap + 31) / 32, (max_t + 31) / 32, b.n);
    cost_kernel<<<grid, 256, 0, s>>>(trk_emb, mean, cov, 0, det_boxes, det_emb, cap, dcount, cap, E, gate, cost, b,
                                     motion_w);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Box-overlap cost of a second association stage: C[t, d] = 1 - IoU(track t's
// predicted box, detection d) in FP64, the track box from its Kalman state
// (cx, cy, a, h): w = a h.  One thread per (track, detection), frame on z.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void iou_cost_kernel(const double* __restrict__ mean, CostBatch b,
                                                       const float* __restrict__ boxes,
                                                       const int* __restrict__ dcount, int cap,
                                                       float* __restrict__ cost) {
    const int f = blockIdx.z;
    const int t = b.begin[f] + blockIdx.y;
    if (t >= b.begin[f + 1]) return;
    int D = dcount[f];
    D = D < cap ? D : cap;
    const double* m = mean + (size_t)t * 8;
    const double w = m[2] * m[3], h = m[3];
    const double ax1 = m[0] - w / 2, ay1 = m[1] - h / 2, ax2 = m[0] + w / 2, ay2 = m[1] + h / 2;
    const double area_a = (ax2 - ax1) * (ay2 - ay1);
    for (int d = blockIdx.x * 256 + threadIdx.x; d < D; d += gridDim.x * 256) {
        const float* bx = boxes + ((size_t)f * cap + d) * 4;
        const double bx1 = bx[0], by1 = bx[1], bx2 = bx[2], by2 = bx[3];
        const double iw = fmax(0.0, fmin(ax2, bx2) - fmax(ax1, bx1));
        const double ih = fmax(0.0, fmin(ay2, by2) - fmax(ay1, by1));
        const double inter = iw * ih;
        const double uni = area_a + (bx2 - bx1) * (by2 - by1) - inter;
        const double iou = uni > 0.0 ? inter / uni : 0.0;
        cost[(size_t)t * cap + d] = (float)(1.0 - iou);
    }
}

hipError_t launch_iou_cost(const double* mean, const CostBatch& b, int max_t, const float* boxes, const int* dcount,
                           int cap, float* cost, hipStream_t s) {
    if (b.n == 0 || max_t == 0) return hipSuccess;
    dim3 grid((cap + 255) / 256 < 8 ? (cap + 255) / 256 : 8, max_t, b.n);
    iou_cost_kernel<<<grid, 256, 0, s>>>(mean, b, boxes, dcount, cap, cost);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Track embedding smoothing f_t <- normalise(m f_t + (1 - m) e_d), one wave per pair.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void emb_update_kernel(const int* pairs, int P, const float* de, int D, float* fe,
                                                         int T, int E, float mom) {
    const int lane = threadIdx.x & 63;
    for (int p = blockIdx.x * 4 + (threadIdx.x >> 6); p < P; p += gridDim.x * 4) {
        const int t = pairs[2 * p], d = pairs[2 * p + 1];
        if (t < 0 || t >= T || d < 0 || d >= D) continue;
        float* f = fe + (size_t)t * E;
        const float* e = de + (size_t)d * E;
        float ss = 0.f;
        for (int c = lane; c < E; c += 64) {
            const float v = mom * f[c] + (1.0f - mom) * e[c];
            ss = __builtin_fmaf(v, v, ss);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
        const float inv = 1.0f / fmaxf(sqrtf(ss), 1e-12f);
        for (int c = lane; c < E; c += 64) f[c] = (mom * f[c] + (1.0f - mom) * e[c]) * inv;
    }
}

hipError_t launch_emb_update(const int* pairs, int P, const float* det_emb, int D, float* trk_emb, int T, int E,
                             float momentum, hipStream_t s) {
    if (P == 0) return hipSuccess;
    const int gx = (P + 3) / 4 < 256 ? (P + 3) / 4 : 256;
    emb_update_kernel<<<gx, 256, 0, s>>>(pairs, P, det_emb, D, trk_emb, T, E, momentum);
    return hipGetLastError();
}

}  // namespace jde
