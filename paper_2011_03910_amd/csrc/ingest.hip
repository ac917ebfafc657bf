// Frame ingest: 8-bit RGB video frames (e.g. FullHD from the capture stage)
// -> the model's NCHW FP32 input in [0, 1] at the batch's frame sizes, in one
// pass: letterbox (aspect-preserving scale, centred, border 0.5), bilinear
// resampling with aligned pixel centres, /255, HWC -> CHW.
//
// Source coordinates are exact: output column u of the resized image samples
// s = ((2u + 1) W_in - new_w) / (2 new_w), computed as an integer quotient and
// remainder, so the interpolation weights are the exact fractions rounded once.
#include "jde_internal.h"

namespace jde {

__device__ __forceinline__ void ingest_coord(int t, int n_out, int n_in, int& i0, int& i1, float& frac) {
    const long long num = (long long)(2 * t + 1) * n_in - n_out;
    const long long den = 2LL * n_out;
    if (num <= 0) {
        i0 = 0;
        frac = 0.f;
    } else {
        long long q = num / den;
        long long r = num - q * den;
        if (q >= n_in - 1) {
            q = n_in - 1;
            r = 0;
        }
        i0 = (int)q;
        frac = (float)r / (float)den;
    }
    i1 = i0 + 1 < n_in ? i0 + 1 : n_in - 1;
}

__global__ __launch_bounds__(256) void ingest_kernel(IngestArgs a) {
    const int f = blockIdx.y;
    const IngestFrame& g = a.fr[f];
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= g.h * g.w) return;
    const int y = p / g.w, x = p - (p / g.w) * g.w;
    float* dst = a.dst + g.dst_off;
    const size_t plane = (size_t)g.h * g.w;
    const int u = x - g.left, v = y - g.top;
    if (u < 0 || u >= g.new_w || v < 0 || v >= g.new_h) {
        dst[p] = 0.5f;
        dst[plane + p] = 0.5f;
        dst[2 * plane + p] = 0.5f;
        return;
    }
    int x0, x1, y0, y1;
    float fx, fy;
    ingest_coord(u, g.new_w, a.src_w, x0, x1, fx);
    ingest_coord(v, g.new_h, a.src_h, y0, y1, fy);
    const unsigned char* src = a.src + (size_t)f * a.src_h * a.src_w * 3;
    const unsigned char* r0 = src + (size_t)y0 * a.src_w * 3;
    const unsigned char* r1 = src + (size_t)y1 * a.src_w * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float p00 = r0[x0 * 3 + c], p01 = r0[x1 * 3 + c];
        const float p10 = r1[x0 * 3 + c], p11 = r1[x1 * 3 + c];
        const float top = p00 * (1.f - fx) + p01 * fx;
        const float bot = p10 * (1.f - fx) + p11 * fx;
        dst[c * plane + p] = (top * (1.f - fy) + bot * fy) / 255.f;
    }
}

hipError_t launch_ingest(const IngestArgs& a, int max_pix, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    ingest_kernel<<<dim3((max_pix + 255) / 256, a.n), 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace jde
