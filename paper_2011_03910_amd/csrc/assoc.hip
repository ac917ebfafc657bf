// Device-side association (Appendix A items 4 and 7): Kalman predict and update
// of the tracks' 8-d constant-velocity state in FP64, and the min-cost
// assignment of every frame of a batch, one workgroup per frame.
//
// The arithmetic follows the host FP64 code of host_track.cpp operation for
// operation, with floating-point contraction off, so the device and the host
// give bit-identical states and the same assignment.
#include "jde_internal.h"

namespace jde {

constexpr double kStdPosD = 1.0 / 20.0;
constexpr double kStdVelD = 1.0 / 160.0;

// ---------------------------------------------------------------------------
// Kalman predict: x <- F x, P <- F P F^T + Q(h), F = [[I, I], [0, I]]; one
// thread per track.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(128) void kf_predict_kernel(int T, double* __restrict__ mean, double* __restrict__ cov) {
#pragma clang fp contract(off)
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double* m = mean + (size_t)t * 8;
    double* Pg = cov + (size_t)t * 64;
    double P[64];
    for (int i = 0; i < 64; ++i) P[i] = Pg[i];
    const double h = m[3];
    const double sd[8] = {kStdPosD * h, kStdPosD * h, 1e-2, kStdPosD * h,
                          kStdVelD * h, kStdVelD * h, 1e-5, kStdVelD * h};
    for (int i = 0; i < 4; ++i) m[i] = m[i] + m[4 + i];
    // rows i < 4 take row i + 4, then columns j < 4 take column j + 4
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 8; ++j) P[i * 8 + j] = P[i * 8 + j] + P[(i + 4) * 8 + j];
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 4; ++j) P[i * 8 + j] = P[i * 8 + j] + P[i * 8 + j + 4];
    for (int i = 0; i < 8; ++i) P[i * 8 + i] = P[i * 8 + i] + sd[i] * sd[i];
    for (int i = 0; i < 64; ++i) Pg[i] = P[i];
}

hipError_t launch_kf_predict(int T, double* mean, double* cov, hipStream_t s) {
    if (T <= 0) return hipSuccess;
    kf_predict_kernel<<<(T + 127) / 128, 128, 0, s>>>(T, mean, cov);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Kalman update of each track with its assigned detection: z = (cx, cy, w/h, h)
// of the detection box, S = H P H^T + R(h), Cholesky, K^T = S^-1 H P, x += K y,
// Joseph form P = (I - K H) P (I - K H)^T + K R K^T, symmetrised.  Track t of
// frame f (rows [tb[f], tb[f+1])) takes box f * cap + det_of_track[t]; tracks
// with det_of_track < 0 are left as they are.  status[t] = 1 if S was not
// positive definite (track unchanged), else 0.
// ---------------------------------------------------------------------------
__device__ bool chol4_dev(const double S[4][4], double L[4][4]) {
#pragma clang fp contract(off)
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) L[i][j] = 0.0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j <= i; ++j) {
            double acc = S[i][j];
            for (int k = 0; k < j; ++k) acc = acc - L[i][k] * L[j][k];
            if (i == j) {
                if (!(acc > 0.0)) return false;
                L[i][i] = sqrt(acc);
            } else {
                L[i][j] = acc / L[j][j];
            }
        }
    return true;
}

__device__ void chol4_solve_dev(const double L[4][4], const double b[4], double x[4]) {
#pragma clang fp contract(off)
    double y[4];
    for (int i = 0; i < 4; ++i) {
        double acc = b[i];
        for (int k = 0; k < i; ++k) acc = acc - L[i][k] * y[k];
        y[i] = acc / L[i][i];
    }
    for (int i = 3; i >= 0; --i) {
        double acc = y[i];
        for (int k = i + 1; k < 4; ++k) acc = acc - L[k][i] * x[k];
        x[i] = acc / L[i][i];
    }
}

__global__ __launch_bounds__(64) void kf_update_kernel(AssocBatch b, const int* __restrict__ det_of_track,
                                                       const float* __restrict__ boxes, int cap,
                                                       double* __restrict__ mean, double* __restrict__ cov,
                                                       int* __restrict__ status) {
#pragma clang fp contract(off)
    const int f = blockIdx.y;
    const int t = b.begin[f] + blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= b.begin[f + 1]) return;
    const int d = det_of_track[t];
    if (status) status[t] = 0;
    if (d < 0) return;
    const float* bx = boxes + ((size_t)f * cap + d) * 4;
    double z[4];
    {
        const double x1 = bx[0], y1 = bx[1], x2 = bx[2], y2 = bx[3];
        const double w = x2 - x1, h = y2 - y1;
        z[0] = (x1 + x2) / 2.0;
        z[1] = (y1 + y2) / 2.0;
        z[2] = w / h;
        z[3] = h;
    }
    double* mg = mean + (size_t)t * 8;
    double* Pg = cov + (size_t)t * 64;
    double m[8], P[64];
    for (int i = 0; i < 8; ++i) m[i] = mg[i];
    for (int i = 0; i < 64; ++i) P[i] = Pg[i];
    const double h = m[3];
    const double r[4] = {kStdPosD * h * kStdPosD * h, kStdPosD * h * kStdPosD * h, 1e-2,
                         kStdPosD * h * kStdPosD * h};
    double S[4][4], L[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) S[i][j] = P[i * 8 + j] + (i == j ? r[i] : 0.0);
    if (!chol4_dev(S, L)) {
        if (status) status[t] = 1;
        return;
    }
    double K[8][4];
    for (int c = 0; c < 8; ++c) {
        const double bb[4] = {P[0 * 8 + c], P[1 * 8 + c], P[2 * 8 + c], P[3 * 8 + c]};
        double x[4];
        chol4_solve_dev(L, bb, x);
        for (int i = 0; i < 4; ++i) K[c][i] = x[i];
    }
    double y[4];
    for (int i = 0; i < 4; ++i) y[i] = z[i] - m[i];
    for (int i = 0; i < 8; ++i) {
        double acc = 0.0;
        for (int j = 0; j < 4; ++j) acc = acc + K[i][j] * y[j];
        m[i] = m[i] + acc;
    }
    double A[8][8];
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) A[i][j] = (i == j ? 1.0 : 0.0) - (j < 4 ? K[i][j] : 0.0);
    double AP[8][8];
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 8; ++k) acc = acc + A[i][k] * P[k * 8 + j];
            AP[i][j] = acc;
        }
    double Pn[8][8];
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 8; ++k) acc = acc + AP[i][k] * A[j][k];
            for (int k = 0; k < 4; ++k) acc = acc + K[i][k] * r[k] * K[j][k];
            Pn[i][j] = acc;
        }
    for (int i = 0; i < 8; ++i) mg[i] = m[i];
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) Pg[i * 8 + j] = 0.5 * (Pn[i][j] + Pn[j][i]);
}

hipError_t launch_kf_update(const AssocBatch& b, int max_t, const int* det_of_track, const float* boxes, int cap,
                            double* mean, double* cov, int* status, hipStream_t s) {
    if (b.n == 0 || max_t == 0) return hipSuccess;
    kf_update_kernel<<<dim3((max_t + 63) / 64, b.n), 64, 0, s>>>(b, det_of_track, boxes, cap, mean, cov, status);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Min-cost assignment per frame (one workgroup each): the shortest augmenting
// path method with row and column potentials (Kuhn-Munkres in the
// Jonker-Volgenant form), on the rows and columns that have at least one
// allowed entry (cost <= max_cost), oriented so that rows <= columns, with
// forbidden entries priced above any feasible total.  Rows are added one at a
// time; each step of a row's search relaxes every unused column in parallel
// and picks the smallest reduced cost by a block reduction (ties to the lowest
// column, as the sequential method scans), so the device takes exactly the
// host's steps.  All state lives in LDS: rows + columns <= kAssignMax each.
// ---------------------------------------------------------------------------
constexpr int kAssignThreads = 256;

struct AssignShared {
    double* u;      // [n + 1]
    double* v;      // [m + 1]
    double* minv;   // [m + 1]
    int* p;         // [m + 1]
    int* way;       // [m + 1]
    int* used;      // [m + 1]
    int* rows;      // [T]  tracks with an allowed entry
    int* cols;      // [D]  detections with an allowed entry
};

__device__ __forceinline__ void argmin_pair(double& v, int& j, double v2, int j2) {
    if (v2 < v || (v2 == v && j2 < j)) {
        v = v2;
        j = j2;
    }
}

__global__ __launch_bounds__(kAssignThreads) void assign_kernel(const float* __restrict__ cost, AssocBatch b,
                                                                const int* __restrict__ dcount, int cap, float max_cost,
                                                                int* __restrict__ det_of_track,
                                                                int* __restrict__ track_of_det,
                                                                int* __restrict__ kept_out, double* __restrict__ total_out,
                                                                int* __restrict__ status) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_n, s_m, s_tr, s_Tr, s_Dr;
    __shared__ double s_red_v[2][kAssignThreads / 64];
    __shared__ int s_red_j[2][kAssignThreads / 64];
    __shared__ double s_sum[kAssignThreads / 64];
    __shared__ int s_cnt[kAssignThreads / 64];
    const int f = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int t0 = b.begin[f];
    const int T = b.begin[f + 1] - t0;
    int D = dcount[f];
    D = D < cap ? D : cap;
    const float* C = cost + (size_t)t0 * cap;
    for (int t = tid; t < T; t += kAssignThreads) det_of_track[t0 + t] = -1;
    for (int d = tid; d < cap; d += kAssignThreads) track_of_det[(size_t)f * cap + d] = -1;
    if (tid == 0) {
        kept_out[f] = 0;
        total_out[f] = 0.0;
        status[f] = 0;
    }
    if (T == 0 || D == 0) return;
    if (T > kAssignMax || D > kAssignMax) {
        if (tid == 0) status[f] = 1;
        return;
    }
    const double mc = (double)max_cost;
    // carve LDS: sizes for the worst orientation (n, m <= max(T, D))
    const int mx = T > D ? T : D;
    AssignShared S;
    {
        unsigned char* q = smem;
        S.u = (double*)q;     q += (size_t)(mx + 1) * 8;
        S.v = (double*)q;     q += (size_t)(mx + 1) * 8;
        S.minv = (double*)q;  q += (size_t)(mx + 1) * 8;
        S.p = (int*)q;        q += (size_t)(mx + 1) * 4;
        S.way = (int*)q;      q += (size_t)(mx + 1) * 4;
        S.used = (int*)q;     q += (size_t)(mx + 1) * 4;
        S.rows = (int*)q;     q += (size_t)T * 4;
        S.cols = (int*)q;
    }
    // rows / columns with an allowed entry, in ascending order
    int* col_ok = S.used;  // scratch flags, reset before the search
    for (int d = tid; d < D; d += kAssignThreads) col_ok[d] = 0;
    int* row_ok = S.p;
    __syncthreads();
    for (int t = tid; t < T; t += kAssignThreads) {
        int any = 0;
        for (int d = 0; d < D; ++d)
            if ((double)C[(size_t)t * cap + d] <= mc) {
                any = 1;
                col_ok[d] = 1;
            }
        row_ok[t] = any;
    }
    __syncthreads();
    if (tid == 0) {
        int k = 0;
        for (int t = 0; t < T; ++t)
            if (row_ok[t]) S.rows[k++] = t;
        s_Tr = k;
        k = 0;
        for (int d = 0; d < D; ++d)
            if (col_ok[d]) S.cols[k++] = d;
        s_Dr = k;
        s_tr = s_Tr > s_Dr;
        s_n = s_tr ? s_Dr : s_Tr;
        s_m = s_tr ? s_Tr : s_Dr;
    }
    __syncthreads();
    const int n = s_n, m = s_m, tr = s_tr;
    if (s_Tr == 0) return;
    const double big = 4.0 * (double)(n + 1) * (mc > 2.0 ? mc : 2.0) + 1.0;
    auto at = [&](int i, int j) -> double {  // 0-based entry of the oriented, reduced problem
        const int t = S.rows[tr ? j : i], d = S.cols[tr ? i : j];
        const double c = (double)C[(size_t)t * cap + d];
        return c <= mc ? c : big;
    };
    for (int j = tid; j <= m; j += kAssignThreads) {
        S.v[j] = 0.0;
        S.p[j] = 0;
        S.way[j] = 0;
    }
    for (int i = tid; i <= n; i += kAssignThreads) S.u[i] = 0.0;
    __syncthreads();
    const double inf = __builtin_inf();
    for (int i = 1; i <= n; ++i) {
        for (int j = tid; j <= m; j += kAssignThreads) {
            S.minv[j] = inf;
            S.used[j] = 0;
        }
        if (tid == 0) S.p[0] = i;
        __syncthreads();
        // One barrier per step.  Column j belongs to thread j % kAssignThreads, which
        // alone reads and writes its used / minv / v / way entries; p does not change
        // during a row's search, and u[i0] of the row being relaxed was last written
        // before the row began (its column joins the tree only now), so only the
        // wave minima need the barrier.  Every thread then finishes the block
        // minimum itself (the same order of comparisons: ties to the lowest column);
        // the minima alternate between two buffers, so a wave one step ahead cannot
        // overwrite what a slower wave still reads.
        int j0 = 0, par = 0;
        while (true) {
            if (j0 % kAssignThreads == tid) S.used[j0] = 1;
            const int i0 = S.p[j0];
            const double ui = S.u[i0];
            double bv = inf;
            int bj = 0x7fffffff;
            for (int j = tid; j <= m; j += kAssignThreads) {
                if (j == 0 || S.used[j]) continue;
                const double cur = at(i0 - 1, j - 1) - ui - S.v[j];
                if (cur < S.minv[j]) {
                    S.minv[j] = cur;
                    S.way[j] = j0;
                }
                argmin_pair(bv, bj, S.minv[j], j);
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double v2 = __shfl_xor(bv, o);
                const int j2 = __shfl_xor(bj, o);
                argmin_pair(bv, bj, v2, j2);
            }
            if (lane == 0) {
                s_red_v[par][wave] = bv;
                s_red_j[par][wave] = bj;
            }
            __syncthreads();
            double delta = s_red_v[par][0];
            int j1 = s_red_j[par][0];
            for (int w = 1; w < kAssignThreads / 64; ++w) argmin_pair(delta, j1, s_red_v[par][w], s_red_j[par][w]);
            for (int j = tid; j <= m; j += kAssignThreads) {
                if (S.used[j]) {
                    S.u[S.p[j]] += delta;
                    S.v[j] -= delta;
                } else {
                    S.minv[j] -= delta;
                }
            }
            j0 = j1;
            par ^= 1;
            if (S.p[j1] == 0) break;
        }
        __syncthreads();  // every thread's last potential update reads p before the path flips it
        if (tid == 0) {
            do {
                const int j1 = S.way[j0];
                S.p[j0] = S.p[j1];
                j0 = j1;
            } while (j0);
        }
        __syncthreads();
    }
    // matched pairs that are allowed; their count and summed cost
    double sum = 0.0;
    int cnt = 0;
    for (int j = 1 + tid; j <= m; j += kAssignThreads) {
        if (!S.p[j]) continue;
        const int i = S.p[j] - 1, jj = j - 1;
        const int t = S.rows[tr ? jj : i], d = S.cols[tr ? i : jj];
        const float c = C[(size_t)t * cap + d];
        if (!((double)c <= mc)) continue;
        det_of_track[t0 + t] = d;
        track_of_det[(size_t)f * cap + d] = t;
        sum += (double)c;
        ++cnt;
    }
    for (int o = 32; o > 0; o >>= 1) {
        sum += __shfl_xor(sum, o);
        cnt += __shfl_xor(cnt, o);
    }
    if (lane == 0) {
        s_sum[wave] = sum;
        s_cnt[wave] = cnt;
    }
    __syncthreads();
    if (tid == 0) {
        double tot = 0.0;
        int k = 0;
        for (int w = 0; w < kAssignThreads / 64; ++w) {
            tot += s_sum[w];
            k += s_cnt[w];
        }
        kept_out[f] = k;
        total_out[f] = tot;
    }
}

size_t assign_lds_bytes(int mx) { return (size_t)(mx + 1) * (3 * 8 + 3 * 4) + (size_t)2 * mx * 4 + 64; }

hipError_t launch_assign(const float* cost, const AssocBatch& b, int max_dim, const int* dcount, int cap,
                         float max_cost, int* det_of_track, int* track_of_det, int* kept, double* total, int* status,
                         hipStream_t s) {
    if (b.n == 0) return hipSuccess;
    const size_t lds = assign_lds_bytes(max_dim);
    // more than the default 64 KB of dynamic LDS for the largest problems
    static const hipError_t attr = hipFuncSetAttribute((const void*)assign_kernel,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)assign_lds_bytes(kAssignMax));
    if (attr != hipSuccess) return attr;
    assign_kernel<<<b.n, kAssignThreads, lds, s>>>(cost, b, dcount, cap, max_cost, det_of_track, track_of_det, kept,
                                                    total, status);
    return hipGetLastError();
}

}  // namespace jde
