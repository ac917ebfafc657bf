// Host FP64 association steps (Appendix A items 4 and 7-9): Kalman filter on
// the 8-d constant-velocity state and the min-cost (Hungarian) assignment.
#include <math.h>
#include <string.h>

#include <limits>
#include <vector>

#include "jde.h"

namespace {

constexpr double kStdPos = 1.0 / 20.0;
constexpr double kStdVel = 1.0 / 160.0;

// Cholesky of a 4x4 SPD matrix (lower, in place in L); false if not PD.
bool chol4(const double S[4][4], double L[4][4]) {
    memset(L, 0, sizeof(double) * 16);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j <= i; ++j) {
            double acc = S[i][j];
            for (int k = 0; k < j; ++k) acc -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(acc > 0.0)) return false;
                L[i][i] = sqrt(acc);
            } else {
                L[i][j] = acc / L[j][j];
            }
        }
    return true;
}

// Solves S x = b for 4-vectors with the Cholesky factor.
void chol4_solve(const double L[4][4], const double b[4], double x[4]) {
    double y[4];
    for (int i = 0; i < 4; ++i) {
        double acc = b[i];
        for (int k = 0; k < i; ++k) acc -= L[i][k] * y[k];
        y[i] = acc / L[i][i];
    }
    for (int i = 3; i >= 0; --i) {
        double acc = y[i];
        for (int k = i + 1; k < 4; ++k) acc -= L[k][i] * x[k];
        x[i] = acc / L[i][i];
    }
}

}  // namespace

extern "C" {

void jde_box_to_z(int n, const float* boxes, double* z) {
    for (int i = 0; i < n; ++i) {
        const double x1 = boxes[4 * i], y1 = boxes[4 * i + 1], x2 = boxes[4 * i + 2], y2 = boxes[4 * i + 3];
        const double w = x2 - x1, h = y2 - y1;
        z[4 * i] = (x1 + x2) / 2.0;
        z[4 * i + 1] = (y1 + y2) / 2.0;
        z[4 * i + 2] = w / h;
        z[4 * i + 3] = h;
    }
}

void jde_kf_initiate(const double z[4], double mean[8], double cov[64]) {
    const double h = z[3];
    for (int i = 0; i < 4; ++i) {
        mean[i] = z[i];
        mean[4 + i] = 0.0;
    }
    const double sd[8] = {2 * kStdPos * h, 2 * kStdPos * h, 1e-2, 2 * kStdPos * h,
                          10 * kStdVel * h, 10 * kStdVel * h, 1e-5, 10 * kStdVel * h};
    for (int i = 0; i < 64; ++i) cov[i] = 0.0;
    for (int i = 0; i < 8; ++i) cov[i * 8 + i] = sd[i] * sd[i];
}

void jde_kf_initiate_n(int n, const double* z, double* mean, double* cov) {
    for (int i = 0; i < n; ++i) jde_kf_initiate(z + 4 * (size_t)i, mean + 8 * (size_t)i, cov + 64 * (size_t)i);
}

void jde_kf_predict(int T, double* mean, double* cov) {
    for (int t = 0; t < T; ++t) {
        double* m = mean + (size_t)t * 8;
        double* P = cov + (size_t)t * 64;
        const double h = m[3];
        const double sd[8] = {kStdPos * h, kStdPos * h, 1e-2, kStdPos * h,
                              kStdVel * h, kStdVel * h, 1e-5, kStdVel * h};
        for (int i = 0; i < 4; ++i) m[i] += m[4 + i];
        // P <- F P F^T with F = [[I, I], [0, I]]: rows then columns i += i+4.
        double Q[64];
        memcpy(Q, P, sizeof Q);
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 8; ++j) Q[i * 8 + j] += P[(i + 4) * 8 + j];
        double R[64];
        memcpy(R, Q, sizeof R);
        for (int i = 0; i < 8; ++i)
            for (int j = 0; j < 4; ++j) R[i * 8 + j] += Q[i * 8 + j + 4];
        for (int i = 0; i < 8; ++i) R[i * 8 + i] += sd[i] * sd[i];
        memcpy(P, R, sizeof R);
    }
}

jde_status jde_kf_update(double mean[8], double cov[64], const double z[4]) {
    const double h = mean[3];
    const double r[4] = {kStdPos * h * kStdPos * h, kStdPos * h * kStdPos * h, 1e-2, kStdPos * h * kStdPos * h};
    double S[4][4], L[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) S[i][j] = cov[i * 8 + j] + (i == j ? r[i] : 0.0);
    if (!chol4(S, L)) return JDE_EINVAL;
    // K^T = S^-1 (H P): column c of K^T solves S x = P[0:4, c].
    double K[8][4];
    for (int c = 0; c < 8; ++c) {
        const double b[4] = {cov[0 * 8 + c], cov[1 * 8 + c], cov[2 * 8 + c], cov[3 * 8 + c]};
        double x[4];
        chol4_solve(L, b, x);
        for (int i = 0; i < 4; ++i) K[c][i] = x[i];
    }
    double y[4];
    for (int i = 0; i < 4; ++i) y[i] = z[i] - mean[i];
    for (int i = 0; i < 8; ++i) {
        double acc = 0.0;
        for (int j = 0; j < 4; ++j) acc += K[i][j] * y[j];
        mean[i] += acc;
    }
    // Joseph form: P' = A P A^T + K R K^T with A = I - K H.
    double A[8][8];
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) A[i][j] = (i == j ? 1.0 : 0.0) - (j < 4 ? K[i][j] : 0.0);
    double AP[8][8];
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 8; ++k) acc += A[i][k] * cov[k * 8 + j];
            AP[i][j] = acc;
        }
    double Pn[8][8];
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 8; ++k) acc += AP[i][k] * A[j][k];
            for (int k = 0; k < 4; ++k) acc += K[i][k] * r[k] * K[j][k];
            Pn[i][j] = acc;
        }
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) cov[i * 8 + j] = 0.5 * (Pn[i][j] + Pn[j][i]);
    return JDE_OK;
}

jde_status jde_kf_update_n(int n, const int* track_idx, const int* det_idx, double* mean, double* cov,
                           const double* z) {
    if (n < 0 || (n > 0 && (!track_idx || !det_idx || !mean || !cov || !z))) return JDE_EINVAL;
    jde_status st = JDE_OK;
    for (int i = 0; i < n; ++i) {
        const size_t t = (size_t)track_idx[i], d = (size_t)det_idx[i];
        if (jde_kf_update(mean + 8 * t, cov + 64 * t, z + 4 * d) != JDE_OK) st = JDE_EINVAL;
    }
    return st;
}

// Shortest-augmenting-path Hungarian method with row/column potentials on an
// n x m matrix (n <= m): rows are added one at a time, each by a Dijkstra-like
// search over reduced costs, and the potentials keep reduced costs >= 0.
int jde_assign(const float* cost, int T, int D, float max_cost, int* det_of_track, int* track_of_det,
               double* total) {
    if (T < 0 || D < 0 || (T > 0 && D > 0 && !cost)) return JDE_EINVAL;
    for (int t = 0; t < T; ++t)
        if (det_of_track) det_of_track[t] = -1;
    for (int d = 0; d < D; ++d)
        if (track_of_det) track_of_det[d] = -1;
    if (total) *total = 0.0;
    if (T == 0 || D == 0) return 0;
    const double mc = (double)max_cost;
    // A track or detection with no allowed entry is never matched: the problem
    // reduces to the rows and columns that have one (same optimum, and the
    // search no longer wades through all-forbidden rows).
    std::vector<int> rows, cols;
    {
        std::vector<char> col_ok(D, 0);
        for (int t = 0; t < T; ++t) {
            bool any = false;
            for (int d = 0; d < D; ++d)
                if ((double)cost[(size_t)t * D + d] <= mc) {
                    any = true;
                    col_ok[d] = 1;
                }
            if (any) rows.push_back(t);
        }
        for (int d = 0; d < D; ++d)
            if (col_ok[d]) cols.push_back(d);
    }
    if (rows.empty()) return 0;
    const int Tr = (int)rows.size(), Dr = (int)cols.size();
    const bool tr = Tr > Dr;
    const int n = tr ? Dr : Tr, m = tr ? Tr : Dr;
    const double big = 4.0 * (double)(n + 1) * (mc > 2.0 ? mc : 2.0) + 1.0;
    // the reduced problem, oriented so that it has n <= m, with forbidden = big
    std::vector<double> red((size_t)n * m);
    for (int a = 0; a < Tr; ++a)
        for (int b = 0; b < Dr; ++b) {
            const float c = cost[(size_t)rows[a] * D + cols[b]];
            red[tr ? (size_t)b * m + a : (size_t)a * m + b] = (double)c <= mc ? (double)c : big;
        }
    auto at = [&](int i, int j) -> double { return red[(size_t)i * m + j]; };  // 0-based
    const double inf = std::numeric_limits<double>::infinity();
    std::vector<double> u(n + 1, 0.0), v(m + 1, 0.0), minv(m + 1);
    std::vector<int> p(m + 1, 0), way(m + 1, 0);
    std::vector<char> used(m + 1);
    for (int i = 1; i <= n; ++i) {
        p[0] = i;
        int j0 = 0;
        std::fill(minv.begin(), minv.end(), inf);
        std::fill(used.begin(), used.end(), 0);
        do {
            used[j0] = 1;
            const int i0 = p[j0];
            double delta = inf;
            int j1 = 0;
            for (int j = 1; j <= m; ++j) {
                if (used[j]) continue;
                const double cur = at(i0 - 1, j - 1) - u[i0] - v[j];
                if (cur < minv[j]) {
                    minv[j] = cur;
                    way[j] = j0;
                }
                if (minv[j] < delta) {
                    delta = minv[j];
                    j1 = j;
                }
            }
            for (int j = 0; j <= m; ++j) {
                if (used[j]) {
                    u[p[j]] += delta;
                    v[j] -= delta;
                } else {
                    minv[j] -= delta;
                }
            }
            j0 = j1;
        } while (p[j0] != 0);
        do {
            const int j1 = way[j0];
            p[j0] = p[j1];
            j0 = j1;
        } while (j0);
    }
    int kept = 0;
    double sum = 0.0;
    for (int j = 1; j <= m; ++j) {
        if (!p[j]) continue;
        const int i = p[j] - 1, jj = j - 1;
        const int t = rows[tr ? jj : i], d = cols[tr ? i : jj];
        const float c = cost[(size_t)t * D + d];
        if (!((double)c <= mc)) continue;
        if (det_of_track) det_of_track[t] = d;
        if (track_of_det) track_of_det[d] = t;
        sum += (double)c;
        ++kept;
    }
    if (total) *total = sum;
    return kept;
}

}  // extern "C"
