// Pose initialisation of the tracking front end (Sec. 3.2.1, Eq. 6-9): RANSAC over
// caller-drawn samples of 2D-3D correspondences, a linear six-point PnP per hypothesis,
// inlier scoring, and Gauss-Newton refinement of the best hypothesis on its inliers.
//
//   k_pnp_hyp    one lane per hypothesis: the 12 x 12 normal matrix of the normalised
//                six-point system in LDS (interleaved across lanes, so every access is
//                conflict free), cyclic Jacobi for its eigenvector of least eigenvalue,
//                the normalisation undone, the sign fixed by det(M) > 0, and the nearest
//                rotation as the orthogonal polar factor (Newton iteration on M), with
//                lambda = trace(R^T M) / 3 (the mean singular value);
//   k_pnp_score  one workgroup per hypothesis streams the correspondences (coalesced SoA)
//                and counts those with positive depth and reprojection error < threshold;
//   k_pnp_refine one workgroup: best hypothesis (highest score, lowest index), then
//                rounds x (inlier selection, iterations x Gauss-Newton step) with FP64
//                block reductions of J^T J and J^T r in a fixed order.
// Everything is float64; the inputs are float32.
#include "gspm_common.h"

namespace gspm {

namespace {

constexpr int kHypLanes = 32;     // hypotheses per workgroup of k_pnp_hyp (57 KB of LDS)
constexpr int kScoreBlock = 256;
constexpr int kRefineBlock = 1024;

struct Pose {
    double R[9];
    double t[3];
};

__device__ inline void se3_exp(const double xi[6], double R[9], double t[3]) {
    const double px = xi[3], py = xi[4], pz = xi[5];
    const double th2 = px * px + py * py + pz * pz, th = sqrt(th2);
    double a, b, c;
    if (th < 1e-8) {
        a = 1.0 - th2 / 6.0;
        b = 0.5 - th2 / 24.0;
        c = 1.0 / 6.0 - th2 / 120.0;
    } else {
        a = sin(th) / th;
        b = (1.0 - cos(th)) / th2;
        c = (th - sin(th)) / (th2 * th);
    }
    const double K[9] = {0.0, -pz, py, pz, 0.0, -px, -py, px, 0.0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) K2[3 * i + j] = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
    double V[9];
    for (int k = 0; k < 9; ++k) {
        const double I = (k % 4 == 0) ? 1.0 : 0.0;
        R[k] = I + a * K[k] + b * K2[k];
        V[k] = I + b * K[k] + c * K2[k];
    }
    for (int i = 0; i < 3; ++i) t[i] = V[3 * i] * xi[0] + V[3 * i + 1] * xi[1] + V[3 * i + 2] * xi[2];
}

// Orthogonal polar factor of a 3x3 matrix with positive determinant (Newton iteration
// X <- (X + X^-T) / 2, which converges quadratically to U V^T of the SVD).
__device__ inline void polar(const double M[9], double R[9]) {
    for (int k = 0; k < 9; ++k) R[k] = M[k];
    for (int it = 0; it < 30; ++it) {
        // cofactor matrix C = det(X) X^-T
        double C[9];
        C[0] = R[4] * R[8] - R[5] * R[7];
        C[1] = R[5] * R[6] - R[3] * R[8];
        C[2] = R[3] * R[7] - R[4] * R[6];
        C[3] = R[2] * R[7] - R[1] * R[8];
        C[4] = R[0] * R[8] - R[2] * R[6];
        C[5] = R[1] * R[6] - R[0] * R[7];
        C[6] = R[1] * R[5] - R[2] * R[4];
        C[7] = R[2] * R[3] - R[0] * R[5];
        C[8] = R[0] * R[4] - R[1] * R[3];
        const double det = R[0] * C[0] + R[1] * C[1] + R[2] * C[2];
        if (!(fabs(det) > 1e-300)) return;
        double d = 0.0;
        for (int k = 0; k < 9; ++k) {
            const double nv = 0.5 * (R[k] + C[k] / det);
            d = fmax(d, fabs(nv - R[k]));
            R[k] = nv;
        }
        if (d < 1e-15) return;
    }
}

__global__ void __launch_bounds__(kHypLanes)
k_pnp_hyp(const float *__restrict__ X, const float *__restrict__ uv, int64_t n, gspm_intrinsics K,
          const int32_t *__restrict__ samples, int H, Pose *__restrict__ poses, int32_t *__restrict__ valid) {
    __shared__ double S[78 * kHypLanes];   // upper triangle of the 12 x 12 matrix, lane-interleaved
    __shared__ double E[144 * kHypLanes];  // eigenvector matrix, lane-interleaved
    const int lane = threadIdx.x;
    const int h = blockIdx.x * kHypLanes + lane;
    // Index of (i, j), i <= j, in the packed upper triangle.
    auto up = [&](int i, int j) -> double & {
        if (i > j) { const int t = i; i = j; j = t; }
        return S[(i * 12 - i * (i - 1) / 2 + (j - i)) * kHypLanes + lane];
    };
    auto ev = [&](int i, int j) -> double & { return E[(i * 12 + j) * kHypLanes + lane]; };
    bool ok = h < H;
    int idx[6];
    for (int k = 0; k < 6; ++k) {
        idx[k] = ok ? samples[6 * (int64_t)h + k] : 0;
        ok = ok && idx[k] >= 0 && idx[k] < n;
    }
    if (!ok)
        for (int k = 0; k < 6; ++k) idx[k] = 0;
    double P3[6][3], x2[6][2], c[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 6; ++k) {
        for (int a = 0; a < 3; ++a) {
            P3[k][a] = X[a * n + idx[k]];
            c[a] += P3[k][a] / 6.0;
        }
        x2[k][0] = ((double)uv[idx[k]] - K.cx) / K.fx;
        x2[k][1] = ((double)uv[n + idx[k]] - K.cy) / K.fy;
    }
    double dm = 0.0;
    for (int k = 0; k < 6; ++k) {
        const double dx = P3[k][0] - c[0], dy = P3[k][1] - c[1], dz = P3[k][2] - c[2];
        dm += sqrt(dx * dx + dy * dy + dz * dz) / 6.0;
    }
    const double s = dm > 0.0 ? sqrt(3.0) / dm : 1.0;
    // Normal matrix A^T A of the rows [Xh 0 -x Xh] and [0 Xh -y Xh].
    for (int i = 0; i < 12; ++i)
        for (int j = i; j < 12; ++j) up(i, j) = 0.0;
    for (int k = 0; k < 6; ++k) {
        const double Xh[4] = {s * (P3[k][0] - c[0]), s * (P3[k][1] - c[1]), s * (P3[k][2] - c[2]), 1.0};
        for (int r = 0; r < 2; ++r) {
            double row[12];
            for (int q = 0; q < 12; ++q) row[q] = 0.0;
            for (int q = 0; q < 4; ++q) {
                row[4 * r + q] = Xh[q];
                row[8 + q] = -x2[k][r] * Xh[q];
            }
            for (int i = 0; i < 12; ++i)
                if (row[i] != 0.0)
                    for (int j = i; j < 12; ++j) up(i, j) += row[i] * row[j];
        }
    }
    // Cyclic Jacobi: S -> diag, E accumulates the rotations (columns = eigenvectors).
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) ev(i, j) = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 20; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < 12; ++i) {
            diag += up(i, i) * up(i, i);
            for (int j = i + 1; j < 12; ++j) off += up(i, j) * up(i, j);
        }
        if (off <= 1e-30 * diag) break;
        for (int p = 0; p < 11; ++p)
            for (int q = p + 1; q < 12; ++q) {
                const double apq = up(p, q);
                if (apq == 0.0) continue;
                const double app = up(p, p), aqq = up(q, q);
                const double theta = (aqq - app) / (2.0 * apq);
                const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double cs = 1.0 / sqrt(tt * tt + 1.0), sn = tt * cs;
                for (int k = 0; k < 12; ++k) {
                    if (k == p || k == q) continue;
                    const double akp = up(k, p), akq = up(k, q);
                    up(k, p) = cs * akp - sn * akq;
                    up(k, q) = sn * akp + cs * akq;
                }
                up(p, p) = app - tt * apq;
                up(q, q) = aqq + tt * apq;
                up(p, q) = 0.0;
                for (int k = 0; k < 12; ++k) {
                    const double ekp = ev(k, p), ekq = ev(k, q);
                    ev(k, p) = cs * ekp - sn * ekq;
                    ev(k, q) = sn * ekp + cs * ekq;
                }
            }
    }
    int m = 0;
    for (int i = 1; i < 12; ++i)
        if (up(i, i) < up(m, m)) m = i;
    double p[12];
    for (int i = 0; i < 12; ++i) p[i] = ev(i, m);
    // Undo the normalisation: M = s Pn[:, :3], p4 = Pn[:, 3] - s Pn[:, :3] c.
    double M[9], p4[3];
    for (int r = 0; r < 3; ++r) {
        for (int a = 0; a < 3; ++a) M[3 * r + a] = s * p[4 * r + a];
        p4[r] = p[4 * r + 3] - (M[3 * r] * c[0] + M[3 * r + 1] * c[1] + M[3 * r + 2] * c[2]);
    }
    const double det = M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
                       M[2] * (M[3] * M[7] - M[4] * M[6]);
    if (det < 0.0) {
        for (int k = 0; k < 9; ++k) M[k] = -M[k];
        for (int k = 0; k < 3; ++k) p4[k] = -p4[k];
    }
    Pose P;
    polar(M, P.R);
    double tr = 0.0;  // trace(R^T M) = sum of the singular values
    for (int k = 0; k < 9; ++k) tr += P.R[k] * M[k];
    const double lam = tr / 3.0;
    ok = ok && det != 0.0 && lam > 0.0;
    for (int k = 0; k < 3; ++k) P.t[k] = ok ? p4[k] / lam : 0.0;
    if (h < H) {
        poses[h] = P;
        valid[h] = ok ? 1 : 0;
    }
}

__device__ inline bool inlier(const Pose &P, double x, double y, double z, double u0, double v0,
                              const gspm_intrinsics &K, double thr2, double r[2], double Y[3]) {
    Y[0] = P.R[0] * x + P.R[1] * y + P.R[2] * z + P.t[0];
    Y[1] = P.R[3] * x + P.R[4] * y + P.R[5] * z + P.t[1];
    Y[2] = P.R[6] * x + P.R[7] * y + P.R[8] * z + P.t[2];
    if (!(Y[2] > 0.0)) return false;
    r[0] = K.fx * Y[0] / Y[2] + K.cx - u0;
    r[1] = K.fy * Y[1] / Y[2] + K.cy - v0;
    return r[0] * r[0] + r[1] * r[1] < thr2;
}

__global__ void __launch_bounds__(kScoreBlock)
k_pnp_score(const float *__restrict__ X, const float *__restrict__ uv, int64_t n, gspm_intrinsics K, double thr2,
            const Pose *__restrict__ poses, const int32_t *__restrict__ valid, int32_t *__restrict__ scores) {
    __shared__ int lds[kScoreBlock / kWave];
    const int h = blockIdx.x;
    const Pose P = poses[h];
    int cnt = 0;
    if (valid[h])
        for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
            double r[2], Y[3];
            cnt += inlier(P, X[k], X[n + k], X[2 * n + k], uv[k], uv[n + k], K, thr2, r, Y) ? 1 : 0;
        }
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if (lane_id() == 0) lds[threadIdx.x / kWave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kScoreBlock / kWave; ++w) t += lds[w];
        scores[h] = valid[h] ? t : -1;
    }
}

// Fixed-order block sum of NV doubles per thread into v (valid in every thread afterwards).
template <int NV>
__device__ inline void block_sum(double v[NV], double *lds) {
    const int wid = threadIdx.x / kWave, lane = lane_id();
    for (int k = 0; k < NV; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    __syncthreads();
    if (lane == 0)
        for (int k = 0; k < NV; ++k) lds[wid * NV + k] = v[k];
    __syncthreads();
    for (int k = 0; k < NV; ++k) {
        double t = 0.0;
        for (int w = 0; w < kRefineBlock / kWave; ++w) t += lds[w * NV + k];
        v[k] = t;
    }
}

__global__ void __launch_bounds__(kRefineBlock)
k_pnp_refine(const float *__restrict__ X, const float *__restrict__ uv, int64_t n, gspm_intrinsics K, double thr2,
             const Pose *__restrict__ poses, const int32_t *__restrict__ scores, int H, int iters, int rounds,
             double *__restrict__ T_out, int32_t *__restrict__ n_inliers, uint8_t *__restrict__ mask,
             const float *__restrict__ T_ak, float *__restrict__ T_n) {
    __shared__ double lds[(kRefineBlock / kWave) * 27];
    __shared__ int best_s, best_h;
    if (threadIdx.x == 0) {
        best_s = -1;
        best_h = 0;
        for (int h = 0; h < H; ++h)
            if (scores[h] > best_s) {
                best_s = scores[h];
                best_h = h;
            }
    }
    __syncthreads();
    Pose P = poses[best_h];
    for (int round = 0; round <= rounds; ++round) {
        // Inliers of the current pose (the last pass only reports them).
        double cnt[1] = {0.0};
        for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
            double r[2], Y[3];
            const bool in = inlier(P, X[k], X[n + k], X[2 * n + k], uv[k], uv[n + k], K, thr2, r, Y);
            if (mask) mask[k] = in ? 1 : 0;
            cnt[0] += in ? 1.0 : 0.0;
        }
        block_sum<1>(cnt, lds);
        if (round == rounds || cnt[0] < 6.0) {
            if (threadIdx.x == 0) *n_inliers = (int32_t)cnt[0];
            if (round == rounds) break;
            continue;
        }
        const Pose P0 = P;  // inlier set of this round: the one of P0
        for (int it = 0; it < iters; ++it) {
            double acc[27];  // 21 entries of J^T J (upper triangle), 6 of J^T r
            for (int k = 0; k < 27; ++k) acc[k] = 0.0;
            for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
                const double x = X[k], y = X[n + k], z = X[2 * n + k], u0 = uv[k], v0 = uv[n + k];
                double r0[2], Y0[3];
                if (!inlier(P0, x, y, z, u0, v0, K, thr2, r0, Y0)) continue;
                double r[2], Y[3];
                (void)inlier(P, x, y, z, u0, v0, K, thr2, r, Y);
                const double iz = 1.0 / Y[2];
                const double Jp[2][3] = {{K.fx * iz, 0.0, -K.fx * Y[0] * iz * iz},
                                         {0.0, K.fy * iz, -K.fy * Y[1] * iz * iz}};
                for (int c = 0; c < 2; ++c) {
                    // d Y / d xi = [I | -[Y]x]: rotation block Y x Jp.
                    const double J[6] = {Jp[c][0], Jp[c][1], Jp[c][2], Y[1] * Jp[c][2] - Y[2] * Jp[c][1],
                                         Y[2] * Jp[c][0] - Y[0] * Jp[c][2], Y[0] * Jp[c][1] - Y[1] * Jp[c][0]};
                    int q = 0;
                    for (int i = 0; i < 6; ++i)
                        for (int j = i; j < 6; ++j) acc[q++] += J[i] * J[j];
                    for (int i = 0; i < 6; ++i) acc[21 + i] += J[i] * r[c];
                }
            }
            block_sum<27>(acc, lds);
            // Solve (H + 1e-9 trace(H) / 6 I) xi = -g by Cholesky (every thread, same result).
            double A[6][6];
            int q = 0;
            for (int i = 0; i < 6; ++i)
                for (int j = i; j < 6; ++j) A[i][j] = A[j][i] = acc[q++];
            const double damp = 1e-9 * (A[0][0] + A[1][1] + A[2][2] + A[3][3] + A[4][4] + A[5][5]) / 6.0;
            for (int i = 0; i < 6; ++i) A[i][i] += damp;
            double L[6][6] = {};
            bool spd = true;
            for (int i = 0; i < 6 && spd; ++i)
                for (int j = 0; j <= i; ++j) {
                    double sum = A[i][j];
                    for (int k = 0; k < j; ++k) sum -= L[i][k] * L[j][k];
                    if (i == j) {
                        if (!(sum > 0.0)) { spd = false; break; }
                        L[i][i] = sqrt(sum);
                    } else {
                        L[i][j] = sum / L[j][j];
                    }
                }
            if (!spd) break;
            double w[6], xi[6];
            for (int i = 0; i < 6; ++i) {
                double sum = -acc[21 + i];
                for (int k = 0; k < i; ++k) sum -= L[i][k] * w[k];
                w[i] = sum / L[i][i];
            }
            for (int i = 5; i >= 0; --i) {
                double sum = w[i];
                for (int k = i + 1; k < 6; ++k) sum -= L[k][i] * xi[k];
                xi[i] = sum / L[i][i];
            }
            double dR[9], dt[3];
            se3_exp(xi, dR, dt);
            Pose Pn;
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j)
                    Pn.R[3 * i + j] = dR[3 * i] * P.R[j] + dR[3 * i + 1] * P.R[3 + j] + dR[3 * i + 2] * P.R[6 + j];
                Pn.t[i] = dR[3 * i] * P.t[0] + dR[3 * i + 1] * P.t[1] + dR[3 * i + 2] * P.t[2] + dt[i];
            }
            P = Pn;
        }
    }
    if (threadIdx.x == 0) {
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) T_out[4 * i + j] = P.R[3 * i + j];
            T_out[4 * i + 3] = P.t[i];
        }
        if (T_n)  // Eq. 9: T_n = T_rel T_ak
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 4; ++j) {
                    double acc = j == 3 ? P.t[i] : 0.0;
                    for (int k = 0; k < 3; ++k) acc += P.R[3 * i + k] * (double)T_ak[4 * k + j];
                    T_n[4 * i + j] = (float)acc;
                }
            }
    }
}

}  // namespace

int64_t pnp_scratch_bytes(int H) { return (int64_t)H * ((int64_t)sizeof(Pose) + 8) + 256; }

hipError_t launch_pnp(const float *X, const float *uv, int64_t n, const gspm_intrinsics &K, const int32_t *samples,
                      int H, double thr, int iters, int rounds, void *scratch, double *T_out, int32_t *n_inliers,
                      uint8_t *mask, int32_t *scores_out, const float *T_ak, float *T_n_out, hipStream_t s) {
    Pose *poses = static_cast<Pose *>(scratch);
    int32_t *valid = reinterpret_cast<int32_t *>(poses + H);
    int32_t *scores = scores_out ? scores_out : valid + H;
    const double thr2 = thr * thr;
    hipLaunchKernelGGL(k_pnp_hyp, dim3((H + kHypLanes - 1) / kHypLanes), dim3(kHypLanes), 0, s, X, uv, n, K, samples,
                       H, poses, valid);
    hipLaunchKernelGGL(k_pnp_score, dim3(H), dim3(kScoreBlock), 0, s, X, uv, n, K, thr2, poses, valid, scores);
    hipLaunchKernelGGL(k_pnp_refine, dim3(1), dim3(kRefineBlock), 0, s, X, uv, n, K, thr2, poses, scores, H, iters,
                       rounds, T_out, n_inliers, mask, T_ak, T_n_out);
    return hipGetLastError();
}

}  // namespace gspm
