// Pose initialisation of the tracking front end (Sec. 3.2.1, Eq. 6-9): RANSAC over
// caller-drawn samples of 2D-3D correspondences, a linear six-point PnP per hypothesis,
// inlier scoring, and Gauss-Newton refinement of the best hypothesis on its inliers.
//
//   k_pnp_hyp     one wave per hypothesis: the 12 x 12 normal matrix of the normalised
//                 six-point system in LDS, cyclic Jacobi with lane k updating row/column k
//                 of every rotation, the eigenvector of least eigenvalue, the normalisation
//                 undone, the sign fixed by det(M) > 0, and the nearest rotation as the
//                 orthogonal polar factor (Newton iteration on M), with lambda =
//                 trace(R^T M) / 3 (the mean singular value);
//   k_pnp_score   one workgroup per hypothesis streams the correspondences (coalesced SoA)
//                 and counts those with positive depth and reprojection error < threshold;
//   k_pnp_pick    the best hypothesis (highest score, lowest index) becomes the pose;
//   k_pnp_mark    inlier mask and count of the current pose (per-block partial counts);
//   k_pnp_accum   per-block FP64 partial sums of J^T J and J^T r over the marked inliers;
//   k_pnp_update  one thread: fixed-order sum of the partials, damped Cholesky solve and
//                 the left update T <- Exp(xi) T (skipped with fewer than 6 inliers).
// Everything is float64; the inputs are float32.
#include "gspm_common.h"

namespace gspm {

namespace {

constexpr int kHypWaves = 4;       // hypotheses (waves) per workgroup of k_pnp_hyp
constexpr int kScoreBlock = 256;
constexpr int kAccBlock = 256;
constexpr int kAccBlocks = 256;    // fixed grid of the accumulation kernels

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

__global__ void __launch_bounds__(kHypWaves * kWave)
k_pnp_hyp(const float *__restrict__ X, const float *__restrict__ uv, int64_t n, gspm_intrinsics K,
          const int32_t *__restrict__ samples, int H, Pose *__restrict__ poses, int32_t *__restrict__ valid) {
    __shared__ double Sm[kHypWaves][144];  // symmetric matrix, full storage
    __shared__ double Em[kHypWaves][144];  // eigenvectors (columns)
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int h = blockIdx.x * kHypWaves + w;
    if (h >= H) return;  // wave-uniform
    double *A = Sm[w], *E = Em[w];
    // Every lane loads the sample (wave-uniform values).
    bool ok = true;
    int idx[6];
    for (int k = 0; k < 6; ++k) {
        idx[k] = samples[6 * (int64_t)h + k];
        ok = ok && idx[k] >= 0 && idx[k] < n;
    }
    if (!ok)
        for (int k = 0; k < 6; ++k) idx[k] = 0;
    double P3[6][3], x2[6][2], c[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            P3[k][a] = X[a * n + idx[k]];
            c[a] += P3[k][a] / 6.0;
        }
        x2[k][0] = ((double)uv[idx[k]] - K.cx) / K.fx;
        x2[k][1] = ((double)uv[n + idx[k]] - K.cy) / K.fy;
    }
    double dm = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double dx = P3[k][0] - c[0], dy = P3[k][1] - c[1], dz = P3[k][2] - c[2];
        dm += sqrt(dx * dx + dy * dy + dz * dz) / 6.0;
    }
    const double s = dm > 0.0 ? sqrt(3.0) / dm : 1.0;
    // Lane l < 144 computes entry (l / 12, l % 12) of A^T A for the rows [Xh 0 -x Xh], [0 Xh -y Xh].
    for (int l = lane; l < 144; l += kWave) {
        const int i = l / 12, j = l % 12;
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double Xh[4] = {s * (P3[k][0] - c[0]), s * (P3[k][1] - c[1]), s * (P3[k][2] - c[2]), 1.0};
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const double ri = i < 8 ? ((i / 4 == r) ? Xh[i % 4] : 0.0) : -x2[k][r] * Xh[i - 8];
                const double rj = j < 8 ? ((j / 4 == r) ? Xh[j % 4] : 0.0) : -x2[k][r] * Xh[j - 8];
                acc += ri * rj;
            }
        }
        A[l] = acc;
        E[l] = i == j ? 1.0 : 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // Cyclic Jacobi; lane k < 12 owns row and column k of each rotation.
    for (int sweep = 0; sweep < 20; ++sweep) {
        double off = 0.0, diag = 0.0;
        if (lane < 12)
            for (int j = 0; j < 12; ++j) {
                const double a = A[lane * 12 + j];
                if (j == lane) diag += a * a; else off += a * a;
            }
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_xor(off, o, kWave);
            diag += __shfl_xor(diag, o, kWave);
        }
        if (off <= 2e-30 * diag) break;  // wave-uniform
        for (int p = 0; p < 11; ++p)
            for (int q = p + 1; q < 12; ++q) {
                const double apq = A[p * 12 + q];
                if (apq == 0.0) continue;  // wave-uniform (LDS broadcast)
                const double app = A[p * 12 + p], aqq = A[q * 12 + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double cs = 1.0 / sqrt(tt * tt + 1.0), sn = tt * cs;
                double akp = 0.0, akq = 0.0, ekp = 0.0, ekq = 0.0;
                if (lane < 12) {
                    akp = A[lane * 12 + p];
                    akq = A[lane * 12 + q];
                    ekp = E[lane * 12 + p];
                    ekq = E[lane * 12 + q];
                }
                __builtin_amdgcn_wave_barrier();
                if (lane < 12) {
                    if (lane != p && lane != q) {
                        const double np_ = cs * akp - sn * akq, nq_ = sn * akp + cs * akq;
                        A[lane * 12 + p] = np_;
                        A[p * 12 + lane] = np_;
                        A[lane * 12 + q] = nq_;
                        A[q * 12 + lane] = nq_;
                    }
                    E[lane * 12 + p] = cs * ekp - sn * ekq;
                    E[lane * 12 + q] = sn * ekp + cs * ekq;
                }
                if (lane == 0) {
                    A[p * 12 + p] = app - tt * apq;
                    A[q * 12 + q] = aqq + tt * apq;
                    A[p * 12 + q] = 0.0;
                    A[q * 12 + p] = 0.0;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
    }
    if (lane != 0) return;
    int m = 0;
    for (int i = 1; i < 12; ++i)
        if (A[i * 13] < A[m * 13]) m = i;
    double p[12];
    for (int i = 0; i < 12; ++i) p[i] = E[i * 12 + m];
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
    poses[h] = P;
    valid[h] = ok ? 1 : 0;
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

// Highest score, lowest index among equal scores (one workgroup of 256).
__global__ void __launch_bounds__(256)
k_pnp_pick(const Pose *__restrict__ poses, const int32_t *__restrict__ scores, int H, Pose *__restrict__ cur) {
    __shared__ long long lds[4];
    // Key orders by score, then by the smaller index: (score + 1) * 2^32 - 1 - h.
    long long best = -1;
    for (int h = threadIdx.x; h < H; h += blockDim.x) {
        const long long key = ((long long)scores[h] + 1) * 4294967296ll + (4294967295ll - h);
        best = key > best ? key : best;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const long long o = __shfl_xor(best, off, 64);
        best = o > best ? o : best;
    }
    if (lane_id() == 0) lds[threadIdx.x / kWave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long b = lds[0];
        for (int w = 1; w < 4; ++w) b = lds[w] > b ? lds[w] : b;
        const int h = b < 0 ? 0 : (int)(4294967295ll - (b & 4294967295ll));
        *cur = poses[h];
    }
}

// Inlier mask of the current pose and per-block inlier counts.
__global__ void __launch_bounds__(kAccBlock)
k_pnp_mark(const float *__restrict__ X, const float *__restrict__ uv, int64_t n, gspm_intrinsics K, double thr2,
           const Pose *__restrict__ cur, uint8_t *__restrict__ mask, int32_t *__restrict__ part) {
    __shared__ int lds[kAccBlock / kWave];
    const Pose P = *cur;
    int cnt = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        double r[2], Y[3];
        const bool in = inlier(P, X[k], X[n + k], X[2 * n + k], uv[k], uv[n + k], K, thr2, r, Y);
        mask[k] = in ? 1 : 0;
        cnt += in ? 1 : 0;
    }
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if (lane_id() == 0) lds[threadIdx.x / kWave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = lds[0] + lds[1] + lds[2] + lds[3];
}

// Per-block partial sums: 21 entries of J^T J (upper triangle), 6 of J^T r.
__global__ void __launch_bounds__(kAccBlock)
k_pnp_accum(const float *__restrict__ X, const float *__restrict__ uv, int64_t n, gspm_intrinsics K,
            const Pose *__restrict__ cur, const uint8_t *__restrict__ mask, double *__restrict__ part) {
    __shared__ double lds[kAccBlock / kWave][27];
    const Pose P = *cur;
    double acc[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) acc[q] = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        if (!mask[k]) continue;
        const double x = X[k], y = X[n + k], z = X[2 * n + k];
        const double Y[3] = {P.R[0] * x + P.R[1] * y + P.R[2] * z + P.t[0], P.R[3] * x + P.R[4] * y + P.R[5] * z + P.t[1],
                             P.R[6] * x + P.R[7] * y + P.R[8] * z + P.t[2]};
        if (!(Y[2] > 0.0)) continue;  // cannot happen for small steps; keeps the sums finite
        const double iz = 1.0 / Y[2];
        const double r[2] = {K.fx * Y[0] * iz + K.cx - (double)uv[k], K.fy * Y[1] * iz + K.cy - (double)uv[n + k]};
        const double Jp[2][3] = {{K.fx * iz, 0.0, -K.fx * Y[0] * iz * iz}, {0.0, K.fy * iz, -K.fy * Y[1] * iz * iz}};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            // d Y / d xi = [I | -[Y]x]: the rotation block is Y x Jp.
            const double J[6] = {Jp[c][0], Jp[c][1], Jp[c][2], Y[1] * Jp[c][2] - Y[2] * Jp[c][1],
                                 Y[2] * Jp[c][0] - Y[0] * Jp[c][2], Y[0] * Jp[c][1] - Y[1] * Jp[c][0]};
            int q = 0;
#pragma unroll
            for (int i = 0; i < 6; ++i)
#pragma unroll
                for (int j = i; j < 6; ++j) acc[q++] += J[i] * J[j];
#pragma unroll
            for (int i = 0; i < 6; ++i) acc[21 + i] += J[i] * r[c];
        }
    }
    const int wid = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        double v = acc[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane_id() == 0) lds[wid][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 27)
        part[(int64_t)blockIdx.x * 27 + threadIdx.x] =
            lds[0][threadIdx.x] + lds[1][threadIdx.x] + lds[2][threadIdx.x] + lds[3][threadIdx.x];
}

// One Gauss-Newton step from the partials (fixed order), unless the inliers are < 6.
__global__ void __launch_bounds__(kAccBlocks)
k_pnp_update(const double *__restrict__ part, const int32_t *__restrict__ cnt_part, int nb, Pose *__restrict__ cur) {
    // Fixed-order reduction of the nb = kAccBlocks partials: thread b holds block b's.
    __shared__ double lds[kAccBlocks / kWave][28];
    const int b = threadIdx.x, wid = b / kWave;
    double v[28];
#pragma unroll
    for (int q = 0; q < 27; ++q) v[q] = b < nb ? part[(int64_t)b * 27 + q] : 0.0;
    v[27] = b < nb ? (double)cnt_part[b] : 0.0;
#pragma unroll
    for (int q = 0; q < 28; ++q) {
        for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
        if (lane_id() == 0) lds[wid][q] = v[q];
    }
    __syncthreads();
    if (b != 0) return;
    double acc[28];
    for (int q = 0; q < 28; ++q) {
        acc[q] = 0.0;
        for (int w = 0; w < kAccBlocks / kWave; ++w) acc[q] += lds[w][q];
    }
    if (acc[27] < 6.0) return;
    double A[6][6];
    int q = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) A[i][j] = A[j][i] = acc[q++];
    const double damp = 1e-9 * (A[0][0] + A[1][1] + A[2][2] + A[3][3] + A[4][4] + A[5][5]) / 6.0;
    for (int i = 0; i < 6; ++i) A[i][i] += damp;
    double L[6][6] = {};
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j <= i; ++j) {
            double sum = A[i][j];
            for (int k = 0; k < j; ++k) sum -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(sum > 0.0)) return;  // not positive definite: keep the pose
                L[i][i] = sqrt(sum);
            } else {
                L[i][j] = sum / L[j][j];
            }
        }
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
    const Pose P = *cur;
    Pose Pn;
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            Pn.R[3 * i + j] = dR[3 * i] * P.R[j] + dR[3 * i + 1] * P.R[3 + j] + dR[3 * i + 2] * P.R[6 + j];
        Pn.t[i] = dR[3 * i] * P.t[0] + dR[3 * i + 1] * P.t[1] + dR[3 * i + 2] * P.t[2] + dt[i];
    }
    *cur = Pn;
}

__global__ void k_pnp_finish(const Pose *__restrict__ cur, const int32_t *__restrict__ cnt_part, int nb,
                             double *__restrict__ T_out, int32_t *__restrict__ n_inliers,
                             const float *__restrict__ T_ak, float *__restrict__ T_n) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const Pose P = *cur;
    int cnt = 0;
    for (int b = 0; b < nb; ++b) cnt += cnt_part[b];
    *n_inliers = cnt;
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) T_out[4 * i + j] = P.R[3 * i + j];
        T_out[4 * i + 3] = P.t[i];
    }
    if (T_n)  // Eq. 9: T_n = T_rel T_ak
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 4; ++j) {
                double acc = j == 3 ? P.t[i] : 0.0;
                for (int k = 0; k < 3; ++k) acc += P.R[3 * i + k] * (double)T_ak[4 * k + j];
                T_n[4 * i + j] = (float)acc;
            }
}

}  // namespace

int64_t pnp_scratch_bytes(int H, int64_t n) {
    return (int64_t)H * ((int64_t)sizeof(Pose) + 8) + 2 * (int64_t)sizeof(Pose) + 8 * 27 * kAccBlocks +
           4 * kAccBlocks + n + 1024;
}

hipError_t launch_pnp(const float *X, const float *uv, int64_t n, const gspm_intrinsics &K, const int32_t *samples,
                      int H, double thr, int iters, int rounds, void *scratch, double *T_out, int32_t *n_inliers,
                      uint8_t *mask, int32_t *scores_out, const float *T_ak, float *T_n_out, hipStream_t s) {
    char *base = static_cast<char *>(scratch);
    Pose *poses = reinterpret_cast<Pose *>(base);
    Pose *cur = poses + H;
    int32_t *valid = reinterpret_cast<int32_t *>(cur + 2);
    int32_t *scores = scores_out ? scores_out : valid + H;
    double *part = reinterpret_cast<double *>(base + (((char *)(valid + 2 * H) - base + 255) & ~(int64_t)255));
    int32_t *cnt_part = reinterpret_cast<int32_t *>(part + 27 * kAccBlocks);
    uint8_t *round_mask = reinterpret_cast<uint8_t *>(cnt_part + kAccBlocks);
    const double thr2 = thr * thr;
    hipLaunchKernelGGL(k_pnp_hyp, dim3((H + kHypWaves - 1) / kHypWaves), dim3(kHypWaves * kWave), 0, s, X, uv, n, K,
                       samples, H, poses, valid);
    hipLaunchKernelGGL(k_pnp_score, dim3(H), dim3(kScoreBlock), 0, s, X, uv, n, K, thr2, poses, valid, scores);
    hipLaunchKernelGGL(k_pnp_pick, dim3(1), dim3(256), 0, s, poses, scores, H, cur);
    for (int round = 0; round < rounds; ++round) {
        hipLaunchKernelGGL(k_pnp_mark, dim3(kAccBlocks), dim3(kAccBlock), 0, s, X, uv, n, K, thr2, cur, round_mask,
                           cnt_part);
        for (int it = 0; it < iters; ++it) {
            hipLaunchKernelGGL(k_pnp_accum, dim3(kAccBlocks), dim3(kAccBlock), 0, s, X, uv, n, K, cur, round_mask,
                               part);
            hipLaunchKernelGGL(k_pnp_update, dim3(1), dim3(kAccBlocks), 0, s, part, cnt_part, kAccBlocks, cur);
        }
    }
    uint8_t *final_mask = mask ? mask : round_mask;
    hipLaunchKernelGGL(k_pnp_mark, dim3(kAccBlocks), dim3(kAccBlock), 0, s, X, uv, n, K, thr2, cur, final_mask,
                       cnt_part);
    hipLaunchKernelGGL(k_pnp_finish, dim3(1), dim3(64), 0, s, cur, cnt_part, kAccBlocks, T_out, n_inliers, T_ak,
                       T_n_out);
    return hipGetLastError();
}

}  // namespace gspm
