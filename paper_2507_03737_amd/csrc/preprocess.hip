// Per-(Gaussian, view) projection and its backward.
//
// Forward (one lane per record r = v * n + g): activations, world covariance
// Sigma = R S S^T R^T (Sec. 3.1, Eq. 1), camera transform, EWA projection to a 2D conic,
// opacity-aware support box, tile rectangle and depth key.  Backward (one lane per
// Gaussian, looping over views): chain rule from the image-plane gradients accumulated
// by the raster backward to means, log-scales, quaternions, opacity logits and colours,
// plus the per-view se(3) pose contribution (Sec. 3.2.2, Eq. 11) reduced per wave.
//
// This geometry is per Gaussian, not per pixel, so it runs in float64 (MI355X's vector
// FP64 rate is half its FP32 rate) and rounds once to the float32 record: the mean2D is
// kept as a hi/lo float pair so that the per-pixel offset keeps float32 precision even
// at 2000-pixel coordinates.
#include "gspm_common.h"

namespace gspm {

namespace {

constexpr double kLog2e = 1.4426950408889634074;

struct Proj {
    bool visible;
    bool clamp_x, clamp_y;
    double mu[3];         // world-frame centre
    double m[3];          // camera-frame centre
    double u, v, z;
    double a;             // sigmoid opacity
    double s[3];          // scales
    double qn[4];         // unit quaternion
    double qnorm;
    double Rq[3][3];      // Gaussian rotation
    double Sc[3][3];      // camera-frame covariance W Sigma W^T
    double W[3][3];       // camera rotation
    double J[2][3];
    double cov[3];        // 2D covariance (xx, xy, yy) incl. eps2d
    double Q[3];          // conic
    int32_t rect[4];      // pixel rect imin, imax, jmin, jmax
};

// The view-independent part of the projection: activated scales and opacity, the unit
// quaternion and its rotation.  False for a quaternion that cannot be normalised.
__device__ inline bool gaussian_frame(const gspm_gaussians &G, int64_t g, int64_t n, Proj &P) {
    P.mu[0] = G.means[g]; P.mu[1] = G.means[n + g]; P.mu[2] = G.means[2 * n + g];
    const double qw = G.quats[g], qx = G.quats[n + g], qy = G.quats[2 * n + g], qz = G.quats[3 * n + g];
    P.s[0] = (double)expf(G.log_scales[g]);
    P.s[1] = (double)expf(G.log_scales[n + g]);
    P.s[2] = (double)expf(G.log_scales[2 * n + g]);
    P.a = (double)(1.0f / (1.0f + expf(-G.opacity_logit[g])));
    P.qnorm = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    if (!(P.qnorm > 0.0) || !isfinite(P.qnorm)) return false;
    const double inv = 1.0 / P.qnorm;
    const double w = qw * inv, x = qx * inv, y = qy * inv, z = qz * inv;
    P.qn[0] = w; P.qn[1] = x; P.qn[2] = y; P.qn[3] = z;
    P.Rq[0][0] = 1.0 - 2.0 * (y * y + z * z); P.Rq[0][1] = 2.0 * (x * y - w * z); P.Rq[0][2] = 2.0 * (x * z + w * y);
    P.Rq[1][0] = 2.0 * (x * y + w * z); P.Rq[1][1] = 1.0 - 2.0 * (x * x + z * z); P.Rq[1][2] = 2.0 * (y * z - w * x);
    P.Rq[2][0] = 2.0 * (x * z - w * y); P.Rq[2][1] = 2.0 * (y * z + w * x); P.Rq[2][2] = 1.0 - 2.0 * (x * x + y * y);
    return true;
}

// The view-dependent part (Eq. 1): camera-frame centre and covariance, the clamped
// Jacobian, the 2D covariance, its conic and the pixel support.  Needs gaussian_frame's
// fields of P.
__device__ inline void project_view(const float *T12, float fx, float fy, float cx, float cy, int W, int H,
                                    const RasterSettings &rs, Proj &P) {
    P.visible = false;
    P.clamp_x = P.clamp_y = false;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) P.W[r][c] = T12[4 * r + c];
    for (int r = 0; r < 3; ++r)
        P.m[r] = P.W[r][0] * P.mu[0] + P.W[r][1] * P.mu[1] + P.W[r][2] * P.mu[2] + (double)T12[4 * r + 3];
    P.z = P.m[2];
    if (!(P.z > (double)rs.near_z) || !isfinite(P.z) || !isfinite(P.m[0]) || !isfinite(P.m[1])) return;
    const double iz = 1.0 / P.z;
    P.u = (double)fx * P.m[0] * iz + (double)cx;
    P.v = (double)fy * P.m[1] * iz + (double)cy;

    // M = W Rq diag(s): Sigma_c = M M^T.
    double M[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            M[r][c] = (P.W[r][0] * P.Rq[0][c] + P.W[r][1] * P.Rq[1][c] + P.W[r][2] * P.Rq[2][c]) * P.s[c];
    for (int r = 0; r < 3; ++r)
        for (int c = r; c < 3; ++c) {
            const double v = M[r][0] * M[c][0] + M[r][1] * M[c][1] + M[r][2] * M[c][2];
            P.Sc[r][c] = v;
            P.Sc[c][r] = v;
        }

    const double limx = (double)rs.jac_clamp * (double)W / (2.0 * (double)fx);
    const double limy = (double)rs.jac_clamp * (double)H / (2.0 * (double)fy);
    double tx = P.m[0] * iz, ty = P.m[1] * iz;
    if (tx < -limx) { tx = -limx; P.clamp_x = true; }
    if (tx > limx) { tx = limx; P.clamp_x = true; }
    if (ty < -limy) { ty = -limy; P.clamp_y = true; }
    if (ty > limy) { ty = limy; P.clamp_y = true; }
    P.J[0][0] = (double)fx * iz; P.J[0][1] = 0.0; P.J[0][2] = -(double)fx * tx * iz;
    P.J[1][0] = 0.0; P.J[1][1] = (double)fy * iz; P.J[1][2] = -(double)fy * ty * iz;

    double JS[2][3];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            JS[r][c] = P.J[r][0] * P.Sc[0][c] + P.J[r][1] * P.Sc[1][c] + P.J[r][2] * P.Sc[2][c];
    P.cov[0] = JS[0][0] * P.J[0][0] + JS[0][1] * P.J[0][1] + JS[0][2] * P.J[0][2] + (double)rs.eps2d;
    P.cov[1] = JS[0][0] * P.J[1][0] + JS[0][1] * P.J[1][1] + JS[0][2] * P.J[1][2];
    P.cov[2] = JS[1][0] * P.J[1][0] + JS[1][1] * P.J[1][1] + JS[1][2] * P.J[1][2] + (double)rs.eps2d;
    const double det = P.cov[0] * P.cov[2] - P.cov[1] * P.cov[1];
    if (!(det > 0.0) || !isfinite(det)) return;
    const double idet = 1.0 / det;
    P.Q[0] = P.cov[2] * idet;
    P.Q[1] = -P.cov[1] * idet;
    P.Q[2] = P.cov[0] * idet;

    if (!(P.a >= (double)rs.alpha_min)) return;
    const double qmax = 2.0 * (double)logf((float)(P.a / (double)rs.alpha_min));
    const double rx = sqrt(qmax * P.cov[0]), ry = sqrt(qmax * P.cov[2]);
    double i0 = ceil(P.u - rx), i1 = floor(P.u + rx), j0 = ceil(P.v - ry), j1 = floor(P.v + ry);
    i0 = fmax(i0, 0.0); j0 = fmax(j0, 0.0);
    i1 = fmin(i1, (double)(W - 1)); j1 = fmin(j1, (double)(H - 1));
    if (i0 > i1 || j0 > j1) return;
    P.rect[0] = (int32_t)i0; P.rect[1] = (int32_t)i1; P.rect[2] = (int32_t)j0; P.rect[3] = (int32_t)j1;
    P.visible = true;
}

__global__ void __launch_bounds__(256)
k_preprocess(gspm_gaussians G, ViewTable vt, const float *__restrict__ T_cw, RasterSettings rs,
             float4 *__restrict__ rec, uint32_t *__restrict__ counts, uint32_t *__restrict__ dkey,
             uint4 *__restrict__ spans, uint32_t *__restrict__ big_list, uint32_t *__restrict__ big_count) {
    // One thread per Gaussian looping over the views: the view-independent part of the
    // projection is computed once.
    const int64_t n = G.n;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    Proj P;
    const bool framed = g < n && gaussian_frame(G, g, n, P);
    for (int v = 0; v < vt.n_views; ++v) {
        const int64_t r = (int64_t)v * n + g;
        bool big = false;
        if (g < n) {
            if (framed)
                project_view(T_cw + 12 * v, vt.fx[v], vt.fy[v], vt.cx[v], vt.cy[v], vt.width[v], vt.height[v], rs, P);
            uint32_t count = 0;
            if (framed && P.visible) {
                const float zf = (float)P.z;
                dkey[r] = __float_as_uint(zf);
                const float uhi = (float)P.u, vhi = (float)P.v;
                const float ulo = (float)(P.u - (double)uhi), vlo = (float)(P.v - (double)vhi);
                const float4 r0 = make_float4(uhi, vhi, ulo, vlo);
                // Factored conic: k Q = L^T L, L = [[a, b], [0, c]], k = log2(e) / 2; c^2 is
                // k det(Q) / Q_xx, which stays positive (det > 0) without cancellation.
                const double kq = 0.5 * kLog2e;
                const double fa = sqrt(kq * P.Q[0]);
                const double fb = kq * P.Q[1] / fa;
                const double fc = sqrt(kq * (P.Q[0] * P.Q[2] - P.Q[1] * P.Q[1]) / P.Q[0]);
                const float4 r1 = make_float4((float)fa, (float)fb, (float)fc, (float)P.a);
                float4 *o = rec + 4 * r;
                o[0] = r0;
                o[1] = r1;
                o[2] = make_float4(G.rgb[g], G.rgb[n + g], G.rgb[2 * n + g], zf);
                if (rs.frame == 0)
                    o[3] = make_float4(G.means[g], G.means[n + g], G.means[2 * n + g], 0.0f);
                else
                    o[3] = make_float4((float)P.m[0], (float)P.m[1], (float)P.m[2], 0.0f);
                // Number of tiles the support meets, row by row (the pair emission repeats this).
                // Records whose support box covers many tiles are counted by whole waves instead.
                Footprint f;
                if (record_footprint(r0, r1, rs.alpha_min, vt.width[v], vt.height[v], f)) {
                    const int T = vt.tile, sh = __builtin_ctz((unsigned)vt.tile);  // a power of two
                    const int rows = (f.j1 >> sh) - (f.j0 >> sh) + 1, cols = (f.i1 >> sh) - (f.i0 >> sh) + 1;
                    if ((uint32_t)(rows * cols) > kBigRecord) {
                        big = true;  // its count may still come out at most kBigRecord: not cached
                        spans[r] = make_uint4(kSpanNone << 16, 0u, 0u, 0u);
                    } else {
                        uint32_t w[kSpanRows] = {1u, 1u, 1u};  // empty rows: first > last
                        uint32_t h[kSpanRows] = {0x00010001u, 0x00010001u, 0x00010001u};  // two rows a word
                        bool narrow = true;  // every tile column below 256
                        for (int ty = f.j0 >> sh, k = 0; ty <= f.j1 >> sh; ++ty, ++k) {
                            int ta, tb;
                            if (row_span(f, T, ty, ta, tb)) {
                                count += (uint32_t)(tb - ta + 1);
                                if (k < (int)kSpanRows) w[k] = (uint32_t)ta | ((uint32_t)tb << 16);
                                if (k < (int)kSpanRowsMax) {
                                    narrow = narrow && tb < 256;
                                    const int q = k >> 1, sft = 16 * (k & 1);
                                    h[q] = (h[q] & ~(0xffffu << sft)) | (((uint32_t)ta | ((uint32_t)tb << 8)) << sft);
                                }
                            }
                        }
                        if (count != 0u) {
                            const uint32_t x0 = (uint32_t)(f.j0 >> sh);
                            if (rows <= (int)kSpanRows)
                                spans[r] = make_uint4(x0 | ((uint32_t)rows << 16), w[0], w[1], w[2]);
                            else if (rows <= (int)kSpanRowsMax && narrow)
                                spans[r] = make_uint4(x0 | ((uint32_t)rows << 16), h[0], h[1], h[2]);
                            else
                                spans[r] = make_uint4(x0 | (kSpanNone << 16), 0u, 0u, 0u);
                        }
                    }
                }
            }
            counts[r] = count;
        }
        const uint32_t slot = wave_append(big_count, big);
        if (big) big_list[slot] = (uint32_t)r;
    }
}

// Exact pair count of the queued large records: one wave per record, one lane per tile row.
__global__ void __launch_bounds__(256)
k_count_big(const float4 *__restrict__ rec, ViewTable vt, RasterSettings rs, int64_t n_per_view,
            uint32_t *__restrict__ counts, const uint32_t *__restrict__ big_list,
            const uint32_t *__restrict__ big_count) {
    const int lane = lane_id();
    const uint32_t n_big = *big_count;
    const uint32_t n_waves = gridDim.x * (blockDim.x / kWave);
    for (uint32_t w = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; w < n_big; w += n_waves) {
        const uint32_t r = big_list[w];
        const int v = (int)(r / (uint32_t)n_per_view);
        Footprint f;
        uint32_t count = 0;
        if (record_footprint(rec[4 * (int64_t)r], rec[4 * (int64_t)r + 1], rs.alpha_min, vt.width[v],
                             vt.height[v], f)) {
            const int T = vt.tile, sh = __builtin_ctz((unsigned)vt.tile);
            for (int ty = (f.j0 >> sh) + lane; ty <= f.j1 >> sh; ty += kWave) {
                int ta, tb;
                if (row_span(f, T, ty, ta, tb)) count += (uint32_t)(tb - ta + 1);
            }
        }
        for (int off = 32; off > 0; off >>= 1) count += __shfl_xor(count, off, 64);
        if (lane == 0) counts[r] = count;
    }
}

// ---------------------------------------------------------------------------------------
// Backward: image-plane gradients -> parameters and pose.

constexpr int kBwdBlock = 256;

constexpr int kBwdWaves = kBwdBlock / kWave;

__global__ void __launch_bounds__(kBwdBlock)
k_preprocess_backward(gspm_gaussians G, ViewTable vt, const float *__restrict__ T_cw, RasterSettings rs,
                      float4 *__restrict__ grad2d, gspm_gaussian_grads out, int want_pose,
                      double *__restrict__ pose_part) {
    // One thread per Gaussian, looping over the views: the Gaussian's parameter gradients
    // are summed over the views in registers and added once (one float atomic per
    // parameter, not one per view), and its parameters stay in cache across the views.
    // The view-independent part of the projection is computed once, and the next view's
    // image-plane gradient row is loaded while this view's is processed.
    // Pose partials per wave and view in FP64.
    const int64_t n = G.n;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double gmu[3] = {0, 0, 0}, gls[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, go = 0.0, gc[3] = {0, 0, 0};
    bool touched = false;
    Proj P;
    const bool framed = g < n && gaussian_frame(G, g, n, P);
    float4 n0 = make_float4(0, 0, 0, 0), n1 = n0, n2 = n0, n3 = n0;
    if (g < n && vt.n_views > 0) {
        const float4 *src = grad2d + 4 * g;
        n0 = src[0]; n1 = src[1]; n2 = src[2]; n3 = src[3];
    }
    for (int v = 0; v < vt.n_views; ++v) {
        double pose[6] = {0, 0, 0, 0, 0, 0};
        bool any = false;
        const float4 q0 = n0, q1 = n1, q2 = n2, q3 = n3;
        if (g < n) {
            if (v + 1 < vt.n_views) {
                const float4 *nxt = grad2d + 4 * ((int64_t)(v + 1) * n + g);
                n0 = nxt[0]; n1 = nxt[1]; n2 = nxt[2]; n3 = nxt[3];
            }
            any = q0.x != 0.f || q0.y != 0.f || q0.z != 0.f || q0.w != 0.f || q1.x != 0.f || q1.y != 0.f ||
                  q1.z != 0.f || q1.w != 0.f || q2.x != 0.f || q2.y != 0.f || q2.z != 0.f || q2.w != 0.f ||
                  q3.x != 0.f;
            if (any) {  // leave the row cleared for the next backward
                float4 *src = grad2d + 4 * ((int64_t)v * n + g);
                const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
                src[0] = z; src[1] = z; src[2] = z; src[3] = z;
            }
        }
        if (any && framed) {
            project_view(T_cw + 12 * v, vt.fx[v], vt.fy[v], vt.cx[v], vt.cy[v], vt.width[v], vt.height[v], rs, P);
            any = P.visible;
        } else {
            any = false;
        }
        {
            if (any) {
                // Moments of g = alpha dL/dalpha over the pixel offsets d = pixel - mean.  With
                // alpha = o 2^e and e = -log2(e) d^T Q d / 2: dL/de = ln 2 g, so
                //   dL/du = sum g (Q d)_x, dL/dv = sum g (Q d)_y, dL/dQ = -sum g d d^T / 2,
                //   dL/do = sum g / o, so the logit's gradient is sum g (1 - o).
                const double R0 = q0.x, Rx = q0.y, Ry = q0.z, Rxx = q0.w, Rxy = q1.x, Ryy = q1.y, gz = q1.z;
                gc[0] += q1.w; gc[1] += q2.x; gc[2] += q2.y;
                const double gp[3] = {q2.z, q2.w, q3.x};
                const double Qa = P.Q[0], Qb = P.Q[1], Qc = P.Q[2];
                const double gu = Qa * Rx + Qb * Ry, gv = Qb * Rx + Qc * Ry;
                const double gQxx = -0.5 * Rxx, gQxy = -Rxy, gQyy = -0.5 * Ryy;
                // d L / d cov2 = -Q Ghat Q with Ghat the symmetric gradient wrt Q.
                const double G00 = gQxx, G01 = 0.5 * gQxy, G11 = gQyy;
                // X = Ghat Q
                const double X00 = G00 * Qa + G01 * Qb, X01 = G00 * Qb + G01 * Qc;
                const double X10 = G01 * Qa + G11 * Qb, X11 = G01 * Qb + G11 * Qc;
                const double H00 = -(Qa * X00 + Qb * X10), H01 = -(Qa * X01 + Qb * X11);
                const double H11 = -(Qb * X01 + Qc * X11);
                // cov2 = J Sc J^T + eps: gradient wrt Sc is J^T H J (H symmetric, off-diagonal H01).
                double GS[3][3];
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l)
                        GS[k][l] = P.J[0][k] * (H00 * P.J[0][l] + H01 * P.J[1][l]) +
                                   P.J[1][k] * (H01 * P.J[0][l] + H11 * P.J[1][l]);
                // d L / d J = 2 H J Sc.
                double JS[2][3];
                for (int r = 0; r < 2; ++r)
                    for (int c = 0; c < 3; ++c)
                        JS[r][c] = P.J[r][0] * P.Sc[0][c] + P.J[r][1] * P.Sc[1][c] + P.J[r][2] * P.Sc[2][c];
                const double gJ00 = 2.0 * (H00 * JS[0][0] + H01 * JS[1][0]);
                const double gJ02 = 2.0 * (H00 * JS[0][2] + H01 * JS[1][2]);
                const double gJ11 = 2.0 * (H01 * JS[0][1] + H11 * JS[1][1]);
                const double gJ12 = 2.0 * (H01 * JS[0][2] + H11 * JS[1][2]);

                // Camera-frame centre.
                const double fx = vt.fx[v], fy = vt.fy[v];
                const double iz = 1.0 / P.z, mx = P.m[0], my = P.m[1];
                double gm[3];
                gm[0] = gu * fx * iz;
                gm[1] = gv * fy * iz;
                gm[2] = -(gu * fx * mx + gv * fy * my) * iz * iz + gz;
                gm[2] += -(gJ00 * P.J[0][0] + gJ11 * P.J[1][1]) * iz;
                if (P.clamp_x) {
                    gm[2] += gJ02 * (-P.J[0][2] * iz);
                } else {
                    gm[0] += gJ02 * (-fx * iz * iz);
                    gm[2] += gJ02 * (-2.0 * P.J[0][2] * iz);
                }
                if (P.clamp_y) {
                    gm[2] += gJ12 * (-P.J[1][2] * iz);
                } else {
                    gm[1] += gJ12 * (-fy * iz * iz);
                    gm[2] += gJ12 * (-2.0 * P.J[1][2] * iz);
                }
                if (rs.frame == 1) { gm[0] += gp[0]; gm[1] += gp[1]; gm[2] += gp[2]; }
                for (int c = 0; c < 3; ++c)
                    gmu[c] += P.W[0][c] * gm[0] + P.W[1][c] * gm[1] + P.W[2][c] * gm[2];
                if (rs.frame == 0) { gmu[0] += gp[0]; gmu[1] += gp[1]; gmu[2] += gp[2]; }

                if (want_pose) {
                    // Translation: dm = rho.  Rotation: dm = phi x m, dSc = [phi]x Sc - Sc [phi]x.
                    pose[0] = gm[0]; pose[1] = gm[1]; pose[2] = gm[2];
                    pose[3] = P.m[1] * gm[2] - P.m[2] * gm[1];
                    pose[4] = P.m[2] * gm[0] - P.m[0] * gm[2];
                    pose[5] = P.m[0] * gm[1] - P.m[1] * gm[0];
                    // A = Sc GS - GS Sc (antisymmetric); d L / d phi += 2 (A12, -A02, A01), GS symmetrised.
                    double Gs[3][3];
                    for (int k = 0; k < 3; ++k)
                        for (int l = 0; l < 3; ++l) Gs[k][l] = 0.5 * (GS[k][l] + GS[l][k]);
                    double A01 = 0, A02 = 0, A12 = 0;
                    for (int k = 0; k < 3; ++k) {
                        A01 += P.Sc[0][k] * Gs[k][1] - Gs[0][k] * P.Sc[k][1];
                        A02 += P.Sc[0][k] * Gs[k][2] - Gs[0][k] * P.Sc[k][2];
                        A12 += P.Sc[1][k] * Gs[k][2] - Gs[1][k] * P.Sc[k][2];
                    }
                    pose[3] += 2.0 * A12;
                    pose[4] += -2.0 * A02;
                    pose[5] += 2.0 * A01;
                }

                // Sc = W Sigma W^T: G_Sigma = W^T GS W; Sigma = (Rq S)(Rq S)^T.
                double T1[3][3], GSig[3][3];
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l)
                        T1[k][l] = P.W[0][k] * GS[0][l] + P.W[1][k] * GS[1][l] + P.W[2][k] * GS[2][l];
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l)
                        GSig[k][l] = T1[k][0] * P.W[0][l] + T1[k][1] * P.W[1][l] + T1[k][2] * P.W[2][l];
                // d L / d M = (GSig + GSig^T) M, M = Rq diag(s).
                double gR[3][3];
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) {
                        double acc = 0.0;
                        for (int b = 0; b < 3; ++b) acc += (GSig[r][b] + GSig[b][r]) * P.Rq[b][c] * P.s[c];
                        gR[r][c] = acc * P.s[c];
                        // gR holds dL/dM * s = dL/dRq; reuse acc for the scale below.
                    }
                for (int c = 0; c < 3; ++c) {
                    // dL/ds_c = sum_r dL/dM_rc Rq_rc = sum_r gR_rc Rq_rc / s_c; dL/dlog s = s dL/ds.
                    double acc = 0.0;
                    for (int r = 0; r < 3; ++r) acc += gR[r][c] * P.Rq[r][c];
                    gls[c] += acc;
                }
                const double w = P.qn[0], x = P.qn[1], y = P.qn[2], z = P.qn[3];
                double gqn[4];
                gqn[0] = 2.0 * (z * (gR[1][0] - gR[0][1]) + y * (gR[0][2] - gR[2][0]) + x * (gR[2][1] - gR[1][2]));
                gqn[1] = 2.0 * (y * (gR[0][1] + gR[1][0]) + z * (gR[0][2] + gR[2][0]) + w * (gR[2][1] - gR[1][2])) -
                         4.0 * x * (gR[1][1] + gR[2][2]);
                gqn[2] = 2.0 * (x * (gR[0][1] + gR[1][0]) + w * (gR[0][2] - gR[2][0]) + z * (gR[1][2] + gR[2][1])) -
                         4.0 * y * (gR[0][0] + gR[2][2]);
                gqn[3] = 2.0 * (w * (gR[1][0] - gR[0][1]) + x * (gR[0][2] + gR[2][0]) + y * (gR[1][2] + gR[2][1])) -
                         4.0 * z * (gR[0][0] + gR[1][1]);
                const double dot = gqn[0] * w + gqn[1] * x + gqn[2] * y + gqn[3] * z;
                const double iq = 1.0 / P.qnorm;
                for (int k = 0; k < 4; ++k) gq[k] += (gqn[k] - P.qn[k] * dot) * iq;
                go += R0 * (1.0 - P.a);
            }
        }
        touched |= any;
        if (want_pose) {
            // The wave's sums in a fixed shuffle order, one partial per wave and view (no
            // block barrier: at 2 waves per SIMD a barrier per view stalls the block).
#pragma unroll
            for (int k = 0; k < 6; ++k)
                for (int off = 32; off > 0; off >>= 1) pose[k] += __shfl_xor(pose[k], off, kWave);
            if (lane_id() == 0) {
                const int64_t gw = (int64_t)blockIdx.x * kBwdWaves + threadIdx.x / kWave;
                double *dst = pose_part + ((int64_t)v * gridDim.x * kBwdWaves + gw) * 6;
                for (int k = 0; k < 6; ++k) dst[k] = pose[k];
            }
        }
    }
    if (g >= n) return;
    if (rs.grads_overwrite) {  // each Gaussian's gradients belong to this thread alone: plain stores
        if (out.means)
            for (int c = 0; c < 3; ++c) out.means[c * n + g] = (float)gmu[c];
        if (out.log_scales)
            for (int c = 0; c < 3; ++c) out.log_scales[c * n + g] = (float)gls[c];
        if (out.quats)
            for (int c = 0; c < 4; ++c) out.quats[c * n + g] = (float)gq[c];
        if (out.opacity_logit) out.opacity_logit[g] = (float)go;
        if (out.rgb)
            for (int c = 0; c < 3; ++c) out.rgb[c * n + g] = (float)gc[c];
        return;
    }
    if (!touched) return;
    if (out.means)
        for (int c = 0; c < 3; ++c) unsafeAtomicAdd(out.means + c * n + g, (float)gmu[c]);
    if (out.log_scales)
        for (int c = 0; c < 3; ++c) unsafeAtomicAdd(out.log_scales + c * n + g, (float)gls[c]);
    if (out.quats)
        for (int c = 0; c < 4; ++c) unsafeAtomicAdd(out.quats + c * n + g, (float)gq[c]);
    if (out.opacity_logit) unsafeAtomicAdd(out.opacity_logit + g, (float)go);
    if (out.rgb)
        for (int c = 0; c < 3; ++c) unsafeAtomicAdd(out.rgb + c * n + g, (float)gc[c]);
}

// One block per (view, pose component); the sum runs in a fixed order (deterministic).
__global__ void __launch_bounds__(256)
k_pose_reduce(const double *__restrict__ part, int64_t nblocks, float *__restrict__ pose_grad, int overwrite) {
    __shared__ double lds[4];
    const int v = blockIdx.x, k = blockIdx.y;
    double acc = 0.0;
    for (int64_t b = threadIdx.x; b < nblocks; b += blockDim.x) acc += part[((int64_t)v * nblocks + b) * 6 + k];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane_id() == 0) lds[threadIdx.x / 64] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float sum = (float)(lds[0] + lds[1] + lds[2] + lds[3]);
        pose_grad[v * 6 + k] = overwrite ? sum : pose_grad[v * 6 + k] + sum;
    }
}

// Zeroes one or two counters in one launch.
__global__ void k_clear2(uint32_t *a, uint32_t *b) {
    if (threadIdx.x == 0) {
        *a = 0u;
        if (b) *b = 0u;
    }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t value, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void k_fill_f32(float *p, float value, int64_t n) {
    const int64_t n4 = n / 4;
    float4 *p4 = reinterpret_cast<float4 *>(p);
    const float4 v4 = make_float4(value, value, value, value);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x)
        p4[i] = v4;
    for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// T <- Exp(xi) T with xi = (rho, phi): rotation by Rodrigues, translation V rho.
__global__ void k_pose_retract(int nv, float *T, const float *xi) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const double r0 = xi[6 * v], r1 = xi[6 * v + 1], r2 = xi[6 * v + 2];
    const double p0 = xi[6 * v + 3], p1 = xi[6 * v + 4], p2 = xi[6 * v + 5];
    const double th2 = p0 * p0 + p1 * p1 + p2 * p2, th = sqrt(th2);
    double A, B, C;
    if (th < 1e-6) {
        A = 1.0 - th2 / 6.0; B = 0.5 - th2 / 24.0; C = 1.0 / 6.0 - th2 / 120.0;
    } else {
        A = sin(th) / th; B = (1.0 - cos(th)) / th2; C = (th - sin(th)) / (th2 * th);
    }
    const double K[3][3] = {{0, -p2, p1}, {p2, 0, -p0}, {-p1, p0, 0}};
    double K2[3][3], R[3][3], V[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) K2[a][b] = K[a][0] * K[0][b] + K[a][1] * K[1][b] + K[a][2] * K[2][b];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const double I = a == b ? 1.0 : 0.0;
            R[a][b] = I + A * K[a][b] + B * K2[a][b];
            V[a][b] = I + B * K[a][b] + C * K2[a][b];
        }
    double Tin[3][4];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 4; ++b) Tin[a][b] = T[12 * v + 4 * a + b];
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b)
            T[12 * v + 4 * a + b] = (float)(R[a][0] * Tin[0][b] + R[a][1] * Tin[1][b] + R[a][2] * Tin[2][b]);
        T[12 * v + 4 * a + 3] = (float)(R[a][0] * Tin[0][3] + R[a][1] * Tin[1][3] + R[a][2] * Tin[2][3] +
                                        V[a][0] * r0 + V[a][1] * r1 + V[a][2] * r2);
    }
}

}  // namespace

static int fill_blocks(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    return (int)(b < 1 ? 1 : b);
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(fill_blocks(n)), dim3(256), 0, s, p, value, n);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, float value, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3(fill_blocks(n / 4 + 1)), dim3(256), 0, s, p, value, n);
    return hipGetLastError();
}

hipError_t launch_preprocess(const gspm_gaussians &g, const ViewTable &vt, const float *T_cw,
                             const RasterSettings &rs, float *records, uint32_t *counts,
                             uint32_t *dkey, uint4 *spans, uint32_t *big_list, uint32_t *big_count,
                             uint32_t *clear_also, hipStream_t s) {
    const int64_t R = g.n * vt.n_views;
    if (R <= 0) return clear_also ? launch_fill_u32(clear_also, 0u, 1, s) : hipSuccess;
    hipLaunchKernelGGL(k_clear2, dim3(1), dim3(64), 0, s, big_count, clear_also);
    hipLaunchKernelGGL(k_preprocess, dim3((unsigned)((g.n + 255) / 256), 1u), dim3(256), 0, s, g,
                       vt, T_cw, rs, reinterpret_cast<float4 *>(records), counts, dkey, spans, big_list, big_count);
    hipLaunchKernelGGL(k_count_big, dim3(1024), dim3(256), 0, s, reinterpret_cast<const float4 *>(records), vt, rs,
                       g.n, counts, big_list, big_count);
    return hipGetLastError();
}

static int64_t bwd_blocks(int64_t n) { return (n + kBwdBlock - 1) / kBwdBlock; }
int64_t pose_partial_blocks(int64_t n) { return bwd_blocks(n) * kBwdWaves; }

hipError_t launch_preprocess_backward(const gspm_gaussians &g, const ViewTable &vt, const float *T_cw,
                                      const RasterSettings &rs, float *grad2d,
                                      const gspm_gaussian_grads &out, bool want_pose,
                                      double *pose_partials, hipStream_t s) {
    if (g.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_preprocess_backward, dim3((unsigned)bwd_blocks(g.n)), dim3(kBwdBlock), 0, s,
                       g, vt, T_cw, rs, reinterpret_cast<float4 *>(grad2d), out, want_pose ? 1 : 0,
                       pose_partials);
    return hipGetLastError();
}

hipError_t launch_pose_reduce(const double *pose_partials, int64_t n_blocks, int n_views, float *pose_grad,
                              bool overwrite, hipStream_t s) {
    if (n_views <= 0 || n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pose_reduce, dim3(n_views, 6), dim3(256), 0, s, pose_partials, n_blocks, pose_grad,
                       overwrite ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_pose_retract(int n_views, float *T_cw, const float *xi, hipStream_t s) {
    hipLaunchKernelGGL(k_pose_retract, dim3((n_views + 63) / 64), dim3(64), 0, s, n_views, T_cw, xi);
    return hipGetLastError();
}

}  // namespace gspm
