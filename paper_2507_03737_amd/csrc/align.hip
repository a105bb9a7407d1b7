// Patch-based pointmap scale alignment (supplementary Alg. 1, behind Sec. 3.3.1) and
// pointmap replacement (Sec. 3.3.2, Eq. 14).
//
// The per-pixel scalar of a pointmap is its norm |X(x)|.  Alg. 1 rescales the prior as
// X^p_iter = sigma' X^p between iterations; norms, patch means and patch standard
// deviations of X^p_iter are then sigma' times those of X^p, so the normalised values
// (|X| - mu) / sd, and with them the set of correct points of a patch, do not depend on
// sigma'.  Only the patch test (candidate or not) does.  The work therefore splits into:
//   k_align_stats   one pass over the pixels (HBM-bound): per patch the means and
//                   standard deviations of |X^r| and |X^p|, and over the pixels that pass
//                   the normalised test, the sums of |X^r| and |X^p| and their count;
//   k_align_iterate one workgroup per view runs the max_iter iterations over the patch
//                   records: candidates under the current sigma', pooled sums over their
//                   correct points, sigma' = sum|X^r| / sum|X^p| (means over the same set).
// Everything after the float32 loads is float64, in the same formulas as the definition,
// so every discrete decision is taken at float64 precision.
//
// Layout: one wave per strip of floor(64 / P) horizontally adjacent P x P patches (as the
// patch-loss kernel): lane l owns image column x0 + l and walks the strip's P rows three
// times (means, spreads, correct points); the rows stay in cache between the passes.
#include <algorithm>

#include "gspm_common.h"

namespace gspm {

namespace {

constexpr int kAlignBlock = 256;
constexpr int kAlignWaves = kAlignBlock / kWave;

struct AlignStrips {
    int32_t n_views;
    int32_t patch, per_wave;
    int32_t npx[kMaxViews];
    int32_t strips_x[kMaxViews];
    int32_t patch_off[kMaxViews + 1];
    int32_t wave_off[kMaxViews + 1];
};

AlignStrips align_strips(const ViewTable &vt, int patch) {
    AlignStrips st;
    st.n_views = vt.n_views;
    st.patch = patch;
    st.per_wave = kWave / patch;
    st.patch_off[0] = 0;
    st.wave_off[0] = 0;
    for (int v = 0; v < vt.n_views; ++v) {
        const int npx = (vt.width[v] + patch - 1) / patch, npy = (vt.height[v] + patch - 1) / patch;
        st.npx[v] = npx;
        st.strips_x[v] = (npx + st.per_wave - 1) / st.per_wave;
        st.patch_off[v + 1] = st.patch_off[v] + npx * npy;
        st.wave_off[v + 1] = st.wave_off[v] + st.strips_x[v] * npy;
    }
    return st;
}

__device__ inline double norm3(const float *X, int64_t a, int64_t plane) {
    const double x = X[a], y = X[a + plane], z = X[a + 2 * plane];
    return sqrt(x * x + y * y + z * z);
}

// Sum of the P column partials of each patch of the strip; lanes < per receive them.
__device__ inline double fold_patch(double x, double (*lds)[kWave], int wid, int lane, int P, int per) {
    lds[wid][lane] = x;
    __syncthreads();
    double t = 0.0;
    if (lane < per)
        for (int k = 0; k < P; ++k) t += lds[wid][lane * P + k];
    __syncthreads();
    return t;
}

__global__ void __launch_bounds__(kAlignBlock)
k_align_stats(ViewTable vt, AlignStrips st, const float *__restrict__ Xr, const float *__restrict__ Xp,
              const float *__restrict__ mask, double eps_r, AlignPatch *__restrict__ out) {
    __shared__ double lds[kAlignWaves][kWave];
    __shared__ double mom[kAlignWaves][4][kWave / 1];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int64_t gw = (int64_t)blockIdx.x * kAlignWaves + wid;
    const bool live = gw < st.wave_off[st.n_views];
    int v = 0;
    for (int k = 1; k < st.n_views; ++k)
        if (gw >= st.wave_off[k]) v = k;
    const int P = st.patch, per = st.per_wave;
    const int lw = live ? (int)(gw - st.wave_off[v]) : 0;
    const int py = lw / st.strips_x[v], sx = lw % st.strips_x[v];
    const int W = vt.width[v], H = vt.height[v];
    const int g = lane / P;                       // patch within the strip
    const int x = sx * per * P + lane;            // image column of this lane
    const bool col = live && g < per && sx * per + g < st.npx[v] && x < W;
    const int y0 = py * P, y1 = min(H, y0 + P);
    const int64_t plane = (int64_t)W * H, o1 = vt.pix_off[v], o3 = 3 * vt.pix_off[v];

    // Pass 1: counts and means.
    double cnt = 0.0, sr = 0.0, sp = 0.0;
    if (col)
        for (int y = y0; y < y1; ++y) {
            const int64_t e = (int64_t)y * W + x;
            if (mask && mask[o1 + e] == 0.f) continue;
            sr += norm3(Xr, o3 + e, plane);
            sp += norm3(Xp, o3 + e, plane);
            cnt += 1.0;
        }
    const double pc = fold_patch(cnt, lds, wid, lane, P, per);
    const double psr = fold_patch(sr, lds, wid, lane, P, per);
    const double psp = fold_patch(sp, lds, wid, lane, P, per);
    if (lane < per) {
        mom[wid][0][lane] = pc > 0.0 ? psr / pc : 0.0;
        mom[wid][1][lane] = pc > 0.0 ? psp / pc : 0.0;
    }
    __syncthreads();
    const double mu_r = (g < per) ? mom[wid][0][g] : 0.0, mu_p = (g < per) ? mom[wid][1][g] : 0.0;

    // Pass 2: population standard deviations.
    double vr = 0.0, vp = 0.0;
    if (col)
        for (int y = y0; y < y1; ++y) {
            const int64_t e = (int64_t)y * W + x;
            if (mask && mask[o1 + e] == 0.f) continue;
            const double a = norm3(Xr, o3 + e, plane) - mu_r, b = norm3(Xp, o3 + e, plane) - mu_p;
            vr += a * a;
            vp += b * b;
        }
    const double pvr = fold_patch(vr, lds, wid, lane, P, per);
    const double pvp = fold_patch(vp, lds, wid, lane, P, per);
    if (lane < per) {
        mom[wid][2][lane] = pc > 0.0 ? sqrt(pvr / pc) : 0.0;
        mom[wid][3][lane] = pc > 0.0 ? sqrt(pvp / pc) : 0.0;
    }
    __syncthreads();
    const double sd_r = (g < per) ? mom[wid][2][g] : 0.0, sd_p = (g < per) ? mom[wid][3][g] : 0.0;

    // Pass 3: the normalised test |(|X^r| - mu_r) / sd_r - (|X^p| - mu_p) / sd_p| < eps_r.
    double csr = 0.0, csp = 0.0, cc = 0.0;
    if (col && sd_r > 0.0 && sd_p > 0.0)
        for (int y = y0; y < y1; ++y) {
            const int64_t e = (int64_t)y * W + x;
            if (mask && mask[o1 + e] == 0.f) continue;
            const double a = norm3(Xr, o3 + e, plane), b = norm3(Xp, o3 + e, plane);
            if (fabs((a - mu_r) / sd_r - (b - mu_p) / sd_p) < eps_r) {
                csr += a;
                csp += b;
                cc += 1.0;
            }
        }
    const double pcsr = fold_patch(csr, lds, wid, lane, P, per);
    const double pcsp = fold_patch(csp, lds, wid, lane, P, per);
    const double pcc = fold_patch(cc, lds, wid, lane, P, per);
    if (live && lane < per && sx * per + lane < st.npx[v]) {
        const int64_t pid = st.patch_off[v] + (int64_t)py * st.npx[v] + sx * per + lane;
        AlignPatch a;
        a.mu_r = mom[wid][0][lane];
        a.mu_p = mom[wid][1][lane];
        a.sd_r = mom[wid][2][lane];
        a.sd_p = mom[wid][3][lane];
        a.cp_sr = pcsr;
        a.cp_sp = pcsp;
        a.n = (int32_t)pc;
        a.cp_n = (int32_t)pcc;
        out[pid] = a;
    }
}

// One workgroup per view: the max_iter iterations of Alg. 1 over the patch records.
__global__ void __launch_bounds__(kAlignBlock)
k_align_iterate(AlignStrips st, const AlignPatch *__restrict__ patches, double delta_mu, double delta_sigma,
                int max_iter, double tau, gspm_align_result *__restrict__ result) {
    __shared__ double lds_a[kAlignWaves], lds_b[kAlignWaves];
    __shared__ long long lds_c[kAlignWaves], lds_n[kAlignWaves];
    const int v = blockIdx.x;
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int p0 = st.patch_off[v], p1 = st.patch_off[v + 1];
    double sigma = 1.0;
    long long cp_total = 0, n_valid = 0;
    for (int it = 0; it < max_iter; ++it) {
        double a = 0.0, b = 0.0;
        long long c = 0, nv = 0;
        for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
            const AlignPatch q = patches[p];
            nv += q.n;
            if (q.n <= 0) continue;
            // Statistics of X^p_iter = sigma' X^p.
            const double mu_p = sigma * q.mu_p, sd_p = sigma * q.sd_p;
            if (fabs(q.mu_r - mu_p) < delta_mu * mu_p && fabs(q.sd_r - sd_p) < delta_sigma * sd_p) {
                a += q.cp_sr;
                b += q.cp_sp;
                c += q.cp_n;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            a += __shfl_xor(a, off, 64);
            b += __shfl_xor(b, off, 64);
            c += __shfl_xor(c, off, 64);
            nv += __shfl_xor(nv, off, 64);
        }
        if (lane == 0) {
            lds_a[wid] = a;
            lds_b[wid] = b;
            lds_c[wid] = c;
            lds_n[wid] = nv;
        }
        __syncthreads();
        double A = 0.0, Bs = 0.0;
        long long C = 0, N = 0;
        for (int w = 0; w < kAlignWaves; ++w) {
            A += lds_a[w];
            Bs += lds_b[w];
            C += lds_c[w];
            N += lds_n[w];
        }
        __syncthreads();
        cp_total = C;
        n_valid = N;
        if (C > 0) sigma = A / Bs;  // mean |X^r[CP]| / mean |X^p[CP]| over the same CP
    }
    if (threadIdx.x == 0) {
        gspm_align_result r;
        r.scale = sigma;
        r.cp = (int32_t)cp_total;
        r.n_valid = (int32_t)n_valid;
        r.insufficient = (double)cp_total < tau * (double)n_valid ? 1 : 0;
        r.pad = 0;
        result[v] = r;
    }
}

// Eq. 14: keep X^r where |X^r - s X^p| <= eps_m |s X^p|, else take s X^p.
__global__ void __launch_bounds__(256)
k_replace(ViewTable vt, const float *__restrict__ Xr, const float *__restrict__ Xp,
          const gspm_align_result *__restrict__ res, double eps_m, float *__restrict__ out,
          uint32_t *__restrict__ replaced) {
    const int v = blockIdx.y;
    const int W = vt.width[v], H = vt.height[v];
    const int64_t plane = (int64_t)W * H, o3 = 3 * vt.pix_off[v];
    const double s = res[v].scale;
    __shared__ uint32_t wave_cnt[256 / kWave];
    uint32_t cnt = 0u;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < plane; e += (int64_t)gridDim.x * blockDim.x) {
        bool rep = false;
        {
            const int64_t a = o3 + e;
            const double r0 = Xr[a], r1 = Xr[a + plane], r2 = Xr[a + 2 * plane];
            const double h0 = s * (double)Xp[a], h1 = s * (double)Xp[a + plane], h2 = s * (double)Xp[a + 2 * plane];
            const double d0 = r0 - h0, d1 = r1 - h1, d2 = r2 - h2;
            const double d = sqrt(d0 * d0 + d1 * d1 + d2 * d2), t = eps_m * sqrt(h0 * h0 + h1 * h1 + h2 * h2);
            rep = !(d <= t);
            out[a] = rep ? (float)h0 : (float)r0;
            out[a + plane] = rep ? (float)h1 : (float)r1;
            out[a + 2 * plane] = rep ? (float)h2 : (float)r2;
        }
        cnt += rep ? 1u : 0u;
    }
    // One atomic per workgroup: the per-view counter sees few updates.
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if (lane_id() == 0) wave_cnt[threadIdx.x / kWave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = wave_cnt[0] + wave_cnt[1] + wave_cnt[2] + wave_cnt[3];
        if (t) atomicAdd(replaced + v, t);
    }
}

}  // namespace

int64_t align_patches(const ViewTable &vt, int patch) { return align_strips(vt, patch).patch_off[vt.n_views]; }

hipError_t launch_align_scale(const ViewTable &vt, const float *Xr, const float *Xp, const float *mask,
                              const gspm_align_params &prm, AlignPatch *patches, gspm_align_result *result,
                              hipStream_t s) {
    const AlignStrips st = align_strips(vt, prm.patch);
    const int64_t waves = st.wave_off[vt.n_views];
    if (waves > 0)
        hipLaunchKernelGGL(k_align_stats, dim3((unsigned)((waves + kAlignWaves - 1) / kAlignWaves)),
                           dim3(kAlignBlock), 0, s, vt, st, Xr, Xp, mask, (double)prm.eps_r, patches);
    hipLaunchKernelGGL(k_align_iterate, dim3(vt.n_views), dim3(kAlignBlock), 0, s, st, patches,
                       (double)prm.delta_mu, (double)prm.delta_sigma, prm.max_iter, (double)prm.tau, result);
    return hipGetLastError();
}

hipError_t launch_replace(const ViewTable &vt, const float *Xr, const float *Xp, const gspm_align_result *result,
                          float eps_m, float *out, uint32_t *replaced, hipStream_t s) {
    hipError_t e = launch_fill_u32(replaced, 0u, vt.n_views, s);
    if (e != hipSuccess) return e;
    int64_t maxp = 1;
    for (int v = 0; v < vt.n_views; ++v) maxp = std::max<int64_t>(maxp, (int64_t)vt.width[v] * vt.height[v]);
    const int64_t bx = std::min<int64_t>((maxp + 255) / 256, 4096);
    hipLaunchKernelGGL(k_replace, dim3((unsigned)bx, (unsigned)vt.n_views), dim3(256), 0, s, vt, Xr, Xp, result,
                       (double)eps_m, out, replaced);
    return hipGetLastError();
}

}  // namespace gspm
