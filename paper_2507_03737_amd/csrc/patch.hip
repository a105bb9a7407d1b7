// Per-patch least-squares scale between a prior pointmap and the rendered one (the scale
// alignment of Sec. 3.3.1, here as the per-patch least-squares estimator), fused with the
// gradient of the mapping loss (Eq. 17 without the isotropic term: the photometric L1
// of Eq. 10 and the pointmap L1 of Eq. 15 against the scale-aligned prior).
//
// One wave per patch.  Pass 1 reduces sum(Xr . Xp), sum |Xp|^2 and the pixel count in
// float64; pass 2 (loss only) revisits the same pixels, which are now in cache, and
// writes sign-based L1 gradients.  Both passes touch each pixel's planes once, so the
// kernel streams at HBM rate.
#include "gspm_common.h"

namespace gspm {

namespace {

__device__ inline double wave_sum_d(double x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ inline float sgn(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }

struct PatchTable {
    int32_t n_views;
    int32_t npx[kMaxViews];          // patches per row
    int32_t patch_off[kMaxViews + 1];
};

__global__ void __launch_bounds__(256)
k_patch_loss(ViewTable vt, PatchTable pt, int P, const float *__restrict__ Xr, const float *__restrict__ Xp,
             const float *__restrict__ mask, const float *__restrict__ rgb, const float *__restrict__ target,
             float alpha, float *__restrict__ scale_out, int32_t *__restrict__ count_out,
             float *__restrict__ loss_out, float *__restrict__ grad_rgb, float *__restrict__ grad_pm) {
    const int lane = lane_id();
    const int64_t gp = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (gp >= pt.patch_off[pt.n_views]) return;  // wave-uniform
    int v = 0;
    for (int k = 1; k < pt.n_views; ++k)
        if (gp >= pt.patch_off[k]) v = k;
    const int lp = (int)(gp - pt.patch_off[v]);
    const int W = vt.width[v], H = vt.height[v];
    const int x0 = (lp % pt.npx[v]) * P, y0 = (lp / pt.npx[v]) * P;
    const int64_t plane = (int64_t)W * H;
    const int64_t o1 = vt.pix_off[v], o3 = 3 * vt.pix_off[v];
    const int npix = P * P;

    double sxy = 0.0, syy = 0.0, cnt = 0.0;
    for (int q = lane; q < npix; q += kWave) {
        const int i = x0 + q % P, j = y0 + q / P;
        if (i >= W || j >= H) continue;
        const int64_t e = (int64_t)j * W + i;
        if (mask && mask[o1 + e] == 0.f) continue;
        const float r0 = Xr[o3 + e], r1 = Xr[o3 + plane + e], r2 = Xr[o3 + 2 * plane + e];
        const float p0 = Xp[o3 + e], p1 = Xp[o3 + plane + e], p2 = Xp[o3 + 2 * plane + e];
        sxy += (double)r0 * p0 + (double)r1 * p1 + (double)r2 * p2;
        syy += (double)p0 * p0 + (double)p1 * p1 + (double)p2 * p2;
        cnt += 1.0;
    }
    sxy = wave_sum_d(sxy);
    syy = wave_sum_d(syy);
    cnt = wave_sum_d(cnt);
    const float s = syy > 0.0 ? (float)(sxy / syy) : 1.0f;
    if (lane == 0) {
        scale_out[gp] = s;
        if (count_out) count_out[gp] = (int32_t)cnt;
    }
    if (!grad_rgb) return;

    const float inv_n = 1.0f / (float)(3 * plane);
    const float wp = alpha * inv_n, wg = (1.0f - alpha) * inv_n;
    double lsum = 0.0;
    for (int q = lane; q < npix; q += kWave) {
        const int i = x0 + q % P, j = y0 + q / P;
        if (i >= W || j >= H) continue;
        const int64_t e = (int64_t)j * W + i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t a = o3 + c * plane + e;
            const float dp = rgb[a] - target[a];
            const float dg = Xr[a] - s * Xp[a];
            grad_rgb[a] = wp * sgn(dp);
            grad_pm[a] = wg * sgn(dg);
            lsum += (double)wp * fabsf(dp) + (double)wg * fabsf(dg);
        }
    }
    lsum = wave_sum_d(lsum);
    if (lane == 0) atomicAdd(loss_out + v, (float)lsum);
}

}  // namespace

hipError_t launch_patch_loss(const ViewTable &vt, const float *Xr, const float *Xp, const float *mask, int patch,
                             const float *rgb, const float *rgb_target, float alpha, float *scale_out,
                             int32_t *count_out, float *loss_out, float *grad_rgb, float *grad_pm, hipStream_t s) {
    PatchTable pt;
    pt.n_views = vt.n_views;
    pt.patch_off[0] = 0;
    for (int v = 0; v < vt.n_views; ++v) {
        const int npx = (vt.width[v] + patch - 1) / patch, npy = (vt.height[v] + patch - 1) / patch;
        pt.npx[v] = npx;
        pt.patch_off[v + 1] = pt.patch_off[v] + npx * npy;
    }
    const int64_t total = pt.patch_off[vt.n_views];
    if (total <= 0) return hipSuccess;
    if (grad_rgb) {
        hipError_t e = launch_fill_f32(loss_out, 0.0f, vt.n_views, s);
        if (e != hipSuccess) return e;
    }
    const int per_block = 256 / kWave;
    hipLaunchKernelGGL(k_patch_loss, dim3((unsigned)((total + per_block - 1) / per_block)), dim3(256), 0, s, vt, pt,
                       patch, Xr, Xp, mask, rgb, rgb_target, alpha, scale_out, count_out, loss_out, grad_rgb, grad_pm);
    return hipGetLastError();
}

}  // namespace gspm
