// Per-patch least-squares scale between a prior pointmap and the rendered one (the scale
// alignment of Sec. 3.3.1, here as the per-patch least-squares estimator), fused with the
// gradient of the mapping loss (Eq. 17 without the isotropic term: the photometric L1
// of Eq. 10 and the pointmap L1 of Eq. 15 against the scale-aligned prior).
//
// One wave per strip of floor(64 / P) horizontally adjacent P x P patches: lane l owns
// image column x0 + l and walks the P rows of the strip, so every load and store is a
// 256-byte row segment.  Column sums (float64) are folded per patch through LDS, the
// scale is formed, and the same lanes revisit their (now cached) pixels to write the
// sign-based L1 gradients.  Loss partials go to one slot per wave and are summed per view
// in a fixed order by a second small kernel.
#include <mutex>

#include "gspm_common.h"

namespace gspm {

// Loss partials of the allocation-free entry point (gspm_window_loss_noalloc): one float64
// slot per wave strip, in a static device array that the code object holds on every GPU
// the library runs on.  In host code this name is only a stand-in for the symbol; kernels
// get the device address that static_loss_partials() looks up.
static __device__ __align__(256) double scratch[kStaticLossPartials];

namespace {

std::mutex g_scratch_mu;
double *g_scratch_addr[kMaxDevices] = {};

}  // namespace

hipError_t static_loss_partials(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // this device's copy of the array
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_addr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

namespace {

constexpr int kPatchBlock = 256;
constexpr int kPatchWaves = kPatchBlock / kWave;

__device__ inline float sgn(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }

struct StripTable {
    int32_t n_views;
    int32_t patch, per_wave;          // P, patches per wave strip
    int32_t npx[kMaxViews];           // patches per row
    int32_t strips_x[kMaxViews];      // strips per patch row
    int32_t patch_off[kMaxViews + 1];
    int32_t wave_off[kMaxViews + 1];
};

__global__ void __launch_bounds__(kPatchBlock)
k_patch_loss(ViewTable vt, StripTable st, const float *__restrict__ Xr, const float *__restrict__ Xp,
             const float *__restrict__ mask, const float *__restrict__ rgb, const float *__restrict__ target,
             float alpha, float *__restrict__ scale_out, int32_t *__restrict__ count_out,
             double *__restrict__ loss_part, float *__restrict__ grad_rgb, float *__restrict__ grad_pm) {
    __shared__ double lds[kPatchWaves][3][kWave];
    __shared__ float scale_lds[kPatchWaves][kWave];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int64_t gw = (int64_t)blockIdx.x * kPatchWaves + wid;
    const bool live = gw < st.wave_off[st.n_views];
    int v = 0;
    for (int k = 1; k < st.n_views; ++k)
        if (gw >= st.wave_off[k]) v = k;
    const int P = st.patch, per = st.per_wave;
    const int lw = live ? (int)(gw - st.wave_off[v]) : 0;
    const int py = lw / st.strips_x[v], sx = lw % st.strips_x[v];
    const int W = vt.width[v], H = vt.height[v];
    const int g = lane / P;                     // patch within the strip
    const int px = sx * per + g;                // patch column
    const int x = sx * per * P + lane;          // image column of this lane
    const bool col = live && g < per && px < st.npx[v] && x < W;
    const int y0 = py * P, y1 = min(H, y0 + P);
    const int64_t plane = (int64_t)W * H, o1 = vt.pix_off[v], o3 = 3 * vt.pix_off[v];

    double sxy = 0.0, syy = 0.0, cnt = 0.0;
    if (col) {
        for (int y = y0; y < y1; ++y) {
            const int64_t e = (int64_t)y * W + x;
            if (mask && mask[o1 + e] == 0.f) continue;
            const float r0 = Xr[o3 + e], r1 = Xr[o3 + plane + e], r2 = Xr[o3 + 2 * plane + e];
            const float p0 = Xp[o3 + e], p1 = Xp[o3 + plane + e], p2 = Xp[o3 + 2 * plane + e];
            sxy += (double)r0 * p0 + (double)r1 * p1 + (double)r2 * p2;
            syy += (double)p0 * p0 + (double)p1 * p1 + (double)p2 * p2;
            cnt += 1.0;
        }
    }
    lds[wid][0][lane] = sxy;
    lds[wid][1][lane] = syy;
    lds[wid][2][lane] = cnt;
    __syncthreads();
    if (live && lane < per) {
        const int pcol = sx * per + lane;
        if (pcol < st.npx[v]) {
            double a = 0.0, b = 0.0, c = 0.0;
            for (int k = 0; k < P; ++k) {
                a += lds[wid][0][lane * P + k];
                b += lds[wid][1][lane * P + k];
                c += lds[wid][2][lane * P + k];
            }
            const float s = b > 0.0 ? (float)(a / b) : 1.0f;
            const int64_t pid = st.patch_off[v] + (int64_t)py * st.npx[v] + pcol;
            scale_out[pid] = s;
            if (count_out) count_out[pid] = (int32_t)c;
            scale_lds[wid][lane] = s;
        }
    }
    __syncthreads();
    if (!grad_rgb) return;

    double lsum = 0.0;
    if (col) {
        const float s = scale_lds[wid][g];
        const float inv_n = 1.0f / (float)(3 * plane);
        const float wp = alpha * inv_n, wg = (1.0f - alpha) * inv_n;
        for (int y = y0; y < y1; ++y) {
            const int64_t e = (int64_t)y * W + x;
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
    }
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
    if (live && lane == 0) loss_part[gw] = lsum;
}

// loss[v] = sum of the wave partials of view v, in wave order.
__global__ void __launch_bounds__(256) k_loss_reduce(StripTable st, const double *__restrict__ part,
                                                     float *__restrict__ loss) {
    __shared__ double lds[4];
    const int v = blockIdx.x;
    double acc = 0.0;
    for (int w = st.wave_off[v] + threadIdx.x; w < st.wave_off[v + 1]; w += blockDim.x) acc += part[w];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane_id() == 0) lds[threadIdx.x / 64] = acc;
    __syncthreads();
    if (threadIdx.x == 0) loss[v] = (float)(lds[0] + lds[1] + lds[2] + lds[3]);
}

StripTable strip_table(const ViewTable &vt, int patch) {
    StripTable st;
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

}  // namespace

int64_t patch_loss_partials(const ViewTable &vt, int patch) {
    return strip_table(vt, patch).wave_off[vt.n_views];
}

hipError_t launch_patch_loss(const ViewTable &vt, const float *Xr, const float *Xp, const float *mask, int patch,
                             const float *rgb, const float *rgb_target, float alpha, float *scale_out,
                             int32_t *count_out, double *loss_part, float *loss_out, float *grad_rgb,
                             float *grad_pm, hipStream_t s) {
    const StripTable st = strip_table(vt, patch);
    const int64_t waves = st.wave_off[vt.n_views];
    if (waves <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_patch_loss, dim3((unsigned)((waves + kPatchWaves - 1) / kPatchWaves)), dim3(kPatchBlock), 0,
                       s, vt, st, Xr, Xp, mask, rgb, rgb_target, alpha, scale_out, count_out, loss_part, grad_rgb,
                       grad_pm);
    if (grad_rgb) hipLaunchKernelGGL(k_loss_reduce, dim3(vt.n_views), dim3(256), 0, s, st, loss_part, loss_out);
    return hipGetLastError();
}

}  // namespace gspm
