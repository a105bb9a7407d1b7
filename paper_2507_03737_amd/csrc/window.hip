// Window management and regularisation around the mapping iteration:
//   - the isotropic regulariser of Eq. 16 (Sec. 3.3.3) and its gradient;
//   - keyframe covisibility, IOU and overlap coefficient of the visible Gaussian sets
//     (supplementary Eq. S1-S2), from the contributing-record marks of a forward;
//   - the median positive depth of each view (the median pointmap depth of the keyframe
//     rule), by radix selection on the float bits.
#include <algorithm>

#include "gspm_common.h"

namespace gspm {

namespace {

constexpr int kIsoBlock = 256;

// Eq. 16 per Gaussian, in float64: s = exp(log_scale), m = mean(s),
// loss = sum_k |s_k - m|, d loss / d log s_k = (sgn(s_k - m) - sum_j sgn(s_j - m) / 3) s_k.
__global__ void __launch_bounds__(kIsoBlock)
k_iso_loss(const float *__restrict__ ls, int64_t n, double weight, double *__restrict__ part,
           float *__restrict__ grad) {
    __shared__ double lds[kIsoBlock / kWave];
    double acc = 0.0;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
        const double s0 = exp((double)ls[g]), s1 = exp((double)ls[n + g]), s2 = exp((double)ls[2 * n + g]);
        const double m = (s0 + s1 + s2) / 3.0;
        const double r0 = s0 - m, r1 = s1 - m, r2 = s2 - m;
        const double g0 = (r0 > 0.0) - (r0 < 0.0), g1 = (r1 > 0.0) - (r1 < 0.0), g2 = (r2 > 0.0) - (r2 < 0.0);
        acc += fabs(r0) + fabs(r1) + fabs(r2);
        if (grad) {
            const double c = (g0 + g1 + g2) / 3.0;
            grad[g] += (float)(weight * (g0 - c) * s0);
            grad[n + g] += (float)(weight * (g1 - c) * s1);
            grad[2 * n + g] += (float)(weight * (g2 - c) * s2);
        }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane_id() == 0) lds[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kIsoBlock / kWave; ++w) t += lds[w];
        part[blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(256)
k_sum_parts(const double *__restrict__ part, int nb, double weight, float *__restrict__ out) {
    __shared__ double lds[4];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += part[b];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane_id() == 0) lds[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = (float)(weight * (lds[0] + lds[1] + lds[2] + lds[3]));
}

// Pairwise counts |G_i and G_j| (i <= j) of the visible sets; the diagonal is |G_i|.
__global__ void __launch_bounds__(256)
k_covis_count(const uint8_t *__restrict__ visible, int64_t n, int V, unsigned long long *__restrict__ counts) {
    __shared__ uint32_t lds[kMaxViews * kMaxViews];
    for (int k = threadIdx.x; k < V * V; k += blockDim.x) lds[k] = 0u;
    __syncthreads();
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
        uint32_t bits = 0u;
        for (int v = 0; v < V; ++v) bits |= visible[(int64_t)v * n + g] ? (1u << v) : 0u;
        for (uint32_t bi = bits; bi; bi &= bi - 1u) {
            const int i = __builtin_ctz(bi);
            for (uint32_t bj = bi; bj; bj &= bj - 1u) atomicAdd(&lds[i * V + __builtin_ctz(bj)], 1u);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < V * V; k += blockDim.x)
        if (lds[k]) atomicAdd(counts + k, (unsigned long long)lds[k]);
}

__global__ void k_covis_finalize(const unsigned long long *__restrict__ counts, int V,
                                 const FrameHeader *__restrict__ hdr, double *__restrict__ iou,
                                 double *__restrict__ oc, int64_t *__restrict__ count_out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= V * V) return;
    const int i = k / V, j = k % V;
    if (hdr->visible == 0u) {  // the forward did not mark contributing records
        iou[k] = oc[k] = __builtin_nan("");
        if (j == 0 && count_out) count_out[i] = -1;
        return;
    }
    const double ci = (double)counts[i * V + i], cj = (double)counts[j * V + j];
    const double inter = (double)counts[min(i, j) * V + max(i, j)];
    const double uni = ci + cj - inter, lo = fmin(ci, cj);
    iou[k] = uni > 0.0 ? inter / uni : 0.0;
    oc[k] = lo > 0.0 ? inter / lo : 0.0;
    if (j == 0 && count_out) count_out[i] = (int64_t)ci;
}

// Radix selection of the lower median of the positive depths of each view, 8 bits per
// round from the top: positive float bit patterns order like the floats.
struct MedianState {
    uint32_t prefix;  // bits selected so far
    uint32_t rank;    // rank of the median among the values that match the prefix
    uint32_t n;       // positive values of the view
    uint32_t pad;
};

__global__ void __launch_bounds__(256)
k_median_hist(ViewTable vt, const float *__restrict__ depth, int round, const MedianState *__restrict__ st,
              uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[256];
    const int v = blockIdx.y;
    h[threadIdx.x] = 0u;
    __syncthreads();
    const int shift = 24 - 8 * round;
    const uint32_t prefix = round ? st[v].prefix : 0u;
    const int64_t np = (int64_t)vt.width[v] * vt.height[v];
    const float *d = depth + vt.pix_off[v];
    // Uniform trip count per wave, so the ballots below see every lane.
    const int lane = lane_id();
    for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x; e0 < np; e0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = e0 + threadIdx.x;
        const float x = e < np ? d[e] : 0.0f;
        const uint32_t b = __float_as_uint(x);
        const bool valid = x > 0.0f && (round == 0 || (b >> (shift + 8)) == prefix);
        const uint32_t bin = (b >> shift) & 255u;
        // Depths cluster in few bins: one LDS atomic per distinct bin of the wave.
        uint64_t active = ballot(valid);
        while (active) {
            const int leader = __ffsll((unsigned long long)active) - 1;
            const uint32_t lb = (uint32_t)__shfl((int)bin, leader, kWave);
            const uint64_t same = ballot(valid && bin == lb);
            if (lane == leader) atomicAdd(&h[lb], (uint32_t)__popcll(same));
            active &= ~same;
        }
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(hist + v * 256 + threadIdx.x, h[threadIdx.x]);
}

__global__ void __launch_bounds__(256)
k_median_select(int round, MedianState *__restrict__ st, uint32_t *__restrict__ hist, float *__restrict__ out) {
    __shared__ uint32_t h[256];
    const int v = blockIdx.x;
    h[threadIdx.x] = hist[v * 256 + threadIdx.x];
    hist[v * 256 + threadIdx.x] = 0u;  // cleared for the next round
    __syncthreads();
    if (threadIdx.x != 0) return;
    MedianState s = st[v];
    if (round == 0) {
        uint32_t n = 0u;
        for (int b = 0; b < 256; ++b) n += h[b];
        s.n = n;
        s.rank = n ? (n - 1u) / 2u : 0u;
        s.prefix = 0u;
    }
    if (s.n != 0u) {
        uint32_t below = 0u;
        int b = 0;
        while (b < 255 && below + h[b] <= s.rank) below += h[b++];
        s.rank -= below;
        s.prefix = (s.prefix << 8) | (uint32_t)b;
    }
    st[v] = s;
    if (round == 3) out[v] = s.n ? __uint_as_float(s.prefix) : 0.0f;
}

}  // namespace

int64_t iso_partials() { return 1024; }

hipError_t launch_iso_loss(const float *log_scales, int64_t n, float weight, double *part, float *loss_out,
                           float *grad, hipStream_t s) {
    const int nb = (int)std::min<int64_t>(iso_partials(), std::max<int64_t>(1, (n + kIsoBlock - 1) / kIsoBlock));
    hipLaunchKernelGGL(k_iso_loss, dim3(nb), dim3(kIsoBlock), 0, s, log_scales, n, (double)weight, part, grad);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, part, nb, (double)weight, loss_out);
    return hipGetLastError();
}

hipError_t launch_covisibility(const uint8_t *visible, int64_t n, int V, const FrameHeader *hdr,
                               unsigned long long *counts, double *iou, double *oc, int64_t *count_out,
                               hipStream_t s) {
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(counts), 0u, 2 * (int64_t)V * V, s);
    if (e != hipSuccess) return e;
    if (n > 0) {
        const int64_t nb = std::min<int64_t>(1024, (n + 255) / 256);
        hipLaunchKernelGGL(k_covis_count, dim3((unsigned)nb), dim3(256), 0, s, visible, n, V, counts);
    }
    hipLaunchKernelGGL(k_covis_finalize, dim3((V * V + 255) / 256), dim3(256), 0, s, counts, V, hdr, iou, oc,
                       count_out);
    return hipGetLastError();
}

int64_t median_scratch_words(int V) { return (int64_t)V * (256 + 4); }

hipError_t launch_median_depth(const ViewTable &vt, const float *depth, uint32_t *scratch, float *out,
                               hipStream_t s) {
    const int V = vt.n_views;
    uint32_t *hist = scratch;
    MedianState *st = reinterpret_cast<MedianState *>(scratch + (int64_t)V * 256);
    hipError_t e = launch_fill_u32(scratch, 0u, median_scratch_words(V), s);
    if (e != hipSuccess) return e;
    int64_t maxp = 1;
    for (int v = 0; v < V; ++v) maxp = std::max<int64_t>(maxp, (int64_t)vt.width[v] * vt.height[v]);
    const unsigned bx = (unsigned)std::min<int64_t>(256, (maxp + 255) / 256);
    for (int round = 0; round < 4; ++round) {
        hipLaunchKernelGGL(k_median_hist, dim3(bx, V), dim3(256), 0, s, vt, depth, round, st, hist);
        hipLaunchKernelGGL(k_median_select, dim3(V), dim3(256), 0, s, round, st, hist, out);
    }
    return hipGetLastError();
}

}  // namespace gspm
