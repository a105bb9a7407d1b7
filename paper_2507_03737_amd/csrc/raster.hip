// Tile rasterizer: front-to-back compositing (Sec. 3.1, Eq. 2; Sec. 3.2.1, Eq. 3-5) and
// its backward.
//
// One workgroup per tile of T x T pixels (T = 8, 16 or 32), one lane per pixel.  The
// tile's depth-ordered record list is streamed through LDS in batches of T*T records
// (one 64-byte record per lane, converted to tile-local coordinates on load); every
// lane walks the batch, and the workgroup stops as soon as all its pixels have reached
// the transmittance floor.
//
// The backward walks the same list front to back and recomputes alpha and
// transmittance exactly as the forward did (same instructions), so no per-fragment
// state is stored: only the per-pixel count of list entries up to the last contributing
// fragment.  The suffix sums that the alpha derivative needs are recovered as
// (sum over all fragments) - (prefix sum), the total coming from the forward's outputs.
// Per-record gradients (13 values) are summed across the 64 lanes of a wave with one
// reduce-scatter (cross-half lane swaps and DPP), after which 13 lanes each hold one
// total and issue one float atomic.
#include "gspm_common.h"

namespace gspm {

namespace {

constexpr float kLn2 = 0.69314718055994530942f;

struct TilePos {
    int v, W, H;
    int i, j;         // pixel coordinates
    bool inside;
    float x0, y0;     // tile origin
    int64_t pix;      // packed pixel index
    int64_t plane;    // W * H of the view
    int64_t pix_off;  // packed offset of the view
};

template <int TILE>
__device__ inline TilePos tile_pos(const ViewTable &vt) {
    TilePos p;
    const int gt = blockIdx.x;
    p.v = find_view(vt, gt);
    const int lt = gt - vt.tile_off[p.v];
    const int tx = lt % vt.tiles_x[p.v], ty = lt / vt.tiles_x[p.v];
    p.W = vt.width[p.v];
    p.H = vt.height[p.v];
    p.i = tx * TILE + (int)(threadIdx.x % TILE);
    p.j = ty * TILE + (int)(threadIdx.x / TILE);
    p.inside = p.i < p.W && p.j < p.H;
    p.x0 = (float)(tx * TILE);
    p.y0 = (float)(ty * TILE);
    p.plane = (int64_t)p.W * p.H;
    p.pix_off = vt.pix_off[p.v];
    p.pix = p.pix_off + (int64_t)p.j * p.W + p.i;
    return p;
}

// Stage record r into LDS slot q, in tile-local pixel coordinates.
__device__ inline void stage(const float4 *__restrict__ rec, uint32_t r, float x0, float y0, float4 *s0,
                             float4 *s1, float4 *s2, float4 *s3, int q) {
    const float4 *src = rec + 4 * (int64_t)r;
    const float4 a = src[0], b = src[1], c = src[2], d = src[3];
    const float ul = (a.x - x0) + a.z;
    const float vl = (a.y - y0) + a.w;
    s0[q] = make_float4(ul, vl, b.x, b.y);
    s1[q] = make_float4(b.z, b.w, c.w, c.x);
    s2[q] = make_float4(c.y, c.z, d.x, d.y);
    s3[q] = make_float4(d.z, __uint_as_float(r), 0.f, 0.f);
}

template <int TILE>
__global__ void __launch_bounds__(TILE *TILE)
k_raster_fwd(ViewTable vt, RasterSettings rs, const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
             const float4 *__restrict__ rec, float *__restrict__ out_rgb, float *__restrict__ out_depth,
             float *__restrict__ out_alpha, float *__restrict__ out_pm, float *__restrict__ t_final,
             uint32_t *__restrict__ last, uint32_t *__restrict__ contrib) {
    constexpr int NT = TILE * TILE;
    __shared__ float4 s0[NT], s1[NT], s2[NT], s3[NT];
    const TilePos tp = tile_pos<TILE>(vt);
    const uint2 rg = ranges[blockIdx.x];
    const float px = (float)(threadIdx.x % TILE), py = (float)(threadIdx.x / TILE);
    const float amin = rs.alpha_min, amax = rs.alpha_max, tmin = rs.t_min;

    float T = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f, X0 = 0.f, X1 = 0.f, X2 = 0.f;
    uint32_t n_last = 0, n_contrib = 0;
    bool done = !tp.inside;
    for (uint32_t base = rg.x; base < rg.y; base += NT) {
        const uint32_t k = base + threadIdx.x;
        if (k < rg.y) stage(rec, vals[k], tp.x0, tp.y0, s0, s1, s2, s3, threadIdx.x);
        __syncthreads();
        const int cnt = (int)min((uint32_t)NT, rg.y - base);
        if (!done) {
            for (int q = 0; q < cnt; ++q) {
                const float4 a = s0[q], b = s1[q];
                float g2;
                const float al = frag_alpha(px - a.x, py - a.y, a.z, a.w, b.x, b.y, amax, g2);
                if (al < amin) continue;
                const float Tn = __fmul_rn(T, __fsub_rn(1.0f, al));
                if (Tn < tmin) {
                    done = true;
                    break;
                }
                const float w = __fmul_rn(al, T);
                const float4 c = s2[q];
                C0 = fmaf(w, b.w, C0);
                C1 = fmaf(w, c.x, C1);
                C2 = fmaf(w, c.y, C2);
                D = fmaf(w, b.z, D);
                X0 = fmaf(w, c.z, X0);
                X1 = fmaf(w, c.w, X1);
                X2 = fmaf(w, s3[q].x, X2);
                T = Tn;
                n_last = base - rg.x + (uint32_t)q + 1u;
                ++n_contrib;
            }
        }
        if (!__syncthreads_or(done ? 0 : 1)) break;
    }
    if (!tp.inside) return;
    const int64_t pix = tp.pix, plane = tp.plane, o3 = 3 * tp.pix_off + (int64_t)tp.j * tp.W + tp.i;
    out_rgb[o3] = fmaf(T, rs.bg[0], C0);
    out_rgb[o3 + plane] = fmaf(T, rs.bg[1], C1);
    out_rgb[o3 + 2 * plane] = fmaf(T, rs.bg[2], C2);
    out_depth[pix] = D;
    out_alpha[pix] = 1.0f - T;
    if (rs.frame == 2) {
        const float rx = ((float)tp.i - vt.cx[tp.v]) / vt.fx[tp.v];
        const float ry = ((float)tp.j - vt.cy[tp.v]) / vt.fy[tp.v];
        X0 = D * rx;
        X1 = D * ry;
        X2 = D;
    }
    out_pm[o3] = X0;
    out_pm[o3 + plane] = X1;
    out_pm[o3 + 2 * plane] = X2;
    t_final[pix] = T;
    last[pix] = n_last;
    contrib[pix] = n_contrib;
}

__device__ inline float load_or0(const float *p, int64_t i) { return p ? p[i] : 0.0f; }

template <int TILE, bool POSE_ONLY>
__global__ void __launch_bounds__(TILE *TILE)
k_raster_bwd(ViewTable vt, RasterSettings rs, const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
             const float4 *__restrict__ rec, const uint32_t *__restrict__ last, const float *__restrict__ t_final,
             gspm_const_images fwd, gspm_const_images up, float *__restrict__ grad2d) {
    constexpr int NT = TILE * TILE;
    __shared__ float4 s0[NT], s1[NT], s2[NT], s3[NT];
    __shared__ uint32_t block_last;
    const TilePos tp = tile_pos<TILE>(vt);
    const uint2 rg = ranges[blockIdx.x];
    const float px = (float)(threadIdx.x % TILE), py = (float)(threadIdx.x / TILE);
    const float amin = rs.alpha_min, amax = rs.alpha_max;
    const int lane = lane_id();

    // Per-pixel upstream gradient and the total sum_k w_k (g . e_k) from the forward outputs.
    uint32_t my_last = 0;
    float gC0 = 0.f, gC1 = 0.f, gC2 = 0.f, gD = 0.f, gA = 0.f, gX0 = 0.f, gX1 = 0.f, gX2 = 0.f;
    float Gtot = 0.f, bgterm = 0.f;
    if (tp.inside) {
        const int64_t pix = tp.pix, plane = tp.plane, o3 = 3 * tp.pix_off + (int64_t)tp.j * tp.W + tp.i;
        my_last = last[pix];
        gC0 = load_or0(up.rgb, o3);
        gC1 = load_or0(up.rgb, o3 + plane);
        gC2 = load_or0(up.rgb, o3 + 2 * plane);
        gD = load_or0(up.depth, pix);
        gA = load_or0(up.alpha, pix);
        gX0 = load_or0(up.pointmap, o3);
        gX1 = load_or0(up.pointmap, o3 + plane);
        gX2 = load_or0(up.pointmap, o3 + 2 * plane);
        const float Tf = t_final[pix];
        if (rs.frame == 2) {
            // Eq. 5: the pointmap is D K^-1 [i, j, 1]^T, a function of the depth only.
            const float rx = ((float)tp.i - vt.cx[tp.v]) / vt.fx[tp.v];
            const float ry = ((float)tp.j - vt.cy[tp.v]) / vt.fy[tp.v];
            gD += gX0 * rx + gX1 * ry + gX2;
            gX0 = gX1 = gX2 = 0.f;
        }
        bgterm = Tf * (gC0 * rs.bg[0] + gC1 * rs.bg[1] + gC2 * rs.bg[2]);
        Gtot = gC0 * fwd.rgb[o3] + gC1 * fwd.rgb[o3 + plane] + gC2 * fwd.rgb[o3 + 2 * plane] - bgterm +
               gD * fwd.depth[pix] + gA * (1.0f - Tf);
        if (rs.frame != 2)
            Gtot += gX0 * fwd.pointmap[o3] + gX1 * fwd.pointmap[o3 + plane] + gX2 * fwd.pointmap[o3 + 2 * plane];
        if (gC0 == 0.f && gC1 == 0.f && gC2 == 0.f && gD == 0.f && gA == 0.f && gX0 == 0.f && gX1 == 0.f &&
            gX2 == 0.f)
            my_last = 0;  // nothing flows back from this pixel
    }
    if (threadIdx.x == 0) block_last = 0;
    __syncthreads();
    // Wave-level bound first, then the block bound.
    uint32_t wave_last = my_last;
    for (int off = 32; off > 0; off >>= 1) wave_last = max(wave_last, (uint32_t)__shfl_xor((int)wave_last, off, 64));
    if (lane == 0) atomicMax(&block_last, wave_last);
    __syncthreads();
    const uint32_t end = rg.x + block_last;

    float T = 1.0f, Pfx = 0.0f;
    for (uint32_t base = rg.x; base < end; base += NT) {
        const uint32_t k = base + threadIdx.x;
        if (k < end) stage(rec, vals[k], tp.x0, tp.y0, s0, s1, s2, s3, threadIdx.x);
        __syncthreads();
        const int cnt = (int)min((uint32_t)NT, end - base);
        const uint32_t rel0 = base - rg.x;
        for (int q = 0; q < cnt; ++q) {
            if (rel0 + (uint32_t)q >= wave_last) break;  // wave-uniform
            const float4 a = s0[q], b = s1[q];
            const float dx = px - a.x, dy = py - a.y;
            float g2;
            const float al = frag_alpha(dx, dy, a.z, a.w, b.x, b.y, amax, g2);
            const bool valid = (rel0 + (uint32_t)q < my_last) && !(al < amin);
            float v[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) v[t] = 0.f;
            if (valid) {
                const float4 c = s2[q];
                const float pz = s3[q].x;
                const float w = __fmul_rn(al, T);
                const float s = gC0 * b.w + gC1 * c.x + gC2 * c.y + gD * b.z + gA + gX0 * c.z + gX1 * c.w + gX2 * pz;
                Pfx = fmaf(w, s, Pfx);
                const float one_m = __fsub_rn(1.0f, al);
                const float dLda = T * s - (Gtot - Pfx + bgterm) * __builtin_amdgcn_rcpf(one_m);
                if (!(b.y * g2 > amax)) {
                    const float Gl = dLda * al * kLn2;
                    v[0] = -Gl * (2.0f * a.z * dx + a.w * dy);
                    v[1] = -Gl * (a.w * dx + 2.0f * b.x * dy);
                    v[2] = Gl * dx * dx;
                    v[3] = Gl * dx * dy;
                    v[4] = Gl * dy * dy;
                    if (!POSE_ONLY) v[5] = dLda * g2;
                }
                v[6] = w * gD;
                if (!POSE_ONLY) {
                    v[7] = w * gC0;
                    v[8] = w * gC1;
                    v[9] = w * gC2;
                }
                v[10] = w * gX0;
                v[11] = w * gX1;
                v[12] = w * gX2;
                T = __fmul_rn(T, one_m);
            }
            if (__ballot(valid) == 0ull) continue;
            const float tot = wave_reduce_scatter16(v);
            const int idx = (lane >> 2) & 15;
            if ((lane & 3) == 0 && idx < kG2Used && tot != 0.f) {
                const uint32_t r = __float_as_uint(s3[q].y);
                unsafeAtomicAdd(grad2d + (int64_t)r * kG2 + idx, tot);
            }
        }
        __syncthreads();
    }
}

}  // namespace

template <int TILE>
static void fwd_launch(const ViewTable &vt, const RasterSettings &rs, const uint2 *ranges, const uint32_t *vals,
                       const float *records, float *rgb, float *depth, float *alpha, float *pm, float *t_final,
                       uint32_t *last, uint32_t *contrib, hipStream_t s) {
    const int n_tiles = vt.tile_off[vt.n_views];
    hipLaunchKernelGGL((k_raster_fwd<TILE>), dim3(n_tiles), dim3(TILE * TILE), 0, s, vt, rs, ranges, vals,
                       reinterpret_cast<const float4 *>(records), rgb, depth, alpha, pm, t_final, last, contrib);
}

hipError_t launch_raster_forward(const ViewTable &vt, const RasterSettings &rs, const uint2 *ranges,
                                 const uint32_t *pair_vals, const float *records, float *rgb, float *depth,
                                 float *alpha, float *pointmap, float *t_final, uint32_t *last, uint32_t *contrib,
                                 hipStream_t s) {
    switch (vt.tile) {
        case 8: fwd_launch<8>(vt, rs, ranges, pair_vals, records, rgb, depth, alpha, pointmap, t_final, last, contrib, s); break;
        case 32: fwd_launch<32>(vt, rs, ranges, pair_vals, records, rgb, depth, alpha, pointmap, t_final, last, contrib, s); break;
        default: fwd_launch<16>(vt, rs, ranges, pair_vals, records, rgb, depth, alpha, pointmap, t_final, last, contrib, s); break;
    }
    return hipGetLastError();
}

template <int TILE, bool POSE_ONLY>
static void bwd_launch(const ViewTable &vt, const RasterSettings &rs, const uint2 *ranges, const uint32_t *vals,
                       const float *records, const uint32_t *last, const float *t_final, const gspm_const_images &fwd,
                       const gspm_const_images &up, float *grad2d, hipStream_t s) {
    const int n_tiles = vt.tile_off[vt.n_views];
    hipLaunchKernelGGL((k_raster_bwd<TILE, POSE_ONLY>), dim3(n_tiles), dim3(TILE * TILE), 0, s, vt, rs, ranges, vals,
                       reinterpret_cast<const float4 *>(records), last, t_final, fwd, up, grad2d);
}

hipError_t launch_raster_backward(const ViewTable &vt, const RasterSettings &rs, const uint2 *ranges,
                                  const uint32_t *pair_vals, const float *records, const uint32_t *last,
                                  const float *t_final, const gspm_const_images &fwd, const gspm_const_images &up,
                                  float *grad2d, bool pose_only, hipStream_t s) {
#define GSPM_BWD(T)                                                                                         \
    (pose_only ? bwd_launch<T, true>(vt, rs, ranges, pair_vals, records, last, t_final, fwd, up, grad2d, s) \
               : bwd_launch<T, false>(vt, rs, ranges, pair_vals, records, last, t_final, fwd, up, grad2d, s))
    switch (vt.tile) {
        case 8: GSPM_BWD(8); break;
        case 32: GSPM_BWD(32); break;
        default: GSPM_BWD(16); break;
    }
#undef GSPM_BWD
    return hipGetLastError();
}

}  // namespace gspm
