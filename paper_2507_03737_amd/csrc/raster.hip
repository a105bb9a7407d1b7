// Tile rasterizer: front-to-back compositing (Sec. 3.1, Eq. 2; Sec. 3.2.1, Eq. 3-5) and
// its backward.
//
// One workgroup per tile of T x T pixels (T = 8, 16 or 32) with T*T/PPT lanes.  Each wave
// owns a compact rectangle of the tile (8 x 8 pixels for PPT = 1, 8 x 16 for PPT = 2, ...)
// and each lane PPT vertically adjacent pixels of one of its columns.  The tile's
// depth-ordered record list is streamed through LDS in batches of one record per lane (a
// 64-byte record, converted to tile-local coordinates on load).  When a tile holds several
// waves, each wave of the forward first tests the whole batch against its own rectangle (one record per
// lane: the maximum of the concave base-2 exponent over the rectangle, against the
// record's threshold, with a rounding margin so that no record a pixel would accept is
// dropped) and then walks only the records that meet it, taken from the ballot mask with
// scalar bit scans.  Binning stays at tile granularity while the per-pixel work is that of
// 8-pixel-wide tiles.  A fragment is rejected on its base-2 exponent against a per-record
// threshold, so the exponential is only evaluated for pixels that composite it; the
// workgroup stops as soon as every pixel has reached the transmittance floor.
//
// The forward also records, per wave, which list entries one of its live pixels accepted
// (one bit per entry and wave, kept in the frame state).  The backward walks only those
// entries, front to back: in the matrix-core form each wave stages its own entries through
// LDS, 32 at a time and with no workgroup barrier; otherwise the workgroup stages batches
// of one record per lane.  It recomputes alpha and transmittance with the same
// instructions as the forward, so no per-fragment state is stored: only the bits and the
// per-pixel count of list entries up to the last contributing fragment.  The suffix sums
// that the alpha derivative needs are carried as a remainder: it starts at the sum over
// all fragments (from the forward's outputs) and each walked fragment subtracts its share.  Per record the wave needs up to 13
// sums over its pixels: the moments of alpha dL/dalpha over the pixel offsets (from which
// the mean, conic and opacity gradients follow) and the colour, depth and point sums.
// With one pixel per lane these are a dense contraction (per-wave constant functions of
// the pixel times per-record pixel values) done on the matrix cores for 8 records at a
// time; with several pixels per lane each lane adds its pixels' contributions and the
// wave adds them up with one reduce-scatter (cross-half lane swaps and DPP) of 8, 12 or
// 16 values.  Either way the atomics are paid once per wave and record.
#include <type_traits>

#include "gspm_common.h"

namespace gspm {

namespace {


struct TilePos {
    int gt;  // global tile index
    int v, W, H;
    int tx, ty;
    float x0, y0;     // tile origin
    int64_t plane;    // W * H of the view
    int64_t pix_off;  // packed offset of the view
};

// Workgroups run the tiles in the given order (heaviest first, so that the long lists do
// not start last and leave the chip idle behind them).
template <int TILE>
__device__ inline TilePos tile_pos(const ViewTable &vt, const uint32_t *order) {
    TilePos p;
    const int gt = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    p.gt = gt;
    p.v = find_view(vt, gt);
    const int lt = gt - vt.tile_off[p.v];
    p.tx = lt % vt.tiles_x[p.v];
    p.ty = lt / vt.tiles_x[p.v];
    p.W = vt.width[p.v];
    p.H = vt.height[p.v];
    p.x0 = (float)(p.tx * TILE);
    p.y0 = (float)(p.ty * TILE);
    p.plane = (int64_t)p.W * p.H;
    p.pix_off = vt.pix_off[p.v];
    return p;
}

// Stage record r into LDS slot q, in tile-local pixel coordinates, with the threshold
// -e_min, e_min = log2(alpha_min / opacity): alpha >= alpha_min exactly when the base-2
// exponent e = -s >= e_min, i.e. s <= -e_min, so rejected pixels never evaluate the
// exponential.
//   s0 = (u, v, a, b), s1 = (c, -e_min, opacity, record index), s2 = (colour, z), s3 = point
// with (a, b, c) the factored conic of the record.
// The acceptance test reads s0 and s1 only.
// With a list position pos, it replaces the point's unused fourth component (one 16-byte
// write instead of that write and a 4-byte one at a 16-byte stride, a 4-way conflict).
__device__ inline void stage(const float4 *__restrict__ rec, uint32_t r, float x0, float y0, float alpha_min,
                             float4 *s0, float4 *s1, float4 *s2, float4 *s3, int q, const uint32_t *pos = nullptr) {
    const float4 *src = rec + 4 * (int64_t)r;
    const float4 a = src[0], b = src[1], c = src[2], d = src[3];
    const float ul = (a.x - x0) + a.z;
    const float vl = (a.y - y0) + a.w;
    s0[q] = make_float4(ul, vl, b.x, b.y);
    s1[q] = make_float4(b.z, -__log2f(alpha_min / b.w), b.w, __uint_as_float(r));
    s2[q] = c;
    s3[q] = pos ? make_float4(d.x, d.y, d.z, __uint_as_float(*pos)) : d;
}

// min(alpha_max, a) for a >= 0, as one median instruction (min would first quiet a
// signalling NaN in the kernel-argument operand, on every call).
__device__ inline float clamp_alpha(float a, float amax) { return __builtin_amdgcn_fmed3f(a, 0.0f, amax); }

// Negated base-2 exponent of a Gaussian at a pixel offset (dx, dy) from its mean, from
// the factored conic and the per-column term a dx: s = -e = (a dx + b dy)^2 + (c dy)^2.
// A NaN offset gives NaN, which fails every threshold test.
__device__ inline float quad_s(float adx, float b, float c, float dy) {
    const float q1 = fmaf(b, dy, adx), q2 = c * dy;
    return fmaf(q1, q1, q2 * q2);
}

// Lane layout of a (TILE, PPT) workgroup: wave w owns a WW x WH pixel rectangle.
template <int TILE, int PPT>
struct Layout {
    static constexpr int NT = TILE * TILE / PPT;  // lanes per workgroup = records per batch
    static constexpr int NW = NT / kWave;         // waves per workgroup
    static constexpr int WH = TILE < 8 * PPT ? TILE : 8 * PPT;
    static constexpr int WW = kWave * PPT / WH;
    static constexpr bool CULL = NW > 1;  // a single wave owns the whole tile: binning culled already
    static_assert(WW * WH == kWave * PPT && TILE % WW == 0 && TILE % WH == 0, "unsupported raster shape");
    int lx, ly;                  // tile-local column and first row of this lane
    float rx0, rx1, ry0, ry1;    // this wave's rectangle of pixel centres, tile-local
    int w;                       // wave index within the workgroup
    __device__ Layout() {
        // The wave index is uniform: keep it (and the rectangle) in scalar registers.
        w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
        const int lane = lane_id();
        const int wx = (w % (TILE / WW)) * WW, wy = (w / (TILE / WW)) * WH;
        lx = wx + lane % WW;
        ly = wy + (lane / WW) * PPT;
        rx0 = (float)wx;
        rx1 = (float)(wx + WW - 1);
        ry0 = (float)wy;
        ry1 = (float)(wy + WH - 1);
    }
};

// Largest value of P d^2 + Q d t + R t^2 (R < 0) over t in [lo, hi], for fixed d.
__device__ inline float edge_max(float P, float Q, float R, float d, float lo, float hi) {
    const float t = fminf(hi, fmaxf(lo, -0.5f * Q * d * __builtin_amdgcn_rcpf(R)));
    return fmaf(fmaf(R, t, Q * d), t, P * d * d);
}

// Whether a staged record (s0 = (u, v, a, b), s1 = (c, -e_min, ...)) can reach its threshold
// at a pixel centre of the rectangle [x0, x1] x [y0, y1].  The exponent is concave with its
// maximum 0 at the mean, so it increases along any segment towards the mean: its maximum
// over the rectangle lies on an edge that faces the mean (a point elsewhere could move
// towards the mean inside the rectangle), or at the mean if that lies inside.  Both are
// covered by two segments: the column x = clamp(u, x0, x1) over [y0, y1] and the row
// y = clamp(v, y0, y1) over [x0, x1], each a one-dimensional concave quadratic (when the
// mean's x lies in [x0, x1], the column passes through the rectangle and the facing row
// holds the maximum; likewise for y).  The margin exceeds the float rounding of this
// evaluation plus that of the per-pixel evaluation (a few units in the last place of the
// sum of the terms' magnitudes), so the test never drops a record that a pixel accepts; it
// may keep a few that none does.
__device__ inline bool meets_rect(const float4 a, const float4 b, float x0, float x1, float y0, float y1) {
    // Expanded coefficients e = A dx^2 + B dx dy + C dy^2 of the factored conic (their
    // rounding is far inside the margin below).
    const float A = -a.z * a.z, B = -2.0f * a.z * a.w, C = -fmaf(a.w, a.w, b.x * b.x);
    const float ax = x0 - a.x, bx = x1 - a.x, ay = y0 - a.y, by = y1 - a.y;
    // Offsets of the column and the row from the mean: 0 where the mean's coordinate lies
    // inside the range, else that of the nearer edge (ax <= bx, ay <= by).
    const float cx = __builtin_amdgcn_fmed3f(0.0f, ax, bx), cy = __builtin_amdgcn_fmed3f(0.0f, ay, by);
    const float m = fmaxf(edge_max(A, B, C, cx, ay, by), edge_max(C, B, A, cy, ax, bx));
    const float DX = fmaxf(fabsf(ax), fabsf(bx)), DY = fmaxf(fabsf(ay), fabsf(by));
    const float S = fmaf(fabsf(A) * DX, DX, fmaf(fabsf(B) * DX, DY, fabsf(C) * DY * DY));
    return m >= -b.y - fmaf(0x1p-16f, S, 0x1p-10f);
}

// Ballot mask of the batch entries [c, c + 64) that this wave must walk.
template <bool CULL>
__device__ inline uint64_t batch_mask(const float4 *s0, const float4 *s1, int c, int cnt, float x0, float x1,
                                      float y0, float y1) {
    const int n = cnt - c;
    if (!CULL) return n >= kWave ? ~0ull : ((1ull << n) - 1ull);
    const int q = c + lane_id();  // below NT: c < cnt <= NT, both multiples of 64 apart from cnt
    const float4 a = s0[q], b = s1[q];
    // Whole 16-byte reads of consecutive records: the parts the test uses, read alone at a
    // 16-byte stride, would meet bank conflicts.
    asm volatile("" ::"v"(a.x), "v"(a.y), "v"(a.z), "v"(a.w), "v"(b.x), "v"(b.y), "v"(b.z), "v"(b.w));
    return ballot(q < cnt && meets_rect(a, b, x0, x1, y0, y1));
}

// FRAME is the pointmap frame (0 world, 1 camera, 2 from the depth, Eq. 5).  In the
// camera frame the depth is the composited point's z and is not accumulated twice; in
// frame 2 the point is not accumulated at all.  COUNT: also write each pixel's number of
// contributing fragments (work statistics).
template <int TILE, int PPT, int FRAME, bool COUNT>
__global__ void __launch_bounds__(TILE *TILE / PPT)
k_raster_fwd(ViewTable vt, RasterSettings rs, const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
             const float4 *__restrict__ rec, float *__restrict__ out_rgb, float *__restrict__ out_depth,
             float *__restrict__ out_alpha, float *__restrict__ out_pm, float *__restrict__ t_final,
             uint32_t *__restrict__ last, uint32_t *__restrict__ contrib, uint8_t *__restrict__ visible,
             const uint32_t *__restrict__ order, uint32_t *__restrict__ tile_work, uint64_t *__restrict__ wmask,
             int64_t wstride, FrameHeader *__restrict__ hdr) {
    using L = Layout<TILE, PPT>;
    constexpr int NT = L::NT;
    __shared__ float4 s0[NT], s1[NT], s2[NT], s3[NT];
    __shared__ uint32_t block_work;
    __shared__ uint32_t block_walk[2];  // COUNT: list entries walked and accepted by the waves
    const TilePos tp = tile_pos<TILE>(vt, order);
    const uint2 rg = ranges[tp.gt];
    const L lay;
    const int lx = lay.lx, ly = lay.ly;
    const float px = (float)lx;
    const float amin = rs.alpha_min, amax = rs.alpha_max, tmin = rs.t_min;
    const int i = tp.tx * TILE + lx;

    float T[PPT], C0[PPT], C1[PPT], C2[PPT], D[PPT], X0[PPT], X1[PPT], X2[PPT];
    // The pixel's tile-local row while it composites; NaN once it has stopped (or if it
    // lies outside the view), which makes the exponent NaN, so that the acceptance test
    // stays one comparison whose lane mask is the wave's ballot as it stands.
    float py[PPT];
    uint32_t n_last[PPT], n_contrib[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        T[k] = 1.0f;
        C0[k] = C1[k] = C2[k] = D[k] = X0[k] = X1[k] = X2[k] = 0.f;
        n_last[k] = n_contrib[k] = 0u;
        const int j = tp.ty * TILE + ly + k;
        py[k] = (i < tp.W && j < tp.H) ? (float)(ly + k) : __builtin_nanf("");
    }
    // Whether any pixel of this lane is still compositing.  Re-evaluated once per 64
    // entries: a wave whose pixels have all stopped walks at most the rest of one mask.
    auto lane_live = [&]() {
        bool l = false;
#pragma unroll
        for (int k = 0; k < PPT; ++k) l |= py[k] == py[k];
        return l;
    };
    uint64_t live = ballot(lane_live());  // lanes with a pixel still compositing
    bool wave_live = live != 0ull;
    // The rectangle of the wave's live pixels, which the chunks are culled against: once
    // pixels stop, the entries that only they would take are not walked.  Scalar bit work on
    // the live-lane mask (lane = column + WW x lane row, PPT pixel rows per lane row).
    float lrx0 = lay.rx0, lrx1 = lay.rx1, lry0 = lay.ry0, lry1 = lay.ry1;
    auto live_rect = [&]() {
        uint64_t cols = live;
#pragma unroll
        for (int sh = 32; sh >= L::WW; sh >>= 1) cols |= cols >> sh;
        cols &= (L::WW >= 64 ? ~0ull : (1ull << L::WW) - 1ull);
        const int c0 = (int)__builtin_ctzll(cols), c1 = 63 - (int)__builtin_clzll(cols);
        const int r0 = (int)__builtin_ctzll(live) / L::WW, r1 = (63 - (int)__builtin_clzll(live)) / L::WW;
        lrx0 = lay.rx0 + (float)c0;
        lrx1 = lay.rx0 + (float)c1;
        lry0 = lay.ry0 + (float)(r0 * PPT);
        lry1 = lay.ry0 + (float)(r1 * PPT + PPT - 1);
    };
    if (wave_live) live_rect();
    uint32_t n_walked = 0u, n_accepted = 0u;  // COUNT: this wave's walked and accepted entries
    // The next batch's record indices are loaded one batch ahead, so staging waits on one
    // global read (the record) rather than two dependent ones.
    uint32_t vnext = rg.x + threadIdx.x < rg.y ? vals[rg.x + threadIdx.x] : 0u;
    for (uint32_t base = rg.x; base < rg.y; base += NT) {
        const uint32_t kk = base + threadIdx.x;
        const uint32_t vcur = vnext;
        if (kk + NT < rg.y) vnext = vals[kk + NT];
        if (kk < rg.y) stage(rec, vcur, tp.x0, tp.y0, amin, s0, s1, s2, s3, threadIdx.x);
        __syncthreads();
        const int cnt = (int)min((uint32_t)NT, rg.y - base);
        for (int c = 0; c < cnt && wave_live; c += kWave) {
            uint64_t m = batch_mask<L::CULL>(s0, s1, c, cnt, lrx0, lrx1, lry0, lry1);
            if (COUNT) n_walked += (uint32_t)__popcll(m);
            uint64_t composited = 0ull;  // entries of this chunk accepted by one of the wave's live pixels
            while (m != 0ull) {
                const int q = c + (int)__builtin_ctzll(m);
                m &= m - 1ull;
                // All four words of the entry at once, before the test: the colour and point
                // reads share the address register, and their latency passes during the test
                // (most walked entries are composited).
                const float4 a = s0[q];
                const float4 b = s1[q];
                const float4 cc = s2[q];
                const float4 d = s3[q];
                // One 16-byte read now rather than a second, split read after the test.
                asm volatile("" ::"v"(b.z), "v"(b.w));
                const float dx = px - a.x;
                const float adx = a.z * dx;
                float sq[PPT];
                bool ok[PPT];
                uint64_t pass = 0ull;
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    sq[k] = quad_s(adx, a.w, b.x, py[k] - a.y);
                    ok[k] = sq[k] <= b.y;
                    pass |= ballot(ok[k]);
                }
                if (pass == 0ull) continue;  // wave-uniform: nothing composites this entry
                // Some live pixel accepts the entry: it is composited there or stops that pixel.
                // The backward walks these entries (a superset of those it finds a valid
                // pixel for; it skips the rest), scalar work only.
                composited |= 1ull << (q - c);
                // Whole 16-byte reads: a 12-byte read of one address for the whole wave keeps
                // the LDS busy twice as long as a 16-byte one.
                asm volatile("" ::"v"(cc.w), "v"(d.w));
                const uint32_t rel = base - rg.x + (uint32_t)q + 1u;
                bool added = false;
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    const float al = fminf(amax, b.z * __builtin_amdgcn_exp2f(-sq[k]));
                    const float Tn = fmaf(-al, T[k], T[k]);  // T (1 - alpha), rounded once
                    const bool add = ok[k] && !(Tn < tmin);
                    const bool stop = ok[k] && !add;  // one comparison; the masks combine in scalar code
                    const float w = add ? __fmul_rn(al, T[k]) : 0.0f;
                    C0[k] = fmaf(w, cc.x, C0[k]);
                    C1[k] = fmaf(w, cc.y, C1[k]);
                    C2[k] = fmaf(w, cc.z, C2[k]);
                    if (FRAME != 1) D[k] = fmaf(w, cc.w, D[k]);
                    if (FRAME != 2) {
                        X0[k] = fmaf(w, d.x, X0[k]);
                        X1[k] = fmaf(w, d.y, X1[k]);
                        X2[k] = fmaf(w, d.z, X2[k]);
                    }
                    T[k] = add ? Tn : T[k];
                    n_last[k] = add ? rel : n_last[k];
                    if (COUNT) n_contrib[k] += add ? 1u : 0u;
                    py[k] = stop ? __builtin_nanf("") : py[k];
                    added |= add;
                }
                if (visible) {  // uniform: marking requested
                    if (ballot(added) != 0ull && lane_id() == 0) visible[__float_as_uint(b.w)] = 1;
                }
            }
            if (COUNT) n_accepted += (uint32_t)__popcll(composited);
            if (composited != 0ull && lane_id() == 0) {
                // Entry q sits at list position base + q; the chunk's bits straddle at most
                // two words of this wave's plane.
                const uint64_t pos = (uint64_t)base + (uint64_t)c;
                uint64_t *w = wmask + (int64_t)lay.w * wstride + (int64_t)(pos >> 6);
                const int sh = (int)(pos & 63u);
                atomicOr((unsigned long long *)w, (unsigned long long)(composited << sh));
                if (sh != 0) atomicOr((unsigned long long *)(w + 1), (unsigned long long)(composited >> (64 - sh)));
            }
            const uint64_t now = ballot(lane_live());
            if (now != live) {  // wave-uniform: some pixels stopped in this chunk
                live = now;
                wave_live = live != 0ull;
                if (wave_live) live_rect();
            }
        }
        if (!__syncthreads_or(lane_live() ? 1 : 0)) break;
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int j = tp.ty * TILE + ly + k;
        if (!(i < tp.W && j < tp.H)) continue;
        const int64_t e = (int64_t)j * tp.W + i;
        const int64_t pix = tp.pix_off + e, o3 = 3 * tp.pix_off + e, plane = tp.plane;
        out_rgb[o3] = fmaf(T[k], rs.bg[0], C0[k]);
        out_rgb[o3 + plane] = fmaf(T[k], rs.bg[1], C1[k]);
        out_rgb[o3 + 2 * plane] = fmaf(T[k], rs.bg[2], C2[k]);
        const float depth = FRAME == 1 ? X2[k] : D[k];
        out_depth[pix] = depth;
        out_alpha[pix] = 1.0f - T[k];
        float x0 = X0[k], x1 = X1[k], x2 = X2[k];
        if (FRAME == 2) {
            const float rx = ((float)i - vt.cx[tp.v]) / vt.fx[tp.v];
            const float ry = ((float)j - vt.cy[tp.v]) / vt.fy[tp.v];
            x0 = depth * rx;
            x1 = depth * ry;
            x2 = depth;
        }
        out_pm[o3] = x0;
        out_pm[o3 + plane] = x1;
        out_pm[o3 + 2 * plane] = x2;
        t_final[pix] = T[k];
        last[pix] = n_last[k];
        if (COUNT) contrib[pix] = n_contrib[k];
    }
    if (COUNT) {  // the launch's walked and accepted (wave, entry) pairs, one atomic pair per workgroup
        if (threadIdx.x == 0) block_walk[0] = block_walk[1] = 0u;
        __syncthreads();
        if (lane_id() == 0) {
            atomicAdd(&block_walk[0], n_walked);
            atomicAdd(&block_walk[1], n_accepted);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            atomicAdd(reinterpret_cast<unsigned long long *>(&hdr->walked), (unsigned long long)block_walk[0]);
            atomicAdd(reinterpret_cast<unsigned long long *>(&hdr->accepted), (unsigned long long)block_walk[1]);
        }
    }
    if (tile_work) {  // uniform
        if (threadIdx.x == 0) block_work = 0u;
        __syncthreads();
        uint32_t m = 0u;
#pragma unroll
        for (int k = 0; k < PPT; ++k) m = max(m, n_last[k]);
        for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off, 64));
        if (lane_id() == 0) atomicMax(&block_work, m);
        __syncthreads();
        if (threadIdx.x == 0) tile_work[tp.gt] = block_work;
    }
}

__device__ inline float load_or0(const float *p, int64_t i) { return p ? p[i] : 0.0f; }

// Which per-record sums the backward forms, in value order, and the accumulator column
// of each: [sum g] [moments of g: 5] [colour: 3] [depth] [point: 3].  A pose-only pass
// (tracking) needs no opacity or colour gradient; the camera frame carries the depth
// gradient in the point's z, and frame 2 has no point term.
template <bool POSE_ONLY, int FRAME>
struct BwdValues {
    static constexpr bool kOpacity = !POSE_ONLY, kColour = !POSE_ONLY;
    static constexpr bool kDepth = FRAME != 1, kPoint = FRAME != 2;
    static constexpr int N = (kOpacity ? 1 : 0) + 5 + (kColour ? 3 : 0) + (kDepth ? 1 : 0) + (kPoint ? 3 : 0);
    static constexpr int NR = N <= 8 ? 8 : (N <= 12 ? 12 : 16);  // reduce-scatter width
    // Column of value k in bits [4k, 4k + 4).
    static constexpr uint64_t columns() {
        uint64_t c = 0;
        int k = 0;
        auto put = [&](int col) { c |= (uint64_t)col << (4 * k++); };
        if (kOpacity) put(0);
        for (int j = 1; j <= 5; ++j) put(j);
        if (kColour) { put(7); put(8); put(9); }
        if (kDepth) put(6);
        if (kPoint) { put(10); put(11); put(12); }
        return c;
    }
    static constexpr uint64_t kColumns = columns();
    // The per-pixel weighted sums (colour, depth, point: weight w times the pixel's upstream
    // gradient), their count and their columns, 4 bits each.
    static constexpr int NW = (kColour ? 3 : 0) + (kDepth ? 1 : 0) + (kPoint ? 3 : 0);
    static constexpr uint32_t kWColumns = (uint32_t)(kColumns >> (4 * (N - NW)));
};

template <int TILE, int PPT, bool POSE_ONLY, int FRAME, bool MX>
__global__ void __launch_bounds__(TILE *TILE / PPT) __attribute__((amdgpu_waves_per_eu(MX && PPT == 1 ? 6 : 1)))
k_raster_bwd(ViewTable vt, RasterSettings rs, const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
             const float4 *__restrict__ rec, const uint32_t *__restrict__ last, const float *__restrict__ t_final,
             gspm_const_images fwd, gspm_const_images up, float *__restrict__ grad2d,
             const uint32_t *__restrict__ order, FrameHeader *__restrict__ hdr, int64_t n_records) {
    // The frame state's layout follows the views, Gaussian count and tile of this call:
    // unless they (and the pointmap frame of the records) are the forward's, and the
    // forward's lists are complete, nothing below may be read.  The test is uniform over
    // the launch; one lane records the refusal for gspm_frame_status.
    if (hdr->magic != kFrameMagic || hdr->overflow != 0u || hdr->sort_stall != 0u || hdr->tile != (uint32_t)TILE ||
        hdr->n_views != (uint32_t)vt.n_views || hdr->n_tiles != (uint32_t)vt.tile_off[vt.n_views] ||
        hdr->n_pixels != (uint64_t)vt.pix_off[vt.n_views] || hdr->n_records != (uint64_t)n_records ||
        hdr->frame != (uint32_t)FRAME) {
        if (blockIdx.x == 0 && threadIdx.x == 0) hdr->bwd_error = 1u;
        return;
    }
    using L = Layout<TILE, PPT>;
    using V = BwdValues<POSE_ONLY, FRAME>;
    constexpr int NT = L::NT;
    // One pixel per lane: the per-record sums are a dense contraction done on the matrix
    // cores (below); each wave keeps its operand columns for kSlots records in LDS.
    constexpr bool kMfma = MX && PPT == 1;
    constexpr int kSlots = 8;
    static_assert(!kMfma || (L::WW == 8 && L::WH == 8), "one pixel per lane means 8 x 8 wave rectangles");
    // Records staged per batch for the whole workgroup; the matrix-core form stages per
    // wave instead (kWS entries at a time), which with its operand buffers leaves room for
    // six workgroups per compute unit (6 waves per SIMD, the register budget's target).
    constexpr int NS = kMfma ? 1 : NT;
    __shared__ float4 s0[NS], s1[NS], s2[NS], s3[NS];
    constexpr int kWS = 32;  // entries a wave stages at a time (matrix-core form)
    constexpr uint32_t kWSMask = kWS >= 32 ? 0xffffffffu : (uint32_t)((1ull << kWS) - 1ull);
    __shared__ float4 mw0[kMfma ? L::NW : 1][kMfma ? kWS : 1], mw1[kMfma ? L::NW : 1][kMfma ? kWS : 1],
        mw2[kMfma ? L::NW : 1][kMfma ? kWS : 1], mw3[kMfma ? L::NW : 1][kMfma ? kWS : 1];
    __shared__ uint32_t block_last;
    // B operand of slot column j (g: j = slot, w: j = 8 + slot) for pixel p = 4 kb + c
    // (kb = 4 q + e): the 16-byte word 64 q + 16 c + (j ^ (c + 4 (q & 1))) holds the four
    // pixels e = 0..3 of (q, c, j).  A flush lane's four values of one q are one 16-byte
    // read, and the 16 lanes of each c read 16 consecutive words in a permuted order, which
    // the LDS serves without conflicts; the XOR spreads the walk's one-column writes of the
    // 64 pixels over all banks (measured: no conflict cycles either way, where the padded
    // layout 272 q + 68 c + 4 j + e took 3.2 per read).
    // Slot s's record (mean, index) follows at kMeta + 4 s: (u, v, -, index).
    constexpr int kBq = 256, kBc = 64, kMeta = 4 * kBq;
    __shared__ __align__(16) float mf_b[kMfma ? L::NW : 1][kMfma ? kMeta + 4 * kSlots : 4];
    const TilePos tp = tile_pos<TILE>(vt, order);
    const uint2 rg = ranges[tp.gt];
    const L lay;
    const int lx = lay.lx, ly = lay.ly;
    const float px = (float)lx;
    const float amin = rs.alpha_min, amax = rs.alpha_max;
    const int i = tp.tx * TILE + lx;
    // Per-pixel upstream gradient and, to start the walk's remainder Rem, the total
    // G = sum_k w_k (g . e_k) + T_final (g_C . bg) that the forward's outputs give.
    uint32_t my_last[PPT];
    float gC0[PPT], gC1[PPT], gC2[PPT], gD[PPT], gA[PPT], gX0[PPT], gX1[PPT], gX2[PPT], Rem[PPT], py[PPT];
    float T[PPT];
    uint32_t thread_last = 0;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        my_last[k] = 0;
        gC0[k] = gC1[k] = gC2[k] = gD[k] = gA[k] = gX0[k] = gX1[k] = gX2[k] = Rem[k] = 0.f;
        T[k] = 1.0f;
        py[k] = (float)(ly + k);
        const int j = tp.ty * TILE + ly + k;
        if (!(i < tp.W && j < tp.H)) continue;
        const int64_t e = (int64_t)j * tp.W + i;
        const int64_t pix = tp.pix_off + e, o3 = 3 * tp.pix_off + e, plane = tp.plane;
        my_last[k] = last[pix];
        gC0[k] = load_or0(up.rgb, o3);
        gC1[k] = load_or0(up.rgb, o3 + plane);
        gC2[k] = load_or0(up.rgb, o3 + 2 * plane);
        gD[k] = load_or0(up.depth, pix);
        gA[k] = load_or0(up.alpha, pix);
        gX0[k] = load_or0(up.pointmap, o3);
        gX1[k] = load_or0(up.pointmap, o3 + plane);
        gX2[k] = load_or0(up.pointmap, o3 + 2 * plane);
        const float Tf = t_final[pix];
        const bool none = gC0[k] == 0.f && gC1[k] == 0.f && gC2[k] == 0.f && gD[k] == 0.f && gA[k] == 0.f &&
                          gX0[k] == 0.f && gX1[k] == 0.f && gX2[k] == 0.f;
        // The rgb output holds sum_k w_k c_k + T_final bg, which is exactly what G needs.
        Rem[k] = gC0[k] * fwd.rgb[o3] + gC1[k] * fwd.rgb[o3 + plane] + gC2[k] * fwd.rgb[o3 + 2 * plane] +
                gD[k] * fwd.depth[pix] + gA[k] * (1.0f - Tf);
        if (FRAME == 2) {
            // Eq. 5: the pointmap is D K^-1 [i, j, 1]^T, a function of the depth only.
            const float rx = ((float)i - vt.cx[tp.v]) / vt.fx[tp.v];
            const float ry = ((float)j - vt.cy[tp.v]) / vt.fy[tp.v];
            const float gXD = gX0[k] * rx + gX1[k] * ry + gX2[k];
            Rem[k] += gXD * fwd.depth[pix];
            gD[k] += gXD;
            gX0[k] = gX1[k] = gX2[k] = 0.f;
        } else {
            Rem[k] += gX0[k] * fwd.pointmap[o3] + gX1[k] * fwd.pointmap[o3 + plane] +
                     gX2[k] * fwd.pointmap[o3 + 2 * plane];
        }
        if (FRAME == 1) {
            // The depth is the point's z: one gradient for both.
            gX2[k] += gD[k];
            gD[k] = 0.f;
        }
        if (none) my_last[k] = 0;  // nothing flows back from this pixel
        thread_last = max(thread_last, my_last[k]);
    }
    if (threadIdx.x == 0) block_last = 0;
    __syncthreads();
    uint32_t wave_last = thread_last;
    for (int off = 32; off > 0; off >>= 1) wave_last = max(wave_last, (uint32_t)__shfl_xor((int)wave_last, off, 64));
    wave_last = (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_last);  // uniform: keep it scalar
    if (lane_id() == 0) atomicMax(&block_last, wave_last);
    __syncthreads();
    const uint32_t end = rg.x + block_last;

    // Matrix-core form of the per-record sums (PPT = 1).  For records j of a wave and its
    // 64 pixels p, every sum is  Out[f][j] = sum_p F_f(p) H_j(p):  the six moments take
    // F = 1, x, y, x^2, xy, y^2 (pixel offsets from the wave rectangle's centre) and
    // H = g = alpha dL/dalpha; the colour, depth and point sums take F = the pixel's
    // upstream gradient and H = w = alpha T.  Out is 16 x 16 with rows f (6 moments, then
    // up to 7 weighted sums) and columns (H in {g, w}) x (8 record slots), the contraction
    // runs over the 64 pixels: 16 v_mfma_f32_16x16x4f32 per 8 records.  The A operand
    // (F, 16 values per lane) is constant for the wave; the B operand (g and w of each
    // slot) is written by the walk.  Lane L supplies A[L % 16][4 kb + L / 16] and
    // B[4 kb + L / 16][L % 16] for step kb and receives D[4 (L / 16) + r][L % 16].
    typedef float v4f __attribute__((ext_vector_type(4)));
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave)), lane = lane_id();
    float Aop[kMfma ? 16 : 1];
    // Byte offset of this lane's pixel in column 0 (bits 4-6 clear), with its word's XOR
    // pattern in bits 4-6: column j's value then sits at (bofs ^ 16 j), one instruction
    // per record.
    const uint32_t bofs =
        4u * (uint32_t)((wv * (kMeta + 4 * kSlots) + (lane >> 4) * kBq + (lane & 3) * kBc + ((lane >> 2) & 3)) |
                        4 * ((lane & 3) + 4 * ((lane >> 4) & 1)));
    int slot = 0;  // filled record slots of this wave (wave-uniform)
    const float cxw = lay.rx0 + 3.5f, cyw = lay.ry0 + 3.5f;
    if constexpr (kMfma) {
        float *buf = mf_b[wv];
        float wg[7];
        int m = 0;
        if (V::kColour) { wg[m++] = gC0[0]; wg[m++] = gC1[0]; wg[m++] = gC2[0]; }
        if (V::kDepth) wg[m++] = gD[0];
        if (V::kPoint) { wg[m++] = gX0[0]; wg[m++] = gX1[0]; wg[m++] = gX2[0]; }
        // Pixel-major at a pitch of 9 words (coprime with the 32 banks): neither these writes
        // nor the reads below meet bank conflicts.
#pragma unroll
        for (int t = 0; t < V::NW; ++t) buf[9 * lane + t] = wg[t];
        __builtin_amdgcn_wave_barrier();
        const int f = lane & 15, c = lane >> 4;
#pragma unroll
        for (int kb = 0; kb < 16; ++kb) {
            const int p = 4 * kb + c;
            const float x = (float)(p & 7) - 3.5f, y = (float)(p >> 3) - 3.5f;
            float av = f == 0 ? 1.0f : f == 1 ? x : f == 2 ? y : f == 3 ? x * x : f == 4 ? x * y : y * y;
            if (f >= 6) av = f < 6 + V::NW ? buf[9 * p + f - 6] : 0.0f;
            Aop[kb] = av;
        }
        __builtin_amdgcn_wave_barrier();  // read before the walk overwrites the buffer
    }
    // What each lane of the flush produces: grad2d column j = lane % 16 of a record, from
    // row f of B column (H, slot) of the product (src: its offset in the transposed block,
    // has: the column is produced at all), and which moment it is (c1..c5: j = 1..5).
    struct FlushLane {
        bool has, c1, c2, c3, c4, c5;
        int src;
    } fl;
    {
        const int j = lane & 15;
        int src_f = j <= 5 && (j > 0 || V::kOpacity) ? j : -1;
#pragma unroll
        for (int m = 0; m < V::NW; ++m)
            if ((int)((V::kWColumns >> (4 * m)) & 15u) == j) src_f = 16 | (6 + m);
        fl.has = src_f >= 0;
        fl.src = fl.has ? (src_f >> 4) * 8 * 20 + (src_f & 15) : 0;
        fl.c1 = j == 1; fl.c2 = j == 2; fl.c3 = j == 3; fl.c4 = j == 4; fl.c5 = j == 5;
    }
    // Contract the first n slots and add the results to the records' rows.
    auto flush = [&](int n) {
        __builtin_amdgcn_wave_barrier();  // the slots are written (a wave's LDS accesses stay in order)
        const int j = lane & 15, c = lane >> 4;
        const float *src0 = mf_b[wv] + kBc * c + 4 * (j ^ c);        // q = 0, 2
        const float *src1 = mf_b[wv] + kBc * c + 4 * (j ^ (c + 4));  // q = 1, 3
        const float4 q0 = *reinterpret_cast<const float4 *>(src0);
        const float4 q1 = *reinterpret_cast<const float4 *>(src1 + kBq);
        const float4 q2 = *reinterpret_cast<const float4 *>(src0 + 2 * kBq);
        const float4 q3 = *reinterpret_cast<const float4 *>(src1 + 3 * kBq);
        const float bq[16] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w,
                              q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w};
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 16; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Aop[kb], bq[kb], acc, 0, 0, 0);
        // Transpose through LDS (over the B operand, read above) so that 16 adjacent lanes
        // hold one record's row (one cache line per record and atomic instruction):
        // dout[20 j + f] for column j, row f (the pitch of 20 keeps the 16-byte writes of a
        // phase in distinct banks).
        float *dout = mf_b[wv];
        *reinterpret_cast<float4 *>(dout + j * 20 + 4 * c) = make_float4(acc[0], acc[1], acc[2], acc[3]);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int sr = 4 * h + c;  // record slot of this lane
            const float4 mt = *reinterpret_cast<const float4 *>(mf_b[wv] + kMeta + 4 * sr);
            const float4 sm = *reinterpret_cast<const float4 *>(dout + sr * 20);  // S0, Sx, Sy, Sxx
            const float val = fl.has ? dout[fl.src + sr * 20] : 0.0f;
            // Moments about the wave centre -> about the record's mean (dx = x - ux):
            // R_x = S_x - ux S0, R_xx = S_xx - 2 ux S_x + ux^2 S0, R_xy = S_xy - uy S_x -
            // ux S_y + ux uy S0, and likewise in y.  The column of each lane picks its
            // coefficients by selects on wave-constant lane masks (no branches).
            const float ux = mt.x - cxw, uy = mt.y - cyw;
            float al = fl.c1 ? -ux : 0.0f;
            al = fl.c2 ? -uy : al;
            al = fl.c3 ? ux * ux : al;
            al = fl.c4 ? ux * uy : al;
            al = fl.c5 ? uy * uy : al;
            float be = fl.c3 ? -2.0f * ux : 0.0f;
            be = fl.c4 ? -uy : be;
            float ga = fl.c4 ? -ux : 0.0f;
            ga = fl.c5 ? -2.0f * uy : ga;
            const float out = fmaf(ga, sm.z, fmaf(be, sm.y, fmaf(al, sm.x, val)));
            const uint32_t rid = __float_as_uint(mt.w);
            if (sr < n && fl.has && out != 0.f) unsafeAtomicAdd(grad2d + (int64_t)rid * kG2 + j, out);
        }
        __builtin_amdgcn_wave_barrier();  // read before later records overwrite the buffer
    };

    // The entries that one of this wave's live pixels accepted in the forward (its bit plane
    // after the pair list): every entry with a valid pixel here, plus the few that only
    // stopped a pixel, so the walk needs no culling test and meets almost no entry without
    // a contribution.
    const int64_t cap = (int64_t)hdr->capacity;
    const uint64_t *plane = wmask_at(vals, cap) + (int64_t)lay.w * wmask_stride(cap);
    // A forward with another number of pixels per lane had other waves: cull instead.
    const bool use_bits = hdr->ppt == (uint32_t)PPT;
    auto wave_bits = [&](uint32_t pos) {  // the 64 bits of list positions pos .. pos + 63
        const uint64_t *wp = plane + (pos >> 6);
        const int sh = (int)(pos & 63u);
        uint64_t m = wp[0] >> sh;
        if (sh != 0) m |= wp[1] << (64 - sh);
        return m;
    };
    // One list entry (its staged record, and its position rel in the tile's list): the
    // per-pixel recomputation and this wave's sums for it.
    auto walk_record = [&](const float4 &a, const float4 &b, const float4 &cc, const float4 &d, uint32_t rel) {
        const float dx = px - a.x;
        const float adx = a.z * dx;
        float sq[PPT];
        bool valid[PPT];
        uint64_t any = 0ull;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            sq[k] = quad_s(adx, a.w, b.x, py[k] - a.y);
            // Two comparisons whose lane masks are combined by a scalar AND.
            valid[k] = rel < my_last[k] && sq[k] <= b.y;
            any |= ballot(valid[k]);
        }
        if constexpr (kMfma) {
            asm volatile("" ::"v"(cc.x), "v"(cc.y), "v"(cc.z), "v"(cc.w));
            // Whole 16-byte reads (a 12-byte read of one address for the whole wave keeps the
            // LDS busy twice as long).
            if constexpr (V::kPoint) asm volatile("" ::"v"(d.x), "v"(d.y), "v"(d.z), "v"(d.w));
        }
        if (any == 0ull) return;  // wave-uniform
        float v[V::NR];
#pragma unroll
        for (int t = V::N; t < V::NR; ++t) v[t] = 0.f;
        // The per-pixel terms, in two forms.  alpha = min(alpha_max, o exp2(-s)) can only be
        // clamped when the opacity o reaches alpha_max (rare), where a clamped alpha passes
        // no gradient; otherwise alpha is o exp2(-s) itself (o exp2(-s) <= o for s >= 0).
        auto pixel_terms = [&](auto may_clamp) {
            constexpr bool kClamp = decltype(may_clamp)::value;
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                // The first pixel assigns, later ones accumulate (x + 0 is not folded).
                auto add = [&](int t, float x) { v[t] = k == 0 ? x : v[t] + x; };
                auto mad = [&](int t, float x, float y) { v[t] = k == 0 ? x * y : fmaf(x, y, v[t]); };
                // Branch-free: an invalid pixel takes alpha = 0, so its weight and its alpha
                // gradient are 0 and T * (1 - 0) leaves T unchanged.
                const float dy = py[k] - a.y;
                const float ao = b.z * __builtin_amdgcn_exp2f(-sq[k]);
                const float al = valid[k] ? (kClamp ? clamp_alpha(ao, amax) : ao) : 0.0f;
                const float w = __fmul_rn(al, T[k]);
                float sv = fmaf(gC0[k], cc.x, fmaf(gC1[k], cc.y, fmaf(gC2[k], cc.z, gA[k])));
                if (V::kDepth) sv = fmaf(gD[k], cc.w, sv);
                if (V::kPoint) sv = fmaf(gX0[k], d.x, fmaf(gX1[k], d.y, fmaf(gX2[k], d.z, sv)));
                // Rem = G - sum of w s over this and earlier fragments: the later fragments'
                // share plus the background term.
                Rem[k] = fmaf(-w, sv, Rem[k]);
                const float one_m = __fsub_rn(1.0f, al);
                const float dLda = T[k] * sv - Rem[k] * __builtin_amdgcn_rcpf(one_m);
                const float g = kClamp && al >= amax ? 0.0f : dLda * al;
                T[k] = fmaf(-al, T[k], T[k]);  // as in the forward
                if constexpr (kMfma) {
                    float *bw = reinterpret_cast<float *>(reinterpret_cast<char *>(&mf_b[0][0]) +
                                                          (bofs ^ (16u * (uint32_t)slot)));
                    bw[0] = g;
                    bw[4 * kSlots] = w;
                    // The slot's record mean and index, stored by lane 0 (whose pixel offset is
                    // 0) behind the B operand, straight from the registers they were read into.
                    if (lane == 0) {
                        *reinterpret_cast<float2 *>(bw + kMeta) = make_float2(a.x, a.y);
                        bw[kMeta + 3] = b.w;
                    }
                    continue;
                }
                const float gdx = g * dx, gdy = g * dy;
                int t = 0;
                if (V::kOpacity) add(t++, g);
                add(t++, gdx);
                add(t++, gdy);
                mad(t++, gdx, dx);
                mad(t++, gdy, dx);
                mad(t++, gdy, dy);
                if (V::kColour) {
                    mad(t++, w, gC0[k]);
                    mad(t++, w, gC1[k]);
                    mad(t++, w, gC2[k]);
                }
                if (V::kDepth) mad(t++, w, gD[k]);
                if (V::kPoint) {
                    mad(t++, w, gX0[k]);
                    mad(t++, w, gX1[k]);
                    mad(t++, w, gX2[k]);
                }
            }
        };
        // The opacity is wave-uniform; both are positive, so their bit patterns order as they do.
        if (__builtin_amdgcn_readfirstlane(__float_as_int(b.z)) >= __float_as_int(amax)) {
            pixel_terms(std::true_type{});
        } else {
            pixel_terms(std::false_type{});
        }
        if constexpr (kMfma) {
            if (++slot == kSlots) {
                flush(kSlots);
                slot = 0;
            }
            return;
        }
        int idx;
        const float tot = wave_reduce_scatter(v, idx);
        if (idx >= 0 && idx < V::N && tot != 0.f) {
            // The record index is wave-uniform: a scalar row base plus the lane's column.
            const uint32_t r = (uint32_t)__builtin_amdgcn_readfirstlane((int)__float_as_uint(b.w));
            const uint32_t col = (uint32_t)((V::kColumns >> (4 * idx)) & 15u);
            unsafeAtomicAdd(grad2d + (int64_t)r * kG2 + col, tot);
        }
    };
    if constexpr (kMfma) {
        // Each wave stages only the entries its bits mark, kWS at a time, in its own LDS
        // area, and walks them with no workgroup barrier.  The entry's list position rides
        // in the staged point's fourth component.
        float4 *w0 = mw0[wv], *w1 = mw1[wv], *w2 = mw2[wv], *w3 = mw3[wv];
        const uint32_t wend = rg.x + wave_last;
        // The next 64 positions' bits and record indices are loaded one step ahead, so that
        // a step waits on one global read (its records) rather than three dependent ones.
        uint64_t m_next = 0ull;
        uint32_t rec_next = 0u;
        if (rg.x < wend) {
            m_next = use_bits ? wave_bits(rg.x) : ~0ull;  // without bits every entry is tested
            rec_next = rg.x + (uint32_t)lane < wend ? vals[rg.x + (uint32_t)lane] : 0u;
        }
        for (uint32_t pos = rg.x; pos < wend; pos += kWave) {
            uint64_t m = m_next;
            const uint32_t rec_here = rec_next;
            const uint32_t np = pos + (uint32_t)kWave;
            if (np < wend) {
                m_next = use_bits ? wave_bits(np) : ~0ull;
                rec_next = np + (uint32_t)lane < wend ? vals[np + (uint32_t)lane] : 0u;
            }
            const uint32_t lim = wend - pos;
            if (lim < (uint32_t)kWave) m &= (1ull << lim) - 1ull;
            // Lane L holds the record index of position pos + L.
            const bool mine = (m >> lane) & 1ull;
            const uint32_t my_rec = rec_here;
#pragma unroll
            for (int h = 0; h < kWave / kWS; ++h) {
                const uint32_t mh = (uint32_t)((m >> (kWS * h)) & kWSMask);
                if (mh == 0u) continue;  // wave-uniform
                const int sub = lane - kWS * h;  // this lane's bit within the half
                if (mine && sub >= 0 && sub < kWS) {
                    const uint32_t si = (uint32_t)__popc(mh & ((1u << sub) - 1u));
                    const uint32_t p = pos + (uint32_t)lane;
                    const uint32_t rel = p - rg.x;
                    stage(rec, my_rec, tp.x0, tp.y0, amin, w0, w1, w2, w3, (int)si, &rel);
                }
                __builtin_amdgcn_wave_barrier();  // staged (a wave's LDS accesses stay in order)
                const int n_st = __popc(mh);
                for (int i = 0; i < n_st; ++i) {
                    const float4 a = w0[i];
                    const float4 b = w1[i];
                    const float4 cc = w2[i];
                    const float4 d = w3[i];
                    // One 16-byte read now rather than a second, split read after the test.
                    asm volatile("" ::"v"(b.z), "v"(b.w));
                    walk_record(a, b, cc, d, __float_as_uint(d.w));
                }
                __builtin_amdgcn_wave_barrier();  // read before the next entries are staged
            }
        }
    } else {
        // The next batch's record indices are loaded one batch ahead, so staging waits on one
        // global read (the record) rather than two dependent ones.
        uint32_t vnext = (threadIdx.x < NS && rg.x + threadIdx.x < end) ? vals[rg.x + threadIdx.x] : 0u;
        for (uint32_t base = rg.x; base < end; base += NS) {
            const uint32_t kk = base + threadIdx.x;
            const uint32_t vcur = vnext;
            if (threadIdx.x < NS && kk + NS < end) vnext = vals[kk + NS];
            const uint64_t bits0 = use_bits ? wave_bits(base) : 0ull;  // read while the batch is staged
            if (threadIdx.x < NS && kk < end) stage(rec, vcur, tp.x0, tp.y0, amin, s0, s1, s2, s3, threadIdx.x);
            __syncthreads();
            const int cnt = (int)min((uint32_t)NS, end - base);
            const uint32_t rel0 = base - rg.x;
            for (int c = 0; c < cnt && rel0 + (uint32_t)c < wave_last; c += kWave) {
                uint64_t m;
                if (use_bits) {
                    m = c == 0 ? bits0 : wave_bits(base + (uint32_t)c);
                    if (cnt - c < kWave) m &= (1ull << (cnt - c)) - 1ull;  // the next tile's entries
                } else {
                    m = batch_mask<L::CULL>(s0, s1, c, cnt, lay.rx0, lay.rx1, lay.ry0, lay.ry1);
                }
                // Entries at or past the wave's last contributing one are not walked.
                const uint32_t lim = wave_last - (rel0 + (uint32_t)c);
                if (lim < (uint32_t)kWave) m &= (1ull << lim) - 1ull;
                while (m != 0ull) {
                    const int q = c + (int)__builtin_ctzll(m);
                    m &= m - 1ull;
                    const uint32_t rel = rel0 + (uint32_t)q;
                    const float4 a = s0[q];
                    const float4 b = s1[q];
                    const float4 cc = s2[q];
                    const float4 d = s3[q];
                    // One 16-byte read now rather than a second, split read after the test.
                    asm volatile("" ::"v"(b.z), "v"(b.w));
                    walk_record(a, b, cc, d, rel);
                }
            }
            __syncthreads();
        }
    }
    if constexpr (kMfma) {
        if (slot > 0) flush(slot);  // wave-uniform
    }
}

}  // namespace

// Launch configurations: (tile, pixels per lane).
#define GSPM_RASTER_CONFIGS(X) X(8, 1) X(16, 1) X(16, 2) X(16, 4) X(32, 1) X(32, 2) X(32, 4)

bool raster_config_supported(int tile, int ppt) {
#define GSPM_CHECK(T_, P_) \
    if (tile == T_ && ppt == P_) return true;
    GSPM_RASTER_CONFIGS(GSPM_CHECK)
#undef GSPM_CHECK
    return false;
}

hipError_t launch_raster_forward(const ViewTable &vt, const RasterSettings &rs, const uint2 *ranges,
                                 const uint32_t *pair_vals, const float *records, float *rgb, float *depth,
                                 float *alpha, float *pointmap, float *t_final, uint32_t *last, uint32_t *contrib,
                                 uint8_t *visible, const uint32_t *order, uint32_t *tile_work, uint64_t *wmask,
                                 int64_t wstride, FrameHeader *hdr, hipStream_t s) {
    const int n_tiles = vt.tile_off[vt.n_views];
    const float4 *rec = reinterpret_cast<const float4 *>(records);
    if (rs.frame < 0 || rs.frame > 2) return hipErrorInvalidValue;
#define GSPM_FWD2(T_, P_, F_, C_)                                                                        \
    hipLaunchKernelGGL((k_raster_fwd<T_, P_, F_, C_>), dim3(n_tiles), dim3(T_ * T_ / P_), 0, s, vt, rs, \
                       ranges, pair_vals, rec, rgb, depth, alpha, pointmap, t_final, last, contrib, visible,   \
                       order, tile_work, wmask, wstride, hdr)
#define GSPM_FWD1(T_, P_, F_)                                                                  \
    do {                                                                                       \
        if (rs.count_work) GSPM_FWD2(T_, P_, F_, true);                                        \
        else GSPM_FWD2(T_, P_, F_, false);                                                     \
    } while (0)
#define GSPM_FWD(T_, P_)                                      \
    if (vt.tile == T_ && vt.ppt == P_) {                      \
        if (rs.frame == 0) GSPM_FWD1(T_, P_, 0);              \
        else if (rs.frame == 1) GSPM_FWD1(T_, P_, 1);         \
        else GSPM_FWD1(T_, P_, 2);                            \
        return hipGetLastError();                             \
    }
    GSPM_RASTER_CONFIGS(GSPM_FWD)
#undef GSPM_FWD
#undef GSPM_FWD2
#undef GSPM_FWD1
    return hipErrorInvalidValue;
}

hipError_t launch_raster_backward(const ViewTable &vt, const RasterSettings &rs, const uint2 *ranges,
                                  const uint32_t *pair_vals, const float *records, const uint32_t *last,
                                  const float *t_final, const gspm_const_images &fwd, const gspm_const_images &up,
                                  float *grad2d, bool pose_only, const uint32_t *order, FrameHeader *hdr,
                                  int64_t n_records, hipStream_t s) {
    const int n_tiles = vt.tile_off[vt.n_views];
    const float4 *rec = reinterpret_cast<const float4 *>(records);
    if (rs.frame < 0 || rs.frame > 2) return hipErrorInvalidValue;
#define GSPM_BWD1(T_, P_, PO_, F_, MX_)                                                                         \
    hipLaunchKernelGGL((k_raster_bwd<T_, P_, PO_, F_, MX_>), dim3(n_tiles), dim3(T_ * T_ / P_), 0, s, vt, rs, \
                       ranges, pair_vals, rec, last, t_final, fwd, up, grad2d, order, hdr, n_records)
#define GSPM_BWD2(T_, P_, PO_, MX_)                            \
    if (rs.frame == 0) GSPM_BWD1(T_, P_, PO_, 0, MX_);         \
    else if (rs.frame == 1) GSPM_BWD1(T_, P_, PO_, 1, MX_);    \
    else GSPM_BWD1(T_, P_, PO_, 2, MX_);
    // The matrix-core form exists at one pixel per lane only (MX = false elsewhere, so no
    // kernel is instantiated twice).
#define GSPM_BWD3(T_, P_, PO_)                                 \
    if (!rs.bwd_lane_reduce) {                                 \
        GSPM_BWD2(T_, P_, PO_, (P_ == 1))                      \
    } else {                                                   \
        GSPM_BWD2(T_, P_, PO_, false)                          \
    }
#define GSPM_BWD(T_, P_)                                  \
    if (vt.tile == T_ && vt.ppt == P_) {                  \
        if (pose_only) {                                  \
            GSPM_BWD3(T_, P_, true)                       \
        } else {                                          \
            GSPM_BWD3(T_, P_, false)                      \
        }                                                 \
        return hipGetLastError();                         \
    }
    GSPM_RASTER_CONFIGS(GSPM_BWD)
#undef GSPM_BWD
#undef GSPM_BWD3
#undef GSPM_BWD2
#undef GSPM_BWD1
    return hipErrorInvalidValue;
}

}  // namespace gspm
