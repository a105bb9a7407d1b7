// Internal declarations shared by the HIP translation units of libgspm (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gspm.h"

namespace gspm {

constexpr int kMaxViews = GSPM_MAX_VIEWS;
constexpr int kWave = 64;

// Per-launch table of the views of a window, passed by value as a kernel argument so
// that a captured graph holds it.  Tiles of all views form one global tile space
// (view v owns [tile_off[v], tile_off[v+1])); pixels are packed the same way.
struct ViewTable {
    int32_t n_views;
    int32_t tile;
    int32_t ppt;  // pixels per lane in the raster kernels
    int32_t width[kMaxViews];
    int32_t height[kMaxViews];
    int32_t tiles_x[kMaxViews];
    int32_t tile_off[kMaxViews + 1];
    int64_t pix_off[kMaxViews + 1];
    float fx[kMaxViews], fy[kMaxViews], cx[kMaxViews], cy[kMaxViews];
};

struct RasterSettings {
    float near_z, alpha_min, alpha_max, t_min, eps2d, jac_clamp;
    float bg[3];
    int32_t frame;  // 0 world, 1 camera, 2 depth back-projection
    int32_t mark_visible;
    int32_t count_work;  // the forward writes each pixel's contributing-fragment count
    int32_t bwd_lane_reduce;  // one pixel per lane: reduce-scatter instead of the matrix cores
    int32_t grads_overwrite;  // the backward writes the gradients instead of adding them
};

// Projected record of one (Gaussian, view) pair: 64 bytes, 4 x float4.
//   r0 = (u_hi, v_hi, u_lo, v_lo)     mean2D as a float32 pair (u = u_hi + u_lo)
//   r1 = (a, b, c, opacity)           factored conic, base 2:
//                                     alpha = opacity * 2^-((a dx + b dy)^2 + (c dy)^2)
//   r2 = (c_r, c_g, c_b, z)           colour and camera depth
//   r3 = (p_x, p_y, p_z, 0)           composited point (world centre or camera centre)
// With k = log2(e) / 2, k Q = L^T L for L = [[a, b], [0, c]] (the Cholesky factor of the
// scaled conic Q).  The exponent is a sum of two squares: an elongated footprint (a near
// Gaussian seen at a grazing angle) would lose ~1e-4 of alpha to cancellation between the
// terms of the expanded form A dx^2 + B dx dy + C dy^2 in float32, the factored form
// keeps it near float32 rounding.
constexpr int kRecFloats = 16;

// Per-record image-plane gradient accumulator (16 floats, 13 used).  With
// g = alpha dL/dalpha per composited fragment (0 where alpha is clamped) and (dx, dy) the
// pixel centre minus the projected mean, the first six are the moments
//   0 sum g, 1 sum g dx, 2 sum g dy, 3 sum g dx^2, 4 sum g dx dy, 5 sum g dy^2,
// from which the mean, conic and opacity gradients follow (d e / d u = log2(e) (Q d)_x,
// d e / d Q = -log2(e) d d^T / 2 for the base-2 exponent e, d alpha / d e = ln 2 alpha);
// then 6 z, 7..9 colour, 10..12 point (sums of w dL/d output).  In the camera pointmap
// frame the depth is the point's z, so its gradient is carried in column 12 and 6 stays 0.
constexpr int kG2 = 16;

// The radix sorts publish 30-bit counts in their look-back words, so a sort takes fewer
// than 2^30 keys: records per window and tile pairs per frame are bounded by this.
constexpr int64_t kMaxSortKeys = int64_t(1) << 30;
constexpr int kScanMaxBlocks = 4096;  // blocks of a device-wide scan (scratch: one word each)

// Records with more tile pairs than this are counted and emitted by whole waves.
constexpr uint32_t kBigRecord = 64;

// Tile-row spans of a record, cached by the counting pass for the emission pass: x = first
// tile row | rows << 16, then the rows (first > last when a row is empty).  Up to
// kSpanRows rows take one word each (first | last tile << 16); kSpanRows + 1 to
// kSpanRowsMax rows take half a word each (first | last tile << 8, the lower half first),
// when every tile column is below 256.  Other records are not cached (rows = kSpanNone)
// and the emission evaluates them again.
constexpr uint32_t kSpanRows = 3;
constexpr uint32_t kSpanRowsMax = 6;
constexpr uint32_t kSpanNone = 0xffffu;

// Row i < rows of a cached span: tiles [ta, tb] of tile row (x & 0xffff) + i.
__device__ inline void span_row(const uint4 sp, int rows, int i, int &ta, int &tb) {
    if (rows <= (int)kSpanRows) {
        const uint32_t w = i == 0 ? sp.y : (i == 1 ? sp.z : sp.w);
        ta = (int)(w & 0xffffu);
        tb = (int)(w >> 16);
    } else {
        const uint32_t w = (i >> 1) == 0 ? sp.y : ((i >> 1) == 1 ? sp.z : sp.w);
        const uint32_t h = (w >> (16 * (i & 1))) & 0xffffu;
        ta = (int)(h & 0xffu);
        tb = (int)(h >> 8);
    }
}

// Frame-state layout (caller-owned device buffer).
struct FrameHeader {
    uint32_t pairs;     // tile pairs produced (or needed, on overflow)
    uint32_t overflow;  // nonzero if pairs > capacity
    uint32_t capacity;
    uint32_t tile;
    uint32_t n_views;
    uint32_t n_tiles;
    uint64_t n_pixels;
    uint64_t n_records;
    uint32_t magic;
    uint32_t visible;     // nonzero if the forward marked contributing records
    uint32_t sort_stall;  // nonzero if a radix sort pass abandoned its look-back
    uint32_t counted;     // nonzero if the forward wrote the contributing-fragment counts
    uint32_t ppt;         // pixels per lane of the forward, whose waves the contribution bits follow
    uint32_t frame;       // pointmap frame of the forward (the records carry that frame's point)
    uint32_t bwd_error;   // set by a backward that found the frame state unusable (see k_raster_bwd)
    uint32_t pad;
    uint64_t walked;      // counting forward: (wave, list entry) pairs its waves walked
    uint64_t accepted;    // counting forward: of those, the ones a live pixel of the wave accepted
};
constexpr uint32_t kFrameMagic = 0x47535046u;  // "GSPF"

struct FrameLayout {
    int64_t header, visible, ranges, t_final, last, contrib, order, records, pair_vals, total;
};

__host__ __device__ inline int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

// Per-wave contribution bits of a forward, stored after the pair list: one plane per wave
// of a tile, in which bit p (p = position in the sorted pair list) is set when one of that
// wave's live pixels accepted entry p (it composited there, or it stopped that pixel).  The
// backward walks these entries only.  Planes are sized for the tile's wave count at one
// pixel per lane.
inline int wmask_planes(int tile) { return tile * tile / kWave; }
__host__ __device__ inline int64_t wmask_stride(int64_t cap) { return cap / 64 + 2; }  // words per plane
inline int64_t wmask_bytes(int64_t cap, int tile) { return align256(wmask_planes(tile) * wmask_stride(cap) * 8); }
// The bits start right after the pair list of a frame whose capacity is cap.
__host__ __device__ inline uint64_t *wmask_at(const uint32_t *pair_vals, int64_t cap) {
    return reinterpret_cast<uint64_t *>(
        reinterpret_cast<char *>(const_cast<uint32_t *>(pair_vals)) + align256(cap * 4));
}

inline FrameLayout frame_layout(int64_t n_tiles, int64_t n_pixels, int64_t n_records, int64_t cap) {
    FrameLayout L;
    int64_t o = 0;
    L.header = o;    o += align256(sizeof(FrameHeader));
    L.visible = o;   o += align256(n_records);  // one byte per record (offset independent of the tile)
    L.ranges = o;    o += align256(n_tiles * 8);
    L.t_final = o;   o += align256(n_pixels * 4);
    L.last = o;      o += align256(n_pixels * 4);
    L.contrib = o;   o += align256(n_pixels * 4);
    L.order = o;     o += align256(2 * n_tiles * 4);  // launch orders of the forward and backward
    L.records = o;   o += align256(n_records * kRecFloats * 4);
    L.pair_vals = o; o += align256(cap * 4);
    L.total = o;
    return L;
}

// ---------------------------------------------------------------------------------------
// Device helpers.

__device__ inline int lane_id() { return __lane_id(); }

// Lane mask of a predicate.  Takes a bool: HIP's __ballot(int) converts the predicate to
// an int and back, which costs two vector instructions per call.
__device__ inline uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Sum over the 64 lanes of a wave using DPP row operations; the total lands in lane 63.
#define GSPM_DPP(x, ctrl, rmask)                                                            \
    __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, (x)), \
                                                          (ctrl), (rmask), 0xf, false))

__device__ inline float wave_sum_to_lane63(float x) {
    x += GSPM_DPP(x, 0xb1, 0xf);   // quad_perm [1,0,3,2]
    x += GSPM_DPP(x, 0x4e, 0xf);   // quad_perm [2,3,0,1]
    x += GSPM_DPP(x, 0x114, 0xf);  // row_shr:4
    x += GSPM_DPP(x, 0x118, 0xf);  // row_shr:8
    x += GSPM_DPP(x, 0x142, 0xa);  // row_bcast:15 into rows 1 and 3
    x += GSPM_DPP(x, 0x143, 0xc);  // row_bcast:31 into rows 2 and 3
    return x;
}

__device__ inline float wave_total(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, wave_sum_to_lane63(x)), 63));
}

#define GSPM_DPP_MOV(x, ctrl)                                                              \
    __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, (x)), \
                                                          (ctrl), 0xf, 0xf, true))

// gfx950 cross-half lane swaps, written as single instructions because this compiler's
// two-result builtins return the first result twice.  After v_permlane32_swap a, b:
// a = (a[0:32], b[0:32]) and b = (a[32:64], b[32:64]); after v_permlane16_swap a, b the
// odd 16-lane rows of a and the even rows of b are exchanged.  One s_nop 1 gives the
// wait states a VALU result needs before a lane-permute reads it; the swaps of a group
// read only registers written before the group.
#define GSPM_SWAP4(op, a0, b0, a1, b1, a2, b2, a3, b3)                                     \
    asm volatile("s_nop 1\n\t" op " %0, %4\n\t" op " %1, %5\n\t" op " %2, %6\n\t" op " %3, %7" \
                 : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(b0), "+v"(b1), "+v"(b2), "+v"(b3))

#define GSPM_SWAP3(op, a0, b0, a1, b1, a2, b2)                                           \
    asm volatile("s_nop 1\n\t" op " %0, %3\n\t" op " %1, %4\n\t" op " %2, %5"                \
                 : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(b0), "+v"(b1), "+v"(b2))
#define GSPM_SWAP2(op, a0, b0, a1, b1) \
    asm volatile("s_nop 1\n\t" op " %0, %2\n\t" op " %1, %3" : "+v"(a0), "+v"(a1), "+v"(b0), "+v"(b1))

// Sum over the 16 lanes of each row; every lane of the row receives it.
__device__ inline float row_sum16(float x) {
    x += GSPM_DPP_MOV(x, 0x128);  // row_ror:8
    x += GSPM_DPP_MOV(x, 0x124);  // row_ror:4
    x += GSPM_DPP_MOV(x, 0x4e);   // quad_perm [2,3,0,1]
    x += GSPM_DPP_MOV(x, 0xb1);   // quad_perm [1,0,3,2]
    return x;
}

// Reduce-scatter of N per-lane values (N = 8, 12 or 16) over a wave of 64 lanes: returns
// the wave-wide sum of v[idx] in the lanes where idx >= 0, one lane per value.  Lane bits
// 5 and 4 are folded with the cross-half swaps, each fold halving the number of live
// values, so a value costs about two instructions instead of six exchanges.
//   N = 16: lane 4q holds v[q] (bits 3 and 2 are folded with DPP as well);
//   N = 12: lane 16 rho + k (k < 3) holds v[3 rho + k];
//   N = 8:  lane 16 rho + k (k < 2) holds v[2 rho + k].
__device__ inline float wave_reduce_scatter(const float (&v)[16], int &idx) {
    const int lane = lane_id();
    float x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = v[k];
    GSPM_SWAP4("v_permlane32_swap_b32", x[0], x[8], x[1], x[9], x[2], x[10], x[3], x[11]);
    GSPM_SWAP4("v_permlane32_swap_b32", x[4], x[12], x[5], x[13], x[6], x[14], x[7], x[15]);
    float a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = x[k] + x[k + 8];  // lanes 0-31: v[k]; lanes 32-63: v[k + 8]
    GSPM_SWAP4("v_permlane16_swap_b32", a[0], a[4], a[1], a[5], a[2], a[6], a[3], a[7]);
    float b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) b[k] = a[k] + a[k + 4];  // even rows keep a[k], odd rows a[k + 4]
    const bool b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1;
    float c[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float send = b3 ? b[k] : b[k + 2];
        const float keep = b3 ? b[k + 2] : b[k];
        c[k] = keep + GSPM_DPP_MOV(send, 0x128);  // row_ror:8 == lane xor 8 within a row
    }
    const float send = b2 ? c[0] : c[1];
    const float keep = b2 ? c[1] : c[0];
    const float from_hi = GSPM_DPP_MOV(send, 0x104);  // row_shl:4: lane l reads lane l + 4
    const float from_lo = GSPM_DPP_MOV(send, 0x114);  // row_shr:4: lane l reads lane l - 4
    float d = keep + (b2 ? from_lo : from_hi);
    d += GSPM_DPP_MOV(d, 0x4e);  // quad_perm [2,3,0,1]
    d += GSPM_DPP_MOV(d, 0xb1);  // quad_perm [1,0,3,2]
    idx = (lane & 3) == 0 ? (lane >> 2) & 15 : -1;
    return d;
}

__device__ inline float wave_reduce_scatter(const float (&v)[12], int &idx) {
    const int lane = lane_id();
    float x[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) x[k] = v[k];
    GSPM_SWAP3("v_permlane32_swap_b32", x[0], x[6], x[1], x[7], x[2], x[8]);
    GSPM_SWAP3("v_permlane32_swap_b32", x[3], x[9], x[4], x[10], x[5], x[11]);
    float a[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) a[k] = x[k] + x[k + 6];  // lanes 0-31: v[k]; lanes 32-63: v[k + 6]
    GSPM_SWAP3("v_permlane16_swap_b32", a[0], a[3], a[1], a[4], a[2], a[5]);
    float b[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) b[k] = row_sum16(a[k] + a[k + 3]);  // row rho: v[3 rho + k]
    // Keep the sums whole in every lane: otherwise the last adds are sunk into branches
    // on the lane's index, which costs more than the two selects.
    asm volatile("" : "+v"(b[0]), "+v"(b[1]), "+v"(b[2]));
    const int r = lane & 15;
    idx = r < 3 ? 3 * (lane >> 4) + r : -1;
    return r == 0 ? b[0] : (r == 1 ? b[1] : b[2]);
}

__device__ inline float wave_reduce_scatter(const float (&v)[8], int &idx) {
    const int lane = lane_id();
    float x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = v[k];
    GSPM_SWAP4("v_permlane32_swap_b32", x[0], x[4], x[1], x[5], x[2], x[6], x[3], x[7]);
    float a[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = x[k] + x[k + 4];  // lanes 0-31: v[k]; lanes 32-63: v[k + 4]
    GSPM_SWAP2("v_permlane16_swap_b32", a[0], a[2], a[1], a[3]);
    float b[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) b[k] = row_sum16(a[k] + a[k + 2]);  // row rho: v[2 rho + k]
    asm volatile("" : "+v"(b[0]), "+v"(b[1]));
    const int r = lane & 15;
    idx = r < 2 ? 2 * (lane >> 4) + r : -1;
    return r == 0 ? b[0] : b[1];
}

// Wave-wide inclusive prefix sum of a uint32 (Hillis-Steele over cross-lane reads).
__device__ inline uint32_t wave_inclusive_scan(uint32_t x) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

// Appends the lanes with pred set to a global queue with one atomic per wave; returns
// each such lane's slot.  Must be reached by every active lane of the wave.
__device__ inline uint32_t wave_append(uint32_t *counter, bool pred) {
    const uint64_t m = ballot(pred);
    if (m == 0ull) return 0u;
    const int lane = lane_id();
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t base = 0u;
    if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = (uint32_t)__shfl((int)base, leader, kWave);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    return base + (uint32_t)__popcll(m & lt);
}

__device__ inline int find_view(const ViewTable &vt, int32_t global_tile) {
    int v = 0;
#pragma unroll 1
    for (int k = 1; k < vt.n_views; ++k)
        if (global_tile >= vt.tile_off[k]) v = k;
    return v;
}

// ---------------------------------------------------------------------------------------
// Support footprint of a record and its exact tile-row spans.
//
// The support of a Gaussian is the ellipse d^T Q d <= q, q = 2 ln(opacity / alpha_min),
// where its alpha reaches alpha_min.  A tile takes a (tile, record) pair exactly when the
// ellipse meets the rectangle spanned by the tile's pixel centres (clipped to the
// support's pixel box).  Per tile row this is an interval of tiles: the ellipse's x-extent
// over the row's y-range is attained at the row's ends or at the ellipse's leftmost /
// rightmost points.  Both the pair count and the pair emission evaluate this in float64
// from the same float32 record fields, so they agree exactly.
constexpr double kSupportMargin = 1e-6;  // relative widening of q, keeps the test conservative

struct Footprint {
    double u, v;            // centre
    double qxx, qxy, qyy;   // conic
    double q;               // support level
    double isyy;            // 1 / Sigma_yy = det(Q) / qxx
    double iqxx;            // 1 / qxx
    double rx, ry;          // support half extents
    double yr;              // y offset of the rightmost support point
    double kx;              // centre-line slope -qxy / qxx
    int i0, i1, j0, j1;     // support pixel box clipped to the image
};

__device__ inline bool record_footprint(const float4 r0, const float4 r1, float alpha_min, int W, int H,
                                        Footprint &f) {
    constexpr double kLn2d = 0.69314718055994530942;
    if (!(r1.w >= alpha_min)) return false;
    f.u = (double)r0.x + (double)r0.z;
    f.v = (double)r0.y + (double)r0.w;
    // Q = L^T L / k with 1 / k = 2 ln 2 (products of two floats are exact in double).
    const double a = r1.x, b = r1.y, c = r1.z;
    f.qxx = 2.0 * kLn2d * (a * a);
    f.qxy = 2.0 * kLn2d * (a * b);
    f.qyy = 2.0 * kLn2d * (b * b + c * c);
    const double det = f.qxx * f.qyy - f.qxy * f.qxy;
    if (!(det > 0.0) || !(f.qxx > 0.0)) return false;
    f.q = 2.0 * log((double)r1.w / (double)alpha_min) * (1.0 + kSupportMargin);
    const double idet = 1.0 / det;
    const double sxx = f.qyy * idet, syy = f.qxx * idet, sxy = -f.qxy * idet;
    f.iqxx = 1.0 / f.qxx;
    f.isyy = det * f.iqxx;
    f.rx = sqrt(f.q * sxx);
    f.ry = sqrt(f.q * syy);
    f.yr = f.rx > 0.0 ? sxy * f.q / f.rx : 0.0;  // = sxy sqrt(q / sxx)
    f.kx = -f.qxy * f.iqxx;
    f.i0 = (int)fmax(0.0, ceil(f.u - f.rx));
    f.i1 = (int)fmin((double)(W - 1), floor(f.u + f.rx));
    f.j0 = (int)fmax(0.0, ceil(f.v - f.ry));
    f.j1 = (int)fmin((double)(H - 1), floor(f.v + f.ry));
    return f.i0 <= f.i1 && f.j0 <= f.j1;
}

// Tiles [ta, tb] of tile row ty that meet the support (false if none).
__device__ inline bool row_span(const Footprint &f, int B, int ty, int &ta, int &tb) {
    const int ja = max(ty * B, f.j0), jb = min(ty * B + B - 1, f.j1);
    if (ja > jb) return false;
    const double ya = fmax((double)ja - f.v, -f.ry), yb = fmin((double)jb - f.v, f.ry);
    if (ya > yb) return false;
    // Half width of the support at height y around the centre line x = kx y.
    const double ha = sqrt(fmax(0.0, (f.q - ya * ya * f.isyy) * f.iqxx));
    const double hb = sqrt(fmax(0.0, (f.q - yb * yb * f.isyy) * f.iqxx));
    const double xr = (f.yr >= ya && f.yr <= yb) ? f.rx : fmax(f.kx * ya + ha, f.kx * yb + hb);
    const double xl = (-f.yr >= ya && -f.yr <= yb) ? -f.rx : fmin(f.kx * ya - ha, f.kx * yb - hb);
    const int ia = max(f.i0, (int)ceil(f.u + xl));
    const int ib = min(f.i1, (int)floor(f.u + xr));
    if (ia > ib) return false;
    const int sh = __builtin_ctz((unsigned)B);  // tile edges are powers of two
    ta = ia >> sh;
    tb = ib >> sh;
    return true;
}

// ---------------------------------------------------------------------------------------
// Host-side launch wrappers (defined in the .hip files).

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t n, hipStream_t s);
hipError_t launch_fill_f32(float *p, float value, int64_t n, hipStream_t s);

// Projects every record and counts its tile pairs, caching the tile-row spans of records
// with pairs in spans [N V]; big_list / big_count are scratch for the records counted by
// whole waves (big_count is zeroed here, and clear_also, if not NULL, in the same launch).
hipError_t launch_preprocess(const gspm_gaussians &g, const ViewTable &vt, const float *T_cw,
                             const RasterSettings &rs, float *records, uint32_t *counts,
                             uint32_t *dkey, uint4 *spans, uint32_t *big_list, uint32_t *big_count,
                             uint32_t *clear_also, hipStream_t s);

// A window of at most 2^kPackShift records carries each live record through the depth sort
// as its index with its pair count in the top bits, so that the pair-offset scan reads
// the counts in depth order without gathering them; a count of kPackCountMax or more is
// looked up by index.
constexpr uint32_t kPackShift = 26;
constexpr uint32_t kPackMask = (1u << kPackShift) - 1u;
constexpr uint32_t kPackCountMax = (1u << (32 - kPackShift)) - 1u;

// Exclusive scan for p < n of: counts[idx[p]] (flag 0), counts[idx[p]] != 0 (flag 1), or
// the pair count packed in idx[p] (flag 2); idx NULL means the identity.  n is
// min(*n_dev, n) when n_dev is given.  Writes offsets[p] and the total to *total.  part:
// scratch of at least scan_partials(n) words.
int64_t scan_partials(int64_t n);
hipError_t launch_scan_indirect(const uint32_t *counts, const uint32_t *idx, int64_t n,
                                uint32_t *offsets, uint32_t *total, uint32_t *part, hipStream_t s,
                                const uint32_t *n_dev = nullptr, int flag = 0, uint32_t *gathered = nullptr,
                                uint32_t *clear = nullptr);

// Compacts (depth key, record index) of the records with counts[r] != 0, in record order,
// and writes their number to *n_live; with pack, the value also carries the pair count
// (see kPackShift).  part: scratch of at least scan_partials(n) words.
hipError_t launch_compact(const uint32_t *counts, const uint32_t *dkey, int64_t n, uint32_t *ckey, uint32_t *cval,
                          uint32_t *n_live, uint32_t *part, bool pack, hipStream_t s);

// Stable LSD radix sort of (key, value) uint32 pairs over the low `bits` key bits, in
// ceil(bits / digit_bits) passes of equal width (digit_bits in [4, 8]).  n_dev: device
// count (may be NULL: n_max is then exact).  Buffers: keys/vals in, tmp, out (the sorted
// result ends in keys_out/vals_out).  scratch: radix_hist_words(n_max, digit_bits) words.
// *stall (device) is set if a pass gave up waiting for an earlier tile (the result is
// then invalid); the caller clears it.  ranges (optional): the keys are tile ids and the
// final pass writes each tile's [first, end) positions; the caller fills it with
// (0xffffffff, 0) beforehand, which empty tiles keep.  keep_keys = false: the final pass
// writes only the values (keys_out then holds an earlier pass's keys).
int64_t radix_hist_words(int64_t n_max, int digit_bits);
hipError_t radix_sort(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_tmp,
                      uint32_t *vals_tmp, uint32_t *keys_out, uint32_t *vals_out, int64_t n_max,
                      const uint32_t *n_dev, int bits, int digit_bits, uint32_t *scratch, uint32_t *stall,
                      uint2 *ranges, hipStream_t s, bool keep_keys = true);

// Emits the (global tile, record) pairs of every record in depth order.  Records with
// more than kBigRecord pairs are queued in big_list (big_count must be zero on entry: the
// pair-offset scan clears it) and emitted by whole waves.  records: the projected records (for the support footprint of records
// whose spans are not cached in spans).  It also fills ranges [n_tiles] with the empty
// range (0xffffffff, 0) that the tile sort's last pass narrows.
// rec_mask: kPackMask if sorted_rec carries packed counts, else all ones.
hipError_t launch_keygen(const uint32_t *sorted_rec, uint32_t rec_mask, const uint32_t *sorted_counts,
                         const uint32_t *offsets, const float *records, const uint4 *spans, const RasterSettings &rs,
                         int64_t n_records, int64_t n_per_view,
                         const ViewTable &vt, uint32_t *pkey, uint32_t *pval, FrameHeader *hdr,
                         uint32_t capacity, const uint32_t *total, uint32_t *big_list, uint32_t *big_count,
                         const uint32_t *n_dev, uint2 *ranges, int64_t n_tiles, hipStream_t s);

hipError_t launch_sum_u64(const uint32_t *x, int64_t n, unsigned long long *out, hipStream_t s);

// Scale alignment (align.hip).  Per patch: statistics of |X^r| and |X^p| and the sums
// over the pixels that pass the normalised correct-point test.
struct AlignPatch {
    double mu_r, sd_r, mu_p, sd_p, cp_sr, cp_sp;
    int32_t n, cp_n;
};
int64_t align_patches(const ViewTable &vt, int patch);
hipError_t launch_align_scale(const ViewTable &vt, const float *Xr, const float *Xp, const float *mask,
                              const gspm_align_params &prm, AlignPatch *patches, gspm_align_result *result,
                              hipStream_t s);
hipError_t launch_replace(const ViewTable &vt, const float *Xr, const float *Xp, const gspm_align_result *result,
                          float eps_m, float *out, uint32_t *replaced, hipStream_t s);

// Pose initialisation (pnp.hip).
int64_t pnp_scratch_bytes(int H, int64_t n);
hipError_t launch_pnp(const float *X, const float *uv, int64_t n, const gspm_intrinsics &K, const int32_t *samples,
                      int H, double thr, int iters, int rounds, void *scratch, double *T_out, int32_t *n_inliers,
                      uint8_t *mask, int32_t *scores_out, const float *T_ak, float *T_n_out, hipStream_t s);

// Regulariser and window management (window.hip).
int64_t iso_partials();
hipError_t launch_iso_loss(const float *log_scales, int64_t n, float weight, double *part, float *loss_out,
                           float *grad, hipStream_t s);
hipError_t launch_covisibility(const uint8_t *visible, int64_t n, int V, const FrameHeader *hdr,
                               unsigned long long *counts, double *iou, double *oc, int64_t *count_out,
                               hipStream_t s);
int64_t median_scratch_words(int V);
hipError_t launch_median_depth(const ViewTable &vt, const float *depth, uint32_t *scratch, float *out,
                               hipStream_t s);

// Launch order of the raster workgroups, heaviest tiles first: the tiles' work is the list
// length (ranges) or a per-tile estimate (work); exactly one of the two is given.  Ranges
// the sort left at (0xffffffff, 0) (tiles without pairs) are reset to (0, 0) on the way.
hipError_t launch_order_tiles(uint2 *ranges, const uint32_t *work, int64_t n_tiles, uint32_t *order,
                              hipStream_t s);

bool raster_config_supported(int tile, int ppt);

// order: workgroup -> tile (NULL: identity).  tile_work (optional) receives each tile's
// largest per-pixel list count up to the last contributing fragment.
hipError_t launch_raster_forward(const ViewTable &vt, const RasterSettings &rs, const uint2 *ranges,
                                 const uint32_t *pair_vals, const float *records, float *rgb,
                                 float *depth, float *alpha, float *pointmap, float *t_final,
                                 uint32_t *last, uint32_t *contrib, uint8_t *visible, const uint32_t *order,
                                 uint32_t *tile_work, uint64_t *wmask, int64_t wstride, FrameHeader *hdr, hipStream_t s);

hipError_t launch_raster_backward(const ViewTable &vt, const RasterSettings &rs, const uint2 *ranges,
                                  const uint32_t *pair_vals, const float *records, const uint32_t *last,
                                  const float *t_final, const gspm_const_images &fwd,
                                  const gspm_const_images &up, float *grad2d, bool pose_only,
                                  const uint32_t *order, FrameHeader *hdr, int64_t n_records, hipStream_t s);

// Image-plane gradient rows -> parameter gradients (added into out) and per-wave pose
// partials; every row read as nonzero is cleared, so grad2d is all zero afterwards.
hipError_t launch_preprocess_backward(const gspm_gaussians &g, const ViewTable &vt, const float *T_cw,
                                      const RasterSettings &rs, float *grad2d,
                                      const gspm_gaussian_grads &out, bool want_pose,
                                      double *pose_partials, hipStream_t s);
int64_t pose_partial_blocks(int64_t n);  // pose partials per view (one per wave of the launch)
hipError_t launch_pose_reduce(const double *pose_partials, int64_t n_blocks, int n_views,
                              float *pose_grad, bool overwrite, hipStream_t s);

int64_t patch_loss_partials(const ViewTable &vt, int patch);
// Slots of the static partials array behind gspm_window_loss_noalloc (1 MiB of float64),
// and the current device's address of that array (looked up once per device).
constexpr int64_t kStaticLossPartials = GSPM_WINDOW_LOSS_NOALLOC_SLOTS;
constexpr int kMaxDevices = 64;
hipError_t static_loss_partials(double **out);
hipError_t launch_patch_loss(const ViewTable &vt, const float *Xr, const float *Xp, const float *mask,
                             int patch, const float *rgb, const float *rgb_target, float alpha,
                             float *scale_out, int32_t *count_out, double *loss_part, float *loss_out,
                             float *grad_rgb, float *grad_pm, hipStream_t s);

hipError_t launch_pose_retract(int n_views, float *T_cw, const float *xi, hipStream_t s);

}  // namespace gspm
