// Host side of the C ABI declared in include/gspm.h: argument validation, scratch
// management and the launch sequences of the forward, backward and loss calls.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "gspm_common.h"

using namespace gspm;

namespace {

thread_local std::string g_last_error;

gspm_status fail(gspm_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
gspm_status fail(gspm_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

gspm_status hip_fail(hipError_t e, const char *where) {
    return fail(GSPM_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define GSPM_HIP(call)                                  \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    int64_t bytes = 0;
};

hipError_t grow(DevBuf &b, int64_t bytes) {
    if (bytes <= b.bytes) return hipSuccess;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        if (e != hipSuccess) return e;
        b.p = nullptr;
        b.bytes = 0;
    }
    bytes = align256(bytes > 256 ? bytes : 256);
    hipError_t e = hipMalloc(&b.p, (size_t)bytes);
    if (e != hipSuccess) return e;
    b.bytes = bytes;
    return hipSuccess;
}

bool finite_pos(float x) { return isfinite(x) && x > 0.0f; }

}  // namespace

struct gspm_ctx {
    // Phase timing: pairs of events recorded around each phase while enabled.
    bool timing = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<int> phase_of;  // per recorded pair
    // Per record (n * V).
    DevBuf counts, big, live, dkey, dval, dkey_tmp, dval_tmp, dkey_s, dval_s, offsets, grad2d, spans;
    // The image-plane gradient rows are all zero: the parameter pass clears every row it
    // reads as nonzero, so only a new allocation or an interrupted backward needs a fill.
    bool grad2d_clean = false;
    // Per pair (capacity).
    DevBuf pkey, pval, pkey_tmp, pval_tmp, pkey_s;
    // Small scratch.
    DevBuf hist, scan_part, misc, pose_part, loss_part, align, aux, pnp, twork;
};

namespace {

// Records a start event on construction and an end event on stop() when timing is on.
struct PhaseTimer {
    gspm_ctx *ctx;
    hipStream_t s;
    int phase;
    hipEvent_t end = nullptr;
    PhaseTimer(gspm_ctx *c, hipStream_t st, int ph) : ctx(c), s(st), phase(ph) {
        if (!ctx->timing) return;
        if (ctx->used + 2 > ctx->pool.size()) {
            for (int k = 0; k < 64; ++k) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) return;
                ctx->pool.push_back(e);
            }
        }
        hipEvent_t b = ctx->pool[ctx->used];
        end = ctx->pool[ctx->used + 1];
        ctx->used += 2;
        ctx->phase_of.push_back(phase);
        (void)hipEventRecord(b, s);
    }
    void stop() {
        if (end) (void)hipEventRecord(end, s);
        end = nullptr;
    }
    ~PhaseTimer() { stop(); }
};

struct Prepared {
    ViewTable vt;
    RasterSettings rs;
    int64_t n_tiles, n_pixels, n_records;
};

gspm_status check_gaussians(const gspm_gaussians *g) {
    if (!g) return fail(GSPM_ERR_INVALID_ARG, "gaussians is NULL");
    if (g->n < 0) return fail(GSPM_ERR_INVALID_ARG, "n = %lld < 0", (long long)g->n);
    if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logit || !g->rgb))
        return fail(GSPM_ERR_INVALID_ARG, "a Gaussian parameter pointer is NULL");
    return GSPM_OK;
}

gspm_status build_views(const gspm_views *views, int32_t tile, ViewTable &vt, int64_t &n_tiles, int64_t &n_pixels) {
    if (!views) return fail(GSPM_ERR_INVALID_ARG, "views is NULL");
    if (views->n_views < 1 || views->n_views > GSPM_MAX_VIEWS)
        return fail(GSPM_ERR_INVALID_ARG, "n_views = %d outside [1, %d]", views->n_views, GSPM_MAX_VIEWS);
    if (!views->intr || !views->T_cw) return fail(GSPM_ERR_INVALID_ARG, "views->intr or views->T_cw is NULL");
    memset(&vt, 0, sizeof(vt));
    vt.n_views = views->n_views;
    vt.tile = tile;
    int64_t toff = 0, poff = 0;
    for (int v = 0; v < views->n_views; ++v) {
        const gspm_intrinsics &k = views->intr[v];
        if (k.width <= 0 || k.height <= 0 || k.width > 16384 || k.height > 16384)
            return fail(GSPM_ERR_INVALID_ARG, "view %d: size %dx%d outside [1, 16384]", v, k.width, k.height);
        if (!finite_pos(k.fx) || !finite_pos(k.fy) || !isfinite(k.cx) || !isfinite(k.cy))
            return fail(GSPM_ERR_INVALID_ARG, "view %d: intrinsics must be finite with fx, fy > 0", v);
        vt.width[v] = k.width;
        vt.height[v] = k.height;
        vt.tiles_x[v] = (k.width + tile - 1) / tile;
        vt.tile_off[v] = (int32_t)toff;
        vt.pix_off[v] = poff;
        vt.fx[v] = k.fx; vt.fy[v] = k.fy; vt.cx[v] = k.cx; vt.cy[v] = k.cy;
        toff += (int64_t)vt.tiles_x[v] * ((k.height + tile - 1) / tile);
        poff += (int64_t)k.width * k.height;
    }
    if (toff > (1ll << 30)) return fail(GSPM_ERR_INVALID_ARG, "too many tiles (%lld)", (long long)toff);
    vt.tile_off[views->n_views] = (int32_t)toff;
    vt.pix_off[views->n_views] = poff;
    n_tiles = toff;
    n_pixels = poff;
    return GSPM_OK;
}

gspm_status prepare(const gspm_gaussians *g, const gspm_views *views, const gspm_settings *s, Prepared &P) {
    gspm_status st = check_gaussians(g);
    if (st) return st;
    if (!s) return fail(GSPM_ERR_INVALID_ARG, "settings is NULL");
    if (s->tile != 8 && s->tile != 16 && s->tile != 32)
        return fail(GSPM_ERR_INVALID_ARG, "tile = %d, expected 8, 16 or 32", s->tile);
    if (!raster_config_supported(s->tile, s->pixels_per_lane))
        return fail(GSPM_ERR_INVALID_ARG, "(tile, pixels_per_lane) = (%d, %d) is not a supported configuration",
                    s->tile, s->pixels_per_lane);
    if (s->sort_digit_bits < 4 || s->sort_digit_bits > 8)
        return fail(GSPM_ERR_INVALID_ARG, "sort_digit_bits = %d outside [4, 8]", s->sort_digit_bits);
    if (s->pointmap_frame < 0 || s->pointmap_frame > 2)
        return fail(GSPM_ERR_INVALID_ARG, "pointmap_frame = %d, expected 0, 1 or 2", s->pointmap_frame);
    if (!(s->alpha_min > 0.0f && s->alpha_min < 1.0f) || !(s->alpha_max >= s->alpha_min && s->alpha_max < 1.0f))
        return fail(GSPM_ERR_INVALID_ARG, "need 0 < alpha_min <= alpha_max < 1");
    if (!(s->t_min > 0.0f && s->t_min < 1.0f)) return fail(GSPM_ERR_INVALID_ARG, "need 0 < t_min < 1");
    if (!(s->near_z > 0.0f) || !isfinite(s->near_z)) return fail(GSPM_ERR_INVALID_ARG, "need near_z > 0");
    if (!(s->eps2d >= 0.0f) || !isfinite(s->eps2d)) return fail(GSPM_ERR_INVALID_ARG, "need eps2d >= 0");
    if (!(s->jac_clamp > 0.0f) || !isfinite(s->jac_clamp)) return fail(GSPM_ERR_INVALID_ARG, "need jac_clamp > 0");
    for (int c = 0; c < 3; ++c)
        if (!isfinite(s->bg[c])) return fail(GSPM_ERR_INVALID_ARG, "bg must be finite");
    st = build_views(views, s->tile, P.vt, P.n_tiles, P.n_pixels);
    if (st) return st;
    P.vt.ppt = s->pixels_per_lane;
    P.n_records = g->n * views->n_views;
    // The radix sorts' look-back words hold 30-bit counts.
    if (P.n_records >= kMaxSortKeys) return fail(GSPM_ERR_INVALID_ARG, "n * n_views must be < 2^30");
    P.rs.near_z = s->near_z;
    P.rs.alpha_min = s->alpha_min;
    P.rs.alpha_max = s->alpha_max;
    P.rs.t_min = s->t_min;
    P.rs.eps2d = s->eps2d;
    P.rs.jac_clamp = s->jac_clamp;
    P.rs.bg[0] = s->bg[0]; P.rs.bg[1] = s->bg[1]; P.rs.bg[2] = s->bg[2];
    P.rs.frame = s->pointmap_frame;
    P.rs.mark_visible = s->mark_visible != 0 ? 1 : 0;
    P.rs.count_work = s->count_work != 0 ? 1 : 0;
    P.rs.bwd_lane_reduce = s->bwd_lane_reduce != 0 ? 1 : 0;
    P.rs.grads_overwrite = s->grads_overwrite != 0 ? 1 : 0;
    return GSPM_OK;
}

int tile_bits(int64_t n_tiles) {
    int b = 1;
    while (b < 32 && ((int64_t)1 << b) < n_tiles) ++b;
    return b;
}

hipError_t ensure_records(gspm_ctx *c, int64_t R, int digit_bits) {
    const int64_t w = R > 0 ? R : 1;
    hipError_t e;
    if ((e = grow(c->counts, 4 * w))) return e;
    if ((e = grow(c->big, 4 * w))) return e;
    if ((e = grow(c->live, 4 * w))) return e;
    if ((e = grow(c->dkey, 4 * w))) return e;
    if ((e = grow(c->dval, 4 * w))) return e;
    if ((e = grow(c->dkey_tmp, 4 * w))) return e;
    if ((e = grow(c->dval_tmp, 4 * w))) return e;
    if ((e = grow(c->dkey_s, 4 * w))) return e;
    if ((e = grow(c->dval_s, 4 * w))) return e;
    if ((e = grow(c->offsets, 4 * w))) return e;
    if ((e = grow(c->spans, 16 * w))) return e;
    if ((e = grow(c->hist, 4 * radix_hist_words(w, digit_bits)))) return e;
    if ((e = grow(c->scan_part, 4 * kScanMaxBlocks))) return e;
    if ((e = grow(c->misc, 256))) return e;
    return hipSuccess;
}

hipError_t ensure_pairs(gspm_ctx *c, int64_t cap, int digit_bits) {
    const int64_t w = cap > 0 ? cap : 1;
    hipError_t e;
    if ((e = grow(c->pkey, 4 * w))) return e;
    if ((e = grow(c->pval, 4 * w))) return e;
    if ((e = grow(c->pkey_tmp, 4 * w))) return e;
    if ((e = grow(c->pval_tmp, 4 * w))) return e;
    if ((e = grow(c->pkey_s, 4 * w))) return e;
    if ((e = grow(c->hist, 4 * radix_hist_words(w, digit_bits)))) return e;
    return hipSuccess;
}

template <typename T>
T *at(void *base, int64_t off) {
    return reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off);
}
template <typename T>
const T *at(const void *base, int64_t off) {
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}

gspm_status backward_common(gspm_ctx *ctx, const gspm_gaussians *g, const gspm_views *views, const gspm_settings *s,
                            const gspm_const_images *fwd_out, const gspm_const_images *grad_out,
                            const void *frame_state, const gspm_gaussian_grads *grads, float *pose_grad,
                            bool pose_only, void *stream) {
    if (!ctx) return fail(GSPM_ERR_INVALID_ARG, "ctx is NULL");
    Prepared P;
    gspm_status st = prepare(g, views, s, P);
    if (st) return st;
    if (!frame_state) return fail(GSPM_ERR_INVALID_ARG, "frame_state is NULL");
    if (!fwd_out || !fwd_out->rgb || !fwd_out->depth || !fwd_out->pointmap)
        return fail(GSPM_ERR_INVALID_ARG, "forward outputs rgb, depth and pointmap are required");
    if (!grad_out) return fail(GSPM_ERR_INVALID_ARG, "grad_out is NULL");
    if (pose_only && !pose_grad) return fail(GSPM_ERR_INVALID_ARG, "pose_grad is NULL");
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    const FrameLayout L = frame_layout(P.n_tiles, P.n_pixels, P.n_records, 0);
    const int64_t R = P.n_records;
    const void *g2_before = ctx->grad2d.p;
    GSPM_HIP(grow(ctx->grad2d, 4 * kG2 * (R > 0 ? R : 1)));
    if (ctx->grad2d.p != g2_before) ctx->grad2d_clean = false;
    const int64_t nb = pose_partial_blocks(g->n);
    GSPM_HIP(grow(ctx->pose_part, 8 * 6 * (nb > 0 ? nb : 1) * P.vt.n_views));
    float *g2 = static_cast<float *>(ctx->grad2d.p);
    if (!ctx->grad2d_clean) GSPM_HIP(launch_fill_f32(g2, 0.0f, ctx->grad2d.bytes / 4, hs));
    ctx->grad2d_clean = false;  // until both passes below have been launched
    PhaseTimer t_rb(ctx, hs, GSPM_PHASE_RASTER_BWD);
    GSPM_HIP(launch_raster_backward(P.vt, P.rs, at<uint2>(frame_state, L.ranges), at<uint32_t>(frame_state, L.pair_vals),
                                    at<float>(frame_state, L.records), at<uint32_t>(frame_state, L.last),
                                    at<float>(frame_state, L.t_final), *fwd_out, *grad_out, g2, pose_only,
                                    at<uint32_t>(frame_state, L.order) + P.n_tiles,
                                    at<FrameHeader>(const_cast<void *>(frame_state), L.header), P.n_records, hs));
    t_rb.stop();
    PhaseTimer t_pb(ctx, hs, GSPM_PHASE_PARAM_BWD);
    gspm_gaussian_grads none = {nullptr, nullptr, nullptr, nullptr, nullptr};
    const gspm_gaussian_grads &out = (pose_only || !grads) ? none : *grads;
    GSPM_HIP(launch_preprocess_backward(*g, P.vt, views->T_cw, P.rs, g2, out, pose_grad != nullptr,
                                        static_cast<double *>(ctx->pose_part.p), hs));
    ctx->grad2d_clean = true;
    if (pose_grad && nb > 0)
        GSPM_HIP(launch_pose_reduce(static_cast<double *>(ctx->pose_part.p), nb, P.vt.n_views, pose_grad,
                                     P.rs.grads_overwrite != 0, hs));
    else if (pose_grad && P.rs.grads_overwrite)  // no Gaussians: the written gradient is zero
        GSPM_HIP(launch_fill_f32(pose_grad, 0.0f, 6 * (int64_t)P.vt.n_views, hs));
    return GSPM_OK;
}

}  // namespace

extern "C" {

gspm_status gspm_create(gspm_ctx **out) {
    if (!out) return fail(GSPM_ERR_INVALID_ARG, "out is NULL");
    *out = new (std::nothrow) gspm_ctx();
    if (!*out) return fail(GSPM_ERR_INTERNAL, "out of host memory");
    return GSPM_OK;
}

void gspm_destroy(gspm_ctx *ctx) {
    if (!ctx) return;
    DevBuf *bufs[] = {&ctx->counts, &ctx->big, &ctx->live, &ctx->dkey, &ctx->dval, &ctx->dkey_tmp, &ctx->dval_tmp,
                      &ctx->dkey_s, &ctx->dval_s, &ctx->offsets, &ctx->grad2d, &ctx->spans, &ctx->pkey, &ctx->pval,
                      &ctx->pkey_tmp, &ctx->pval_tmp, &ctx->pkey_s, &ctx->hist, &ctx->scan_part, &ctx->misc,
                      &ctx->pose_part, &ctx->loss_part, &ctx->align, &ctx->aux, &ctx->pnp, &ctx->twork};
    for (DevBuf *b : bufs)
        if (b->p) (void)hipFree(b->p);
    for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    delete ctx;
}

gspm_status gspm_reserve(gspm_ctx *ctx, int64_t max_records, int64_t max_pairs, int64_t max_tiles) {
    if (!ctx) return fail(GSPM_ERR_INVALID_ARG, "ctx is NULL");
    if (max_records < 0 || max_pairs < 0 || max_tiles < 0) return fail(GSPM_ERR_INVALID_ARG, "negative size");
    if (max_pairs >= kMaxSortKeys || max_records >= kMaxSortKeys)
        return fail(GSPM_ERR_INVALID_ARG, "sizes must be < 2^30");
    (void)max_tiles;
    GSPM_HIP(ensure_records(ctx, max_records, 8));
    GSPM_HIP(ensure_pairs(ctx, max_pairs, 8));
    const void *g2_before = ctx->grad2d.p;
    GSPM_HIP(grow(ctx->grad2d, 4 * kG2 * (max_records > 0 ? max_records : 1)));
    if (ctx->grad2d.p != g2_before) ctx->grad2d_clean = false;
    return GSPM_OK;
}

int64_t gspm_frame_state_bytes(const gspm_views *views, int64_t n_gaussians, int64_t max_pairs, int32_t tile) {
    if (tile != 8 && tile != 16 && tile != 32) {
        fail(GSPM_ERR_INVALID_ARG, "tile = %d, expected 8, 16 or 32", tile);
        return -1;
    }
    if (n_gaussians < 0 || max_pairs < 0) {
        fail(GSPM_ERR_INVALID_ARG, "negative size");
        return -1;
    }
    ViewTable vt;
    int64_t nt, np;
    if (build_views(views, tile, vt, nt, np) != GSPM_OK) return -1;
    return frame_layout(nt, np, n_gaussians * views->n_views, max_pairs).total + wmask_bytes(max_pairs, tile);
}

gspm_status gspm_render_forward(gspm_ctx *ctx, const gspm_gaussians *g, const gspm_views *views,
                                const gspm_settings *s, const gspm_images *out, void *frame_state,
                                int64_t frame_state_bytes, void *stream) {
    if (!ctx) return fail(GSPM_ERR_INVALID_ARG, "ctx is NULL");
    Prepared P;
    gspm_status st = prepare(g, views, s, P);
    if (st) return st;
    if (!out || !out->rgb || !out->depth || !out->alpha || !out->pointmap)
        return fail(GSPM_ERR_INVALID_ARG, "all four output planes are required");
    if (!frame_state) return fail(GSPM_ERR_INVALID_ARG, "frame_state is NULL");
    const FrameLayout L0 = frame_layout(P.n_tiles, P.n_pixels, P.n_records, 0);
    if (frame_state_bytes < L0.total)
        return fail(GSPM_ERR_INVALID_ARG, "frame_state_bytes = %lld < %lld (no room for pairs)",
                    (long long)frame_state_bytes, (long long)L0.total);
    // The pair list and, after it, the per-wave contribution bits: the largest capacity
    // whose two regions fit.
    const int64_t avail = frame_state_bytes - L0.pair_vals;
    auto need = [&](int64_t c) { return align256(c * 4) + wmask_bytes(c, P.vt.tile); };
    if (avail < need(0))
        return fail(GSPM_ERR_INVALID_ARG, "frame_state_bytes = %lld < %lld (no room for pairs)",
                    (long long)frame_state_bytes, (long long)(L0.pair_vals + need(0)));
    int64_t cap = 0;
    for (int64_t hi = avail / 4 + 1; hi - cap > 1;) {  // need(cap) fits, need(hi) does not
        const int64_t mid = cap + (hi - cap) / 2;
        if (need(mid) <= avail) cap = mid; else hi = mid;
    }
    if (cap >= kMaxSortKeys) cap = kMaxSortKeys - 1;
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    const int db = s->sort_digit_bits;
    const int64_t R = P.n_records;
    GSPM_HIP(ensure_records(ctx, R, db));
    GSPM_HIP(ensure_pairs(ctx, cap, db));

    FrameHeader *hdr = at<FrameHeader>(frame_state, L0.header);
    uint2 *ranges = at<uint2>(frame_state, L0.ranges);
    float *records = at<float>(frame_state, L0.records);
    uint32_t *pair_vals = at<uint32_t>(frame_state, L0.pair_vals);
    uint32_t *total = static_cast<uint32_t *>(ctx->misc.p);
    uint32_t *counts = static_cast<uint32_t *>(ctx->counts.p);
    uint32_t *hist = static_cast<uint32_t *>(ctx->hist.p);
    uint32_t *part = static_cast<uint32_t *>(ctx->scan_part.p);

    // 1. Project every (Gaussian, view) record.
    PhaseTimer t_pre(ctx, hs, GSPM_PHASE_PREPROCESS);
    GSPM_HIP(launch_preprocess(*g, P.vt, views->T_cw, P.rs, records, counts, static_cast<uint32_t *>(ctx->dkey.p),
                               static_cast<uint4 *>(ctx->spans.p), static_cast<uint32_t *>(ctx->big.p), total + 1,
                               &hdr->sort_stall, hs));
    t_pre.stop();
    // Device-side counts: total[0] tile pairs, total[1] queued large records, total[2] live records.
    uint32_t *n_live = total + 2;
    // Small enough windows carry each live record's pair count through the depth sort.
    const bool pack = R <= (int64_t)kPackMask + 1;
    if (R > 0) {
        // 2. Keep the records that have tile pairs (in record order) and sort them by float32
        //    depth (stable, so ties keep record order).
        PhaseTimer t_ds(ctx, hs, GSPM_PHASE_DEPTH_SORT);
        GSPM_HIP(launch_compact(counts, static_cast<uint32_t *>(ctx->dkey.p), R, static_cast<uint32_t *>(ctx->dval.p),
                                static_cast<uint32_t *>(ctx->live.p), n_live, part, pack, hs));
        GSPM_HIP(radix_sort(static_cast<uint32_t *>(ctx->dval.p), static_cast<uint32_t *>(ctx->live.p),
                            static_cast<uint32_t *>(ctx->dkey_tmp.p), static_cast<uint32_t *>(ctx->dval_tmp.p),
                            static_cast<uint32_t *>(ctx->dkey_s.p), static_cast<uint32_t *>(ctx->dval_s.p), R, n_live,
                            32, db, hist, &hdr->sort_stall, nullptr, hs, false));
        t_ds.stop();
    }
    PhaseTimer t_bin(ctx, hs, GSPM_PHASE_BINNING);
    if (R > 0) {
        // 3. Offsets of each live record's tile pairs, in depth order.
        // The sorted depth keys are no longer needed: their buffer receives the pair counts
        // in depth order, unpacked (or gathered) once by the scan.
        GSPM_HIP(launch_scan_indirect(counts, static_cast<uint32_t *>(ctx->dval_s.p), R,
                                      static_cast<uint32_t *>(ctx->offsets.p), total, part, hs, n_live, pack ? 2 : 0,
                                      static_cast<uint32_t *>(ctx->dkey_s.p), total + 1));  // + the emitter's queue count
    } else {
        GSPM_HIP(launch_fill_u32(total, 0u, 3, hs));
    }
    // 4. Emit (tile, record) pairs; the header gets the pair count and overflow flag.
    GSPM_HIP(launch_keygen(static_cast<uint32_t *>(ctx->dval_s.p), pack ? kPackMask : 0xffffffffu,
                           static_cast<uint32_t *>(ctx->dkey_s.p),
                           static_cast<uint32_t *>(ctx->offsets.p),
                           records, static_cast<const uint4 *>(ctx->spans.p), P.rs, R, g->n > 0 ? g->n : 1, P.vt,
                           static_cast<uint32_t *>(ctx->pkey.p),
                           static_cast<uint32_t *>(ctx->pval.p), hdr, (uint32_t)cap, total,
                           static_cast<uint32_t *>(ctx->big.p), total + 1, n_live, ranges, P.n_tiles, hs));
    t_bin.stop();
    // 5. Stable sort by tile id; its final pass writes the per-tile ranges (6).
    if (cap > 0) {
        PhaseTimer t_ts(ctx, hs, GSPM_PHASE_TILE_SORT);
        GSPM_HIP(radix_sort(static_cast<uint32_t *>(ctx->pkey.p), static_cast<uint32_t *>(ctx->pval.p),
                            static_cast<uint32_t *>(ctx->pkey_tmp.p), static_cast<uint32_t *>(ctx->pval_tmp.p),
                            static_cast<uint32_t *>(ctx->pkey_s.p), pair_vals, cap, &hdr->pairs,
                            tile_bits(P.n_tiles), db, hist, &hdr->sort_stall, ranges, hs, false));
        t_ts.stop();
    }
    // Heaviest tiles first: by list length for the forward; the forward measures each
    // tile's contributing depth, which orders the backward.
    uint32_t *order = at<uint32_t>(frame_state, L0.order);
    GSPM_HIP(grow(ctx->twork, 4 * (P.n_tiles > 0 ? P.n_tiles : 1)));
    uint32_t *twork = static_cast<uint32_t *>(ctx->twork.p);
    GSPM_HIP(launch_order_tiles(ranges, nullptr, P.n_tiles, order, hs));
    // 7. Composite (optionally marking the records that contribute to a pixel).
    uint8_t *visible = nullptr;
    if (P.rs.mark_visible) {
        visible = at<uint8_t>(frame_state, L0.visible);
        GSPM_HIP(launch_fill_u32(reinterpret_cast<uint32_t *>(visible), 0u, (R + 3) / 4, hs));
    }
    uint64_t *wmask = wmask_at(pair_vals, cap);
    const int64_t wstride = wmask_stride(cap);
    GSPM_HIP(launch_fill_u32(reinterpret_cast<uint32_t *>(wmask), 0u,
                             2 * wstride * (P.vt.tile * P.vt.tile / P.vt.ppt / kWave), hs));
    PhaseTimer t_fwd(ctx, hs, GSPM_PHASE_RASTER_FWD);
    GSPM_HIP(launch_raster_forward(P.vt, P.rs, ranges, pair_vals, records, out->rgb, out->depth, out->alpha,
                                   out->pointmap, at<float>(frame_state, L0.t_final), at<uint32_t>(frame_state, L0.last),
                                   at<uint32_t>(frame_state, L0.contrib), visible, order, twork, wmask, wstride, hdr,
                                   hs));
    GSPM_HIP(launch_order_tiles(nullptr, twork, P.n_tiles, order + P.n_tiles, hs));
    return GSPM_OK;
}

gspm_status gspm_frame_status(const void *frame_state, void *stream, int64_t *pairs) {
    if (!frame_state) return fail(GSPM_ERR_INVALID_ARG, "frame_state is NULL");
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    GSPM_HIP(hipStreamSynchronize(hs));
    FrameHeader h;
    GSPM_HIP(hipMemcpy(&h, frame_state, sizeof(h), hipMemcpyDeviceToHost));
    if (h.magic != kFrameMagic) return fail(GSPM_ERR_INVALID_ARG, "frame_state was not written by a forward");
    if (pairs) *pairs = h.pairs;
    if (h.sort_stall) return fail(GSPM_ERR_INTERNAL, "a radix sort pass stopped waiting for an earlier tile");
    if (h.overflow)
        return fail(GSPM_ERR_CAPACITY, "tile pairs %u exceed the frame state's capacity %u", h.pairs, h.capacity);
    if (h.bwd_error)
        return fail(GSPM_ERR_INVALID_ARG,
                    "a backward refused this frame state: its views, Gaussian count, tile or pointmap frame "
                    "differ from the forward's; its gradients were not computed");
    return GSPM_OK;
}

gspm_status gspm_frame_work(gspm_ctx *ctx, const gspm_views *views, int64_t n_gaussians, int32_t tile,
                            const void *frame_state, void *stream, int64_t *out) {
    if (!ctx || !frame_state || !out) return fail(GSPM_ERR_INVALID_ARG, "ctx, frame_state and out are required");
    if (tile != 8 && tile != 16 && tile != 32) return fail(GSPM_ERR_INVALID_ARG, "tile must be 8, 16 or 32");
    if (n_gaussians < 0) return fail(GSPM_ERR_INVALID_ARG, "n_gaussians < 0");
    ViewTable vt;
    int64_t nt, np;
    gspm_status st = build_views(views, tile, vt, nt, np);
    if (st) return st;
    const FrameLayout L = frame_layout(nt, np, n_gaussians * views->n_views, 0);
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    GSPM_HIP(grow(ctx->misc, 256));
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(static_cast<char *>(ctx->misc.p) + 64);
    unsigned long long host[2];
    GSPM_HIP(launch_sum_u64(at<uint32_t>(frame_state, L.contrib), np, acc, hs));
    GSPM_HIP(launch_sum_u64(at<uint32_t>(frame_state, L.last), np, acc + 1, hs));
    FrameHeader h;
    GSPM_HIP(hipMemcpyAsync(host, acc, sizeof(host), hipMemcpyDeviceToHost, hs));
    GSPM_HIP(hipMemcpyAsync(&h, frame_state, sizeof(h), hipMemcpyDeviceToHost, hs));
    GSPM_HIP(hipStreamSynchronize(hs));
    if (h.magic != kFrameMagic) return fail(GSPM_ERR_INVALID_ARG, "frame_state was not written by a forward");
    if (!h.counted) return fail(GSPM_ERR_INVALID_ARG, "the forward did not count its work (settings.count_work = 0)");
    out[0] = h.pairs;
    out[1] = (int64_t)host[0];
    out[2] = (int64_t)host[1];
    out[3] = (int64_t)h.walked;
    out[4] = (int64_t)h.accepted;
    return GSPM_OK;
}

gspm_status gspm_render_backward(gspm_ctx *ctx, const gspm_gaussians *g, const gspm_views *views,
                                 const gspm_settings *s, const gspm_const_images *fwd_out,
                                 const gspm_const_images *grad_out, const void *frame_state,
                                 const gspm_gaussian_grads *grads, float *pose_grad, void *stream) {
    if (!grads && !pose_grad) return fail(GSPM_ERR_INVALID_ARG, "nothing to compute: grads and pose_grad are NULL");
    return backward_common(ctx, g, views, s, fwd_out, grad_out, frame_state, grads, pose_grad, false, stream);
}

gspm_status gspm_pose_backward(gspm_ctx *ctx, const gspm_gaussians *g, const gspm_views *views,
                               const gspm_settings *s, const gspm_const_images *fwd_out,
                               const gspm_const_images *grad_out, const void *frame_state, float *pose_grad,
                               void *stream) {
    return backward_common(ctx, g, views, s, fwd_out, grad_out, frame_state, nullptr, pose_grad, true, stream);
}

static gspm_status patch_common(gspm_ctx *ctx, const gspm_views *views, const float *Xr, const float *Xp,
                                const float *mask, int32_t patch, const float *rgb, const float *rgb_target,
                                float alpha, float *scale_out, int32_t *count_out, float *loss_out, float *grad_rgb,
                                float *grad_pm, void *stream) {
    ViewTable vt;
    int64_t nt, np;
    gspm_status st = build_views(views, 16, vt, nt, np);
    if (st) return st;
    if (patch < 1 || patch > 64) return fail(GSPM_ERR_INVALID_ARG, "patch = %d outside [1, 64]", patch);
    if (!Xr || !Xp || !scale_out) return fail(GSPM_ERR_INVALID_ARG, "Xr, Xp and scale_out are required");
    double *part = nullptr;
    if (grad_rgb) {
        GSPM_HIP(grow(ctx->loss_part, 8 * (patch_loss_partials(vt, patch) + 1)));
        part = static_cast<double *>(ctx->loss_part.p);
    }
    GSPM_HIP(launch_patch_loss(vt, Xr, Xp, mask, patch, rgb, rgb_target, alpha, scale_out, count_out, part, loss_out,
                               grad_rgb, grad_pm, reinterpret_cast<hipStream_t>(stream)));
    return GSPM_OK;
}

gspm_status gspm_patch_scale_align(const gspm_views *views, const float *Xr, const float *Xp, const float *mask,
                                   int32_t patch, float *scale_out, int32_t *count_out, void *stream) {
    return patch_common(nullptr, views, Xr, Xp, mask, patch, nullptr, nullptr, 0.0f, scale_out, count_out, nullptr,
                        nullptr, nullptr, stream);
}

gspm_status gspm_window_loss(gspm_ctx *ctx, const gspm_views *views, const float *rgb, const float *rgb_target,
                             const float *pm, const float *Xp, int32_t patch, float alpha, float *scale_out,
                             float *loss_out, float *grad_rgb, float *grad_pm, void *stream) {
    if (!ctx) return fail(GSPM_ERR_INVALID_ARG, "ctx is NULL");
    if (!rgb || !rgb_target || !loss_out || !grad_rgb || !grad_pm)
        return fail(GSPM_ERR_INVALID_ARG, "rgb, rgb_target, loss_out, grad_rgb and grad_pm are required");
    if (!(alpha >= 0.0f && alpha <= 1.0f)) return fail(GSPM_ERR_INVALID_ARG, "alpha must lie in [0, 1]");
    return patch_common(ctx, views, pm, Xp, nullptr, patch, rgb, rgb_target, alpha, scale_out, nullptr, loss_out,
                        grad_rgb, grad_pm, stream);
}

gspm_status gspm_window_loss_noalloc(const gspm_views *views, const float *rgb, const float *rgb_target,
                                     const float *pm, const float *Xp, int32_t patch, float alpha, float *scale_out,
                                     float *loss_out, float *grad_rgb, float *grad_pm, void *stream) {
    if (!rgb || !rgb_target || !pm || !Xp || !scale_out || !loss_out || !grad_rgb || !grad_pm)
        return fail(GSPM_ERR_INVALID_ARG, "rgb, rgb_target, pm, Xp, scale_out, loss_out, grad_rgb and grad_pm are required");
    if (!(alpha >= 0.0f && alpha <= 1.0f)) return fail(GSPM_ERR_INVALID_ARG, "alpha must lie in [0, 1]");
    if (patch < 1 || patch > 64) return fail(GSPM_ERR_INVALID_ARG, "patch = %d outside [1, 64]", patch);
    ViewTable vt;
    int64_t nt, np;
    gspm_status st = build_views(views, 16, vt, nt, np);
    if (st) return st;
    const int64_t need = patch_loss_partials(vt, patch);
    if (need > kStaticLossPartials)
        return fail(GSPM_ERR_INVALID_ARG, "the window needs %lld loss partials, more than the %lld this call holds",
                    (long long)need, (long long)kStaticLossPartials);
    double *part = nullptr;
    GSPM_HIP(static_loss_partials(&part));
    GSPM_HIP(launch_patch_loss(vt, pm, Xp, nullptr, patch, rgb, rgb_target, alpha, scale_out, nullptr, part, loss_out,
                               grad_rgb, grad_pm, reinterpret_cast<hipStream_t>(stream)));
    return GSPM_OK;
}

gspm_status gspm_align_scale(gspm_ctx *ctx, const gspm_views *views, const float *Xr, const float *Xp,
                             const float *mask, const gspm_align_params *prm, gspm_align_result *result,
                             void *stream) {
    if (!ctx) return fail(GSPM_ERR_INVALID_ARG, "ctx is NULL");
    if (!Xr || !Xp || !prm || !result) return fail(GSPM_ERR_INVALID_ARG, "Xr, Xp, params and result are required");
    if (prm->patch < 2 || prm->patch > 64) return fail(GSPM_ERR_INVALID_ARG, "patch = %d outside [2, 64]", prm->patch);
    if (prm->max_iter < 1) return fail(GSPM_ERR_INVALID_ARG, "max_iter must be >= 1");
    if (!(prm->delta_mu > 0.0f) || !(prm->delta_sigma > 0.0f) || !(prm->eps_r > 0.0f) || !(prm->tau >= 0.0f))
        return fail(GSPM_ERR_INVALID_ARG, "delta_mu, delta_sigma, eps_r must be > 0 and tau >= 0");
    ViewTable vt;
    int64_t nt, np;
    gspm_status st = build_views(views, 16, vt, nt, np);
    if (st) return st;
    GSPM_HIP(grow(ctx->align, (int64_t)sizeof(AlignPatch) * (align_patches(vt, prm->patch) + 1)));
    GSPM_HIP(launch_align_scale(vt, Xr, Xp, mask, *prm, static_cast<AlignPatch *>(ctx->align.p), result,
                                reinterpret_cast<hipStream_t>(stream)));
    return GSPM_OK;
}

gspm_status gspm_replace_pointmap(const gspm_views *views, const float *Xr, const float *Xp,
                                  const gspm_align_result *result, float eps_m, float *Xr_hat,
                                  int32_t *replaced_out, void *stream) {
    if (!Xr || !Xp || !result || !Xr_hat || !replaced_out)
        return fail(GSPM_ERR_INVALID_ARG, "Xr, Xp, result, Xr_hat and replaced_out are required");
    if (Xr_hat == Xr || Xr_hat == Xp) return fail(GSPM_ERR_INVALID_ARG, "Xr_hat may not alias Xr or Xp");
    if (!(eps_m >= 0.0f)) return fail(GSPM_ERR_INVALID_ARG, "eps_m must be >= 0");
    ViewTable vt;
    int64_t nt, np;
    gspm_status st = build_views(views, 16, vt, nt, np);
    if (st) return st;
    GSPM_HIP(launch_replace(vt, Xr, Xp, result, eps_m, Xr_hat, reinterpret_cast<uint32_t *>(replaced_out),
                            reinterpret_cast<hipStream_t>(stream)));
    return GSPM_OK;
}

gspm_status gspm_pnp_ransac(gspm_ctx *ctx, const float *X, const float *uv, int64_t n, const gspm_intrinsics *K,
                            const int32_t *samples, const gspm_pnp_params *prm, double *T_out, int32_t *n_inliers,
                            uint8_t *inlier_mask, int32_t *scores, const float *T_ak, float *T_n_out,
                            void *stream) {
    if (!ctx) return fail(GSPM_ERR_INVALID_ARG, "ctx is NULL");
    if (!X || !uv || !K || !samples || !prm || !T_out || !n_inliers)
        return fail(GSPM_ERR_INVALID_ARG, "X, uv, K, samples, params, T_out and n_inliers are required");
    if (n < 6 || n > (1ll << 31)) return fail(GSPM_ERR_INVALID_ARG, "n = %lld outside [6, 2^31]", (long long)n);
    if (prm->n_hypotheses < 1 || prm->n_hypotheses > (1 << 20))
        return fail(GSPM_ERR_INVALID_ARG, "n_hypotheses = %d outside [1, 2^20]", prm->n_hypotheses);
    if (!(prm->threshold > 0.0f) || !std::isfinite(prm->threshold) || prm->iterations < 0 || prm->rounds < 0)
        return fail(GSPM_ERR_INVALID_ARG, "threshold must be > 0, iterations and rounds >= 0");
    if (!finite_pos(K->fx) || !finite_pos(K->fy) || !std::isfinite(K->cx) || !std::isfinite(K->cy))
        return fail(GSPM_ERR_INVALID_ARG, "invalid intrinsics");
    GSPM_HIP(grow(ctx->pnp, pnp_scratch_bytes(prm->n_hypotheses, n)));
    GSPM_HIP(launch_pnp(X, uv, n, *K, samples, prm->n_hypotheses, (double)prm->threshold, prm->iterations,
                        prm->rounds, ctx->pnp.p, T_out, n_inliers, inlier_mask, scores,
                        (T_ak && T_n_out) ? T_ak : nullptr, (T_ak && T_n_out) ? T_n_out : nullptr,
                        reinterpret_cast<hipStream_t>(stream)));
    return GSPM_OK;
}

gspm_status gspm_iso_loss(gspm_ctx *ctx, const gspm_gaussians *g, float weight, float *loss_out,
                          float *grad_log_scales, void *stream) {
    if (!ctx) return fail(GSPM_ERR_INVALID_ARG, "ctx is NULL");
    if (!g || g->n < 0 || (g->n > 0 && !g->log_scales)) return fail(GSPM_ERR_INVALID_ARG, "Gaussians are invalid");
    if (!loss_out) return fail(GSPM_ERR_INVALID_ARG, "loss_out is required");
    if (!std::isfinite(weight)) return fail(GSPM_ERR_INVALID_ARG, "weight must be finite");
    GSPM_HIP(grow(ctx->aux, 8 * iso_partials()));
    GSPM_HIP(launch_iso_loss(g->log_scales, g->n, weight, static_cast<double *>(ctx->aux.p), loss_out,
                             grad_log_scales, reinterpret_cast<hipStream_t>(stream)));
    return GSPM_OK;
}

gspm_status gspm_covisibility(gspm_ctx *ctx, const gspm_views *views, int64_t n_gaussians, const void *frame_state,
                              double *iou_out, double *oc_out, int64_t *count_out, void *stream) {
    if (!ctx) return fail(GSPM_ERR_INVALID_ARG, "ctx is NULL");
    if (!frame_state || !iou_out || !oc_out) return fail(GSPM_ERR_INVALID_ARG, "frame_state, iou_out, oc_out required");
    if (n_gaussians < 0) return fail(GSPM_ERR_INVALID_ARG, "n_gaussians < 0");
    ViewTable vt;
    int64_t nt, np;
    gspm_status st = build_views(views, 16, vt, nt, np);
    if (st) return st;
    const FrameLayout L = frame_layout(0, 0, n_gaussians * vt.n_views, 0);
    const int V = vt.n_views;
    GSPM_HIP(grow(ctx->aux, 8 * (int64_t)V * V));
    GSPM_HIP(launch_covisibility(at<uint8_t>(frame_state, L.visible), n_gaussians, V,
                                 at<FrameHeader>(frame_state, L.header),
                                 static_cast<unsigned long long *>(ctx->aux.p), iou_out, oc_out, count_out,
                                 reinterpret_cast<hipStream_t>(stream)));
    return GSPM_OK;
}

gspm_status gspm_median_depth(gspm_ctx *ctx, const gspm_views *views, const float *depth, float *median_out,
                              void *stream) {
    if (!ctx) return fail(GSPM_ERR_INVALID_ARG, "ctx is NULL");
    if (!depth || !median_out) return fail(GSPM_ERR_INVALID_ARG, "depth and median_out are required");
    ViewTable vt;
    int64_t nt, np;
    gspm_status st = build_views(views, 16, vt, nt, np);
    if (st) return st;
    GSPM_HIP(grow(ctx->aux, 4 * median_scratch_words(vt.n_views)));
    GSPM_HIP(launch_median_depth(vt, depth, static_cast<uint32_t *>(ctx->aux.p), median_out,
                                 reinterpret_cast<hipStream_t>(stream)));
    return GSPM_OK;
}

gspm_status gspm_pose_retract(int32_t n_views, float *T_cw, const float *xi, void *stream) {
    if (n_views < 1 || n_views > GSPM_MAX_VIEWS) return fail(GSPM_ERR_INVALID_ARG, "n_views out of range");
    if (!T_cw || !xi) return fail(GSPM_ERR_INVALID_ARG, "T_cw and xi are required");
    GSPM_HIP(launch_pose_retract(n_views, T_cw, xi, reinterpret_cast<hipStream_t>(stream)));
    return GSPM_OK;
}

gspm_status gspm_timing_enable(gspm_ctx *ctx, int32_t on) {
    if (!ctx) return fail(GSPM_ERR_INVALID_ARG, "ctx is NULL");
    ctx->timing = on != 0;
    return GSPM_OK;
}

gspm_status gspm_timing_collect(gspm_ctx *ctx, double *ms_out, int64_t *counts_out) {
    if (!ctx) return fail(GSPM_ERR_INVALID_ARG, "ctx is NULL");
    for (size_t k = 0; k < ctx->phase_of.size(); ++k) {
        hipEvent_t b = ctx->pool[2 * k], e = ctx->pool[2 * k + 1];
        GSPM_HIP(hipEventSynchronize(e));
        float ms = 0.0f;
        GSPM_HIP(hipEventElapsedTime(&ms, b, e));
        const int ph = ctx->phase_of[k];
        if (ms_out) ms_out[ph] += ms;
        if (counts_out) counts_out[ph] += 1;
    }
    ctx->phase_of.clear();
    ctx->used = 0;
    return GSPM_OK;
}

const char *gspm_last_error(void) { return g_last_error.c_str(); }

const char *gspm_version(void) { return "gspm 0.1 gfx950"; }

}  // extern "C"
