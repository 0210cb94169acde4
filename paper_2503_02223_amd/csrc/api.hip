// Host side of the C ABI: argument validation (before any launch), the state
// buffer layout, and the launch sequence of each call.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "ctx.hpp"
#include "dqo_device.hpp"

namespace {

using namespace dqo;

bool tile_ok(int tw, int th) {
    return (tw == 16 && th == 16) || (tw == 8 && th == 8) || (tw == 16 && th == 8) || (tw == 32 && th == 8) ||
           (tw == 8 && th == 32);
}

int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

int key_bits(int64_t tiles_total) {
    int b = 0;
    while (b < 32 && (tiles_total - 1) >> b) ++b;
    return b;
}

struct Geo {
    dqo_layout L;
    int64_t items;
    int depth_blocks, scan_blocks, pair_blocks, pair_passes, pair_first_buf;
    int64_t lb_words;
    // scratch sub-offsets (relative to DQO_BUF_SCRATCH)
    int64_t off_dk1, off_dv1, off_dk2, off_dv2, off_pk1, off_pv1, off_sched, off_sums, off_pose, off_written, off_sbase, off_seg,
        off_sgbase, off_tlast, off_ckpt, off_lbd, off_lbs, off_lbp;
    int64_t seg_cap, ckpt_cap;
    bool tile_sort;     // per-tile depth order (dqo_depth_order TILE)
    int tile_sort_lds;  // pairs of a tile sorted in LDS
};

int validate_frame(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams) {
    if (!ctx) return DQO_EINVAL;
    if (!d || !cams) return fail(ctx, DQO_EINVAL, "frame descriptor and cameras must not be NULL");
    if (d->dtype != DQO_F32 && d->dtype != DQO_F64) return fail(ctx, DQO_EINVAL, "dtype %d unknown", d->dtype);
    if (d->n < 0) return fail(ctx, DQO_EINVAL, "n = %lld < 0", (long long)d->n);
    if (d->n_views < 1 || d->n_views > DQO_MAX_VIEWS)
        return fail(ctx, DQO_EINVAL, "n_views = %d outside [1, %d]", d->n_views, DQO_MAX_VIEWS);
    if (d->K < 0 || d->K > DQO_MAX_K) return fail(ctx, DQO_EINVAL, "K = %d outside [0, %d]", d->K, DQO_MAX_K);
    if (d->pair_capacity < 0 || d->pair_capacity > (int64_t(1) << 30))
        return fail(ctx, DQO_EINVAL, "pair_capacity = %lld outside [0, 2^30]", (long long)d->pair_capacity);
    if ((int64_t)d->n * d->n_views > (int64_t(1) << 31) - 1)
        return fail(ctx, DQO_EINVAL, "n * n_views must be < 2^31");
    if (d->segments) {
        for (int v = 0; v < d->n_views; ++v) {
            const int64_t first = d->segments[2 * v], count = d->segments[2 * v + 1];
            if (first < 0 || count < 0 || first + count > d->n)
                return fail(ctx, DQO_EINVAL, "segment of view %d = [%lld, +%lld) outside [0, %lld)", v,
                            (long long)first, (long long)count, (long long)d->n);
        }
    }
    if (d->jobs) {
        for (int v = 0; v < d->n_views; ++v)
            if (d->jobs[v] < -1 || d->jobs[v] >= d->K)
                return fail(ctx, DQO_EINVAL, "job of view %d = %d outside [-1, K = %d)", v, d->jobs[v], d->K);
    }
    const int W = cams[0].width, H = cams[0].height;
    if (W < 1 || H < 1 || W > 32767 || H > 32767) return fail(ctx, DQO_EINVAL, "image size %dx%d invalid", W, H);
    for (int v = 0; v < d->n_views; ++v) {
        const dqo_camera& c = cams[v];
        if (c.width != W || c.height != H) return fail(ctx, DQO_EINVAL, "all views must share width and height");
        bool fin = isfinite(c.fx) && isfinite(c.fy) && isfinite(c.cx) && isfinite(c.cy);
        for (int k = 0; k < 9; ++k) fin = fin && isfinite(c.R[k]);
        for (int k = 0; k < 3; ++k) fin = fin && isfinite(c.t[k]);
        if (!fin) return fail(ctx, DQO_EINVAL, "camera %d has non-finite entries", v);
    }
    if (!tile_ok(ctx->cfg.tile_w, ctx->cfg.tile_h))
        return fail(ctx, DQO_EINVAL, "tile %dx%d not supported", ctx->cfg.tile_w, ctx->cfg.tile_h);
    return DQO_OK;
}

Geo geometry(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams) {
    Geo g;
    memset(&g, 0, sizeof(g));
    const int tw = ctx->cfg.tile_w, th = ctx->cfg.tile_h;
    const int W = cams[0].width, H = cams[0].height;
    g.L.tiles_x = (W + tw - 1) / tw;
    g.L.tiles_y = (H + th - 1) / th;
    const int64_t tiles_total = (int64_t)g.L.tiles_x * g.L.tiles_y * d->n_views;
    g.L.pair_key_bits = key_bits(tiles_total);
    g.pair_passes = (g.L.pair_key_bits + kRadixBits - 1) / kRadixBits;
    g.pair_first_buf = g.pair_passes & 1;
    g.items = (int64_t)d->n * d->n_views;
    const int64_t M = g.items, cap = d->pair_capacity;
    const int order = ctx->cfg.depth_order;
    g.tile_sort = order == DQO_DEPTH_ORDER_TILE;  // AUTO: GLOBAL
    g.tile_sort_lds = ctx->cfg.tile_sort_lds > 0 ? ctx->cfg.tile_sort_lds : 4096;
    const int64_t ts = d->dtype == DQO_F64 ? 8 : 4;
    g.depth_blocks = (int)((M + kDepthNt * depth_ipt(M) - 1) / (kDepthNt * depth_ipt(M)));
    g.scan_blocks = (int)((M + kScanTile - 1) / kScanTile);
    g.pair_blocks = (int)((cap + kPairTileMin - 1) / kPairTileMin);
    int64_t sz[DQO_BUF_COUNT];
    sz[DQO_BUF_SPLATS] = M * kSplatWords * ts;
    sz[DQO_BUF_RECTS] = M * 8;
    sz[DQO_BUF_COUNTS] = M * 4;
    sz[DQO_BUF_OFFSETS] = M * 4;
    sz[DQO_BUF_DEPTH_KEYS] = M * 4;
    sz[DQO_BUF_DEPTH_ORDER] = M * 4;
    sz[DQO_BUF_PAIR_KEYS] = cap * 4;
    sz[DQO_BUF_PAIR_VALS] = cap * 4;
    sz[DQO_BUF_RANGES] = tiles_total * 8;
    sz[DQO_BUF_PARTIALS] = cap * kGradWords * ts;
    sz[DQO_BUF_CONTROL] = (int64_t)sizeof(Ctrl);
    int64_t so = 0;
    g.off_dk1 = so; so = align256(so + M * 4);
    g.off_dv1 = so; so = align256(so + M * 4);
    g.off_dk2 = so; so = align256(so + M * 4);
    g.off_dv2 = so; so = align256(so + M * 4);
    g.off_pk1 = so; so = align256(so + cap * 4);
    g.off_pv1 = so; so = align256(so + cap * 4);
    g.off_sched = so; so = align256(so + tiles_total * 4);
    g.off_sums = so; so = align256(so + M * kGradWords * ts);
    g.off_pose = so; so = align256(so + (int64_t)d->n_views * ((d->n + 255) / 256) * 6 * 8);
    g.off_written = so; so = align256(so + cap);
    g.off_sbase = so; so = align256(so + (int64_t)g.scan_blocks * 4);
    // segment boundaries (64-pixel tiles, frames the backward segments):
    // sum over tiles of ceil(range / L) - 1 <= cap / L
    g.ckpt_cap = (tw * th == kWave && tiles_total <= kSegTilesMax) ? cap / kSegLen + 1 : 0;
    g.seg_cap = tiles_total + g.ckpt_cap;
    g.off_seg = so; so = align256(so + g.seg_cap * 16);
    g.off_sgbase = so; so = align256(so + tiles_total * 4);
    g.off_tlast = so; so = align256(so + tiles_total * 4);
    g.off_ckpt = so; so = align256(so + g.ckpt_cap * 6 * kWave * ts);
    // look-back words: every block's, then every group's (grouped look-back)
    g.off_lbd = so; so = align256(so + (int64_t)kMaxDepthPasses * lb_blocks(g.depth_blocks) * kRadixBins * 8);
    g.off_lbs = so; so = align256(so + (int64_t)lb_blocks(g.scan_blocks) * (kRadixBins + 1) * 8);
    g.off_lbp = so; so = align256(so + (int64_t)kMaxPairPasses * lb_blocks(g.pair_blocks) * kRadixBins * 8);
    g.lb_words = (so - g.off_lbd) / 8;
    sz[DQO_BUF_SCRATCH] = so;
    int64_t off = 0;
    for (int b = 0; b < DQO_BUF_COUNT; ++b) {
        g.L.offset[b] = off;
        g.L.bytes[b] = sz[b];
        off = align256(off + sz[b]);
    }
    g.L.total = off;
    return g;
}

StatePtrs state_ptrs(const Geo& g, void* state) {
    StatePtrs s;
    char* b = (char*)state;
    s.splats = b + g.L.offset[DQO_BUF_SPLATS];
    s.rects = (short4*)(b + g.L.offset[DQO_BUF_RECTS]);
    s.counts = (uint32_t*)(b + g.L.offset[DQO_BUF_COUNTS]);
    s.offsets = (uint32_t*)(b + g.L.offset[DQO_BUF_OFFSETS]);
    char* sc = b + g.L.offset[DQO_BUF_SCRATCH];
    s.depth_keys[0] = (uint32_t*)(b + g.L.offset[DQO_BUF_DEPTH_KEYS]);
    s.depth_vals[0] = (uint32_t*)(b + g.L.offset[DQO_BUF_DEPTH_ORDER]);
    s.depth_keys[1] = (uint32_t*)(sc + g.off_dk1);
    s.depth_vals[1] = (uint32_t*)(sc + g.off_dv1);
    s.depth_keys[2] = (uint32_t*)(sc + g.off_dk2);
    s.depth_vals[2] = (uint32_t*)(sc + g.off_dv2);
    s.pair_keys[0] = (uint32_t*)(b + g.L.offset[DQO_BUF_PAIR_KEYS]);
    s.pair_vals[0] = (uint32_t*)(b + g.L.offset[DQO_BUF_PAIR_VALS]);
    s.pair_keys[1] = (uint32_t*)(sc + g.off_pk1);
    s.pair_vals[1] = (uint32_t*)(sc + g.off_pv1);
    s.ranges = (uint32_t*)(b + g.L.offset[DQO_BUF_RANGES]);
    s.partials = b + g.L.offset[DQO_BUF_PARTIALS];
    s.schedule = (uint32_t*)(sc + g.off_sched);
    s.sums = sc + g.off_sums;
    s.pose_partials = (double*)(sc + g.off_pose);
    s.written = (uint8_t*)(sc + g.off_written);
    s.scan_base = (uint32_t*)(sc + g.off_sbase);
    s.seg_list = (uint4*)(sc + g.off_seg);
    s.seg_base = (uint32_t*)(sc + g.off_sgbase);
    s.tile_last = (int32_t*)(sc + g.off_tlast);
    s.ckpt = sc + g.off_ckpt;
    s.seg_cap = g.seg_cap;
    s.ckpt_cap = g.ckpt_cap;
    s.ctrl = (Ctrl*)(b + g.L.offset[DQO_BUF_CONTROL]);
    s.lb_depth = (uint64_t*)(sc + g.off_lbd);
    s.lb_scan = (uint64_t*)(sc + g.off_lbs);
    s.lb_pair = (uint64_t*)(sc + g.off_lbp);
    s.items = g.items;
    s.capacity = g.L.bytes[DQO_BUF_PAIR_KEYS] / 4;
    s.depth_blocks = g.depth_blocks;
    s.scan_blocks = g.scan_blocks;
    s.pair_blocks = g.pair_blocks;
    s.pair_passes = g.pair_passes;
    s.pair_first_buf = g.pair_first_buf;
    s.tile_sort = g.tile_sort;
    s.tile_sort_lds = g.tile_sort_lds;
#ifndef DQO_FUSED_EMIT
#define DQO_FUSED_EMIT 1
#endif
    s.fused_emit = DQO_FUSED_EMIT && g.pair_passes >= 1 && g.scan_blocks <= scan_emit_resident(true);
    // One histogram copy per 64 producer workgroups (up to kHistCopies): enough
    // to spread the atomics, few enough for the radix passes to sum cheaply.
    const int64_t proj_blocks = (g.items + 256 * kProjItems - 1) / (256 * kProjItems);
    s.hist_copies_depth = (int)std::max<int64_t>(1, std::min<int64_t>(kHistCopies, proj_blocks / 64));
    s.hist_copies_pair = (int)std::max<int64_t>(1, std::min<int64_t>(kHistCopies, g.scan_blocks / 64));
    return s;
}

template <typename T>
Frame<T> make_frame(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams, const Geo& g, void* state) {
    Frame<T> f;
    memset(&f, 0, sizeof(f));
    const dqo_config& c = ctx->cfg;
    for (int v = 0; v < d->n_views; ++v) {
        DevCam<T>& dc = f.views.cam[v];
        for (int k = 0; k < 9; ++k) dc.R[k] = (T)cams[v].R[k];
        for (int k = 0; k < 3; ++k) dc.t[k] = (T)cams[v].t[k];
        dc.fx = (T)cams[v].fx;
        dc.fy = (T)cams[v].fy;
        dc.cx = (T)cams[v].cx;
        dc.cy = (T)cams[v].cy;
        dc.limx = (T)(1.3 * 0.5 * cams[v].width / cams[v].fx);
        dc.limy = (T)(1.3 * 0.5 * cams[v].height / cams[v].fy);
        dc.seg_lo = d->segments ? (int32_t)d->segments[2 * v] : 0;
        dc.seg_hi = d->segments ? (int32_t)(d->segments[2 * v] + d->segments[2 * v + 1]) : (int32_t)d->n;
        const int W = cams[0].width, H = cams[0].height;
        int32_t x0 = 0, y0 = 0, x1 = W, y1 = H;
        if (d->windows) {
            x0 = std::max(0, d->windows[4 * v]);
            y0 = std::max(0, d->windows[4 * v + 1]);
            x1 = std::min(W, d->windows[4 * v + 2]);
            y1 = std::min(H, d->windows[4 * v + 3]);
            if (x1 <= x0 || y1 <= y0) x0 = y0 = x1 = y1 = 0;
        }
        dc.win_x0 = x0;
        dc.win_y0 = y0;
        dc.win_x1 = x1;
        dc.win_y1 = y1;
        const int tw = ctx->cfg.tile_w, th = ctx->cfg.tile_h;
        dc.tile_x0 = x0 / tw;
        dc.tile_y0 = y0 / th;
        dc.tile_x1 = x1 > x0 ? (x1 - 1) / tw : -1;
        dc.tile_y1 = y1 > y0 ? (y1 - 1) / th : -1;
        dc.job = d->jobs ? d->jobs[v] : -1;
    }
    f.views.n_views = d->n_views;
    f.views.W = cams[0].width;
    f.views.H = cams[0].height;
    f.views.tile_w = c.tile_w;
    f.views.tile_h = c.tile_h;
    f.views.tiles_x = g.L.tiles_x;
    f.views.tiles_y = g.L.tiles_y;
    f.views.tiles_per_view = g.L.tiles_x * g.L.tiles_y;
    f.consts.z_near = (T)c.z_near;
    f.consts.dilation = (T)c.dilation;
    f.consts.q_max = (T)c.q_max;
    f.consts.alpha_min = (T)c.alpha_min;
    f.consts.alpha_max = (T)c.alpha_max;
    f.consts.t_min = (T)c.t_min;
    for (int k = 0; k < 3; ++k) f.consts.bg[k] = (T)c.bg[k];
    f.n = d->n;
    f.K = d->K;
    if (state) f.s = state_ptrs(g, state);  // the image-space passes need only the views
    return f;
}

int check_quadric_inputs(const dqo_ctx* ctx, int32_t n_obj, int64_t n_boxes, const double* boxes,
                         const int32_t* box_obj, const int32_t* box_view, int32_t n_views, const double* P) {
    if (n_obj < 0 || n_boxes < 0 || n_views < 0) return fail(ctx, DQO_EINVAL, "negative size");
    if (n_obj > 65535) return fail(ctx, DQO_EINVAL, "n_obj too large");
    if (n_boxes > 0 && (!boxes || !box_obj || !box_view || !P || n_views < 1))
        return fail(ctx, DQO_EINVAL, "boxes, box_obj, box_view and P are required");
    return DQO_OK;
}

int check_increment_cfg(const dqo_ctx* ctx, const dqo_increment_cfg* c) {
    if (!c) return fail(ctx, DQO_EINVAL, "increment config must not be NULL");
    if (!(c->theta_alpha >= 0 && c->theta_alpha <= 1)) return fail(ctx, DQO_EINVAL, "theta_alpha outside [0, 1]");
    if (!(c->theta_d >= 0) || !(c->theta_c >= 0)) return fail(ctx, DQO_EINVAL, "theta_d and theta_c must be >= 0");
    if (!(c->og_opacity > 0 && c->og_opacity < 1) || !(c->tg_opacity > 0 && c->tg_opacity < 1))
        return fail(ctx, DQO_EINVAL, "OG and TG opacities must lie in (0, 1)");
    return DQO_OK;
}

int check_images(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_images* img, bool need_probs_ok) {
    if (!img) return fail(ctx, DQO_EINVAL, "images must not be NULL");
    if (!img->color || !img->depth || !img->t_final || !img->last)
        return fail(ctx, DQO_EINVAL, "images: color, depth, t_final and last are required");
    if (img->probs && d->K < 1) return fail(ctx, DQO_EINVAL, "probs requested with K = 0");
    if (img->id_map && !img->probs) return fail(ctx, DQO_EINVAL, "id_map needs probs");
    if (img->p_target && !img->target) return fail(ctx, DQO_EINVAL, "p_target needs target");
    if (need_probs_ok && img->probs) {
        const int64_t ts = d->dtype == DQO_F64 ? 8 : 4;
        if ((int64_t)d->K * ctx->cfg.tile_w * ctx->cfg.tile_h * ts > 65536)
            return fail(ctx, DQO_EINVAL, "K = %d instance channels do not fit in LDS for this tile and dtype", d->K);
    }
    return DQO_OK;
}

template <typename F>
int run(const dqo_ctx* ctx, const char* what, F&& fn) {
    hipError_t e = fn();
    if (e != hipSuccess) return hip_fail(ctx, e, what);
    ctx->err[0] = 0;
    return DQO_OK;
}

int check_loss_args(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams, const dqo_images* img,
                    const dqo_targets* tgt, const dqo_loss_weights* w, double* loss, const dqo_image_grads* gr) {
    int rc = validate_frame(ctx, d, cams);
    if (rc) return rc;
    if (!img || !img->color || !img->depth || !img->p_target)
        return fail(ctx, DQO_EINVAL, "object_loss needs color, depth and p_target images");
    if (!tgt || !tgt->color || !tgt->depth) return fail(ctx, DQO_EINVAL, "object_loss needs target color and depth");
    if (!w || !loss) return fail(ctx, DQO_EINVAL, "weights and loss must not be NULL");
    if (!(w->ce_eps > 0)) return fail(ctx, DQO_EINVAL, "ce_eps must be > 0");
    if (gr && (!gr->d_color || !gr->d_depth || !gr->d_p_target))
        return fail(ctx, DQO_EINVAL, "object_loss gradients need d_color, d_depth and d_p_target");
    if (d->jobs && !tgt->id) {
        for (int v = 0; v < d->n_views; ++v)
            if (d->jobs[v] >= 0) return fail(ctx, DQO_EINVAL, "per-object jobs need the target ids");
    }
    return DQO_OK;
}

int enqueue_loss(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams, const dqo_images* img,
                 const dqo_targets* tgt, const dqo_loss_weights* w, double* loss, const dqo_image_grads* gr,
                 double* partials, uint32_t* n_valid, void* stream) {
    dqo_image_grads none;
    memset(&none, 0, sizeof(none));
    const int64_t HW = (int64_t)cams[0].width * cams[0].height;
    const dqo_image_grads& g = gr ? *gr : none;
    // each view's window and job, as the render kernels see them
    Geo geo = geometry(ctx, d, cams);
    Frame<float> f = make_frame<float>(ctx, d, cams, geo, nullptr);
    LossViewsHost lv;
    memset(&lv, 0, sizeof(lv));
    for (int v = 0; v < d->n_views; ++v) {
        const DevCam<float>& c = f.views.cam[v];
        lv.win[v][0] = c.win_x0;
        lv.win[v][1] = c.win_y0;
        lv.win[v][2] = c.win_x1;
        lv.win[v][3] = c.win_y1;
        lv.job[v] = c.job;
    }
    lv.W = cams[0].width;
    return run(ctx, "object_loss", [&] {
        if (d->dtype == DQO_F32)
            return launch_object_loss<float>(HW, d->n_views, *img, *tgt, *w, loss, g, lv, partials, n_valid,
                                             (hipStream_t)stream);
        return launch_object_loss<double>(HW, d->n_views, *img, *tgt, *w, loss, g, lv, partials, n_valid,
                                          (hipStream_t)stream);
    });
}

}  // namespace

extern "C" {

void dqo_config_default(dqo_config* c) {
    if (!c) return;
    c->tile_w = 16;
    c->tile_h = 16;
    c->z_near = 0.2;
    c->dilation = 0.3;
    c->q_max = 9.0;
    c->alpha_min = 1.0 / 255.0;
    c->alpha_max = 0.99;
    c->t_min = 1e-4;
    c->bg[0] = c->bg[1] = c->bg[2] = 0.0;
    c->depth_order = DQO_DEPTH_ORDER_AUTO;
    c->tile_sort_lds = 0;
}

int dqo_ctx_create(dqo_ctx** out, const dqo_config* cfg) {
    if (!out) return DQO_EINVAL;
    dqo_config c;
    dqo_config_default(&c);
    if (cfg) c = *cfg;
    if (!tile_ok(c.tile_w, c.tile_h)) return DQO_EINVAL;
    if (!(c.alpha_min > 0 && c.alpha_max <= 1 && c.alpha_min < c.alpha_max && c.t_min > 0 && c.t_min < 1 &&
          c.q_max > 0 && c.dilation >= 0 && c.z_near > 0 && c.depth_order >= DQO_DEPTH_ORDER_AUTO &&
          c.depth_order <= DQO_DEPTH_ORDER_TILE && c.tile_sort_lds >= 0 && c.tile_sort_lds <= 4096))
        return DQO_EINVAL;
    dqo_ctx* x = new dqo_ctx;
    x->cfg = c;
    x->err[0] = 0;
    *out = x;
    return DQO_OK;
}

int dqo_ctx_destroy(dqo_ctx* ctx) {
    delete ctx;
    return DQO_OK;
}

const char* dqo_last_error(const dqo_ctx* ctx) { return ctx ? ctx->err : "NULL context"; }

const char* dqo_version(void) { return "dqo 0.2 gfx950"; }

const char* dqo_status_string(int code) {
    switch (code) {
        case DQO_OK: return "ok";
        case DQO_EINVAL: return "invalid argument";
        case DQO_ECAPACITY: return "pair capacity exceeded";
        case DQO_ENONFINITE: return "non-finite input";
        case DQO_EDEGENERATE: return "degenerate input";
        case DQO_EHIP: return "HIP runtime error";
        case DQO_EINTERNAL: return "internal device wait bound exceeded";
        default: return "unknown status";
    }
}

int dqo_state_layout(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams, dqo_layout* out) {
    int rc = validate_frame(ctx, d, cams);
    if (rc) return rc;
    if (!out) return fail(ctx, DQO_EINVAL, "layout output must not be NULL");
    *out = geometry(ctx, d, cams).L;
    return DQO_OK;
}

int dqo_state_init(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams, void* state, void* stream) {
    int rc = validate_frame(ctx, d, cams);
    if (rc) return rc;
    if (!state) return fail(ctx, DQO_EINVAL, "state must not be NULL");
    Geo g = geometry(ctx, d, cams);
    StatePtrs s = state_ptrs(g, state);
    return run(ctx, "state_init", [&] {
        hipError_t e = launch_clear_ctrl(s.ctrl, s.lb_depth, g.lb_words, (hipStream_t)stream);
        if (e != hipSuccess) return e;
        return launch_zero_words(s.ranges, g.L.bytes[DQO_BUF_RANGES] / 4, (hipStream_t)stream);
    });
}

int dqo_read_status(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams, void* state,
                    uint32_t* status, int64_t* num_pairs, void* stream) {
    int rc = validate_frame(ctx, d, cams);
    if (rc) return rc;
    if (!state) return fail(ctx, DQO_EINVAL, "state must not be NULL");
    Geo g = geometry(ctx, d, cams);
    StatePtrs s = state_ptrs(g, state);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "read_status sync");
    uint32_t h[3];
    e = hipMemcpy(h, s.ctrl, sizeof(h), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "read_status copy");
    if (status) *status = h[0];
    if (num_pairs) *num_pairs = h[2];
    if (h[0] & DQO_STATUS_TIMEOUT) return fail(ctx, DQO_EINTERNAL, "a device wait exceeded its bound");
    if (h[0] & DQO_STATUS_OVERFLOW)
        return fail(ctx, DQO_ECAPACITY, "pair list needs %u entries, capacity %lld", h[2],
                    (long long)d->pair_capacity);
    if (h[0] & DQO_STATUS_NONFINITE) return fail(ctx, DQO_ENONFINITE, "non-finite Gaussian parameters");
    ctx->err[0] = 0;
    return DQO_OK;
}

int dqo_clear_status(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams, void* state,
                     void* stream) {
    int rc = validate_frame(ctx, d, cams);
    if (rc) return rc;
    if (!state) return fail(ctx, DQO_EINVAL, "state must not be NULL");
    Geo g = geometry(ctx, d, cams);
    StatePtrs s = state_ptrs(g, state);
    return run(ctx, "clear_status", [&] { return launch_clear_status(s.ctrl, (hipStream_t)stream); });
}

int dqo_project_cull_bin(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams, const void* params,
                         const int32_t* ids, void* state, void* stream) {
    int rc = validate_frame(ctx, d, cams);
    if (rc) return rc;
    if (!state || (d->n > 0 && (!params || !ids)))
        return fail(ctx, DQO_EINVAL, "params, ids and state must not be NULL");
    Geo g = geometry(ctx, d, cams);
    if (d->dtype == DQO_F32) {
        Frame<float> f = make_frame<float>(ctx, d, cams, g, state);
        return run(ctx, "project_cull_bin", [&] {
            return launch_project_bin<float>(f, (const float*)params, ids, (hipStream_t)stream);
        });
    }
    Frame<double> f = make_frame<double>(ctx, d, cams, g, state);
    return run(ctx, "project_cull_bin",
               [&] { return launch_project_bin<double>(f, (const double*)params, ids, (hipStream_t)stream); });
}

int dqo_sort(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams, void* state, void* stream) {
    int rc = validate_frame(ctx, d, cams);
    if (rc) return rc;
    if (!state) return fail(ctx, DQO_EINVAL, "state must not be NULL");
    Geo g = geometry(ctx, d, cams);
    StatePtrs s = state_ptrs(g, state);
    const int tiles_total = g.L.tiles_x * g.L.tiles_y * d->n_views;
    return run(ctx, "sort", [&] {
        // also clears the written marks of the pairs (the render backward
        // writes only the pairs that contribute in their tile, and marks them)
        return launch_pair_sort(s, tiles_total, (hipStream_t)stream);
    });
}

int dqo_render_forward(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams, const void* state,
                       const dqo_images* img, void* stream) {
    int rc = validate_frame(ctx, d, cams);
    if (rc) return rc;
    if (!state) return fail(ctx, DQO_EINVAL, "state must not be NULL");
    rc = check_images(ctx, d, img, true);
    if (rc) return rc;
    Geo g = geometry(ctx, d, cams);
    if (d->dtype == DQO_F32) {
        Frame<float> f = make_frame<float>(ctx, d, cams, g, (void*)state);
        return run(ctx, "render_forward", [&] { return launch_render_forward<float>(f, *img, (hipStream_t)stream); });
    }
    Frame<double> f = make_frame<double>(ctx, d, cams, g, (void*)state);
    return run(ctx, "render_forward", [&] { return launch_render_forward<double>(f, *img, (hipStream_t)stream); });
}

int dqo_object_loss(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams, const dqo_images* img,
                    const dqo_targets* tgt, const dqo_loss_weights* w, double* loss, const dqo_image_grads* gr,
                    void* state, void* stream) {
    int rc = check_loss_args(ctx, d, cams, img, tgt, w, loss, gr);
    if (rc) return rc;
    if (!state) return fail(ctx, DQO_EINVAL, "state must not be NULL");
    Geo g = geometry(ctx, d, cams);
    StatePtrs s = state_ptrs(g, state);
    return enqueue_loss(ctx, d, cams, img, tgt, w, loss, gr, &s.ctrl->loss_partials[0][0], &s.ctrl->n_valid,
                        stream);
}

// The allocation-free object loss: its per-workgroup partial sums and the
// valid-depth count live in `scratch`, one copy per device, whose address
// is taken once per device (a __device__ symbol's host-side name is not a
// device address: kernels get the address from hipGetSymbolAddress).
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};

int scratch_address(const dqo_ctx* ctx, void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(ctx, e, "object_loss_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kNoAllocMaxDevices)
        return fail(ctx, DQO_EINVAL, "object_loss_noalloc: device %d beyond the %d supported", dev,
                    kNoAllocMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(ctx, e, "object_loss_noalloc: hipGetSymbolAddress(scratch)");
        if (!p) return fail(ctx, DQO_EHIP, "object_loss_noalloc: no device address for scratch");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DQO_OK;
}
}  // namespace

int dqo_object_loss_noalloc(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams,
                            const dqo_images* img, const dqo_targets* tgt, const dqo_loss_weights* w, double* loss,
                            const dqo_image_grads* gr, void* stream) {
    int rc = check_loss_args(ctx, d, cams, img, tgt, w, loss, gr);
    if (rc) return rc;
    const int64_t npix = (int64_t)cams[0].width * cams[0].height * d->n_views;
    const int blocks = loss_partial_blocks(npix);
    if ((int64_t)blocks * kLossParts + 1 > kNoAllocScratchDoubles)
        return fail(ctx, DQO_EINVAL, "object_loss_noalloc: %d partial rows exceed the scratch of %d", blocks,
                    (kNoAllocScratchDoubles - 1) / kLossParts);
    void* sp = nullptr;
    rc = scratch_address(ctx, &sp);
    if (rc) return rc;
    double* partials = (double*)sp;
    uint32_t* n_valid = (uint32_t*)(partials + (kNoAllocScratchDoubles - 1));
    return enqueue_loss(ctx, d, cams, img, tgt, w, loss, gr, partials, n_valid, stream);
}

int dqo_render_backward(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams, void* state,
                        const dqo_images* img, const dqo_image_grads* gr, void* stream) {
    int rc = validate_frame(ctx, d, cams);
    if (rc) return rc;
    if (!state) return fail(ctx, DQO_EINVAL, "state must not be NULL");
    rc = check_images(ctx, d, img, false);
    if (rc) return rc;
    if (!gr || !gr->d_color) return fail(ctx, DQO_EINVAL, "render_backward needs d_color");
    if (gr->d_p_target && !img->target) return fail(ctx, DQO_EINVAL, "d_p_target needs images.target");
    if (gr->d_probs && d->K < 1) return fail(ctx, DQO_EINVAL, "d_probs with K = 0");
    Geo g = geometry(ctx, d, cams);
    if (d->dtype == DQO_F32) {
        Frame<float> f = make_frame<float>(ctx, d, cams, g, state);
        return run(ctx, "render_backward",
                   [&] { return launch_render_backward<float>(f, *img, *gr, (hipStream_t)stream); });
    }
    Frame<double> f = make_frame<double>(ctx, d, cams, g, state);
    return run(ctx, "render_backward",
               [&] { return launch_render_backward<double>(f, *img, *gr, (hipStream_t)stream); });
}

int dqo_project_backward(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams, const void* params,
                         const void* state, void* grads, void* stream) {
    int rc = validate_frame(ctx, d, cams);
    if (rc) return rc;
    if (!state || (d->n > 0 && (!params || !grads)))
        return fail(ctx, DQO_EINVAL, "params, state and grads must not be NULL");
    Geo g = geometry(ctx, d, cams);
    if (d->dtype == DQO_F32) {
        Frame<float> f = make_frame<float>(ctx, d, cams, g, (void*)state);
        return run(ctx, "project_backward", [&] {
            return launch_project_backward<float>(f, (const float*)params, (float*)grads, (hipStream_t)stream);
        });
    }
    Frame<double> f = make_frame<double>(ctx, d, cams, g, (void*)state);
    return run(ctx, "project_backward", [&] {
        return launch_project_backward<double>(f, (const double*)params, (double*)grads, (hipStream_t)stream);
    });
}

int dqo_pose_backward(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams, const void* params,
                      const void* state, double* pose_grads, void* stream) {
    int rc = validate_frame(ctx, d, cams);
    if (rc) return rc;
    if (!state || !pose_grads || (d->n > 0 && !params))
        return fail(ctx, DQO_EINVAL, "params, state and pose_grads must not be NULL");
    Geo g = geometry(ctx, d, cams);
    if (d->dtype == DQO_F32) {
        Frame<float> f = make_frame<float>(ctx, d, cams, g, (void*)state);
        return run(ctx, "pose_backward", [&] {
            return launch_pose_backward<float>(f, (const float*)params, pose_grads, (hipStream_t)stream);
        });
    }
    Frame<double> f = make_frame<double>(ctx, d, cams, g, (void*)state);
    return run(ctx, "pose_backward", [&] {
        return launch_pose_backward<double>(f, (const double*)params, pose_grads, (hipStream_t)stream);
    });
}

int dqo_project_backward_adam(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams, void* params,
                              const void* state, void* m, void* v, const dqo_adam* hp, int64_t* d_step, void* grads,
                              void* stream) {
    int rc = validate_frame(ctx, d, cams);
    if (rc) return rc;
    if (!state || !hp || !d_step || (d->n > 0 && (!params || !m || !v)))
        return fail(ctx, DQO_EINVAL, "params, state, m, v, hyper-parameters and the step counter are required");
    if (!(hp->beta1 >= 0 && hp->beta1 < 1 && hp->beta2 >= 0 && hp->beta2 < 1 && hp->eps >= 0))
        return fail(ctx, DQO_EINVAL, "adam betas must lie in [0, 1) and eps >= 0");
    Geo g = geometry(ctx, d, cams);
    if (d->dtype == DQO_F32) {
        Frame<float> f = make_frame<float>(ctx, d, cams, g, (void*)state);
        return run(ctx, "project_backward_adam", [&] {
            return launch_project_backward_adam<float>(f, (float*)params, (float*)grads, (float*)m, (float*)v, *hp,
                                                       d_step, (hipStream_t)stream);
        });
    }
    Frame<double> f = make_frame<double>(ctx, d, cams, g, (void*)state);
    return run(ctx, "project_backward_adam", [&] {
        return launch_project_backward_adam<double>(f, (double*)params, (double*)grads, (double*)m, (double*)v, *hp,
                                                    d_step, (hipStream_t)stream);
    });
}

int dqo_incremental_masks(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams,
                          const dqo_images* img, const dqo_targets* tgt, const dqo_increment_cfg* cfg,
                          uint8_t* masks, int32_t* obj_counts, void* stream) {
    int rc = validate_frame(ctx, d, cams);
    if (rc) return rc;
    if ((rc = check_increment_cfg(ctx, cfg))) return rc;
    if (d->K < 1) return fail(ctx, DQO_EINVAL, "incremental masks need K >= 1");
    if (!img || !img->color || !img->depth || !img->p_target)
        return fail(ctx, DQO_EINVAL, "incremental masks need rendered color, depth and p_target");
    if (!tgt || !tgt->color || !tgt->depth || !tgt->id)
        return fail(ctx, DQO_EINVAL, "incremental masks need target color, depth and id");
    if (!masks || !obj_counts) return fail(ctx, DQO_EINVAL, "masks and obj_counts must not be NULL");
    Geo g = geometry(ctx, d, cams);
    if (d->dtype == DQO_F32) {
        Frame<float> f = make_frame<float>(ctx, d, cams, g, nullptr);
        return run(ctx, "incremental_masks", [&] {
            return launch_incremental_masks<float>(f, *img, *tgt, *cfg, masks, obj_counts, (hipStream_t)stream);
        });
    }
    Frame<double> f = make_frame<double>(ctx, d, cams, g, nullptr);
    return run(ctx, "incremental_masks", [&] {
        return launch_incremental_masks<double>(f, *img, *tgt, *cfg, masks, obj_counts, (hipStream_t)stream);
    });
}

int dqo_densify(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams, const dqo_targets* tgt,
                const uint8_t* masks, const dqo_increment_cfg* cfg, int64_t n_old, int64_t n_cap, void* params,
                int32_t* ids, int64_t* counts, void* stream) {
    int rc = validate_frame(ctx, d, cams);
    if (rc) return rc;
    if ((rc = check_increment_cfg(ctx, cfg))) return rc;
    if (!tgt || !tgt->color || !tgt->depth || !tgt->id)
        return fail(ctx, DQO_EINVAL, "densify needs target color, depth and id");
    if (!masks || !counts) return fail(ctx, DQO_EINVAL, "masks and counts must not be NULL");
    if (n_old < 0 || n_cap < n_old || n_cap > (int64_t(1) << 31) - 1)
        return fail(ctx, DQO_EINVAL, "need 0 <= n_old <= n_cap < 2^31 (n_old %lld, n_cap %lld)", (long long)n_old,
                    (long long)n_cap);
    if (n_cap > n_old && (!params || !ids)) return fail(ctx, DQO_EINVAL, "params and ids must not be NULL");
    Geo g = geometry(ctx, d, cams);
    if (d->dtype == DQO_F32) {
        Frame<float> f = make_frame<float>(ctx, d, cams, g, nullptr);
        return run(ctx, "densify", [&] {
            return launch_densify<float>(f, *tgt, masks, *cfg, n_old, n_cap, (float*)params, ids, counts,
                                         (hipStream_t)stream);
        });
    }
    Frame<double> f = make_frame<double>(ctx, d, cams, g, nullptr);
    return run(ctx, "densify", [&] {
        return launch_densify<double>(f, *tgt, masks, *cfg, n_old, n_cap, (double*)params, ids, counts,
                                      (hipStream_t)stream);
    });
}

int dqo_adam_step(const dqo_ctx* ctx, int32_t dtype, void* params, const void* grads, void* m, void* v, int64_t n,
                  const dqo_adam* hp, int64_t step, void* stream) {
    if (!ctx) return DQO_EINVAL;
    if (dtype != DQO_F32 && dtype != DQO_F64) return fail(ctx, DQO_EINVAL, "dtype %d unknown", dtype);
    if (n < 0 || step < 1 || !hp) return fail(ctx, DQO_EINVAL, "need n >= 0, step >= 1 and hyper-parameters");
    if (n > 0 && (!params || !grads || !m || !v)) return fail(ctx, DQO_EINVAL, "adam buffers must not be NULL");
    if (!(hp->beta1 >= 0 && hp->beta1 < 1 && hp->beta2 >= 0 && hp->beta2 < 1 && hp->eps >= 0))
        return fail(ctx, DQO_EINVAL, "adam betas must lie in [0, 1) and eps >= 0");
    if (dtype == DQO_F32)
        return run(ctx, "adam", [&] {
            return launch_adam<float>((float*)params, (const float*)grads, (float*)m, (float*)v, n, *hp, step,
                                      nullptr, (hipStream_t)stream);
        });
    return run(ctx, "adam", [&] {
        return launch_adam<double>((double*)params, (const double*)grads, (double*)m, (double*)v, n, *hp, step,
                                   nullptr, (hipStream_t)stream);
    });
}

int dqo_adam_step_counted(const dqo_ctx* ctx, int32_t dtype, void* params, const void* grads, void* m, void* v,
                          int64_t n, const dqo_adam* hp, int64_t* d_step, void* stream) {
    if (!ctx) return DQO_EINVAL;
    if (dtype != DQO_F32 && dtype != DQO_F64) return fail(ctx, DQO_EINVAL, "dtype %d unknown", dtype);
    if (n < 0 || !hp || !d_step) return fail(ctx, DQO_EINVAL, "need n >= 0, hyper-parameters and a step counter");
    if (n > 0 && (!params || !grads || !m || !v)) return fail(ctx, DQO_EINVAL, "adam buffers must not be NULL");
    if (!(hp->beta1 >= 0 && hp->beta1 < 1 && hp->beta2 >= 0 && hp->beta2 < 1 && hp->eps >= 0))
        return fail(ctx, DQO_EINVAL, "adam betas must lie in [0, 1) and eps >= 0");
    if (dtype == DQO_F32)
        return run(ctx, "adam", [&] {
            return launch_adam<float>((float*)params, (const float*)grads, (float*)m, (float*)v, n, *hp, 1, d_step,
                                      (hipStream_t)stream);
        });
    return run(ctx, "adam", [&] {
        return launch_adam<double>((double*)params, (const double*)grads, (double*)m, (double*)v, n, *hp, 1, d_step,
                                   (hipStream_t)stream);
    });
}

int dqo_id_boxes(const dqo_ctx* ctx, const int32_t* id_map, int32_t n_views, int32_t width, int32_t height,
                 int32_t K, double* boxes, int32_t* box_obj, int32_t* box_view, void* stream) {
    if (!ctx) return DQO_EINVAL;
    if (n_views < 1 || n_views > DQO_MAX_VIEWS || width < 1 || height < 1 || K < 1 || K > DQO_MAX_K)
        return fail(ctx, DQO_EINVAL, "id_boxes: bad sizes");
    if (!id_map || !boxes || !box_obj || !box_view) return fail(ctx, DQO_EINVAL, "id_boxes: NULL buffer");
    return run(ctx, "id_boxes", [&] {
        return launch_id_boxes(id_map, n_views, width, height, K, boxes, box_obj, box_view, (hipStream_t)stream);
    });
}

int dqo_fit_dual_quadric(const dqo_ctx* ctx, int32_t n_obj, int64_t n_boxes, const double* boxes,
                         const int32_t* box_obj, const int32_t* box_view, int32_t n_views, const double* P,
                         const int32_t* img_wh, double border, double* Q, double* mu, double* R, double* axes,
                         int32_t* status, void* stream) {
    if (!ctx) return DQO_EINVAL;
    if (n_obj < 0 || n_boxes < 0 || n_views < 0) return fail(ctx, DQO_EINVAL, "negative size");
    if (n_boxes > 0 && (!boxes || !box_obj || !box_view || !P || n_views < 1))
        return fail(ctx, DQO_EINVAL, "boxes, box_obj, box_view and P are required");
    if (n_obj > 0 && (!Q || !mu || !R || !axes || !status))
        return fail(ctx, DQO_EINVAL, "quadric outputs must not be NULL");
    if (n_obj > 65535) return fail(ctx, DQO_EINVAL, "n_obj too large");
    return run(ctx, "fit_dual_quadric", [&] {
        return launch_fit_quadric(n_obj, n_boxes, boxes, box_obj, box_view, n_views, P, img_wh, border, Q, mu, R,
                                  axes, status, (hipStream_t)stream);
    });
}

int dqo_quadric_iou_grad(const dqo_ctx* ctx, int32_t n_obj, int64_t n_boxes, const double* boxes,
                         const int32_t* box_obj, const int32_t* box_view, int32_t n_views, const double* P,
                         const int32_t* img_wh, const double* theta, double* loss, double* grad, double* box_iou,
                         void* stream) {
    if (!ctx) return DQO_EINVAL;
    int rc = check_quadric_inputs(ctx, n_obj, n_boxes, boxes, box_obj, box_view, n_views, P);
    if (rc) return rc;
    if (n_obj > 0 && (!theta || !loss || !grad)) return fail(ctx, DQO_EINVAL, "theta, loss and grad are required");
    return run(ctx, "quadric_iou_grad", [&] {
        return launch_quadric_iou_grad(n_obj, n_views, n_boxes, boxes, box_obj, box_view, P, img_wh, theta, loss,
                                       grad, box_iou, (hipStream_t)stream);
    });
}

int dqo_refine_quadrics(const dqo_ctx* ctx, int32_t n_obj, int64_t n_boxes, const double* boxes,
                        const int32_t* box_obj, const int32_t* box_view, int32_t n_views, const double* P,
                        const int32_t* img_wh, const int32_t* status, const dqo_refine_cfg* cfg, double* mu,
                        double* R, double* axes, double* Q, double* loss, double* box_iou, void* stream) {
    if (!ctx) return DQO_EINVAL;
    int rc = check_quadric_inputs(ctx, n_obj, n_boxes, boxes, box_obj, box_view, n_views, P);
    if (rc) return rc;
    if (!cfg) return fail(ctx, DQO_EINVAL, "refine config must not be NULL");
    if (cfg->iterations < 0 || cfg->iterations > 1000000)
        return fail(ctx, DQO_EINVAL, "iterations = %d outside [0, 1e6]", cfg->iterations);
    if (!(cfg->lr_mu >= 0) || !(cfg->lr_rot >= 0) || !(cfg->lr_axes >= 0) || !isfinite(cfg->lr_mu) ||
        !isfinite(cfg->lr_rot) || !isfinite(cfg->lr_axes))
        return fail(ctx, DQO_EINVAL, "learning rates must be finite and >= 0");
    if (!(cfg->beta1 >= 0 && cfg->beta1 < 1) || !(cfg->beta2 >= 0 && cfg->beta2 < 1) || !(cfg->eps > 0))
        return fail(ctx, DQO_EINVAL, "need 0 <= beta1, beta2 < 1 and eps > 0");
    if (n_obj > 0 && (!mu || !R || !axes || !loss)) return fail(ctx, DQO_EINVAL, "mu, R, axes and loss are required");
    return run(ctx, "refine_quadrics", [&] {
        return launch_refine_quadrics(n_obj, n_views, n_boxes, boxes, box_obj, box_view, P, img_wh, status, *cfg, mu,
                                      R, axes, Q, loss, box_iou, (hipStream_t)stream);
    });
}

int dqo_associate(const dqo_ctx* ctx, int32_t n_obj, const double* mu, const double* R, const double* axes,
                  int64_t n_det, const double* boxes, const int32_t* det_frame, int32_t n_frames, const double* P,
                  const int32_t* img_wh, double iou_min, double* iou, int32_t* match, double* occ, void* stream) {
    if (!ctx) return DQO_EINVAL;
    if (n_obj < 0 || n_obj > 65535 || n_det < 0 || n_frames < 0) return fail(ctx, DQO_EINVAL, "bad sizes");
    if ((int64_t)n_obj * n_det > (int64_t(1) << 31) || n_det > (int64_t(1) << 15))
        return fail(ctx, DQO_EINVAL, "n_obj * n_det must be < 2^31 and n_det <= 32768");
    if (n_det > 0 && (!boxes || !det_frame || !match || n_frames < 1 || !P || !img_wh))
        return fail(ctx, DQO_EINVAL, "boxes, det_frame, P, img_wh and match are required");
    if (n_obj > 0 && n_det > 0 && (!mu || !R || !axes || !iou))
        return fail(ctx, DQO_EINVAL, "object quadrics and iou are required");
    if (!isfinite(iou_min)) return fail(ctx, DQO_EINVAL, "iou_min must be finite");
    return run(ctx, "associate", [&] {
        return launch_associate(n_obj, mu, R, axes, n_det, boxes, det_frame, n_frames, P, img_wh, iou_min, iou, match,
                                occ, (hipStream_t)stream);
    });
}

int dqo_quadric_distance(const dqo_ctx* ctx, int32_t na, const double* mu_a, const double* R_a, const double* axes_a,
                         int32_t nb, const double* mu_b, const double* R_b, const double* axes_b, double tau,
                         double* qd, void* stream) {
    if (!ctx) return DQO_EINVAL;
    if (na < 0 || nb < 0 || (int64_t)na * nb > (int64_t(1) << 31)) return fail(ctx, DQO_EINVAL, "bad sizes");
    if ((int64_t)na * nb > 0 && (!mu_a || !R_a || !axes_a || !mu_b || !R_b || !axes_b || !qd))
        return fail(ctx, DQO_EINVAL, "quadric buffers and qd must not be NULL");
    if (!(tau >= 0) || !isfinite(tau)) return fail(ctx, DQO_EINVAL, "tau must be finite and >= 0");
    return run(ctx, "quadric_distance", [&] {
        return launch_quadric_distance(na, mu_a, R_a, axes_a, nb, mu_b, R_b, axes_b, tau, qd, (hipStream_t)stream);
    });
}

int dqo_associate_decide(const dqo_ctx* ctx, int64_t n_det, int32_t n_obj, const int32_t* match, const double* qd_obs,
                         const double* occ, const double* qd_det, const int32_t* label, double qd_min, double t_occ,
                         double qd_occ, int32_t* fine, int32_t* parent, int32_t* root, int32_t* obj, void* stream) {
    if (!ctx) return DQO_EINVAL;
    if (n_det < 0 || n_obj < 0 || n_det > (int64_t(1) << 15)) return fail(ctx, DQO_EINVAL, "bad sizes (n_det <= 32768)");
    if ((int64_t)n_obj * n_det > (int64_t(1) << 31)) return fail(ctx, DQO_EINVAL, "n_obj * n_det must be < 2^31");
    if (!isfinite(qd_min) || !isfinite(t_occ) || !isfinite(qd_occ)) return fail(ctx, DQO_EINVAL, "thresholds must be finite");
    if (n_det > 0 && (!match || !occ || !qd_det || !label || !fine || !parent || !root || !obj))
        return fail(ctx, DQO_EINVAL, "match, occ, qd_det, label and the four outputs are required");
    if (n_det > 0 && n_obj > 0 && !qd_obs) return fail(ctx, DQO_EINVAL, "qd_obs is required when n_obj > 0");
    return run(ctx, "associate_decide", [&] {
        return launch_associate_decide(n_det, n_obj, match, qd_obs, occ, qd_det, label, qd_min, t_occ, qd_occ, fine,
                                       parent, root, obj, (hipStream_t)stream);
    });
}

}  // extern "C"
