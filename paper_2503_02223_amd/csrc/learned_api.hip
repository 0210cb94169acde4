// Host side of the learned-initialization C ABI: the parameter layout,
// argument validation (before any launch) and the launch sequences.
#include <math.h>
#include <string.h>

#include "ctx.hpp"
#include "dqo_device.hpp"
#include "dqo_learned.h"
#include "net.hpp"

namespace dqo {
namespace net {

void layout(dqo_net_layout* L) {
    static const int cin[4] = {5, 32, 64, 64}, cout[4] = {32, 64, 64, 6};
    static const int cinp[4] = {16, 32, 64, 64}, coutp[4] = {32, 64, 64, 16};
    memset(L, 0, sizeof(*L));
    int64_t off = 0, wk = 0;
    for (int l = 0; l < DQO_NET_LAYERS; ++l) {
        L->cin[l] = cin[l];
        L->cout[l] = cout[l];
        L->cin_pad[l] = cinp[l];
        L->cout_pad[l] = coutp[l];
        L->w_offset[l] = off;
        off += (int64_t)coutp[l] * 9 * cinp[l];
        L->b_offset[l] = off;
        off += coutp[l];
        L->wk_offset[l] = wk;
        wk += (int64_t)coutp[l] * 9 * cinp[l];
    }
    L->n_params = off;
    L->w_elems = wk;
}

}  // namespace net
}  // namespace dqo

using namespace dqo;

namespace {

int check_crops(const dqo_ctx* ctx, int B, int H, int W) {
    if (!ctx) return DQO_EINVAL;
    if (B < 1 || H < 16 || W < 16 || H > 4096 || W > 4096 || H % 16 || W % 16)
        return fail(ctx, DQO_EINVAL, "crop batch %d x %d x %d invalid (H, W multiples of 16 in [16, 4096])", B, H,
                    W);
    if ((int64_t)B * H * W > (int64_t(1) << 28)) return fail(ctx, DQO_EINVAL, "B * H * W must be <= 2^28");
    return DQO_OK;
}

int done(const dqo_ctx* ctx, hipError_t e, const char* where) { return e == hipSuccess ? DQO_OK : hip_fail(ctx, e, where); }

int make_cams(const dqo_ctx* ctx, int B, const dqo_camera* cams, net::InitCams* out) {
    if (!cams) return fail(ctx, DQO_EINVAL, "cams must not be NULL");
    if (B > DQO_MAX_VIEWS) return fail(ctx, DQO_EINVAL, "at most %d crops per initialization call", DQO_MAX_VIEWS);
    memset(out, 0, sizeof(*out));
    for (int b = 0; b < B; ++b) {
        const dqo_camera& c = cams[b];
        bool fin = isfinite(c.fx) && isfinite(c.fy) && isfinite(c.cx) && isfinite(c.cy) && c.fx > 0 && c.fy > 0;
        for (int k = 0; k < 9; ++k) fin = fin && isfinite(c.R[k]);
        for (int k = 0; k < 3; ++k) fin = fin && isfinite(c.t[k]);
        if (!fin) return fail(ctx, DQO_EINVAL, "camera %d invalid", b);
        for (int k = 0; k < 9; ++k) out->R[b][k] = (float)c.R[k];
        for (int k = 0; k < 3; ++k) out->t[b][k] = (float)c.t[k];
        out->fx[b] = (float)c.fx;
        out->fy[b] = (float)c.fy;
        out->cx[b] = (float)c.cx;
        out->cy[b] = (float)c.cy;
    }
    return DQO_OK;
}

}  // namespace

extern "C" {

int dqo_net_layout_get(dqo_net_layout* out) {
    if (!out) return DQO_EINVAL;
    net::layout(out);
    return DQO_OK;
}

int dqo_net_workspace_size(int32_t B, int32_t H, int32_t W, int64_t* bytes) {
    if (!bytes || B < 1 || H < 16 || W < 16 || H % 16 || W % 16 || H > 4096 || W > 4096) return DQO_EINVAL;
    *bytes = net::carve(nullptr, B, H, W, nullptr);
    return DQO_OK;
}

int dqo_net_pack(const dqo_ctx* ctx, const float* theta, uint16_t* wf, uint16_t* wt, void* stream) {
    if (!ctx) return DQO_EINVAL;
    if (!theta || !wf || !wt) return fail(ctx, DQO_EINVAL, "theta, wf and wt must not be NULL");
    dqo_net_layout L;
    net::layout(&L);
    return done(ctx, net::launch_pack(L, theta, wf, wt, (hipStream_t)stream), "dqo_net_pack");
}

int dqo_net_forward(const dqo_ctx* ctx, int32_t B, int32_t H, int32_t W, const float* rgbdm, const uint16_t* wf,
                    const float* theta, void* workspace, float* out, void* stream) {
    int rc = check_crops(ctx, B, H, W);
    if (rc) return rc;
    if (!rgbdm || !wf || !theta || !workspace || !out)
        return fail(ctx, DQO_EINVAL, "rgbdm, wf, theta, workspace and out must not be NULL");
    dqo_net_layout L;
    net::layout(&L);
    net::Work w;
    net::carve(workspace, B, H, W, &w);
    return done(ctx, net::launch_forward(L, w, B, H, W, rgbdm, wf, theta, out, (hipStream_t)stream),
                "dqo_net_forward");
}

int dqo_net_loss(const dqo_ctx* ctx, int32_t B, int32_t H, int32_t W, const float* rgbdm, const float* out,
                 const float* labels, const double* chan_w, double* loss, void* workspace, void* stream) {
    int rc = check_crops(ctx, B, H, W);
    if (rc) return rc;
    if (!rgbdm || !out || !labels || !chan_w || !loss || !workspace)
        return fail(ctx, DQO_EINVAL, "rgbdm, out, labels, chan_w, loss and workspace must not be NULL");
    for (int c = 0; c < 5; ++c)
        if (!(chan_w[c] >= 0.0) || !isfinite(chan_w[c])) return fail(ctx, DQO_EINVAL, "chan_w[%d] invalid", c);
    net::Work w;
    net::carve(workspace, B, H, W, &w);
    return done(ctx, net::launch_loss(w, B, H, W, rgbdm, out, labels, chan_w, loss, (hipStream_t)stream),
                "dqo_net_loss");
}

int dqo_net_backward(const dqo_ctx* ctx, int32_t B, int32_t H, int32_t W, const uint16_t* wt, void* workspace,
                     float* grad, void* stream) {
    int rc = check_crops(ctx, B, H, W);
    if (rc) return rc;
    if (!wt || !workspace || !grad) return fail(ctx, DQO_EINVAL, "wt, workspace and grad must not be NULL");
    dqo_net_layout L;
    net::layout(&L);
    net::Work w;
    net::carve(workspace, B, H, W, &w);
    return done(ctx, net::launch_backward(L, w, B, H, W, wt, grad, (hipStream_t)stream), "dqo_net_backward");
}

int dqo_adam_flat(const dqo_ctx* ctx, float* params, const float* grads, float* m, float* v, int64_t n, double lr,
                  double beta1, double beta2, double eps, int64_t* d_step, void* stream) {
    if (!ctx) return DQO_EINVAL;
    if (n < 0) return fail(ctx, DQO_EINVAL, "n < 0");
    if (!d_step || (n > 0 && (!params || !grads || !m || !v)))
        return fail(ctx, DQO_EINVAL, "params, grads, m, v and d_step must not be NULL");
    if (!(beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps >= 0 && isfinite(lr)))
        return fail(ctx, DQO_EINVAL, "Adam hyper-parameters invalid");
    dqo_adam hp;
    memset(&hp, 0, sizeof(hp));
    hp.lr[0] = lr;
    hp.beta1 = beta1;
    hp.beta2 = beta2;
    hp.eps = eps;
    return done(ctx, launch_adam<float>(params, grads, m, v, n, hp, 1, d_step, (hipStream_t)stream, 1),
                "dqo_adam_flat");
}

int dqo_init_gaussians(const dqo_ctx* ctx, int32_t B, int32_t H, int32_t W, const float* rgbdm,
                       const dqo_camera* cams, const int64_t* offsets, const float* pred, const int32_t* use_pred,
                       int64_t n, float* params, int32_t* ids, int32_t obj_id, void* stream) {
    int rc = check_crops(ctx, B, H, W);
    if (rc) return rc;
    if (!rgbdm || !offsets || n < 0 || (n > 0 && (!params || !ids)))
        return fail(ctx, DQO_EINVAL, "rgbdm, offsets, params and ids must be given and n >= 0");
    net::InitCams ic;
    rc = make_cams(ctx, B, cams, &ic);
    if (rc) return rc;
    return done(ctx, net::launch_init(B, H, W, rgbdm, ic, offsets, pred, use_pred, n, params, ids, obj_id,
                                      (hipStream_t)stream),
                "dqo_init_gaussians");
}

int dqo_init_labels(const dqo_ctx* ctx, int32_t B, int32_t H, int32_t W, const float* rgbdm,
                    const dqo_camera* cams, const int64_t* offsets, const float* params, int64_t n, float* labels,
                    void* stream) {
    int rc = check_crops(ctx, B, H, W);
    if (rc) return rc;
    if (!rgbdm || !offsets || !labels || n < 0 || (n > 0 && !params))
        return fail(ctx, DQO_EINVAL, "rgbdm, offsets, params and labels must be given and n >= 0");
    net::InitCams ic;
    rc = make_cams(ctx, B, cams, &ic);
    if (rc) return rc;
    return done(ctx, net::launch_labels(B, H, W, rgbdm, ic, offsets, params, n, labels, (hipStream_t)stream),
                "dqo_init_labels");
}

int dqo_net_fallback(const dqo_ctx* ctx, int32_t B, int32_t H, int32_t W, const float* rgbdm, const float* out,
                     double threshold, int32_t* use_pred, float* mean_logerr, void* stream) {
    int rc = check_crops(ctx, B, H, W);
    if (rc) return rc;
    if (!rgbdm || !out || !use_pred) return fail(ctx, DQO_EINVAL, "rgbdm, out and use_pred must not be NULL");
    return done(ctx, net::launch_fallback(B, H, W, rgbdm, out, (float)threshold, use_pred, mean_logerr,
                                          (hipStream_t)stream),
                "dqo_net_fallback");
}

int dqo_masked_psnr(const dqo_ctx* ctx, int32_t V, int32_t H, int32_t W, const float* color, const float* rgbdm,
                    double* psnr, void* stream) {
    if (!ctx) return DQO_EINVAL;
    if (V < 1 || H < 1 || W < 1) return fail(ctx, DQO_EINVAL, "sizes must be positive");
    if (!color || !rgbdm || !psnr) return fail(ctx, DQO_EINVAL, "color, rgbdm and psnr must not be NULL");
    return done(ctx, net::launch_psnr(V, H, W, color, rgbdm, psnr, (hipStream_t)stream), "dqo_masked_psnr");
}

}  // extern "C"
