// Workspace of the learned-initialization network and its launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dqo_learned.h"

namespace dqo {
namespace net {

constexpr int kMaxSplits = 128;  // pixel splits of the weight-gradient GEMMs

// Views into the caller's workspace for a batch of B crops of H x W.
struct Work {
    int splits;
    uint16_t *x0, *a1, *a2, *a3;  // BF16 NHWC activations: 16, 32, 64, 64 channels
    uint16_t *g4, *gA, *gB;       // BF16 NHWC activation gradients: 16, 64, 64 channels
    float* part;                  // [splits][64 * 9 * 64] partial weight gradients
    float* part_b;                // [splits][64] partial bias gradients
    float* dmin;                  // [B] smallest valid depth per crop
    int32_t* cnt;                 // [pixel blocks] valid-pixel counts
    int64_t* total;               // valid pixels of the batch
    double* lpart;                // [pixel blocks][2] loss partial sums
};

inline int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// Carves the workspace (ws == nullptr: only computes the size).
inline int64_t carve(void* ws, int B, int H, int W, Work* w) {
    const int64_t P = (int64_t)B * H * W;
    const int64_t nblk = (P + 255) / 256;
    const int64_t n_tiles = (int64_t)B * (H / 16) * (W / 16);
    const int splits = (int)(n_tiles < kMaxSplits ? n_tiles : kMaxSplits);
    const int64_t sizes[] = {P * 16 * 2, P * 32 * 2, P * 64 * 2, P * 64 * 2, P * 16 * 2, P * 64 * 2, P * 64 * 2,
                             (int64_t)splits * 64 * 9 * 64 * 4, (int64_t)splits * 64 * 4, (int64_t)B * 4, nblk * 4,
                             8, nblk * 16};
    int64_t off[13], total = 0;
    for (int i = 0; i < 13; ++i) {
        off[i] = total;
        total = align256(total + sizes[i]);
    }
    if (ws && w) {
        char* b = (char*)ws;
        w->splits = splits;
        w->x0 = (uint16_t*)(b + off[0]);
        w->a1 = (uint16_t*)(b + off[1]);
        w->a2 = (uint16_t*)(b + off[2]);
        w->a3 = (uint16_t*)(b + off[3]);
        w->g4 = (uint16_t*)(b + off[4]);
        w->gA = (uint16_t*)(b + off[5]);
        w->gB = (uint16_t*)(b + off[6]);
        w->part = (float*)(b + off[7]);
        w->part_b = (float*)(b + off[8]);
        w->dmin = (float*)(b + off[9]);
        w->cnt = (int32_t*)(b + off[10]);
        w->total = (int64_t*)(b + off[11]);
        w->lpart = (double*)(b + off[12]);
    }
    return total;
}

void layout(dqo_net_layout* L);
hipError_t launch_pack(const dqo_net_layout& L, const float* theta, uint16_t* wf, uint16_t* wt, hipStream_t st);
hipError_t launch_forward(const dqo_net_layout& L, const Work& w, int B, int H, int W, const float* rgbdm,
                          const uint16_t* wf, const float* theta, float* out, hipStream_t st);
hipError_t launch_loss(const Work& w, int B, int H, int W, const float* rgbdm, const float* out, const float* labels,
                       const double* chan_w, double* loss, hipStream_t st);
hipError_t launch_backward(const dqo_net_layout& L, const Work& w, int B, int H, int W, const uint16_t* wt,
                           float* grad, hipStream_t st);
hipError_t launch_fallback(int B, int H, int W, const float* rgbdm, const float* out, float thr, int32_t* use_pred,
                           float* mean_out, hipStream_t st);
hipError_t launch_psnr(int V, int H, int W, const float* color, const float* rgbdm, double* psnr, hipStream_t st);

// Crop cameras for the initialization kernels (passed by value).
struct InitCams {
    float R[DQO_MAX_VIEWS][9];
    float t[DQO_MAX_VIEWS][3];
    float fx[DQO_MAX_VIEWS], fy[DQO_MAX_VIEWS], cx[DQO_MAX_VIEWS], cy[DQO_MAX_VIEWS];
};

hipError_t launch_init(int B, int H, int W, const float* rgbdm, const InitCams& cams, const int64_t* offsets,
                       const float* pred, const int32_t* use_pred, int64_t n, float* params, int32_t* ids,
                       int32_t obj_id, hipStream_t st);
hipError_t launch_labels(int B, int H, int W, const float* rgbdm, const InitCams& cams, const int64_t* offsets,
                         const float* params, int64_t n, float* labels, hipStream_t st);

}  // namespace net
}  // namespace dqo
