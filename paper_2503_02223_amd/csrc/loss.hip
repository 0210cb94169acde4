// Object loss of Eq. (10)-(14) read as L1 colour + L1 depth (valid target
// depth only) + object cross-entropy on the rendered instance probability, with
// a fixed-order (bitwise reproducible) reduction in double precision, and the
// upstream gradients it feeds into the render backward.
#include <type_traits>

#include "dqo_device.hpp"

namespace dqo {

constexpr int kLossThreads = 256;

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_down(v, d);
    return v;
}

// Which pixels each term counts (whole images and whole-scene views unless
// the frame gives windows or per-object jobs).
struct LossViews {
    int32_t win[DQO_MAX_VIEWS][4];  // x0, y0, x1, y1
    int32_t job[DQO_MAX_VIEWS];     // -1 whole scene, else the job's object
    int32_t W;
};

// Pixel i (view v, pixel p): in the view's window (every term) and a colour
// pixel (colour and depth terms: a whole-scene view, or the job's object).
__device__ __forceinline__ void loss_masks(const LossViews& lv, const int32_t* __restrict__ tid, int64_t i,
                                           int64_t v, int64_t p, bool& in_win, bool& colour) {
    const int u = (int)(p % lv.W), y = (int)(p / lv.W);
    in_win = u >= lv.win[v][0] && u < lv.win[v][2] && y >= lv.win[v][1] && y < lv.win[v][3];
    const int job = lv.job[v];
    colour = in_win && (job < 0 || (tid && tid[i] == job));
}

// Per-workgroup partial sums, kLossParts per workgroup: colour residuals,
// depth residuals, depth pixels, cross-entropy, colour pixels, window pixels.
// MASKED: the frame has pixel windows or per-object jobs; without them every
// pixel counts for every term and the pixel counts are known on the host.
template <typename T, bool MASKED>
__global__ __launch_bounds__(kLossThreads) void loss_partial_kernel(const T* __restrict__ C, const T* __restrict__ D,
                                                                    const T* __restrict__ pt, const T* __restrict__ tC,
                                                                    const T* __restrict__ tD,
                                                                    const int32_t* __restrict__ tid, LossViews lv,
                                                                    int64_t HW, int V, double eps,
                                                                    double* __restrict__ partials) {
    __shared__ double s_part[kLossThreads / kWave][kLossParts];
    const int64_t npix = HW * V;
    double acc[kLossParts] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * kLossThreads + threadIdx.x; i < npix;
         i += (int64_t)gridDim.x * kLossThreads) {
        const int64_t v = i / HW, p = i - v * HW;
        bool in_win = true, colour = true;
        if constexpr (MASKED) loss_masks(lv, tid, i, v, p, in_win, colour);
        if (colour) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int64_t k = (v * 3 + c) * HW + p;
                acc[0] += fabs((double)C[k] - (double)tC[k]);
            }
            if constexpr (MASKED) acc[4] += 1.0;
            const double td = (double)tD[i];
            if (td > 0) {
                acc[1] += fabs((double)D[i] - td);
                acc[2] += 1.0;
            }
        }
        if (in_win) {
            acc[3] += -log(fmax((double)pt[i], eps));
            if constexpr (MASKED) acc[5] += 1.0;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int kParts = MASKED ? 6 : 4;
#pragma unroll
    for (int c = 0; c < kParts; ++c) {
        acc[c] = wave_sum_d(acc[c]);
        if (lane == 0) s_part[wave][c] = acc[c];
    }
    __syncthreads();
    if (threadIdx.x < kParts) {
        double a = 0;
        for (int w = 0; w < kLossThreads / kWave; ++w) a += s_part[w][threadIdx.x];
        partials[kLossParts * blockIdx.x + threadIdx.x] = a;
    }
}

// Totals of the per-block partials: wave c (of 4) sums components c and
// c + 4, lane l taking blocks l, l + 64, ... in order, then a fixed shuffle
// tree combines the lanes (deterministic for a given block count).  Every
// thread of the block must call it; the totals land in s_tot.
// npix >= 0: an unmasked frame, whose colour and window pixel counts are npix.
__device__ __forceinline__ void loss_totals(const double* partials, int nblocks, double npix, double* s_tot) {
    const int lane = threadIdx.x & 63, c = threadIdx.x >> 6;
    const int halves = npix >= 0 ? 1 : 2;
    for (int h = 0; h < halves; ++h) {
        double a = 0;
        for (int b = lane; b < nblocks; b += 64) a += partials[kLossParts * b + c + 4 * h];
        a = wave_sum_d(a);
        if (lane == 0) s_tot[c + 4 * h] = a;
    }
    if (npix >= 0 && threadIdx.x < 2) s_tot[4 + threadIdx.x] = npix;
    __syncthreads();
}

__device__ __forceinline__ void write_loss(const double* tot, double w_rgb, double w_d, double lam, double* loss,
                                           uint32_t* n_valid) {
    const double nv = tot[2], nc = tot[4], no = tot[5];
    const double l_rgb = nc > 0 ? tot[0] / (3.0 * nc) : 0.0;
    const double l_d = nv > 0 ? tot[1] / nv : 0.0;
    const double l_obj = no > 0 ? tot[3] / no : 0.0;
    loss[0] = w_rgb * l_rgb + w_d * l_d + lam * l_obj;
    loss[1] = l_rgb;
    loss[2] = l_d;
    loss[3] = l_obj;
    *n_valid = (uint32_t)nv;
}

// The loss alone (no gradients requested).
__global__ __launch_bounds__(kLossThreads) void loss_final_kernel(const double* __restrict__ partials, int nblocks,
                                                                  double npix, double w_rgb, double w_d, double lam,
                                                                  double* loss, uint32_t* n_valid) {
    __shared__ double s_tot[kLossParts];
    loss_totals(partials, nblocks, npix, s_tot);
    if (threadIdx.x == 0) write_loss(s_tot, w_rgb, w_d, lam, loss, n_valid);
}

template <typename T>
__device__ __forceinline__ T sgn(T x) { return (x > T(0)) ? T(1) : ((x < T(0)) ? T(-1) : T(0)); }

template <typename T, bool MASKED>
__global__ __launch_bounds__(kLossThreads) void loss_grad_kernel(const T* __restrict__ C, const T* __restrict__ D,
                                                                 const T* __restrict__ pt, const T* __restrict__ tC,
                                                                 const T* __restrict__ tD,
                                                                 const int32_t* __restrict__ tid, LossViews lv,
                                                                 int64_t HW, int V, double w_rgb, double w_d,
                                                                 double lam, double eps,
                                                                 const double* __restrict__ partials, int nblocks,
                                                                 uint32_t* __restrict__ n_valid,
                                                                 double* __restrict__ loss, T* __restrict__ gC,
                                                                 T* __restrict__ gD, T* __restrict__ gP) {
    // Every block forms the totals itself (the pixel counts scale the
    // gradients); block 0 also writes the loss.
    __shared__ double s_tot[kLossParts];
    loss_totals(partials, nblocks, MASKED ? -1.0 : (double)(HW * V), s_tot);
    const int64_t npix = HW * V;
    if (blockIdx.x == 0 && threadIdx.x == 0) write_loss(s_tot, w_rgb, w_d, lam, loss, n_valid);
    const int64_t i = (int64_t)blockIdx.x * kLossThreads + threadIdx.x;
    if (i >= npix) return;
    const double nc = s_tot[4], nv = s_tot[2], no = s_tot[5];
    const T crgb = nc > 0 ? (T)(w_rgb / (3.0 * nc)) : T(0);
    const T cd = nv > 0 ? (T)(w_d / nv) : T(0);
    const T cobj = no > 0 ? (T)(-lam / no) : T(0);
    const int64_t v = i / HW, p = i - v * HW;
    bool in_win = true, colour = true;
    if constexpr (MASKED) loss_masks(lv, tid, i, v, p, in_win, colour);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t k = (v * 3 + c) * HW + p;
        gC[k] = colour ? crgb * sgn<T>(C[k] - tC[k]) : T(0);
    }
    const T td = tD[i];
    gD[i] = (colour && td > T(0)) ? cd * sgn<T>(D[i] - td) : T(0);
    const T q = pt[i];
    gP[i] = (in_win && (double)q >= eps) ? cobj / q : T(0);
}

int loss_partial_blocks(int64_t npix) {
    int64_t blocks = (npix + kLossThreads - 1) / kLossThreads;
    if (blocks > kLossBlocks - 1) blocks = kLossBlocks - 1;
    if (blocks < 1) blocks = 1;
    return (int)blocks;
}

template <typename T>
hipError_t launch_object_loss(int64_t HW, int V, const dqo_images& img, const dqo_targets& tgt,
                              const dqo_loss_weights& w, double* loss, const dqo_image_grads& g,
                              const LossViewsHost& views, double* partials, uint32_t* n_valid, hipStream_t st) {
    LossViews lv;
    for (int v = 0; v < DQO_MAX_VIEWS; ++v) {
        for (int k = 0; k < 4; ++k) lv.win[v][k] = views.win[v][k];
        lv.job[v] = views.job[v];
    }
    lv.W = views.W;
    const int64_t npix = HW * V;
    const int blocks = loss_partial_blocks(npix);
    bool masked = false;
    for (int v = 0; v < V; ++v)
        masked = masked || lv.job[v] >= 0 || lv.win[v][0] != 0 || lv.win[v][1] != 0 ||
                 (int64_t)lv.win[v][2] * lv.win[v][3] != HW || lv.win[v][2] != views.W;
    const unsigned gblocks = (unsigned)((npix + kLossThreads - 1) / kLossThreads);
    auto launch = [&](auto masked_tag) {
        constexpr bool MK = decltype(masked_tag)::value;
        hipLaunchKernelGGL((loss_partial_kernel<T, MK>), dim3(blocks), dim3(kLossThreads), 0, st, (const T*)img.color,
                           (const T*)img.depth, (const T*)img.p_target, (const T*)tgt.color, (const T*)tgt.depth,
                           tgt.id, lv, HW, V, w.ce_eps, partials);
        if (npix > 0 && g.d_color) {
            hipLaunchKernelGGL((loss_grad_kernel<T, MK>), dim3(gblocks), dim3(kLossThreads), 0, st,
                               (const T*)img.color, (const T*)img.depth, (const T*)img.p_target, (const T*)tgt.color,
                               (const T*)tgt.depth, tgt.id, lv, HW, V, w.w_rgb, w.w_depth, w.lambda, w.ce_eps,
                               (const double*)partials, blocks, n_valid, loss, (T*)g.d_color, (T*)g.d_depth,
                               (T*)g.d_p_target);
        } else {
            hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(kLossThreads), 0, st, (const double*)partials, blocks,
                               MK ? -1.0 : (double)npix, w.w_rgb, w.w_depth, w.lambda, loss, n_valid);
        }
    };
    if (masked)
        launch(std::true_type{});
    else
        launch(std::false_type{});
    return hipGetLastError();
}

template hipError_t launch_object_loss<float>(int64_t, int, const dqo_images&, const dqo_targets&,
                                              const dqo_loss_weights&, double*, const dqo_image_grads&,
                                              const LossViewsHost&, double*, uint32_t*, hipStream_t);
template hipError_t launch_object_loss<double>(int64_t, int, const dqo_images&, const dqo_targets&,
                                               const dqo_loss_weights&, double*, const dqo_image_grads&,
                                               const LossViewsHost&, double*, uint32_t*, hipStream_t);

}  // namespace dqo
