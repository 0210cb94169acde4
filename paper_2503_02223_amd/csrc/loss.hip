// Object loss of Eq. (10)-(14) read as L1 colour + L1 depth (valid target
// depth only) + object cross-entropy on the rendered instance probability, with
// a fixed-order (bitwise reproducible) reduction in double precision, and the
// upstream gradients it feeds into the render backward.
#include "dqo_device.hpp"

namespace dqo {

constexpr int kLossThreads = 256;

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_down(v, d);
    return v;
}

template <typename T>
__global__ __launch_bounds__(kLossThreads) void loss_partial_kernel(const T* __restrict__ C, const T* __restrict__ D,
                                                                    const T* __restrict__ pt, const T* __restrict__ tC,
                                                                    const T* __restrict__ tD, int64_t HW, int V,
                                                                    double eps, Ctrl* ctrl) {
    __shared__ double s_part[kLossThreads / kWave][4];
    const int64_t npix = HW * V;
    double s_rgb = 0, s_d = 0, s_nv = 0, s_obj = 0;
    for (int64_t i = (int64_t)blockIdx.x * kLossThreads + threadIdx.x; i < npix;
         i += (int64_t)gridDim.x * kLossThreads) {
        const int64_t v = i / HW, p = i - v * HW;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t k = (v * 3 + c) * HW + p;
            s_rgb += fabs((double)C[k] - (double)tC[k]);
        }
        const double td = (double)tD[i];
        if (td > 0) {
            s_d += fabs((double)D[i] - td);
            s_nv += 1.0;
        }
        s_obj += -log(fmax((double)pt[i], eps));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    s_rgb = wave_sum_d(s_rgb);
    s_d = wave_sum_d(s_d);
    s_nv = wave_sum_d(s_nv);
    s_obj = wave_sum_d(s_obj);
    if (lane == 0) {
        s_part[wave][0] = s_rgb;
        s_part[wave][1] = s_d;
        s_part[wave][2] = s_nv;
        s_part[wave][3] = s_obj;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double a = 0;
        for (int w = 0; w < kLossThreads / kWave; ++w) a += s_part[w][threadIdx.x];
        ctrl->loss_partials[blockIdx.x][threadIdx.x] = a;
    }
}

// Totals of the per-block partials: wave c sums component c, lane l taking
// blocks l, l + 64, ... in order, then a fixed shuffle tree combines the
// lanes (deterministic for a given block count).  Every thread of the block
// must call it; the totals land in s_tot.
__device__ __forceinline__ void loss_totals(const Ctrl* ctrl, int nblocks, double* s_tot) {
    const int lane = threadIdx.x & 63, c = threadIdx.x >> 6;
    double a = 0;
    for (int b = lane; b < nblocks; b += 64) a += ctrl->loss_partials[b][c];
    a = wave_sum_d(a);
    if (lane == 0) s_tot[c] = a;
    __syncthreads();
}

__device__ __forceinline__ void write_loss(const double* tot, int64_t npix, double w_rgb, double w_d, double lam,
                                           double* loss, Ctrl* ctrl) {
    const double nv = tot[2];
    const double l_rgb = npix ? tot[0] / (3.0 * (double)npix) : 0.0;
    const double l_d = nv > 0 ? tot[1] / nv : 0.0;
    const double l_obj = npix ? tot[3] / (double)npix : 0.0;
    loss[0] = w_rgb * l_rgb + w_d * l_d + lam * l_obj;
    loss[1] = l_rgb;
    loss[2] = l_d;
    loss[3] = l_obj;
    ctrl->n_valid = (uint32_t)nv;
}

// The loss alone (no gradients requested).
__global__ __launch_bounds__(kLossThreads) void loss_final_kernel(Ctrl* ctrl, int nblocks, int64_t npix,
                                                                  double w_rgb, double w_d, double lam,
                                                                  double* loss) {
    __shared__ double s_tot[4];
    loss_totals(ctrl, nblocks, s_tot);
    if (threadIdx.x == 0) write_loss(s_tot, npix, w_rgb, w_d, lam, loss, ctrl);
}

template <typename T>
__device__ __forceinline__ T sgn(T x) { return (x > T(0)) ? T(1) : ((x < T(0)) ? T(-1) : T(0)); }

template <typename T>
__global__ __launch_bounds__(kLossThreads) void loss_grad_kernel(const T* __restrict__ C, const T* __restrict__ D,
                                                                 const T* __restrict__ pt, const T* __restrict__ tC,
                                                                 const T* __restrict__ tD, int64_t HW, int V,
                                                                 double w_rgb, double w_d, double lam, double eps,
                                                                 Ctrl* __restrict__ ctrl, int nblocks,
                                                                 double* __restrict__ loss, T* __restrict__ gC,
                                                                 T* __restrict__ gD, T* __restrict__ gP) {
    // Every block forms the totals itself (the valid-depth count scales the
    // depth gradient); block 0 also writes the loss.
    __shared__ double s_tot[4];
    loss_totals(ctrl, nblocks, s_tot);
    const int64_t npix = HW * V;
    if (blockIdx.x == 0 && threadIdx.x == 0) write_loss(s_tot, npix, w_rgb, w_d, lam, loss, ctrl);
    const int64_t i = (int64_t)blockIdx.x * kLossThreads + threadIdx.x;
    if (i >= npix) return;
    const T crgb = (T)(w_rgb / (3.0 * (double)npix));
    const uint32_t nv = (uint32_t)s_tot[2];
    const T cd = nv ? (T)(w_d / (double)nv) : T(0);
    const T cobj = (T)(-lam / (double)npix);
    const int64_t v = i / HW, p = i - v * HW;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t k = (v * 3 + c) * HW + p;
        gC[k] = crgb * sgn<T>(C[k] - tC[k]);
    }
    const T td = tD[i];
    gD[i] = (td > T(0)) ? cd * sgn<T>(D[i] - td) : T(0);
    const T q = pt[i];
    gP[i] = ((double)q >= eps) ? cobj / q : T(0);
}

template <typename T>
hipError_t launch_object_loss(const Frame<T>& f, const dqo_images& img, const dqo_targets& tgt,
                              const dqo_loss_weights& w, double* loss, const dqo_image_grads& g, hipStream_t st) {
    const int64_t HW = (int64_t)f.views.W * f.views.H;
    const int V = f.views.n_views;
    const int64_t npix = HW * V;
    int blocks = (int)((npix + kLossThreads - 1) / kLossThreads);
    if (blocks > kLossBlocks - 1) blocks = kLossBlocks - 1;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(loss_partial_kernel<T>, dim3(blocks), dim3(kLossThreads), 0, st, (const T*)img.color,
                       (const T*)img.depth, (const T*)img.p_target, (const T*)tgt.color, (const T*)tgt.depth, HW, V,
                       w.ce_eps, f.s.ctrl);
    if (npix > 0 && g.d_color) {
        hipLaunchKernelGGL(loss_grad_kernel<T>, dim3((unsigned)((npix + kLossThreads - 1) / kLossThreads)),
                           dim3(kLossThreads), 0, st, (const T*)img.color, (const T*)img.depth,
                           (const T*)img.p_target, (const T*)tgt.color, (const T*)tgt.depth, HW, V, w.w_rgb,
                           w.w_depth, w.lambda, w.ce_eps, f.s.ctrl, blocks, loss, (T*)g.d_color, (T*)g.d_depth,
                           (T*)g.d_p_target);
    } else {
        hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(kLossThreads), 0, st, f.s.ctrl, blocks, npix, w.w_rgb,
                           w.w_depth, w.lambda, loss);
    }
    return hipGetLastError();
}

template hipError_t launch_object_loss<float>(const Frame<float>&, const dqo_images&, const dqo_targets&,
                                              const dqo_loss_weights&, double*, const dqo_image_grads&,
                                              hipStream_t);
template hipError_t launch_object_loss<double>(const Frame<double>&, const dqo_images&, const dqo_targets&,
                                               const dqo_loss_weights&, double*, const dqo_image_grads&,
                                               hipStream_t);

}  // namespace dqo
