// Gaussians spawned from RGB-D crops, one per valid pixel in raster order
// (plain back-projection, optionally corrected by the network's per-pixel
// prediction), and the training labels read back from converged Gaussians.
// One workgroup per crop: each thread takes a contiguous run of pixels, and a
// workgroup scan of the valid counts gives every valid pixel its column.
#include "dqo_device.hpp"
#include "net.hpp"

namespace dqo {
namespace net {

constexpr int kInitThreads = 1024;

__device__ __forceinline__ bool valid_at(const float* c, int HW, int i) {
    return c[4 * HW + i] > 0.5f && c[3 * HW + i] > 0.0f;
}

// Exclusive scan of one value per thread over the workgroup (kInitThreads).
__device__ int block_exclusive_scan(int v, int* s) {
    const int tid = threadIdx.x;
    s[tid] = v;
    __syncthreads();
    for (int k = 1; k < kInitThreads; k <<= 1) {
        const int add = tid >= k ? s[tid - k] : 0;
        __syncthreads();
        s[tid] += add;
        __syncthreads();
    }
    const int incl = s[tid];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kInitThreads) void init_kernel(int H, int W, const float* __restrict__ rgbdm,
                                                            InitCams cams, const int64_t* __restrict__ offsets,
                                                            const float* __restrict__ pred,
                                                            const int32_t* __restrict__ use_pred, int64_t n,
                                                            float* __restrict__ params, int32_t* __restrict__ ids,
                                                            int32_t obj_id) {
    __shared__ int s_scan[kInitThreads];
    const int b = blockIdx.x, HW = H * W;
    const float* c = rgbdm + (size_t)b * 5 * HW;
    const int chunk = (HW + kInitThreads - 1) / kInitThreads;
    const int i0 = min(HW, (int)threadIdx.x * chunk), i1 = min(HW, i0 + chunk);
    int cnt = 0;
    for (int i = i0; i < i1; ++i) cnt += valid_at(c, HW, i) ? 1 : 0;
    int rank = block_exclusive_scan(cnt, s_scan);
    const int64_t first = offsets[b], last = min(offsets[b + 1], n);
    const bool corr = pred != nullptr && (use_pred == nullptr || use_pred[b] != 0);
    const float fx = cams.fx[b], fy = cams.fy[b], cx = cams.cx[b], cy = cams.cy[b];
    const float* R = cams.R[b];
    const float* t = cams.t[b];
    for (int i = i0; i < i1; ++i) {
        if (!valid_at(c, HW, i)) continue;
        const int64_t col = first + rank++;
        if (col < 0 || col >= last) continue;
        const int v = i / W, u = i - v * W;
        const float d = c[3 * HW + i];
        const float xc[3] = {d * ((float)u + 0.5f - cx) / fx - t[0], d * ((float)v + 0.5f - cy) / fy - t[1],
                             d - t[2]};
        float ls = logf(d / fx), eta = logf(9.0f);
        float rgb[3] = {c[i], c[HW + i], c[2 * HW + i]};
        if (corr) {
            const float* pp = pred + (size_t)b * 6 * HW + i;
            ls += pp[0];
            eta = pp[HW];
            rgb[0] += pp[2 * HW];
            rgb[1] += pp[3 * HW];
            rgb[2] += pp[4 * HW];
        }
        float vals[kParams];
        // world mean = R^T (x_c - t)
        vals[0] = R[0] * xc[0] + R[3] * xc[1] + R[6] * xc[2];
        vals[1] = R[1] * xc[0] + R[4] * xc[1] + R[7] * xc[2];
        vals[2] = R[2] * xc[0] + R[5] * xc[1] + R[8] * xc[2];
        vals[3] = vals[4] = vals[5] = ls;
        vals[6] = 1.0f;
        vals[7] = vals[8] = vals[9] = 0.0f;
        vals[10] = eta;
        vals[11] = rgb[0];
        vals[12] = rgb[1];
        vals[13] = rgb[2];
#pragma unroll
        for (int r = 0; r < kParams; ++r) params[(int64_t)r * n + col] = vals[r];
        ids[col] = obj_id;
    }
}

__global__ __launch_bounds__(kInitThreads) void labels_kernel(int H, int W, const float* __restrict__ rgbdm,
                                                              InitCams cams, const int64_t* __restrict__ offsets,
                                                              const float* __restrict__ params, int64_t n,
                                                              float* __restrict__ labels) {
    __shared__ int s_scan[kInitThreads];
    const int b = blockIdx.x, HW = H * W;
    const float* c = rgbdm + (size_t)b * 5 * HW;
    float* lab = labels + (size_t)b * 5 * HW;
    const int chunk = (HW + kInitThreads - 1) / kInitThreads;
    const int i0 = min(HW, (int)threadIdx.x * chunk), i1 = min(HW, i0 + chunk);
    int cnt = 0;
    for (int i = i0; i < i1; ++i) cnt += valid_at(c, HW, i) ? 1 : 0;
    int rank = block_exclusive_scan(cnt, s_scan);
    const int64_t first = offsets[b], last = min(offsets[b + 1], n);
    const float fx = cams.fx[b];
    for (int i = i0; i < i1; ++i) {
        float l[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        if (valid_at(c, HW, i)) {
            const int64_t col = first + rank++;
            if (col >= 0 && col < last) {
                const float d = c[3 * HW + i];
                l[0] = (params[3 * n + col] + params[4 * n + col] + params[5 * n + col]) / 3.0f - logf(d / fx);
                l[1] = params[10 * n + col];
                l[2] = params[11 * n + col] - c[i];
                l[3] = params[12 * n + col] - c[HW + i];
                l[4] = params[13 * n + col] - c[2 * HW + i];
            }
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) lab[k * HW + i] = l[k];
    }
}

hipError_t launch_init(int B, int H, int W, const float* rgbdm, const InitCams& cams, const int64_t* offsets,
                       const float* pred, const int32_t* use_pred, int64_t n, float* params, int32_t* ids,
                       int32_t obj_id, hipStream_t st) {
    hipLaunchKernelGGL(init_kernel, dim3(B), dim3(kInitThreads), 0, st, H, W, rgbdm, cams, offsets, pred, use_pred,
                       n, params, ids, obj_id);
    return hipGetLastError();
}

hipError_t launch_labels(int B, int H, int W, const float* rgbdm, const InitCams& cams, const int64_t* offsets,
                         const float* params, int64_t n, float* labels, hipStream_t st) {
    hipLaunchKernelGGL(labels_kernel, dim3(B), dim3(kInitThreads), 0, st, H, W, rgbdm, cams, offsets, params, n,
                       labels);
    return hipGetLastError();
}

}  // namespace net
}  // namespace dqo
