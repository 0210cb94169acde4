// Adam over the structure-of-arrays parameter block [rows][n] (rows = 14 for
// Gaussians, 1 for a flat vector) with one learning rate per row.  The update follows PyTorch's order of operations:
// m <- m + (1 - b1)(g - m); v <- b2 v + (1 - b2) g^2;
// p <- p - (lr / bc1) * m / (sqrt(v) / sqrt(bc2) + eps).
// The bias corrections come either from the host (step known at launch) or
// from a step counter in device memory (graph-capturable: the same launch
// replays every iteration).
#include "adam_common.hpp"

namespace dqo {

// Step size and 1/sqrt(bc2) of this row: from the host, or from the device
// step counter (computed once per workgroup).
template <typename T>
__device__ __forceinline__ void step_factors(const AdamArgs<T>& a, const int64_t* d_step, int row, T& ss, T& isb) {
    if (!d_step) {
        ss = a.step_size[row];
        isb = a.inv_sqrt_bc2;
        return;
    }
    __shared__ T s_f[2];
    if (threadIdx.x == 0) device_step_factors<T>(a, *d_step, row, s_f[0], s_f[1]);
    __syncthreads();
    ss = s_f[0];
    isb = s_f[1];
}

template <typename T>
__global__ __launch_bounds__(256) void adam_kernel(T* __restrict__ p, const T* __restrict__ g, T* __restrict__ m,
                                                   T* __restrict__ v, int64_t n, AdamArgs<T> a,
                                                   const int64_t* __restrict__ d_step) {
    const int row = blockIdx.y;
    T ss, isb;
    step_factors(a, d_step, row, ss, isb);
    const int64_t base = (int64_t)row * n;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        T pp = p[base + i], mm = m[base + i], vv = v[base + i];
        adam_one(pp, g[base + i], mm, vv, ss, isb, a);
        p[base + i] = pp;
        m[base + i] = mm;
        v[base + i] = vv;
    }
}

// float4 path when rows are 16-byte aligned (n % 4 == 0).
__global__ __launch_bounds__(256) void adam_kernel_vec4(float4* __restrict__ p, const float4* __restrict__ g,
                                                        float4* __restrict__ m, float4* __restrict__ v, int64_t n4,
                                                        AdamArgs<float> a, const int64_t* __restrict__ d_step) {
    const int row = blockIdx.y;
    float ss, isb;
    step_factors(a, d_step, row, ss, isb);
    const int64_t base = (int64_t)row * n4;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += (int64_t)gridDim.x * 256) {
        float4 pp = p[base + i], mm = m[base + i], vv = v[base + i];
        const float4 gg = g[base + i];
        adam_one(pp.x, gg.x, mm.x, vv.x, ss, isb, a);
        adam_one(pp.y, gg.y, mm.y, vv.y, ss, isb, a);
        adam_one(pp.z, gg.z, mm.z, vv.z, ss, isb, a);
        adam_one(pp.w, gg.w, mm.w, vv.w, ss, isb, a);
        p[base + i] = pp;
        m[base + i] = mm;
        v[base + i] = vv;
    }
}

__global__ void step_increment_kernel(int64_t* d_step) { *d_step += 1; }

template <typename T>
hipError_t launch_adam(T* p, const T* g, T* m, T* v, int64_t n, const dqo_adam& hp, int64_t step, int64_t* d_step,
                       hipStream_t st, int rows) {
    if (n == 0) {
        if (d_step) hipLaunchKernelGGL(step_increment_kernel, dim3(1), dim3(1), 0, st, d_step);
        return hipGetLastError();
    }
    const AdamArgs<T> a = make_adam_args<T>(hp, step);
    bool vec = sizeof(T) == 4 && (n % 4) == 0 && ((uintptr_t)p % 16) == 0 && ((uintptr_t)g % 16) == 0 &&
               ((uintptr_t)m % 16) == 0 && ((uintptr_t)v % 16) == 0;
    const int64_t len = vec ? n / 4 : n;
    int gx = (int)((len + 255) / 256);
    if (gx > 4096) gx = 4096;
    bool done = false;
    if constexpr (sizeof(T) == 4) {
        if (vec) {
            hipLaunchKernelGGL(adam_kernel_vec4, dim3(gx, rows), dim3(256), 0, st, (float4*)p, (const float4*)g,
                               (float4*)m, (float4*)v, len, a, (const int64_t*)d_step);
            done = true;
        }
    }
    if (!done)
        hipLaunchKernelGGL(adam_kernel<T>, dim3(gx, rows), dim3(256), 0, st, p, g, m, v, n, a,
                           (const int64_t*)d_step);
    if (d_step) hipLaunchKernelGGL(step_increment_kernel, dim3(1), dim3(1), 0, st, d_step);
    return hipGetLastError();
}

template hipError_t launch_adam<float>(float*, const float*, float*, float*, int64_t, const dqo_adam&, int64_t,
                                       int64_t*, hipStream_t, int);
template hipError_t launch_adam<double>(double*, const double*, double*, double*, int64_t, const dqo_adam&, int64_t,
                                        int64_t*, hipStream_t, int);

}  // namespace dqo
