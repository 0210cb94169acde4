// Adam over the structure-of-arrays parameter block [rows][n] (rows = 14 for
// Gaussians, 1 for a flat vector) with one learning rate per row.  The update follows PyTorch's order of operations:
// m <- m + (1 - b1)(g - m); v <- b2 v + (1 - b2) g^2;
// p <- p - (lr / bc1) * m / (sqrt(v) / sqrt(bc2) + eps).
// The bias corrections come either from the host (step known at launch) or
// from a step counter in device memory (graph-capturable: the same launch
// replays every iteration).
#include "adam_common.hpp"

namespace dqo {

// One thread per column (four columns with float4 when the rows allow it),
// all rows of that column in an unrolled loop, so that every per-row value is
// read at a constant index.  The step sizes come from the host, or from the
// device step counter (computed once per workgroup into LDS).
template <typename T>
__device__ __forceinline__ void row_factors(const AdamArgs<T>& a, const int64_t* d_step, T* s_ss, T* s_isb) {
    if (!d_step) return;
    if (threadIdx.x == 0) device_step_table<T>(a, *d_step, s_ss, s_isb);
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(256) void adam_kernel(T* __restrict__ p, const T* __restrict__ g, T* __restrict__ m,
                                                   T* __restrict__ v, int64_t n, int rows, AdamArgs<T> a,
                                                   const int64_t* __restrict__ d_step) {
    __shared__ T s_ss[kParams];
    __shared__ T s_isb;
    row_factors(a, d_step, s_ss, &s_isb);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
#pragma unroll
        for (int r = 0; r < kParams; ++r) {
            if (r >= rows) break;
            const T ss = d_step ? s_ss[r] : a.step_size[r];
            const T isb = d_step ? s_isb : a.inv_sqrt_bc2;
            const int64_t k = (int64_t)r * n + i;
            T pp = p[k], mm = m[k], vv = v[k];
            adam_one(pp, g[k], mm, vv, ss, isb, a);
            p[k] = pp;
            m[k] = mm;
            v[k] = vv;
        }
    }
}

// float4 path when rows are 16-byte aligned (n % 4 == 0); n4 = n / 4.
__global__ __launch_bounds__(256) void adam_kernel_vec4(float4* __restrict__ p, const float4* __restrict__ g,
                                                        float4* __restrict__ m, float4* __restrict__ v, int64_t n4,
                                                        int rows, AdamArgs<float> a,
                                                        const int64_t* __restrict__ d_step) {
    __shared__ float s_ss[kParams];
    __shared__ float s_isb;
    row_factors(a, d_step, s_ss, &s_isb);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += (int64_t)gridDim.x * 256) {
#pragma unroll
        for (int r = 0; r < kParams; ++r) {
            if (r >= rows) break;
            const float ss = d_step ? s_ss[r] : a.step_size[r];
            const float isb = d_step ? s_isb : a.inv_sqrt_bc2;
            const int64_t k = (int64_t)r * n4 + i;
            float4 pp = p[k], mm = m[k], vv = v[k];
            const float4 gg = g[k];
            adam_one(pp.x, gg.x, mm.x, vv.x, ss, isb, a);
            adam_one(pp.y, gg.y, mm.y, vv.y, ss, isb, a);
            adam_one(pp.z, gg.z, mm.z, vv.z, ss, isb, a);
            adam_one(pp.w, gg.w, mm.w, vv.w, ss, isb, a);
            p[k] = pp;
            m[k] = mm;
            v[k] = vv;
        }
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
    if (rows < 1 || rows > kParams) return hipErrorInvalidValue;
    int gx = (int)((len + 255) / 256);
    if (gx > 8192) gx = 8192;
    bool done = false;
    if constexpr (sizeof(T) == 4) {
        if (vec) {
            hipLaunchKernelGGL(adam_kernel_vec4, dim3(gx), dim3(256), 0, st, (float4*)p, (const float4*)g,
                               (float4*)m, (float4*)v, len, rows, a, (const int64_t*)d_step);
            done = true;
        }
    }
    if (!done)
        hipLaunchKernelGGL(adam_kernel<T>, dim3(gx), dim3(256), 0, st, p, g, m, v, n, rows, a,
                           (const int64_t*)d_step);
    if (d_step) hipLaunchKernelGGL(step_increment_kernel, dim3(1), dim3(1), 0, st, d_step);
    return hipGetLastError();
}

template hipError_t launch_adam<float>(float*, const float*, float*, float*, int64_t, const dqo_adam&, int64_t,
                                       int64_t*, hipStream_t, int);
template hipError_t launch_adam<double>(double*, const double*, double*, double*, int64_t, const dqo_adam&, int64_t,
                                        int64_t*, hipStream_t, int);

}  // namespace dqo
