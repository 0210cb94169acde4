// Adam update shared by the optimizer kernels and the fused project-backward
// + Adam kernel, so that both perform the same arithmetic.  The update
// follows PyTorch's order of operations:
// m <- m + (1 - b1)(g - m); v <- b2 v + (1 - b2) g^2;
// p <- p - (lr / bc1) * m / (sqrt(v) / sqrt(bc2) + eps).
#pragma once
#include <math.h>

#include "dqo_device.hpp"

namespace dqo {

template <typename T>
struct AdamArgs {
    double lr[kParams];
    double beta1, beta2;
    T b1c, b2, b2c, eps;
    T step_size[kParams];  // lr / bc1 per row (host step)
    T inv_sqrt_bc2;        // (host step)
};

template <typename T>
inline AdamArgs<T> make_adam_args(const dqo_adam& hp, int64_t step) {
    AdamArgs<T> a;
    for (int r = 0; r < kParams; ++r) a.lr[r] = hp.lr[r];
    a.beta1 = hp.beta1;
    a.beta2 = hp.beta2;
    a.b1c = (T)(1.0 - hp.beta1);
    a.b2 = (T)hp.beta2;
    a.b2c = (T)(1.0 - hp.beta2);
    a.eps = (T)hp.eps;
    const double bc1 = 1.0 - pow(hp.beta1, (double)(step > 0 ? step : 1));
    const double bc2 = 1.0 - pow(hp.beta2, (double)(step > 0 ? step : 1));
    for (int r = 0; r < kParams; ++r) a.step_size[r] = (T)(hp.lr[r] / bc1);
    a.inv_sqrt_bc2 = (T)(1.0 / sqrt(bc2));
    return a;
}

// No multiply-add contraction: every kernel that inlines the update then
// rounds it the same way.
template <typename T>
__device__ __forceinline__ void adam_one(T& p, T g, T& m, T& v, T ss, T isb, const AdamArgs<T>& a) {
#pragma clang fp contract(off)
    m = m + a.b1c * (g - m);
    v = v * a.b2 + a.b2c * g * g;
    const T denom = sqrt(v) * isb + a.eps;
    p = p - ss * (m / denom);
}

// Step sizes of every row and 1/sqrt(bc2) for step t = prev + 1 (device step
// counter), computed by one thread.  Rows are indexed with constants only: a
// kernel argument array indexed at run time is copied to per-thread scratch
// by every thread (216 bytes each, measured to nearly triple the Adam time).
template <typename T>
__device__ __forceinline__ void device_step_table(const AdamArgs<T>& a, int64_t prev, T* ss, T* isb) {
    const double t = (double)(prev + 1);
    const double bc1 = 1.0 - pow(a.beta1, t);
    const double bc2 = 1.0 - pow(a.beta2, t);
#pragma unroll
    for (int r = 0; r < kParams; ++r) ss[r] = (T)(a.lr[r] / bc1);
    *isb = (T)(1.0 / sqrt(bc2));
}

}  // namespace dqo
