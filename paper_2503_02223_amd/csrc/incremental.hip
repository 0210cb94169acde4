// Incremental update (Eq. (7)-(8)): unstable-pixel masks per object from a
// loss-mode render, and new Gaussians back-projected at those pixels.
#include "dqo_device.hpp"

namespace dqo {

constexpr int kMaskThreads = 256;
constexpr int kDensThreads = 1024;

template <typename T>
struct IncCfg {
    T theta_alpha, theta_d, theta_c3;  // theta_c3 = 3 theta_c (the colour test compares the channel sum)
    T eta_og, eta_tg;                  // opacity logits of OG and TG Gaussians
};

// One thread per pixel; per-object counts aggregated in LDS, then added to
// the global counters (integer atomics: the totals are exact).
template <typename T>
__global__ __launch_bounds__(kMaskThreads) void masks_kernel(int64_t P, int64_t HW, int K, const T* __restrict__ C,
                                                             const T* __restrict__ D, const T* __restrict__ pt,
                                                             const T* __restrict__ tc, const T* __restrict__ td,
                                                             const int32_t* __restrict__ tid, IncCfg<T> cfg,
                                                             uint8_t* __restrict__ masks,
                                                             int32_t* __restrict__ counts) {
    __shared__ int32_t s_cnt[DQO_MAX_K * 2];
    for (int k = threadIdx.x; k < 2 * K; k += kMaskThreads) s_cnt[k] = 0;
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * kMaskThreads + threadIdx.x;
    if (p < P) {
        const int64_t v = p / HW, i = p - v * HW;
        const int t = tid[p];
        uint8_t m = 0;
        if (t >= 0 && t < K) {
            const T dobs = td[p];
            const bool geo = pt[p] < cfg.theta_alpha || (dobs > T(0) && fabs(D[p] - dobs) > cfg.theta_d);
            const T e = fabs(C[(v * 3 + 0) * HW + i] - tc[(v * 3 + 0) * HW + i]) +
                        fabs(C[(v * 3 + 1) * HW + i] - tc[(v * 3 + 1) * HW + i]) +
                        fabs(C[(v * 3 + 2) * HW + i] - tc[(v * 3 + 2) * HW + i]);
            const bool rgb = e > cfg.theta_c3;
            m = (uint8_t)((geo ? 1 : 0) | (rgb ? 2 : 0));
            if (geo) atomicAdd(&s_cnt[2 * t], 1);
            if (rgb) atomicAdd(&s_cnt[2 * t + 1], 1);
        }
        masks[p] = m;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 2 * K; k += kMaskThreads)
        if (s_cnt[k]) atomicAdd(&counts[k], s_cnt[k]);
}

__device__ __forceinline__ bool spawns(uint8_t m, float d) { return m != 0 && d > 0.0f; }
__device__ __forceinline__ bool spawns(uint8_t m, double d) { return m != 0 && d > 0.0; }

// Exclusive scan of one value per thread over the workgroup (kDensThreads).
__device__ int dens_block_scan(int v, int* s) {
    const int tid = threadIdx.x;
    s[tid] = v;
    __syncthreads();
    for (int k = 1; k < kDensThreads; k <<= 1) {
        const int add = tid >= k ? s[tid - k] : 0;
        __syncthreads();
        s[tid] += add;
        __syncthreads();
    }
    const int incl = s[tid];
    __syncthreads();
    return incl - v;
}

// Pass 1 (one workgroup per view): the number of Gaussians each view adds.
template <typename T>
__global__ __launch_bounds__(kDensThreads) void densify_count_kernel(int64_t HW, const uint8_t* __restrict__ masks,
                                                                     const T* __restrict__ td,
                                                                     int64_t* __restrict__ counts) {
    __shared__ int s[kDensThreads];
    const int v = blockIdx.x;
    int c = 0;
    for (int64_t i = threadIdx.x; i < HW; i += kDensThreads) c += spawns(masks[v * HW + i], td[v * HW + i]) ? 1 : 0;
    const int excl = dens_block_scan(c, s);
    if (threadIdx.x == kDensThreads - 1) counts[1 + v] = (int64_t)(excl + c);
}

// Pass 2 (one workgroup per view): each thread takes a contiguous run of
// pixels, a workgroup scan gives every spawning pixel its column.
template <typename T>
__global__ __launch_bounds__(kDensThreads) void densify_write_kernel(Views<T> V, int64_t HW, int W,
                                                                     const uint8_t* __restrict__ masks,
                                                                     const T* __restrict__ tc,
                                                                     const T* __restrict__ td,
                                                                     const int32_t* __restrict__ tid, IncCfg<T> cfg,
                                                                     int64_t n_old, int64_t n_cap, T* __restrict__ params,
                                                                     int32_t* __restrict__ ids, int64_t* __restrict__ counts) {
    __shared__ int s[kDensThreads];
    const int v = blockIdx.x;
    int64_t base = n_old;
    for (int u = 0; u < v; ++u) base += counts[1 + u];
    if (v == 0 && threadIdx.x == 0) {
        int64_t tot = 0;
        for (int u = 0; u < V.n_views; ++u) tot += counts[1 + u];
        counts[0] = tot;
    }
    const int64_t chunk = (HW + kDensThreads - 1) / kDensThreads;
    const int64_t i0 = min(HW, (int64_t)threadIdx.x * chunk), i1 = min(HW, i0 + chunk);
    int c = 0;
    for (int64_t i = i0; i < i1; ++i) c += spawns(masks[v * HW + i], td[v * HW + i]) ? 1 : 0;
    int rank = dens_block_scan(c, s);
    const DevCam<T>& cam = V.cam[v];
    for (int64_t i = i0; i < i1; ++i) {
        const uint8_t m = masks[v * HW + i];
        const T d = td[v * HW + i];
        if (!spawns(m, d)) continue;
        const int64_t col = base + rank++;
        if (col < n_old || col >= n_cap) continue;
        const int py = (int)(i / W), px = (int)(i - (int64_t)py * W);
        const T xc0 = d * ((T(px) + T(0.5) - cam.cx) / cam.fx) - cam.t[0];
        const T xc1 = d * ((T(py) + T(0.5) - cam.cy) / cam.fy) - cam.t[1];
        const T xc2 = d - cam.t[2];
        const T* R = cam.R;
        T vals[kParams];
        vals[0] = R[0] * xc0 + R[3] * xc1 + R[6] * xc2;  // R^T (x_c - t)
        vals[1] = R[1] * xc0 + R[4] * xc1 + R[7] * xc2;
        vals[2] = R[2] * xc0 + R[5] * xc1 + R[8] * xc2;
        vals[3] = vals[4] = vals[5] = log(d / cam.fx);
        vals[6] = T(1);
        vals[7] = vals[8] = vals[9] = T(0);
        vals[10] = (m & 1) ? cfg.eta_og : cfg.eta_tg;
        vals[11] = tc[(v * 3 + 0) * HW + i];
        vals[12] = tc[(v * 3 + 1) * HW + i];
        vals[13] = tc[(v * 3 + 2) * HW + i];
#pragma unroll
        for (int r = 0; r < kParams; ++r) params[(int64_t)r * n_cap + col] = vals[r];
        ids[col] = tid[v * HW + i];
    }
}

template <typename T>
IncCfg<T> inc_cfg(const dqo_increment_cfg& c) {
    IncCfg<T> g;
    g.theta_alpha = (T)c.theta_alpha;
    g.theta_d = (T)c.theta_d;
    g.theta_c3 = (T)(3.0 * c.theta_c);
    g.eta_og = (T)log(c.og_opacity / (1.0 - c.og_opacity));
    g.eta_tg = (T)log(c.tg_opacity / (1.0 - c.tg_opacity));
    return g;
}

template <typename T>
hipError_t launch_incremental_masks(const Frame<T>& f, const dqo_images& img, const dqo_targets& tgt,
                                    const dqo_increment_cfg& cfg, uint8_t* masks, int32_t* counts, hipStream_t st) {
    const int64_t HW = (int64_t)f.views.W * f.views.H, P = HW * f.views.n_views;
    hipError_t e = launch_zero_words((uint32_t*)counts, 2 * (int64_t)f.K, st);
    if (e != hipSuccess) return e;
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(masks_kernel<T>, dim3((unsigned)((P + kMaskThreads - 1) / kMaskThreads)), dim3(kMaskThreads),
                       0, st, P, HW, f.K, (const T*)img.color, (const T*)img.depth, (const T*)img.p_target,
                       (const T*)tgt.color, (const T*)tgt.depth, tgt.id, inc_cfg<T>(cfg), masks, counts);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_densify(const Frame<T>& f, const dqo_targets& tgt, const uint8_t* masks,
                          const dqo_increment_cfg& cfg, int64_t n_old, int64_t n_cap, T* params, int32_t* ids,
                          int64_t* counts, hipStream_t st) {
    const int64_t HW = (int64_t)f.views.W * f.views.H;
    const int V = f.views.n_views;
    hipLaunchKernelGGL(densify_count_kernel<T>, dim3(V), dim3(kDensThreads), 0, st, HW, masks, (const T*)tgt.depth,
                       counts);
    hipLaunchKernelGGL(densify_write_kernel<T>, dim3(V), dim3(kDensThreads), 0, st, f.views, HW, f.views.W, masks,
                       (const T*)tgt.color, (const T*)tgt.depth, tgt.id, inc_cfg<T>(cfg), n_old, n_cap, params,
                       ids, counts);
    return hipGetLastError();
}

template hipError_t launch_incremental_masks<float>(const Frame<float>&, const dqo_images&, const dqo_targets&,
                                                    const dqo_increment_cfg&, uint8_t*, int32_t*, hipStream_t);
template hipError_t launch_incremental_masks<double>(const Frame<double>&, const dqo_images&, const dqo_targets&,
                                                     const dqo_increment_cfg&, uint8_t*, int32_t*, hipStream_t);
template hipError_t launch_densify<float>(const Frame<float>&, const dqo_targets&, const uint8_t*,
                                          const dqo_increment_cfg&, int64_t, int64_t, float*, int32_t*, int64_t*,
                                          hipStream_t);
template hipError_t launch_densify<double>(const Frame<double>&, const dqo_targets&, const uint8_t*,
                                           const dqo_increment_cfg&, int64_t, int64_t, double*, int32_t*, int64_t*,
                                           hipStream_t);

}  // namespace dqo
