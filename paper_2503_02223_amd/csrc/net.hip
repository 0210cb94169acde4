// The learned-initialization network on the matrix cores: 3x3 convolutions as
// implicit GEMMs with BF16 operands and FP32 accumulation
// (v_mfma_f32_16x16x32_bf16, or 16x16x16 when a layer has 16 input
// channels), plus the input packing, training loss, weight packing, the
// per-crop fallback decision and a masked PSNR.
//
// Activations are NHWC BF16 with the channel count padded to a multiple of
// 16.  A convolution workgroup (4 waves) owns a 16 x 16 pixel tile of one
// image for every output channel: the 18 x 18 input halo and the layer's
// weights [cout][9][cin] are staged in LDS (16-byte padded rows), and wave w
// computes tile rows 4w..4w+3 (four M-blocks of 16 pixels) against all
// output-channel N-blocks, the K loop running over the 9 taps x cin.
// Weight gradients are GEMMs over pixels: one workgroup per (pixel split,
// tap column) accumulates the three taps' dW_tap[cout][cin] over its tiles
// from transposed LDS copies of the activation window and the output
// gradient (transposed in registers, 8x8 blocks of 16-bit values); a second
// kernel sums the splits in a fixed order.
#include "dqo_device.hpp"
#include "dqo_learned.h"
#include "net.hpp"

namespace dqo {
namespace net {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float x) {  // round to nearest even
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bool valid_px(const float* rgbdm, int64_t plane, int64_t base) {
    return rgbdm[base + 4 * plane] > 0.5f && rgbdm[base + 3 * plane] > 0.0f;
}

constexpr int kT = 16;       // output tile edge (pixels)
constexpr int kHalo = kT + 2;

enum { kEpiRelu = 0, kEpiGate = 1, kEpiOut = 2 };

template <int CIN, int COUT, int EPI>
__global__ __launch_bounds__(256) void conv3x3_kernel(int H, int W, const uint16_t* __restrict__ in,
                                                      const uint16_t* __restrict__ wk, const float* __restrict__ bias,
                                                      const uint16_t* __restrict__ gate, uint16_t* __restrict__ out_bf,
                                                      float* __restrict__ out_f, int nout) {
    constexpr int PIX = CIN + 8;       // LDS elements per halo pixel (16-byte pad)
    constexpr int WROW = 9 * CIN + 8;  // LDS elements per output channel of weights
    constexpr int KS = (CIN % 32 == 0) ? 32 : 16;
    constexpr int NT = COUT / 16;
    static_assert(CIN % 16 == 0 && COUT % 16 == 0, "channels must be multiples of 16");
    __shared__ __attribute__((aligned(16))) uint16_t s_in[kHalo * kHalo * PIX];
    __shared__ __attribute__((aligned(16))) uint16_t s_w[COUT * WROW];
    const int tiles_x = W / kT, tiles_y = H / kT;
    const int img = blockIdx.x / (tiles_x * tiles_y);
    const int t = blockIdx.x - img * tiles_x * tiles_y;
    const int ty0 = (t / tiles_x) * kT, tx0 = (t % tiles_x) * kT;
    const int tid = threadIdx.x;
    constexpr int WCH = 9 * CIN / 8;
    for (int c = tid; c < COUT * WCH; c += 256) {
        const int co = c / WCH, k8 = c - co * WCH;
        *reinterpret_cast<uint4*>(s_w + co * WROW + k8 * 8) =
            *reinterpret_cast<const uint4*>(wk + (size_t)co * 9 * CIN + k8 * 8);
    }
    constexpr int CCH = CIN / 8;
    for (int c = tid; c < kHalo * kHalo * CCH; c += 256) {
        const int pix = c / CCH, c8 = c - pix * CCH;
        const int hy = pix / kHalo, hx = pix - hy * kHalo;
        const int y = ty0 + hy - 1, x = tx0 + hx - 1;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (y >= 0 && y < H && x >= 0 && x < W)
            v = *reinterpret_cast<const uint4*>(in + (((size_t)img * H + y) * W + x) * CIN + c8 * 8);
        *reinterpret_cast<uint4*>(s_in + pix * PIX + c8 * 8) = v;
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    floatx4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3, dx = tap - 3 * dy;
#pragma unroll
        for (int kc = 0; kc < CIN; kc += KS) {
            if constexpr (KS == 32) {
                bf16x8_t a[4], b[NT];
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    a[m] = *reinterpret_cast<const bf16x8_t*>(s_in + ((wave * 4 + m + dy) * kHalo + lr + dx) * PIX +
                                                              kc + 8 * lg);
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    b[n] = *reinterpret_cast<const bf16x8_t*>(s_w + (n * 16 + lr) * WROW + tap * CIN + kc + 8 * lg);
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int n = 0; n < NT; ++n)
                        acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b[n], acc[m][n], 0, 0, 0);
            } else {
                short4_t a[4], b[NT];
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    a[m] = *reinterpret_cast<const short4_t*>(s_in + ((wave * 4 + m + dy) * kHalo + lr + dx) * PIX +
                                                              kc + 4 * lg);
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    b[n] = *reinterpret_cast<const short4_t*>(s_w + (n * 16 + lr) * WROW + tap * CIN + kc + 4 * lg);
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int n = 0; n < NT; ++n)
                        acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[m], b[n], acc[m][n], 0, 0, 0);
            }
        }
    }
    // acc[m][n][r] = output at pixel (row 4 wave + m, column 4 lg + r), channel 16 n + lr
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int y = ty0 + wave * 4 + m;
        const int x0 = tx0 + 4 * lg;
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int co = n * 16 + lr;
            if constexpr (EPI == kEpiOut) {
                if (co < nout) {
                    const float b0 = bias[co];
                    float4 v = make_float4(acc[m][n][0] + b0, acc[m][n][1] + b0, acc[m][n][2] + b0, acc[m][n][3] + b0);
                    *reinterpret_cast<float4*>(out_f + (((size_t)img * nout + co) * H + y) * W + x0) = v;
                }
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const size_t o = (((size_t)img * H + y) * W + x0 + r) * COUT + co;
                    float v;
                    if constexpr (EPI == kEpiRelu) {
                        v = fmaxf(acc[m][n][r] + bias[co], 0.0f);
                    } else {
                        v = bf2f(gate[o]) > 0.0f ? acc[m][n][r] : 0.0f;
                    }
                    out_bf[o] = f2bf(v);
                }
            }
        }
    }
}

// Stages C channels of ROWS x 16 pixels (row-major; image rows y0..,
// columns x0..x0+15) into LDS transposed, channel-major rows of KP elements,
// from NHWC BF16 (zero outside the image).  Each thread takes a block of 8
// consecutive pixels (half a row) x 8 channels: 8 16-byte loads, an 8x8
// transpose of the 16-bit values in registers (v_perm_b32), and 8 16-byte
// stores, one per channel.  Consecutive lanes take consecutive pixel groups,
// so 16 lanes' stores cover the 64 LDS banks once.
template <int C, int KP, int ROWS>
__device__ __forceinline__ void stage_transposed(uint16_t* __restrict__ s, const uint16_t* __restrict__ src, int img,
                                                 int H, int W, int y0, int x0, int tid) {
    constexpr int PG = ROWS * kT / 8;  // pixel groups
    constexpr int NB = PG * (C / 8);
    for (int b = tid; b < NB; b += 256) {
        const int pg = b % PG, cg = b / PG;
        const int px0 = pg * 8;
        const int y = y0 + px0 / kT, xb = x0 + px0 % kT;
        uint4 r[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int x = xb + k;
            r[k] = make_uint4(0u, 0u, 0u, 0u);
            if (y >= 0 && y < H && x >= 0 && x < W)
                r[k] = *reinterpret_cast<const uint4*>(src + (((size_t)img * H + y) * W + x) * C + cg * 8);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            // channel cg*8 + j: dword d of pixel k holds channels 2d (low half) and 2d+1
            const uint32_t sel = (j & 1) ? 0x07060302u : 0x05040100u;
            uint32_t o[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint4 lo = r[2 * e], hi = r[2 * e + 1];
                const uint32_t a = (j >> 1) == 0 ? lo.x : (j >> 1) == 1 ? lo.y : (j >> 1) == 2 ? lo.z : lo.w;
                const uint32_t c = (j >> 1) == 0 ? hi.x : (j >> 1) == 1 ? hi.y : (j >> 1) == 2 ? hi.z : hi.w;
                o[e] = __builtin_amdgcn_perm(c, a, sel);  // pixels 2e (low half) and 2e+1
            }
            *reinterpret_cast<uint4*>(s + (cg * 8 + j) * KP + px0) = make_uint4(o[0], o[1], o[2], o[3]);
        }
    }
}

// Partial weight gradients of the three taps (dy, dx), dy = -1, 0, 1, of one
// column dx = blockIdx.y - 1, over one pixel split:
// part[split][co][tap][ci] = sum over the split's pixels p of g[p][co] * act[p + (dy, dx)][ci],
// part_b[split][co] = sum_p g[p][co] (written by the centre-column workgroups).
// Per tile the output gradient is staged once and the activations once, as
// 18 rows (the tile's rows -1..16 shifted by dx), so a tap's operand is that
// copy offset by dy rows; a wave's A operand serves its three taps.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void conv3x3_wgrad_kernel(int H, int W, int n_tiles, int tiles_per_split,
                                                            const uint16_t* __restrict__ act,
                                                            const uint16_t* __restrict__ g, float* __restrict__ part,
                                                            float* __restrict__ part_b) {
    constexpr int KP = kT * kT + 8;        // LDS row of the output gradient (pixels of a tile) + 16-byte pad
    constexpr int KA = (kT + 2) * kT + 8;  // LDS row of the activations (18 x 16 pixels) + pad
    constexpr int MT = COUT / 16, NTL = CIN / 16, PAIRS = MT * NTL, PER_WAVE = (PAIRS + 3) / 4;
    __shared__ __attribute__((aligned(16))) uint16_t s_g[COUT * KP];
    __shared__ __attribute__((aligned(16))) uint16_t s_a[CIN * KA];
    const int split = blockIdx.x, dxi = blockIdx.y, dx = dxi - 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int tiles_x = W / kT, tiles_img = tiles_x * (H / kT);
    floatx4 acc[PER_WAVE][3];
#pragma unroll
    for (int i = 0; i < PER_WAVE; ++i)
#pragma unroll
        for (int d = 0; d < 3; ++d) acc[i][d] = floatx4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.0f;
    const int t_begin = split * tiles_per_split;
    const int t_end = min(n_tiles, t_begin + tiles_per_split);
    for (int t = t_begin; t < t_end; ++t) {
        const int img = t / tiles_img, tt = t - img * tiles_img;
        const int ty0 = (tt / tiles_x) * kT, tx0 = (tt % tiles_x) * kT;
        __syncthreads();
        stage_transposed<COUT, KP, kT>(s_g, g, img, H, W, ty0, tx0, tid);
        stage_transposed<CIN, KA, kT + 2>(s_a, act, img, H, W, ty0 - 1, tx0 + dx, tid);
        __syncthreads();
#pragma unroll 2
        for (int k0 = 0; k0 < kT * kT; k0 += 32) {
#pragma unroll
            for (int i = 0; i < PER_WAVE; ++i) {
                const int pr = wave + 4 * i;
                if (pr < PAIRS) {
                    const int mt = pr / NTL, nt = pr - mt * NTL;
                    const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(s_g + (mt * 16 + lr) * KP + k0 + 8 * lg);
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        // output pixel k reads activation row (k / 16) + d of the staged copy
                        const bf16x8_t b =
                            *reinterpret_cast<const bf16x8_t*>(s_a + (nt * 16 + lr) * KA + k0 + 8 * lg + d * kT);
                        acc[i][d] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][d], 0, 0, 0);
                    }
                }
            }
        }
        if (dxi == 1 && tid < COUT)
            for (int px = 0; px < kT * kT; ++px) bsum += bf2f(s_g[tid * KP + px]);
    }
    // acc[i][d][r] = dW[co = 16 mt + 4 lg + r][tap = 3 d + dxi][ci = 16 nt + lr]
#pragma unroll
    for (int i = 0; i < PER_WAVE; ++i) {
        const int pr = wave + 4 * i;
        if (pr < PAIRS) {
            const int mt = pr / NTL, nt = pr - mt * NTL;
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int co = mt * 16 + 4 * lg + r, ci = nt * 16 + lr;
                    part[((size_t)split * COUT + co) * 9 * CIN + (3 * d + dxi) * CIN + ci] = acc[i][d][r];
                }
        }
    }
    if (dxi == 1 && tid < COUT) part_b[split * COUT + tid] = bsum;
}

// Sums the splits' partial weight gradients: a workgroup takes 64 entries,
// its four waves a quarter of the splits each (split q, q + 4, ... in order),
// and the four partial sums are added in wave order (a fixed order: the
// result does not depend on timing).
__global__ __launch_bounds__(256) void wgrad_reduce_kernel(int S, int64_t E, int cout, const float* __restrict__ part,
                                                           const float* __restrict__ part_b, float* __restrict__ gw,
                                                           float* __restrict__ gb) {
    __shared__ float s_sum[4][64];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t e = (int64_t)blockIdx.x * 64 + lane;  // entries E.. are the biases
    const bool is_w = e < E, is_b = !is_w && e < E + cout;
    const float* src = is_w ? part + e : part_b + (e - E);
    const int64_t stride = is_w ? E : (int64_t)cout;
    float s = 0.0f;
    if (is_w || is_b)
        for (int k0 = q; k0 < S; k0 += 32) {
            // eight loads in flight, then added in split order
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = (k0 + 4 * j < S) ? src[(int64_t)(k0 + 4 * j) * stride] : 0.0f;
#pragma unroll
            for (int j = 0; j < 8; ++j) s += v[j];
        }
    s_sum[q][lane] = s;
    __syncthreads();
    if (q == 0 && (is_w || is_b)) {
        const float t = ((s_sum[0][lane] + s_sum[1][lane]) + s_sum[2][lane]) + s_sum[3][lane];
        if (is_w) gw[e] = t;
        else gb[e - E] = t;
    }
}

// Smallest valid depth of each crop (one workgroup per crop).
__global__ __launch_bounds__(256) void dmin_kernel(int HW, const float* __restrict__ rgbdm, float* __restrict__ dmin) {
    const int b = blockIdx.x;
    const float* base = rgbdm + (size_t)b * 5 * HW;
    float m = INFINITY;
    for (int i = threadIdx.x; i < HW; i += 256) {
        const float d = base[3 * HW + i];
        if (base[4 * HW + i] > 0.5f && d > 0.0f) m = fminf(m, d);
    }
    __shared__ float s[256];
    s[threadIdx.x] = m;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) s[threadIdx.x] = fminf(s[threadIdx.x], s[threadIdx.x + k]);
        __syncthreads();
    }
    if (threadIdx.x == 0) dmin[b] = s[0];
}

// NHWC16 BF16 input: r, g, b, 4 (d - d_min) / d_min (valid pixels), valid, zeros.
__global__ __launch_bounds__(256) void input_kernel(int64_t P, int HW, const float* __restrict__ rgbdm,
                                                    const float* __restrict__ dmin, uint16_t* __restrict__ x0) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const int64_t b = p / HW, i = p - b * HW;
    const int64_t base = b * 5 * HW + i;
    const bool ok = valid_px(rgbdm, HW, base);
    float rel = 0.0f;
    if (ok) {
        const float dm = dmin[b];
        rel = 4.0f * __fdiv_rn(rgbdm[base + 3 * HW] - dm, dm);
    }
    uint32_t w[8];
    w[0] = (uint32_t)f2bf(rgbdm[base]) | ((uint32_t)f2bf(rgbdm[base + HW]) << 16);
    w[1] = (uint32_t)f2bf(rgbdm[base + 2 * HW]) | ((uint32_t)f2bf(rel) << 16);
    w[2] = (uint32_t)f2bf(ok ? 1.0f : 0.0f);
#pragma unroll
    for (int k = 3; k < 8; ++k) w[k] = 0u;
    uint4* dst = reinterpret_cast<uint4*>(x0 + p * 16);
    dst[0] = make_uint4(w[0], w[1], w[2], w[3]);
    dst[1] = make_uint4(w[4], w[5], w[6], w[7]);
}

// theta -> BF16 forward copy (same order) and transposed copy [cin][9 - 1 - tap][cout].
__global__ __launch_bounds__(256) void pack_kernel(int cin, int cout, const float* __restrict__ w,
                                                   uint16_t* __restrict__ wf, uint16_t* __restrict__ wt) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= cout * 9 * cin) return;
    const int co = e / (9 * cin), r = e - co * 9 * cin, tap = r / cin, ci = r - tap * cin;
    const uint16_t h = f2bf(w[e]);
    wf[e] = h;
    wt[(ci * 9 + (8 - tap)) * cout + co] = h;
}

__global__ __launch_bounds__(256) void count_kernel(int64_t P, int HW, const float* __restrict__ rgbdm,
                                                    int32_t* __restrict__ cnt) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int c = 0;
    if (p < P) {
        const int64_t b = p / HW, i = p - b * HW;
        c = valid_px(rgbdm, HW, b * 5 * HW + i) ? 1 : 0;
    }
    __shared__ int s[256];
    s[threadIdx.x] = c;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) cnt[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void count_total_kernel(int nblk, const int32_t* __restrict__ cnt,
                                                          int64_t* __restrict__ total) {
    __shared__ int64_t s[256];
    int64_t c = 0;
    for (int i = threadIdx.x; i < nblk; i += 256) c += cnt[i];
    s[threadIdx.x] = c;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = s[0];
}

struct ChanW {
    float w[5];
};

// Per valid pixel: the loss terms and dL/dout (BF16, NHWC16, zero elsewhere).
__global__ __launch_bounds__(256) void loss_kernel(int64_t P, int HW, const float* __restrict__ rgbdm,
                                                   const float* __restrict__ out, const float* __restrict__ lab,
                                                   ChanW cw, const int64_t* __restrict__ total,
                                                   uint16_t* __restrict__ g4, double* __restrict__ part) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double l_all = 0.0, l_fit = 0.0;
    if (p < P) {
        const int64_t b = p / HW, i = p - b * HW;
        const bool ok = valid_px(rgbdm, HW, b * 5 * HW + i);
        uint32_t w[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
        if (ok) {
            const float inv_m = 1.0f / (float)max(*total, (int64_t)1);
            float e[5], s = 0.0f;
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                e[c] = out[(b * 6 + c) * HW + i] - lab[(b * 5 + c) * HW + i];
                s += cw.w[c] * e[c] * e[c];
            }
            const float r = logf(s + 1e-4f);
            const float d5 = out[(b * 6 + 5) * HW + i] - r;
            l_all = (double)s + (double)d5 * d5;
            l_fit = (double)s;
            uint16_t h[6];
#pragma unroll
            for (int c = 0; c < 5; ++c) h[c] = f2bf(2.0f * cw.w[c] * e[c] * inv_m);
            h[5] = f2bf(2.0f * d5 * inv_m);
            w[0] = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
            w[1] = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
            w[2] = (uint32_t)h[4] | ((uint32_t)h[5] << 16);
        }
        uint4* dst = reinterpret_cast<uint4*>(g4 + p * 16);
        dst[0] = make_uint4(w[0], w[1], w[2], w[3]);
        dst[1] = make_uint4(w[4], w[5], w[6], w[7]);
    }
    __shared__ double s0[256], s1[256];
    s0[threadIdx.x] = l_all;
    s1[threadIdx.x] = l_fit;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) {
            s0[threadIdx.x] += s0[threadIdx.x + k];
            s1[threadIdx.x] += s1[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0[0];
        part[2 * blockIdx.x + 1] = s1[0];
    }
}

__global__ __launch_bounds__(256) void loss_final_kernel(int nblk, const double* __restrict__ part,
                                                         const int64_t* __restrict__ total, double* __restrict__ loss) {
    __shared__ double s0[256], s1[256];
    double a = 0.0, f = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 256) {
        a += part[2 * i];
        f += part[2 * i + 1];
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = f;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) {
            s0[threadIdx.x] += s0[threadIdx.x + k];
            s1[threadIdx.x] += s1[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double m = (double)max(*total, (int64_t)1);
        loss[0] = s0[0] / m;
        loss[1] = s1[0] / m;
    }
}

// Mean predicted log-error over each crop's valid pixels and the decision.
__global__ __launch_bounds__(256) void fallback_kernel(int HW, const float* __restrict__ rgbdm,
                                                       const float* __restrict__ out, float thr,
                                                       int32_t* __restrict__ use_pred, float* __restrict__ mean_out) {
    const int b = blockIdx.x;
    float s = 0.0f;
    int c = 0;
    for (int i = threadIdx.x; i < HW; i += 256)
        if (valid_px(rgbdm, HW, (int64_t)b * 5 * HW + i)) {
            s += out[((int64_t)b * 6 + 5) * HW + i];
            ++c;
        }
    __shared__ float ss[256];
    __shared__ int sc[256];
    ss[threadIdx.x] = s;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) {
            ss[threadIdx.x] += ss[threadIdx.x + k];
            sc[threadIdx.x] += sc[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float mean = sc[0] > 0 ? ss[0] / (float)sc[0] : INFINITY;
        use_pred[b] = mean <= thr ? 1 : 0;
        if (mean_out) mean_out[b] = mean;
    }
}

__global__ __launch_bounds__(256) void psnr_kernel(int HW, const float* __restrict__ color,
                                                   const float* __restrict__ rgbdm, double* __restrict__ psnr) {
    const int v = blockIdx.x;
    double s = 0.0;
    int c = 0;
    for (int i = threadIdx.x; i < HW; i += 256) {
        const int64_t base = (int64_t)v * 5 * HW + i;
        if (valid_px(rgbdm, HW, base)) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double e = (double)color[((int64_t)v * 3 + k) * HW + i] - (double)rgbdm[base + k * HW];
                s += e * e;
            }
            ++c;
        }
    }
    __shared__ double ss[256];
    __shared__ int sc[256];
    ss[threadIdx.x] = s;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) {
            ss[threadIdx.x] += ss[threadIdx.x + k];
            sc[threadIdx.x] += sc[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) psnr[v] = sc[0] > 0 ? 10.0 * log10(3.0 * sc[0] / ss[0]) : 0.0;
}

// ------------------------------------------------------------------ launchers
template <int CIN, int COUT, int EPI>
static void conv(int B, int H, int W, const uint16_t* in, const uint16_t* wk, const float* bias, const uint16_t* gate,
                 uint16_t* out_bf, float* out_f, int nout, hipStream_t st) {
    const int blocks = B * (H / kT) * (W / kT);
    hipLaunchKernelGGL((conv3x3_kernel<CIN, COUT, EPI>), dim3(blocks), dim3(256), 0, st, H, W, in, wk, bias, gate,
                       out_bf, out_f, nout);
}

template <int CIN, int COUT>
static void wgrad(const Work& w, int B, int H, int W, const uint16_t* act, const uint16_t* g, float* gw, float* gb,
                  hipStream_t st) {
    const int n_tiles = B * (H / kT) * (W / kT);
    const int S = w.splits;
    const int per = (n_tiles + S - 1) / S;
    hipLaunchKernelGGL((conv3x3_wgrad_kernel<CIN, COUT>), dim3(S, 3), dim3(256), 0, st, H, W, n_tiles, per, act, g,
                       w.part, w.part_b);
    const int64_t E = (int64_t)COUT * 9 * CIN;
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((unsigned)((E + COUT + 63) / 64)), dim3(256), 0, st, S, E, COUT, w.part,
                       w.part_b, gw, gb);
}

hipError_t launch_pack(const dqo_net_layout& L, const float* theta, uint16_t* wf, uint16_t* wt, hipStream_t st) {
    for (int l = 0; l < DQO_NET_LAYERS; ++l) {
        const int ci = L.cin_pad[l], co = L.cout_pad[l];
        const int E = co * 9 * ci;
        hipLaunchKernelGGL(pack_kernel, dim3((E + 255) / 256), dim3(256), 0, st, ci, co, theta + L.w_offset[l],
                           wf + L.wk_offset[l], wt + L.wk_offset[l]);
    }
    return hipGetLastError();
}

hipError_t launch_forward(const dqo_net_layout& L, const Work& w, int B, int H, int W, const float* rgbdm,
                          const uint16_t* wf, const float* theta, float* out, hipStream_t st) {
    const int HW = H * W;
    const int64_t P = (int64_t)B * HW;
    const unsigned pb = (unsigned)((P + 255) / 256);
    hipLaunchKernelGGL(dmin_kernel, dim3(B), dim3(256), 0, st, HW, rgbdm, w.dmin);
    hipLaunchKernelGGL(input_kernel, dim3(pb), dim3(256), 0, st, P, HW, rgbdm, w.dmin, w.x0);
    conv<16, 32, kEpiRelu>(B, H, W, w.x0, wf + L.wk_offset[0], theta + L.b_offset[0], nullptr, w.a1, nullptr, 0, st);
    conv<32, 64, kEpiRelu>(B, H, W, w.a1, wf + L.wk_offset[1], theta + L.b_offset[1], nullptr, w.a2, nullptr, 0, st);
    conv<64, 64, kEpiRelu>(B, H, W, w.a2, wf + L.wk_offset[2], theta + L.b_offset[2], nullptr, w.a3, nullptr, 0, st);
    conv<64, 16, kEpiOut>(B, H, W, w.a3, wf + L.wk_offset[3], theta + L.b_offset[3], nullptr, nullptr, out,
                          DQO_NET_OUT, st);
    return hipGetLastError();
}

hipError_t launch_loss(const Work& w, int B, int H, int W, const float* rgbdm, const float* out, const float* labels,
                       const double* chan_w, double* loss, hipStream_t st) {
    const int HW = H * W;
    const int64_t P = (int64_t)B * HW;
    const int nblk = (int)((P + 255) / 256);
    ChanW cw;
    for (int c = 0; c < 5; ++c) cw.w[c] = (float)chan_w[c];
    hipLaunchKernelGGL(count_kernel, dim3(nblk), dim3(256), 0, st, P, HW, rgbdm, w.cnt);
    hipLaunchKernelGGL(count_total_kernel, dim3(1), dim3(256), 0, st, nblk, w.cnt, w.total);
    hipLaunchKernelGGL(loss_kernel, dim3(nblk), dim3(256), 0, st, P, HW, rgbdm, out, labels, cw, w.total, w.g4,
                       w.lpart);
    hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, st, nblk, w.lpart, w.total, loss);
    return hipGetLastError();
}

hipError_t launch_backward(const dqo_net_layout& L, const Work& w, int B, int H, int W, const uint16_t* wt,
                           float* grad, hipStream_t st) {
    wgrad<64, 16>(w, B, H, W, w.a3, w.g4, grad + L.w_offset[3], grad + L.b_offset[3], st);
    conv<16, 64, kEpiGate>(B, H, W, w.g4, wt + L.wk_offset[3], nullptr, w.a3, w.gA, nullptr, 0, st);
    wgrad<64, 64>(w, B, H, W, w.a2, w.gA, grad + L.w_offset[2], grad + L.b_offset[2], st);
    conv<64, 64, kEpiGate>(B, H, W, w.gA, wt + L.wk_offset[2], nullptr, w.a2, w.gB, nullptr, 0, st);
    wgrad<32, 64>(w, B, H, W, w.a1, w.gB, grad + L.w_offset[1], grad + L.b_offset[1], st);
    conv<64, 32, kEpiGate>(B, H, W, w.gB, wt + L.wk_offset[1], nullptr, w.a1, w.gA, nullptr, 0, st);
    wgrad<16, 32>(w, B, H, W, w.x0, w.gA, grad + L.w_offset[0], grad + L.b_offset[0], st);
    return hipGetLastError();
}

hipError_t launch_fallback(int B, int H, int W, const float* rgbdm, const float* out, float thr, int32_t* use_pred,
                           float* mean_out, hipStream_t st) {
    hipLaunchKernelGGL(fallback_kernel, dim3(B), dim3(256), 0, st, H * W, rgbdm, out, thr, use_pred, mean_out);
    return hipGetLastError();
}

hipError_t launch_psnr(int V, int H, int W, const float* color, const float* rgbdm, double* psnr, hipStream_t st) {
    hipLaunchKernelGGL(psnr_kernel, dim3(V), dim3(256), 0, st, H * W, color, rgbdm, psnr);
    return hipGetLastError();
}

}  // namespace net
}  // namespace dqo
