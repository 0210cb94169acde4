// Projection, culling and binning of Gaussians into pixel tiles, and the chain
// rule back through the projection.
//
// Each (view, Gaussian) item is projected with the EWA splatting model the
// method inherits from 3D Gaussian Splatting: the 3D covariance
// R diag(s^2) R^T of the Gaussian (the quadric shape of Eq. (2)) is pushed
// through the perspective Jacobian, a 0.3 px^2 dilation is added, and its
// inverse (the conic) is stored with the 2D mean, opacity, depth and colour in
// one 12-word record so that the render kernels gather one record per pair.
//
// Binning is factorised: items are first sorted by depth (4 radix passes over
// the float bits of z), then each item's tile pairs are emitted in depth order
// by a scan over the sorted items; a later stable sort by tile id then yields
// the (tile, depth, index) order with far fewer bytes than sorting 64-bit
// (tile, depth) keys over all pairs.
#include "adam_common.hpp"
#include <algorithm>

#include "dqo_device.hpp"
#include "sort_common.hpp"

namespace dqo {

// Starts a frame: new look-back epoch, counters and the histogram copies in
// use cleared (workgroup c clears copy c of each).
__global__ __launch_bounds__(256) void prep_kernel(Ctrl* ctrl, int copies_depth, int copies_pair) {
    const int t = threadIdx.x, c = blockIdx.x;
    if (c == 0) {
        if (t == 0) ctrl->epoch = ctrl->epoch + 1u;
        if (t < kNumCounters) ctrl->counters[t] = 0u;
        if (t == 0) ctrl->num_pairs = 0u;
        if (t < 2 * kHistCopies) (&ctrl->dkey_range[0][0])[t] = 0u;
    }
    if (c < copies_depth)
        for (int p = 0; p < kMaxDepthPasses; ++p) ctrl->hist_depth[c][p][t] = 0u;
    if (c < copies_pair)
        for (int p = 0; p < kMaxPairPasses; ++p) ctrl->hist_pair[c][p][t] = 0u;
}

template <typename T>
__device__ __forceinline__ void store_splat(T* dst, const T (&w)[kSplatWords]) {
#pragma unroll
    for (int k = 0; k < kSplatWords; ++k) dst[k] = w[k];
}
template <>
__device__ __forceinline__ void store_splat<float>(float* dst, const float (&w)[kSplatWords]) {
    float4* d = reinterpret_cast<float4*>(dst);
    d[0] = make_float4(w[0], w[1], w[2], w[3]);
    d[1] = make_float4(w[4], w[5], w[6], w[7]);
    d[2] = make_float4(w[8], w[9], w[10], w[11]);
    d[3] = make_float4(w[12], w[13], w[14], w[15]);
}

template <typename T>
struct Proj {
    T x, y, z;        // camera-frame mean
    T R[9];           // rotation of the normalised quaternion
    T qn[4], qnorm;
    T s[3];           // scales
    T U[6];           // J W R diag(s) (2x3)
    T s00, s01, s11;  // 2D covariance incl. dilation
    T det;
    T A, B, C;        // conic
    T mx, my;
    T o;
    T ux, uy;  // x/z and y/z as used in the Jacobian (after the frustum limit)
    bool ux_clamped, uy_clamped;
    bool visible;
};

template <typename T>
__device__ __forceinline__ void project_item(const DevCam<T>& c, const Consts<T>& cs, const T (&p)[kParams],
                                             Proj<T>& r) {
    const T* W = c.R;
    r.x = W[0] * p[0] + W[1] * p[1] + W[2] * p[2] + c.t[0];
    r.y = W[3] * p[0] + W[4] * p[1] + W[5] * p[2] + c.t[1];
    r.z = W[6] * p[0] + W[7] * p[1] + W[8] * p[2] + c.t[2];
    r.o = T(1) / (T(1) + exp(-p[10]));
    r.qnorm = sqrt(p[6] * p[6] + p[7] * p[7] + p[8] * p[8] + p[9] * p[9]);
    const T inv = T(1) / r.qnorm;
    r.qn[0] = p[6] * inv; r.qn[1] = p[7] * inv; r.qn[2] = p[8] * inv; r.qn[3] = p[9] * inv;
    quat_rot(r.qn[0], r.qn[1], r.qn[2], r.qn[3], r.R);
    r.s[0] = exp(p[3]); r.s[1] = exp(p[4]); r.s[2] = exp(p[5]);
    r.visible = r.z > cs.z_near;
    if (!r.visible) return;
    const T iz = T(1) / r.z;
    // The Jacobian is evaluated at x/z, y/z limited to the frustum widened by 30%.
    const T ux = r.x * iz, uy = r.y * iz;
    r.ux = fmin(fmax(ux, -c.limx), c.limx);
    r.uy = fmin(fmax(uy, -c.limy), c.limy);
    r.ux_clamped = ux > c.limx || ux < -c.limx;
    r.uy_clamped = uy > c.limy || uy < -c.limy;
    const T j00 = c.fx * iz, j02 = -c.fx * r.ux * iz;
    const T j11 = c.fy * iz, j12 = -c.fy * r.uy * iz;
    T T2[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T2[k] = j00 * W[k] + j02 * W[6 + k];
        T2[3 + k] = j11 * W[3 + k] + j12 * W[6 + k];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            r.U[a * 3 + b] = (T2[a * 3 + 0] * r.R[0 + b] + T2[a * 3 + 1] * r.R[3 + b] + T2[a * 3 + 2] * r.R[6 + b]) * r.s[b];
    r.s00 = r.U[0] * r.U[0] + r.U[1] * r.U[1] + r.U[2] * r.U[2] + cs.dilation;
    r.s01 = r.U[0] * r.U[3] + r.U[1] * r.U[4] + r.U[2] * r.U[5];
    r.s11 = r.U[3] * r.U[3] + r.U[4] * r.U[4] + r.U[5] * r.U[5] + cs.dilation;
    r.det = r.s00 * r.s11 - r.s01 * r.s01;
    if (!(r.det > T(0))) { r.visible = false; return; }
    const T idet = T(1) / r.det;
    r.A = r.s11 * idet;
    r.B = -r.s01 * idet;
    r.C = r.s00 * idet;
    r.mx = c.fx * r.x * iz + c.cx;
    r.my = c.fy * r.y * iz + c.cy;
}

template <typename T>
__global__ __launch_bounds__(256) void project_kernel(Views<T> V, Consts<T> cs, int64_t n, int64_t M,
                                                      const T* __restrict__ params, const int32_t* __restrict__ ids,
                                                      T* __restrict__ splats, short4* __restrict__ rects,
                                                      uint32_t* __restrict__ counts, uint32_t* __restrict__ dkeys,
                                                      uint32_t* __restrict__ dvals, uint32_t* __restrict__ ranges,
                                                      int64_t range_words, int copies, Ctrl* ctrl,
                                                      uint32_t* __restrict__ pair_hist0, int copies_pair) {
    __shared__ uint32_t s_hist[kRadixBins];  // low byte of the depth keys
    __shared__ uint32_t s_krange[2];         // visible depth keys: max of ~key, max of key
    // Low-byte histogram of the pairs' tile ids (when the emission sorts by
    // that byte itself): a difference array over the 256 digits, one range
    // per rectangle row, and the count of whole 256-tile cycles.
    __shared__ uint32_t s_pd[kRadixBins + 1];
    __shared__ uint32_t s_pall;
    __shared__ uint32_t s_tmp[256 / kWave];
    const int tid = threadIdx.x;
    // Tile ranges start empty: the sort writes only the bounds of tiles that hold pairs.
    for (int64_t w = (int64_t)blockIdx.x * 256 + tid; w < range_words; w += (int64_t)gridDim.x * 256) ranges[w] = 0u;
    s_hist[tid] = 0u;
    s_pd[tid] = 0u;
    if (tid < 2) s_krange[tid] = 0u;
    if (tid == 0) {
        s_pd[kRadixBins] = 0u;
        s_pall = 0u;
    }
    __syncthreads();
    // kProjItems items per thread (coalesced per item step): fewer workgroups
    // flush histogram counts to the shared copies.
    uint32_t kmin_inv = 0u, kmax = 0u;  // visible depth keys: max of ~key, max of key
    for (int it = 0; it < kProjItems; ++it) {
        const int64_t i = ((int64_t)blockIdx.x * kProjItems + it) * 256 + tid;
        if (i < M) {
            const int v = (int)(i / n);
            const int64_t g = i - (int64_t)v * n;
            const bool in_seg = g >= V.cam[v].seg_lo && g < V.cam[v].seg_hi;
            T p[kParams];
            bool finite = true;
#pragma unroll
            for (int r = 0; r < kParams; ++r) {
                p[r] = in_seg ? params[(int64_t)r * n + g] : T(0);
                finite = finite && isfinite(p[r]);
            }
            if (!finite) atomicOr(&ctrl->status, (uint32_t)DQO_STATUS_NONFINITE);
            Proj<T> pr;
            pr.visible = false;
            if (finite && in_seg) project_item(V.cam[v], cs, p, pr);
            uint32_t cnt = 0;
            short4 rc = make_short4(0, 0, -1, -1);
            T w[kSplatWords];
#pragma unroll
            for (int k = 0; k < kSplatWords; ++k) w[k] = T(0);
            if (pr.visible) {
                const T ex = T(3) * sqrt(pr.s00), ey = T(3) * sqrt(pr.s11);
                T x0 = floor((pr.mx - ex) / T(V.tile_w)), x1 = floor((pr.mx + ex) / T(V.tile_w));
                T y0 = floor((pr.my - ey) / T(V.tile_h)), y1 = floor((pr.my + ey) / T(V.tile_h));
                // tiles of the view's window only (the whole image unless windowed)
                x0 = max(x0, T(V.cam[v].tile_x0));
                y0 = max(y0, T(V.cam[v].tile_y0));
                x1 = min(x1, T(V.cam[v].tile_x1));
                y1 = min(y1, T(V.cam[v].tile_y1));
                if (x0 <= x1 && y0 <= y1) {
                    rc = make_short4((short)x0, (short)y0, (short)x1, (short)y1);
                    cnt = (uint32_t)(rc.z - rc.x + 1) * (uint32_t)(rc.w - rc.y + 1);
                    if (pair_hist0) {
                        // row y holds tiles t0 + y * tiles_x + [0, tw): digits [a, a + tw mod 256) mod 256
                        const uint32_t tw = (uint32_t)(rc.z - rc.x + 1), rem = tw & (kRadixBins - 1);
                        const uint32_t t0 = (uint32_t)v * (uint32_t)V.tiles_per_view + (uint32_t)rc.x;
                        if (tw >> kRadixBits) atomicAdd(&s_pall, (tw >> kRadixBits) * (uint32_t)(rc.w - rc.y + 1));
                        if (rem)
                            for (int y = rc.y; y <= rc.w; ++y) {
                                const uint32_t a = (t0 + (uint32_t)y * (uint32_t)V.tiles_x) & (kRadixBins - 1);
                                const uint32_t b = a + rem;
                                atomicAdd(&s_pd[a], 1u);
                                if (b <= (uint32_t)kRadixBins) {
                                    atomicAdd(&s_pd[b], 0xFFFFFFFFu);
                                } else {
                                    atomicAdd(&s_pd[0], 1u);
                                    atomicAdd(&s_pd[b - kRadixBins], 0xFFFFFFFFu);
                                }
                            }
                    }
                }
                w[0] = pr.mx; w[1] = pr.my; w[2] = pr.A; w[3] = pr.B; w[4] = pr.C; w[5] = pr.o; w[6] = pr.z;
                w[7] = id_to_word<T>(ids[g]);
                w[8] = p[11]; w[9] = p[12]; w[10] = p[13];
                // the tile rectangle for the render backward's pair slots
                // (the first slot, kSpSlot, is written by the scan)
                w[kSpRect] = id_to_word<T>((int)((uint32_t)(uint16_t)rc.x | ((uint32_t)(uint16_t)rc.y << 16)));
                w[kSpRectW] = id_to_word<T>(rc.z - rc.x + 1);
            }
            store_splat<T>(splats + i * kSplatWords, w);
            rects[i] = rc;
            counts[i] = cnt;
            const uint32_t key = pr.visible ? __float_as_uint((float)pr.z) : 0xffffffffu;
            dkeys[i] = key;
            dvals[i] = (uint32_t)i;
            // the depth passes count their later digits themselves (relative to the smallest key)
            atomicAdd(&s_hist[key & 255u], 1u);
            if (pr.visible) {
                kmin_inv = max(kmin_inv, ~key);
                kmax = max(kmax, key);
            }
        }
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        kmin_inv = max(kmin_inv, (uint32_t)__shfl_xor(kmin_inv, d));
        kmax = max(kmax, (uint32_t)__shfl_xor(kmax, d));
    }
    if ((tid & (kWave - 1)) == 0) {
        atomicMax(&s_krange[0], kmin_inv);
        atomicMax(&s_krange[1], kmax);
    }
    __syncthreads();
    if (tid < 2 && s_krange[tid]) atomicMax(&ctrl->dkey_range[blockIdx.x % kHistCopies][tid], s_krange[tid]);
    {
        const uint32_t c = s_hist[tid];
        if (c) atomicAdd(&ctrl->hist_depth[blockIdx.x % copies][0][tid], c);
    }
    if (pair_hist0) {  // uniform
        const uint32_t d = s_pd[tid];
        const uint32_t c = block_exclusive_scan<256>(d, s_tmp) + d + s_pall;
        if (c) atomicAdd(&pair_hist0[(size_t)(blockIdx.x % copies_pair) * kMaxPairPasses * kRadixBins + tid], c);
    }
}

// Scan of the tile counts in depth order and emission of (tile, item) pairs.
// When the grid fits on the device at once, each block obtains its offset by
// decoupled look-back (blocks ordered by workgroup index).  Larger grids would
// wait on a chain as long as the grid, so they scan in two levels first: the
// pair count of every block, then one workgroup's scan of those counts; the
// emission then reads its block's offset and waits on nothing (eight
// keyframes, 9.6M items: 206 -> 211 training steps/s).
__global__ __launch_bounds__(kScanThreads) void scan_block_sums_kernel(const uint32_t* __restrict__ order,
                                                                      const uint32_t* __restrict__ counts, uint32_t M,
                                                                      uint32_t* __restrict__ sums) {
    __shared__ uint32_t s_tmp[kScanThreads / kWave];
    const int tid = threadIdx.x;
    const uint32_t base = blockIdx.x * (uint32_t)kScanTile;
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < kScanIpt; ++k) {
        const uint32_t q = base + tid * kScanIpt + k;
        if (q < M) v += counts[order ? min(order[q], M - 1) : q];
    }
    const uint32_t excl = block_exclusive_scan<kScanThreads>(v, s_tmp);
    if (tid == kScanThreads - 1) sums[blockIdx.x] = excl + v;
}

// Exclusive scan of the block counts in place (one workgroup), the pair total
// and the overflow flag.
__global__ __launch_bounds__(kScanThreads) void scan_block_base_kernel(uint32_t* __restrict__ sums, int nblocks,
                                                                      uint32_t cap, Ctrl* __restrict__ ctrl) {
    __shared__ uint32_t s_tmp[kScanThreads / kWave];
    __shared__ uint32_t s_carry;
    const int tid = threadIdx.x;
    if (tid == 0) s_carry = 0u;
    __syncthreads();
    for (int c0 = 0; c0 < nblocks; c0 += kScanThreads) {
        const int i = c0 + tid;
        const uint32_t v = i < nblocks ? sums[i] : 0u;
        const uint32_t excl = block_exclusive_scan<kScanThreads>(v, s_tmp);
        const uint32_t carry = s_carry;
        if (i < nblocks) sums[i] = carry + excl;
        __syncthreads();
        if (tid == kScanThreads - 1) s_carry = carry + excl + v;
        __syncthreads();
    }
    if (tid == 0) {
        const uint32_t total = s_carry;
        ctrl->num_pairs = total;
        if (total > cap) atomicOr(&ctrl->status, (uint32_t)DQO_STATUS_OVERFLOW);
    }
}

// FUSED: the emission also performs the first pass of the pair sort, by the
// low byte of the tile id: each pair goes straight to its place in the pass's
// stable digit order.  That place is the digit's global start (from the
// per-digit totals the projection counted) + the digit's pairs in earlier
// blocks (decoupled look-back per digit, a 257th channel carrying the pair
// count) + those of earlier wavefronts of the block (counted per wavefront
// from the tile rectangles, one difference-array range per rectangle row) +
// those earlier in the wavefront's own emission rounds (match ballots and a
// running count per digit).  Needs the whole grid on the device at once.
template <typename T, bool FUSED>
__global__ __launch_bounds__(kScanThreads) void scan_emit_kernel(
    const uint32_t* __restrict__ order, const uint32_t* __restrict__ counts, const short4* __restrict__ rects,
    uint32_t* __restrict__ offsets, T* __restrict__ splats, uint32_t* __restrict__ pkeys, uint32_t* __restrict__ pvals, uint32_t M,
    uint32_t cap, int64_t n, int tiles_x, int tiles_per_view, int pair_passes, int copies, uint64_t* lb, Ctrl* ctrl,
    const uint32_t* __restrict__ block_base) {
    __shared__ uint32_t s_incl[kScanTile];
    __shared__ uint32_t s_rec[kScanTile];
    __shared__ uint32_t s_tbase[kScanTile];
    __shared__ short4 s_rect[kScanTile];
    __shared__ uint16_t s_nzq[kScanThreads / kWave][kWave];
    __shared__ uint8_t s_start[kScanThreads / kWave][kWave];
    __shared__ uint32_t s_hist[kMaxPairPasses][kRadixBins];
    __shared__ uint32_t s_tmp[kScanThreads / kWave];
    __shared__ uint32_t s_base, s_bid, s_agg, s_ticket;
    constexpr int kWaves = kScanThreads / kWave;
    constexpr int kCh = FUSED ? kRadixBins + 1 : 1;  // look-back channels (FUSED: 256 digits, then the count)
    // FUSED: per wavefront, the digit difference array, then the digit
    // counts, then the running output position of each digit
    __shared__ uint32_t s_wd[FUSED ? kWaves : 1][kRadixBins + 1];
    __shared__ uint32_t s_wall[FUSED ? kWaves : 1];
    // FUSED: a block of up to kStage pairs is staged in LDS in its digit
    // order and written out in runs (one per digit), so stores coalesce;
    // longer blocks store each pair where it goes.  s_gb: output position of
    // the block's staged pair 0 of each digit, minus the digit's staged start.
    constexpr int kStage = FUSED ? 12 * kScanThreads : 1;
    __shared__ uint32_t s_pk[kStage], s_pv[kStage];
    __shared__ uint32_t s_gb[FUSED ? kRadixBins : 1];
    const int tid = threadIdx.x;
    // The block's records at its workgroup index (the order in force unless a
    // ticket is drawn), loaded before anything waits; order is a permutation
    // of [0, M) (the depth order), or the identity.
    uint32_t c[kScanIpt], rec[kScanIpt], sum = 0;
    auto load_recs = [&](uint32_t b) {
#pragma unroll
        for (int k = 0; k < kScanIpt; ++k) {
            const uint32_t q = b * (uint32_t)kScanTile + tid * kScanIpt + k;
            rec[k] = q < M ? (order ? min(order[q], M - 1) : q) : 0xffffffffu;
        }
    };
    load_recs(blockIdx.x);
    const uint32_t epoch = ctrl->epoch;
    if (tid == 0) {
        // Single-level scans chain every block to its predecessor by
        // workgroup index, which needs the whole grid on the device at once;
        // once a bounded wait has given up (status bit), the order comes from
        // a ticket instead.  The two-level scan waits on nothing.
        const bool ticket = !block_base && (ctrl->status & (uint32_t)DQO_STATUS_TIMEOUT) != 0u;
        s_bid = ticket ? atomicAdd(&ctrl->counters[kCounterScan], 1u) : blockIdx.x;
        s_ticket = ticket ? 1u : 0u;
    }
    if (tid < kRadixBins) {
        for (int p = 0; p < kMaxPairPasses; ++p) s_hist[p][tid] = 0u;
    }
    uint32_t gcount = 0;  // FUSED: pairs of digit tid over the frame (tid < 256)
    if constexpr (FUSED) {
        for (int i = tid; i < kWaves * (kRadixBins + 1); i += kScanThreads) (&s_wd[0][0])[i] = 0u;
        if (tid < kWaves) s_wall[tid] = 0u;
        if (tid < kRadixBins)
            for (int c = 0; c < copies; ++c) gcount += ctrl->hist_pair[c][0][tid];
    }
    __syncthreads();
    const uint32_t bid = s_bid;
    const uint32_t base = bid * (uint32_t)kScanTile;
    if (base >= M) return;
    if (bid != blockIdx.x) load_recs(bid);
    // The block's records with their counts and tile rectangles, gathered
    // with every load in flight at once and kept in LDS for the emission.
    short4 rc[kScanIpt];
#pragma unroll
    for (int k = 0; k < kScanIpt; ++k) {
        const bool ok = rec[k] != 0xffffffffu;
        c[k] = ok ? counts[rec[k]] : 0u;
        rc[k] = ok ? rects[rec[k]] : make_short4(0, 0, -1, -1);
    }
#pragma unroll
    for (int k = 0; k < kScanIpt; ++k) {
        const uint32_t q = tid * kScanIpt + k;
        s_rec[q] = rec[k];
        s_rect[q] = rc[k];
        s_tbase[q] = rec[k] != 0xffffffffu ? (uint32_t)(rec[k] / (uint32_t)n) * (uint32_t)tiles_per_view : 0u;
        sum += c[k];
        if constexpr (FUSED) {
            if (c[k]) {
                // row y holds tiles t0 + y * tiles_x + [0, tw): digits [a, a + tw mod 256) mod 256
                const int wv = tid >> 6;
                const uint32_t tw = (uint32_t)(rc[k].z - rc[k].x + 1), rem = tw & (kRadixBins - 1);
                const uint32_t t0 = s_tbase[q] + (uint32_t)rc[k].x;
                if (tw >> kRadixBits) atomicAdd(&s_wall[wv], (tw >> kRadixBits) * (uint32_t)(rc[k].w - rc[k].y + 1));
                if (rem)
                    for (int y = rc[k].y; y <= rc[k].w; ++y) {
                        const uint32_t a = (t0 + (uint32_t)y * (uint32_t)tiles_x) & (kRadixBins - 1), b = a + rem;
                        atomicAdd(&s_wd[wv][a], 1u);
                        if (b <= (uint32_t)kRadixBins) {
                            atomicAdd(&s_wd[wv][b], 0xFFFFFFFFu);
                        } else {
                            atomicAdd(&s_wd[wv][0], 1u);
                            atomicAdd(&s_wd[wv][b - kRadixBins], 0xFFFFFFFFu);
                        }
                    }
            }
        }
    }
    const uint32_t texcl = block_exclusive_scan<kScanThreads>(sum, s_tmp);
    uint32_t run = texcl;
#pragma unroll
    for (int k = 0; k < kScanIpt; ++k) {
        run += c[k];
        s_incl[tid * kScanIpt + k] = run;
    }
    if (tid == kScanThreads - 1) s_agg = run;
    __syncthreads();
    const uint32_t agg = s_agg;
    const int lane = tid & (kWave - 1), wave = tid >> 6;
    uint32_t dtotal = 0;  // FUSED: pairs of digit tid in this block (tid < 256)
    if constexpr (FUSED) {
        // each wavefront turns its difference array into digit counts (lane l: digits 4l .. 4l + 3)
        uint32_t d4[4], run = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            run += s_wd[wave][4 * lane + j];
            d4[j] = run;
        }
        const uint32_t off = wave_inclusive_scan(run, lane) - run + s_wall[wave];
#pragma unroll
        for (int j = 0; j < 4; ++j) s_wd[wave][4 * lane + j] = off + d4[j];
        __syncthreads();
        // digit owners: the block's count and each wavefront's exclusive offset
        if (tid < kRadixBins) {
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t cw = s_wd[w][tid];
                s_wd[w][tid] = dtotal;
                dtotal += cw;
            }
        }
    }
    const int lb_thread = FUSED ? kScanThreads - 1 : 0;  // FUSED: a wavefront of its own for the count
    if (tid == lb_thread) {
        if (block_base) {
            s_base = block_base[bid];
        } else {
            // all blocks start at once unless the ticket order is in force
            uint64_t* ch = lb + (kCh - 1);
            const uint32_t excl = (s_ticket || !DQO_LB_GROUPED)
                                      ? lookback_exclusive(ch, kCh, (int)bid, agg, epoch, &ctrl->status)
                                      : lookback_grouped(ch, ch + (size_t)gridDim.x * kCh, kCh, (int)bid, agg, epoch,
                                                         &ctrl->status);
            s_base = excl;
            if (base + kScanTile >= M) {
                const uint32_t total = excl + agg;
                ctrl->num_pairs = total;
                if (total > cap) atomicOr(&ctrl->status, (uint32_t)DQO_STATUS_OVERFLOW);
            }
        }
    }
    if constexpr (FUSED) {
        // digit owners: the digit's pairs in earlier blocks (a digit no pair
        // has anywhere needs no chain), then the wavefronts' start positions
        uint32_t excl = 0;
        if (tid < kRadixBins && gcount)
            excl = (s_ticket || !DQO_LB_GROUPED)
                       ? lookback_exclusive(lb + tid, kCh, (int)bid, dtotal, epoch, &ctrl->status)
                       : lookback_grouped(lb + tid, lb + (size_t)gridDim.x * kCh + tid, kCh, (int)bid, dtotal, epoch,
                                          &ctrl->status);
        const uint32_t gdig = block_exclusive_scan<kScanThreads>(tid < kRadixBins ? gcount : 0u, s_tmp);
        const uint32_t dstart = block_exclusive_scan<kScanThreads>(tid < kRadixBins ? dtotal : 0u, s_tmp);
        if (tid < kRadixBins) {
            s_gb[tid] = gdig + excl - dstart;  // mod 2^32; staged positions of the digit start at dstart
            for (int w = 0; w < kWaves; ++w) s_wd[w][tid] += dstart;
        }
    }
    __syncthreads();
    const uint32_t gbase = s_base;
#pragma unroll
    for (int k = 0; k < kScanIpt; ++k) {
        const uint32_t q = tid * kScanIpt + k;
        if (base + q < M) {
            const uint32_t first = gbase + s_incl[q] - c[k];
            offsets[s_rec[q]] = first;
            // also in the splat record, beside the rectangle (unused when the item has no pairs)
            if (c[k]) splats[(size_t)s_rec[q] * kSplatWords + kSpSlot] = id_to_word<T>((int)first);
        }
    }
    // Emission, one wavefront per group of 64 consecutive records: each round
    // writes 64 consecutive pair slots.  The record owning slot o is the last
    // record with pairs that starts at or before o; within a round it is found
    // from a 64-bit mask of the record starts that fall in the round (one flag
    // byte per slot in LDS, read back through a ballot) and a population
    // count, instead of a search.
    const uint64_t lt = lane ? (~0ull >> (kWave - lane)) : 0ull;
    const bool staged = FUSED && agg <= (uint32_t)kStage;
    constexpr int kGroups = kScanTile / (kScanThreads / kWave) / kWave;
#pragma unroll 1
    for (int g = 0; g < kGroups; ++g) {
        const int q = (wave * kGroups + g) * kWave + lane;
        const uint32_t incl = s_incl[q];
        const uint32_t excl = q ? s_incl[q - 1] : 0u;
        const bool has = incl > excl;
        const uint32_t g0 = __shfl(excl, 0), g1 = __shfl(incl, kWave - 1);
        const uint64_t nzmask = __ballot(has);
        if (has) s_nzq[wave][__popcll(nzmask & lt)] = (uint16_t)q;
        __builtin_amdgcn_wave_barrier();
        for (uint32_t r0 = g0; r0 < g1; r0 += kWave) {
            s_start[wave][lane] = 0;
            if (has && excl >= r0 && excl < r0 + kWave) s_start[wave][excl - r0] = 1;
            __builtin_amdgcn_wave_barrier();
            const uint64_t marks = __ballot(s_start[wave][lane] != 0);
            __builtin_amdgcn_wave_barrier();
            const uint32_t before = (uint32_t)__popcll(__ballot(has && excl < r0));
            const uint32_t o = r0 + (uint32_t)lane;
            const bool valid = o < g1;
            uint32_t tile = 0u, item = 0u;
            if (valid) {
                const uint32_t k = (uint32_t)__popcll(marks & ((2ull << lane) - 1ull));
                const int qo = s_nzq[wave][before + k - 1];
                const uint32_t j = o - (qo ? s_incl[qo - 1] : 0u);
                const short4 rq = s_rect[qo];
                const uint32_t w = (uint32_t)(rq.z - rq.x + 1);
                // j / w from the reciprocal, corrected to the exact quotient
                uint32_t ty = (uint32_t)((float)j * __builtin_amdgcn_rcpf((float)w));
                if (ty * w > j) --ty;
                else if ((ty + 1u) * w <= j) ++ty;
                const uint32_t tx = j - ty * w;
                tile = s_tbase[qo] + ((uint32_t)rq.y + ty) * (uint32_t)tiles_x + (uint32_t)rq.x + tx;
                item = s_rec[qo];
            }
            uint32_t gpos = gbase + o;
            if constexpr (FUSED) {
                // rank among this round's pairs of the same low byte, after the
                // wavefront's earlier pairs of that byte
                const uint32_t d = tile & (kRadixBins - 1);
                uint64_t peers = __ballot(valid);
#pragma unroll
                for (int b = 0; b < kRadixBits; ++b) {
                    const bool bit = (d >> b) & 1u;
                    const uint64_t bb = __ballot(bit);
                    peers &= bit ? bb : ~bb;
                }
                uint32_t pos0 = 0u;
                if (valid) pos0 = s_wd[wave][d];
                if (valid && (peers >> lane) == 1ull) s_wd[wave][d] = pos0 + (uint32_t)__popcll(peers);
                const uint32_t lpos = pos0 + (uint32_t)__popcll(peers & lt);
                if (valid && staged) {
                    s_pk[lpos] = tile;
                    s_pv[lpos] = item;
                }
                gpos = staged ? cap : s_gb[d] + lpos;  // staged pairs are stored below
            }
            if (valid && gpos < cap) {
                pkeys[gpos] = tile;
                pvals[gpos] = item;
            }
            if (valid)
                for (int p = FUSED ? 1 : 0; p < pair_passes; ++p) atomicAdd(&s_hist[p][(tile >> (8 * p)) & 255u], 1u);
        }
    }
    __syncthreads();
    if (staged) {  // uniform: the block's runs, one per digit
        for (uint32_t q = tid; q < agg; q += kScanThreads) {
            const uint32_t k = s_pk[q];
            const uint32_t o = s_gb[k & (kRadixBins - 1)] + q;
            if (o < cap) {
                pkeys[o] = k;
                pvals[o] = s_pv[q];
            }
        }
    }
    if (tid < kRadixBins)
        for (int p = FUSED ? 1 : 0; p < pair_passes; ++p) {
            const uint32_t h = s_hist[p][tid];
            if (h) atomicAdd(&ctrl->hist_pair[blockIdx.x % copies][p][tid], h);
        }
}

int scan_emit_resident(bool fused) {
    return fused ? std::min(resident_blocks<scan_emit_kernel<float, true>, kScanThreads>(),
                            resident_blocks<scan_emit_kernel<double, true>, kScanThreads>())
                 : std::min(resident_blocks<scan_emit_kernel<float, false>, kScanThreads>(),
                            resident_blocks<scan_emit_kernel<double, false>, kScanThreads>());
}

template <typename T>
hipError_t launch_project_bin(const Frame<T>& f, const T* params, const int32_t* ids, hipStream_t st) {
    const StatePtrs& s = f.s;
    hipLaunchKernelGGL(prep_kernel, dim3((unsigned)std::max(1, std::max(s.hist_copies_depth, s.hist_copies_pair))),
                       dim3(256), 0, st, s.ctrl, s.hist_copies_depth, s.hist_copies_pair);
    const int64_t M = s.items;
    const int64_t range_words = 2 * (int64_t)f.views.tiles_per_view * f.views.n_views;
    if (M == 0) return launch_zero_words(s.ranges, range_words, st);
    hipLaunchKernelGGL(project_kernel<T>, dim3((unsigned)((M + 256 * kProjItems - 1) / (256 * kProjItems))), dim3(256),
                       0, st, f.views, f.consts,
                       f.n, M, params, ids, (T*)s.splats, s.rects, s.counts, s.depth_keys[0], s.depth_vals[0],
                       s.ranges, range_words, s.hist_copies_depth, s.ctrl,
                       s.fused_emit ? &s.ctrl->hist_pair[0][0][0] : nullptr, s.hist_copies_pair);
    // Below 2^18 items the 2048-item blocks run as 1024 threads x 2 items
    // (4 wavefronts per SIMD instead of 1 hide more of the load latency:
    // 12.6 -> 12.0 us per pass at 200k items); the block length is the same.
#ifndef DQO_DEPTH_SMALL_NT
#define DQO_DEPTH_SMALL_NT 1024
#endif
    const int dnt = M < (int64_t(1) << 18) ? DQO_DEPTH_SMALL_NT : kDepthNt;
    const int dipt = kDepthNt * depth_ipt(M) / dnt;
    // Buffers of the four passes: 0 -> 1 -> 2 -> 1 -> 0, or 0 -> 1 -> 2 -> 0
    // when three passes suffice (decided on the device from the key range).
    static const int kIn[kMaxDepthPasses] = {0, 1, 2, 1}, kOut[kMaxDepthPasses] = {1, 2, 1, 0};
    for (int p = 0; p < (s.tile_sort ? 0 : kMaxDepthPasses); ++p) {
        const DepthRel rel{p, p == 2 ? s.depth_keys[0] : nullptr, p == 2 ? s.depth_vals[0] : nullptr,
                           p + 1 < kMaxDepthPasses ? &s.ctrl->hist_depth[0][p + 1][0] : nullptr};
        hipError_t e = launch_radix_pass(s.depth_keys[kIn[p]], s.depth_vals[kIn[p]], s.depth_keys[kOut[p]],
                                         s.depth_vals[kOut[p]], nullptr, (uint32_t)M, p * kRadixBits,
                                         &s.ctrl->hist_depth[0][p][0], kMaxDepthPasses * kRadixBins, s.hist_copies_depth,
                                         s.lb_depth + (size_t)p * lb_blocks(s.depth_blocks) * kRadixBins,
                                         &s.ctrl->counters[kCounterDepth + p], s.ctrl, st, dnt, dipt, &rel);
        if (e != hipSuccess) return e;
    }
    // the fused emission writes the first pair pass's output buffer
    const int pf = s.pair_first_buf ^ (s.fused_emit ? 1 : 0);
    const bool two_level = s.scan_blocks > scan_emit_resident(s.fused_emit);
    if (two_level) {
        hipLaunchKernelGGL(scan_block_sums_kernel, dim3((unsigned)s.scan_blocks), dim3(kScanThreads), 0, st,
                           item_order(s), s.counts, (uint32_t)M, s.scan_base);
        hipLaunchKernelGGL(scan_block_base_kernel, dim3(1), dim3(kScanThreads), 0, st, s.scan_base, s.scan_blocks,
                           (uint32_t)s.capacity, s.ctrl);
    }
    auto emit = s.fused_emit ? scan_emit_kernel<T, true> : scan_emit_kernel<T, false>;
    hipLaunchKernelGGL(emit, dim3((unsigned)s.scan_blocks), dim3(kScanThreads), 0, st, item_order(s),
                       s.counts, s.rects, s.offsets, (T*)s.splats, s.pair_keys[pf], s.pair_vals[pf], (uint32_t)M,
                       (uint32_t)s.capacity, f.n, f.views.tiles_x, f.views.tiles_per_view, s.pair_passes,
                       s.hist_copies_pair, s.lb_scan, s.ctrl, two_level ? (const uint32_t*)s.scan_base : nullptr);
    return hipGetLastError();
}

// ---------------------------------------------------------------- backward
// Clears the written marks of the pairs of this frame.  The render backward
// writes the partials of the pairs that contribute somewhere in their tile and
// marks them; the per-item sums read the partials of marked pairs only, so the
// partials themselves are never cleared.
__global__ __launch_bounds__(256) void clear_written_kernel(uint32_t* __restrict__ words,
                                                            const Ctrl* __restrict__ ctrl, uint32_t cap) {
    const uint32_t n = (min(ctrl->num_pairs, cap) + 3u) / 4u;  // marks are bytes, cleared four at a time
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) words[i] = 0u;
}

hipError_t launch_clear_written(const StatePtrs& s, hipStream_t st) {
    if (s.capacity == 0) return hipSuccess;
    hipLaunchKernelGGL(clear_written_kernel, dim3(256), dim3(256), 0, st, (uint32_t*)s.written, s.ctrl,
                       (uint32_t)s.capacity);
    return hipGetLastError();
}

// Per-item totals of the pair partials (those of pairs the render backward
// marked written; the others count as zero).  An item's (tile, Gaussian)
// partials occupy consecutive slots, and items that are consecutive in depth
// order occupy consecutive slot ranges, so one wavefront takes 64 consecutive
// items and reads their slots 64 at a time, coalesced.  Each round sums the
// slots of every item by a segmented scan over the lanes (a fixed tree per
// segment) and adds the segment totals to the item's accumulator in LDS in
// round order: the result does not depend on timing.
constexpr int kSlotWaves = 4;
#ifndef DQO_SLOT_BATCH
#define DQO_SLOT_BATCH 4
#endif
constexpr int kSlotBatch = DQO_SLOT_BATCH;  // rounds of 64 slots whose loads are issued together

// Lane-shifted copy of x by DPP (row_shr:n within 16-lane rows, or the
// row_bcast:15 / row_bcast:31 steps across rows); lanes without a source get 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_shift(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWS, 0xF, true));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_shift(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROWS, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROWS, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Inclusive scan of v over the lanes within segments: lane l sums lanes
// [seg_lo, l], where seg_lo (the first lane of l's segment) is the same for
// all lanes of a segment.  Row-local shifts by 1, 2, 4, 8, then the last lane
// of rows 0 and 2 into rows 1 and 3, then lane 31 into rows 2 and 3.
template <typename T>
__device__ __forceinline__ T segmented_scan(T v, int lane, int seg_lo) {
    T t;
    t = dpp_shift<0x111, 0xF>(v); if (lane - 1 >= seg_lo && (lane & 15) >= 1) v += t;
    t = dpp_shift<0x112, 0xF>(v); if (lane - 2 >= seg_lo && (lane & 15) >= 2) v += t;
    t = dpp_shift<0x114, 0xF>(v); if (lane - 4 >= seg_lo && (lane & 15) >= 4) v += t;
    t = dpp_shift<0x118, 0xF>(v); if (lane - 8 >= seg_lo && (lane & 15) >= 8) v += t;
    t = dpp_shift<0x142, 0xA>(v); if ((lane & 16) && (lane & ~15) - 1 >= seg_lo) v += t;
    t = dpp_shift<0x143, 0xC>(v); if (lane >= 32 && 31 >= seg_lo) v += t;
    return v;
}

template <typename T>
__global__ __launch_bounds__(kSlotWaves * kWave) void slot_sum_kernel(const uint32_t* __restrict__ order,
                                                                      const uint32_t* __restrict__ counts,
                                                                      const uint32_t* __restrict__ offsets,
                                                                      const T* __restrict__ partials,
                                                                      const uint8_t* __restrict__ written, uint32_t M,
                                                                      uint32_t cap, T* __restrict__ sums) {
    __shared__ T s_acc[kSlotWaves][kWave][kGradWords + 1];
    __shared__ uint16_t s_nz[kSlotWaves][kWave];
    __shared__ uint8_t s_start[kSlotWaves][kWave];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
    const uint64_t lt = lane ? (~0ull >> (kWave - lane)) : 0ull;
    const uint32_t q = ((uint32_t)blockIdx.x * kSlotWaves + wave) * kWave + lane;
    uint32_t rec = 0, c = 0, off = 0;
    if (q < M) {
        rec = order ? min(order[q], M - 1) : q;  // emission order: depth order, or item order
        c = counts[rec];
        off = offsets[rec];
    }
#pragma unroll
    for (int k = 0; k < kGradWords; ++k) s_acc[wave][lane][k] = T(0);
    const bool has = c > 0;
    const uint64_t nzmask = __ballot(has);
    if (nzmask == 0ull) return;  // wave-uniform; no barrier follows
    if (has) s_nz[wave][__popcll(nzmask & lt)] = (uint16_t)lane;
    const int first = __ffsll((unsigned long long)nzmask) - 1, lastl = 63 - __clzll(nzmask);
    const uint32_t S0 = __shfl(off, first);
    const uint32_t S1 = (uint32_t)min((uint64_t)cap, (uint64_t)__shfl(off, lastl) + __shfl(c, lastl));
    __builtin_amdgcn_wave_barrier();
    // Rounds of 64 slots, kSlotBatch at a time: the marks of the batch's
    // rounds are loaded together, then their marked partials together, so a
    // batch costs two memory round trips instead of two per round.
    for (uint32_t b0 = S0; b0 < S1; b0 += kSlotBatch * kWave) {
        bool mk[kSlotBatch];
        T vb[kSlotBatch][kGradWords];
#pragma unroll
        for (int q = 0; q < kSlotBatch; ++q) {
            const uint32_t s = b0 + q * kWave + (uint32_t)lane;
            mk[q] = s < S1 && written[s] != 0;
        }
#pragma unroll
        for (int q = 0; q < kSlotBatch; ++q) {
            const uint32_t s = b0 + q * kWave + (uint32_t)lane;
#pragma unroll
            for (int k = 0; k < kGradWords; ++k) vb[q][k] = mk[q] ? partials[(size_t)s * kGradWords + k] : T(0);
        }
#pragma unroll
        for (int q = 0; q < kSlotBatch; ++q) {
            const uint32_t r0 = b0 + q * kWave;
            if (r0 >= S1) break;  // wave-uniform
            s_start[wave][lane] = 0;
            if (has && off >= r0 && off < r0 + kWave) s_start[wave][off - r0] = 1;
            __builtin_amdgcn_wave_barrier();
            const uint64_t marks = __ballot(s_start[wave][lane] != 0);
            __builtin_amdgcn_wave_barrier();
            const uint32_t before = (uint32_t)__popcll(__ballot(has && off < r0));
            const uint32_t s = r0 + (uint32_t)lane;
            const bool live = s < S1;
            const uint64_t upto = marks & ((2ull << lane) - 1ull);
            int owner = 0;
            if (live) owner = s_nz[wave][before + (uint32_t)__popcll(upto) - 1u];
            const int seg_lo = upto ? 63 - __clzll(upto) : 0;
            T v[kGradWords];
#pragma unroll
            for (int k = 0; k < kGradWords; ++k) v[k] = segmented_scan<T>(vb[q][k], lane, seg_lo);
            const bool seg_end = live && (lane == kWave - 1 || ((marks >> (lane + 1)) & 1ull) || s + 1u >= S1);
            if (seg_end) {
#pragma unroll
                for (int k = 0; k < kGradWords; ++k) s_acc[wave][owner][k] += v[k];
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (has && (uint64_t)off + c <= cap) {
#pragma unroll
        for (int k = 0; k < kGradWords; ++k) sums[(size_t)rec * kGradWords + k] = s_acc[wave][lane][k];
    }
}

// Chain rule of one (view, Gaussian) item from its pair-partial totals d
// (mean2d, conic, o dL/do, colour, depth) to the 14 parameters (out) and to
// the camera-frame mean (dpc); false when the item is culled.
template <typename T>
__device__ __forceinline__ bool item_backward(const DevCam<T>& c, const Consts<T>& cs, const T (&p)[kParams],
                                              const T (&d)[kGradWords], Proj<T>& pr, T (&out)[kParams],
                                              T (&dpc)[3]) {
    project_item(c, cs, p, pr);
    if (!pr.visible) return false;
    const T* W = c.R;
    // conic -> 2D covariance: G_S = -Ci Gc Ci with Gc = [[dA, dB/2], [dB/2, dC]]
    const T hB = T(0.5) * d[3];
    const T a00 = pr.A * d[2] + pr.B * hB, a01 = pr.A * hB + pr.B * d[4];
    const T a10 = pr.B * d[2] + pr.C * hB, a11 = pr.B * hB + pr.C * d[4];
    const T gs00 = -(a00 * pr.A + a01 * pr.B);
    const T gs01 = -(a00 * pr.B + a01 * pr.C);
    const T gs11 = -(a10 * pr.B + a11 * pr.C);
    // Sigma2 = U U^T + dil I: dU = 2 G_S U
    T dU[6];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        dU[b] = T(2) * (gs00 * pr.U[b] + gs01 * pr.U[3 + b]);
        dU[3 + b] = T(2) * (gs01 * pr.U[b] + gs11 * pr.U[3 + b]);
    }
    // U = T2 M with T2 = J W, M = R diag(s)
    const T iz = T(1) / pr.z;
    const T j00 = c.fx * iz, j02 = -c.fx * pr.ux * iz;
    const T j11 = c.fy * iz, j12 = -c.fy * pr.uy * iz;
    T T2[6], Mm[9];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T2[k] = j00 * W[k] + j02 * W[6 + k];
        T2[3 + k] = j11 * W[3 + k] + j12 * W[6 + k];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) Mm[a * 3 + b] = pr.R[a * 3 + b] * pr.s[b];
    T dT2[6], dM[9];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            dT2[a * 3 + k] = dU[a * 3 + 0] * Mm[k * 3 + 0] + dU[a * 3 + 1] * Mm[k * 3 + 1] +
                             dU[a * 3 + 2] * Mm[k * 3 + 2];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int b = 0; b < 3; ++b) dM[k * 3 + b] = T2[k] * dU[b] + T2[3 + k] * dU[3 + b];
    // dJ = dT2 W^T (only the four nonzero entries of J matter)
    const T dj00 = dT2[0] * W[0] + dT2[1] * W[1] + dT2[2] * W[2];
    const T dj02 = dT2[0] * W[6] + dT2[1] * W[7] + dT2[2] * W[8];
    const T dj11 = dT2[3] * W[3] + dT2[4] * W[4] + dT2[5] * W[5];
    const T dj12 = dT2[3] * W[6] + dT2[4] * W[7] + dT2[5] * W[8];
    const T iz2 = iz * iz, iz3 = iz2 * iz;
    // A clamped ratio is a constant: J02 = -fx lim / z then depends on z alone.
    T dpx = d[0] * c.fx * iz;
    T dpy = d[1] * c.fy * iz;
    T dpz = dj00 * (-c.fx * iz2) + dj11 * (-c.fy * iz2) + d[0] * (-c.fx * pr.x * iz2) +
            d[1] * (-c.fy * pr.y * iz2) + d[9];
    if (pr.ux_clamped) {
        dpz += dj02 * (c.fx * pr.ux * iz2);
    } else {
        dpx += dj02 * (-c.fx * iz2);
        dpz += dj02 * (T(2) * c.fx * pr.x * iz3);
    }
    if (pr.uy_clamped) {
        dpz += dj12 * (c.fy * pr.uy * iz2);
    } else {
        dpy += dj12 * (-c.fy * iz2);
        dpz += dj12 * (T(2) * c.fy * pr.y * iz3);
    }
    dpc[0] = dpx;
    dpc[1] = dpy;
    dpc[2] = dpz;
    out[0] = W[0] * dpx + W[3] * dpy + W[6] * dpz;
    out[1] = W[1] * dpx + W[4] * dpy + W[7] * dpz;
    out[2] = W[2] * dpx + W[5] * dpy + W[8] * dpz;
    // M = R diag(s)
    T dR[9];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        T ds = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ds += dM[a * 3 + b] * pr.R[a * 3 + b];
            dR[a * 3 + b] = dM[a * 3 + b] * pr.s[b];
        }
        out[3 + b] = ds * pr.s[b];
    }
    // R(q) with q normalised
    const T w = pr.qn[0], x = pr.qn[1], y = pr.qn[2], z = pr.qn[3];
    T dq[4];
    dq[0] = T(2) * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = T(2) * (y * dR[1] + z * dR[2] + y * dR[3] - w * dR[5] + z * dR[6] + w * dR[7]) -
            T(4) * x * (dR[4] + dR[8]);
    dq[2] = T(2) * (x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7]) -
            T(4) * y * (dR[0] + dR[8]);
    dq[3] = T(2) * (-w * dR[1] + x * dR[2] + w * dR[3] + y * dR[5] + x * dR[6] + y * dR[7]) -
            T(4) * z * (dR[0] + dR[4]);
    const T dot = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
    const T iq = T(1) / pr.qnorm;
#pragma unroll
    for (int k = 0; k < 4; ++k) out[6 + k] = (dq[k] - pr.qn[k] * dot) * iq;
    out[10] = d[5] * (T(1) - pr.o);  // d[5] = o dL/do, sigmoid opacity
    out[11] = d[6];
    out[12] = d[7];
    out[13] = d[8];
    return true;
}

template <typename T>
__device__ __forceinline__ void project_backward_one(const Views<T>& V, const Consts<T>& cs, int64_t n, int64_t g,
                                                     T* __restrict__ params, const uint32_t* __restrict__ counts,
                                                     const uint32_t* __restrict__ offsets,
                                                     const T* __restrict__ sums, uint32_t cap, T* __restrict__ grads,
                                                     T* __restrict__ am, T* __restrict__ av, const AdamArgs<T>& aa,
                                                     const T* s_ss, T s_isb, bool adam) {
    T p[kParams], mm[kParams], vv[kParams];
#pragma unroll
    for (int r = 0; r < kParams; ++r) p[r] = params[(int64_t)r * n + g];
    if (adam) {  // the moments are loaded with the parameters, not after the gradient
#pragma unroll
        for (int r = 0; r < kParams; ++r) {
            mm[r] = am[(int64_t)r * n + g];
            vv[r] = av[(int64_t)r * n + g];
        }
    }
    T acc[kParams];
#pragma unroll
    for (int r = 0; r < kParams; ++r) acc[r] = T(0);
    for (int v = 0; v < V.n_views; ++v) {
        if (g < V.cam[v].seg_lo || g >= V.cam[v].seg_hi) continue;
        const int64_t item = (int64_t)v * n + g;
        const uint32_t cnt = counts[item];
        if (cnt == 0) continue;
        const uint32_t off = offsets[item];
        if ((uint64_t)off + cnt > cap) continue;
        T d[kGradWords];
#pragma unroll
        for (int k = 0; k < kGradWords; ++k) d[k] = sums[(size_t)item * kGradWords + k];
        const DevCam<T>& c = V.cam[v];
        Proj<T> pr;
        T out[kParams], dpc[3];
        if (!item_backward<T>(c, cs, p, d, pr, out, dpc)) continue;
#pragma unroll
        for (int r = 0; r < kParams; ++r) acc[r] += out[r];
    }
    if (adam) {
        if (grads) {
#pragma unroll
            for (int r = 0; r < kParams; ++r) grads[(int64_t)r * n + g] = acc[r];
        }
#pragma unroll
        for (int r = 0; r < kParams; ++r) {
            const int64_t i = (int64_t)r * n + g;
            T pp = p[r];
            adam_one<T>(pp, acc[r], mm[r], vv[r], s_ss[r], s_isb, aa);
            params[i] = pp;
            am[i] = mm[r];
            av[i] = vv[r];
        }
    } else {
#pragma unroll
        for (int r = 0; r < kParams; ++r) grads[(int64_t)r * n + g] = acc[r];
    }
}

// Per-Gaussian gradients from the per-item totals (chain rule through the
// projection, summed over the views).  With moment buffers given, the Adam
// update of dqo_adam_step_counted is applied at once to params, m and v, and
// the last workgroup to finish advances the device step.  One kernel serves
// both uses (a run-time switch), so the gradient is the same compiled
// arithmetic whether or not Adam follows.
template <typename T>
__global__ __launch_bounds__(256) void project_backward_kernel(Views<T> V, Consts<T> cs, int64_t n,
                                                               T* __restrict__ params,
                                                               const uint32_t* __restrict__ counts,
                                                               const uint32_t* __restrict__ offsets,
                                                               const T* __restrict__ sums, uint32_t cap,
                                                               T* __restrict__ grads, T* __restrict__ am,
                                                               T* __restrict__ av, AdamArgs<T> aa,
                                                               int64_t* d_step, uint32_t* done) {
    __shared__ T s_ss[kParams];
    __shared__ T s_isb;
    const bool adam = am != nullptr;  // uniform over the grid
    if (adam) {
        if (threadIdx.x == 0) device_step_table<T>(aa, *d_step, s_ss, &s_isb);
        __syncthreads();
    }
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g < n) project_backward_one<T>(V, cs, n, g, params, counts, offsets, sums, cap, grads, am, av, aa, s_ss, s_isb,
                                       adam);
    if (adam) {
        // Every workgroup read the step before it counts itself done (its
        // value was consumed before the barrier above, so the read has
        // completed): the last one advances it and re-arms the counter.  No
        // fence is needed for that order, and an agent-scope fence here
        // writes back and invalidates the L2 once per workgroup (it made the
        // fused kernel ~30 us slower at 200k Gaussians).
        if (threadIdx.x == 0) {
            if (atomicAdd(done, 1u) == gridDim.x - 1u) {
                atomicAdd((unsigned long long*)d_step, 1ull);
                atomicExch(done, 0u);
            }
        }
    }
}


template <typename T>
hipError_t launch_project_backward(const Frame<T>& f, const T* params, T* grads, hipStream_t st) {
    if (f.n == 0) return hipSuccess;
    const int64_t M = f.s.items;
    hipLaunchKernelGGL(slot_sum_kernel<T>, dim3((unsigned)((M + kSlotWaves * kWave - 1) / (kSlotWaves * kWave))),
                       dim3(kSlotWaves * kWave), 0, st, item_order(f.s), f.s.counts, f.s.offsets,
                       (const T*)f.s.partials, f.s.written, (uint32_t)M, (uint32_t)f.s.capacity, (T*)f.s.sums);
    hipLaunchKernelGGL((project_backward_kernel<T>), dim3((unsigned)((f.n + 255) / 256)), dim3(256), 0, st,
                       f.views, f.consts, f.n, const_cast<T*>(params), f.s.counts, f.s.offsets, (const T*)f.s.sums,
                       (uint32_t)f.s.capacity, grads, (T*)nullptr, (T*)nullptr, AdamArgs<T>{}, (int64_t*)nullptr,
                       (uint32_t*)nullptr);
    return hipGetLastError();
}

// Camera-pose gradient of every view (tracking): each (view, Gaussian) item
// contributes, through the rigid-motion identity (moving the camera renders
// what moving every Gaussian by the inverse world motion renders),
// dL/dtau += g and dL/dw += p x g + R dL/dphi, where g is the gradient of the
// camera-frame mean p and phi a world-frame left rotation of the item's
// quaternion (s, u): dL/dphi = (-u dL/ds + s dL/du + u x dL/du) / 2.  Blocks
// reduce in a fixed order (shuffle tree, then waves in order) into per-block
// partials in double precision; pose_final_kernel sums them in block order.
__device__ __forceinline__ double pose_wave_sum(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_down(v, d);
    return v;
}

template <typename T>
__global__ __launch_bounds__(256) void pose_grad_kernel(Views<T> V, Consts<T> cs, int64_t n,
                                                        const T* __restrict__ params,
                                                        const uint32_t* __restrict__ counts,
                                                        const uint32_t* __restrict__ offsets,
                                                        const T* __restrict__ sums, uint32_t cap,
                                                        double* __restrict__ partials) {
    __shared__ double s_w[4][6];
    const int v = blockIdx.y;
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double pose[6] = {0, 0, 0, 0, 0, 0};
    const DevCam<T>& c = V.cam[v];
    if (g < n && g >= c.seg_lo && g < c.seg_hi) {
        const int64_t item = (int64_t)v * n + g;
        const uint32_t cnt = counts[item];
        const uint32_t off = offsets[item];
        if (cnt > 0 && (uint64_t)off + cnt <= cap) {
            T p[kParams], d[kGradWords], out[kParams], dpc[3];
#pragma unroll
            for (int r = 0; r < kParams; ++r) p[r] = params[(int64_t)r * n + g];
#pragma unroll
            for (int k = 0; k < kGradWords; ++k) d[k] = sums[(size_t)item * kGradWords + k];
            Proj<T> pr;
            if (item_backward<T>(c, cs, p, d, pr, out, dpc)) {
                const T qs = p[6], u0 = p[7], u1 = p[8], u2 = p[9];
                const T ds = out[6], du0 = out[7], du1 = out[8], du2 = out[9];
                const T f0 = T(0.5) * (-u0 * ds + qs * du0 + (u1 * du2 - u2 * du1));
                const T f1 = T(0.5) * (-u1 * ds + qs * du1 + (u2 * du0 - u0 * du2));
                const T f2 = T(0.5) * (-u2 * ds + qs * du2 + (u0 * du1 - u1 * du0));
                const T* R = c.R;
                pose[0] = (double)(pr.y * dpc[2] - pr.z * dpc[1] + R[0] * f0 + R[1] * f1 + R[2] * f2);
                pose[1] = (double)(pr.z * dpc[0] - pr.x * dpc[2] + R[3] * f0 + R[4] * f1 + R[5] * f2);
                pose[2] = (double)(pr.x * dpc[1] - pr.y * dpc[0] + R[6] * f0 + R[7] * f1 + R[8] * f2);
                pose[3] = (double)dpc[0];
                pose[4] = (double)dpc[1];
                pose[5] = (double)dpc[2];
            }
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double t = pose_wave_sum(pose[k]);
        if (lane == 0) s_w[wave][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const double t = ((s_w[0][threadIdx.x] + s_w[1][threadIdx.x]) + s_w[2][threadIdx.x]) + s_w[3][threadIdx.x];
        partials[((size_t)v * gridDim.x + blockIdx.x) * 6 + threadIdx.x] = t;
    }
}

// One wavefront per (view, component): lane l sums blocks l, l + 64, ... in
// order, then a fixed shuffle tree.
__global__ __launch_bounds__(384) void pose_final_kernel(const double* __restrict__ partials, int nblocks,
                                                         double* __restrict__ out) {
    const int v = blockIdx.x, k = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double a = 0.0;
    for (int b = lane; b < nblocks; b += 64) a += partials[((size_t)v * nblocks + b) * 6 + k];
    a = pose_wave_sum(a);
    if (lane == 0) out[v * 6 + k] = a;
}

template <typename T>
hipError_t launch_pose_backward(const Frame<T>& f, const T* params, double* pose, hipStream_t st) {
    const int V = f.views.n_views;
    if (f.n == 0) return launch_zero_words((uint32_t*)pose, 12 * (int64_t)V, st);
    const int64_t M = f.s.items;
    hipLaunchKernelGGL(slot_sum_kernel<T>, dim3((unsigned)((M + kSlotWaves * kWave - 1) / (kSlotWaves * kWave))),
                       dim3(kSlotWaves * kWave), 0, st, item_order(f.s), f.s.counts, f.s.offsets,
                       (const T*)f.s.partials, f.s.written, (uint32_t)M, (uint32_t)f.s.capacity, (T*)f.s.sums);
    const int blocks = (int)((f.n + 255) / 256);
    hipLaunchKernelGGL(pose_grad_kernel<T>, dim3((unsigned)blocks, (unsigned)V), dim3(256), 0, st, f.views, f.consts,
                       f.n, params, f.s.counts, f.s.offsets, (const T*)f.s.sums, (uint32_t)f.s.capacity,
                       f.s.pose_partials);
    hipLaunchKernelGGL(pose_final_kernel, dim3((unsigned)V), dim3(384), 0, st, (const double*)f.s.pose_partials,
                       blocks, pose);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_project_backward_adam(const Frame<T>& f, T* params, T* grads, T* m, T* v, const dqo_adam& hp,
                                        int64_t* d_step, hipStream_t st) {
    if (f.n == 0) return launch_adam<T>(params, grads, m, v, 0, hp, 1, d_step, st, kParams);  // advances the step
    const int64_t M = f.s.items;
    hipLaunchKernelGGL(slot_sum_kernel<T>, dim3((unsigned)((M + kSlotWaves * kWave - 1) / (kSlotWaves * kWave))),
                       dim3(kSlotWaves * kWave), 0, st, item_order(f.s), f.s.counts, f.s.offsets,
                       (const T*)f.s.partials, f.s.written, (uint32_t)M, (uint32_t)f.s.capacity, (T*)f.s.sums);
    hipLaunchKernelGGL((project_backward_kernel<T>), dim3((unsigned)((f.n + 255) / 256)), dim3(256), 0, st,
                       f.views, f.consts, f.n, params, f.s.counts, f.s.offsets, (const T*)f.s.sums,
                       (uint32_t)f.s.capacity, grads, m, v, make_adam_args<T>(hp, 1), d_step,
                       &f.s.ctrl->counters[kCounterAdam]);
    return hipGetLastError();
}

__global__ void clear_ctrl_kernel(Ctrl* ctrl, uint64_t* lb, int64_t lb_words) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t* c = reinterpret_cast<uint32_t*>(ctrl);
    const int64_t cw = (int64_t)(sizeof(Ctrl) / 4);
    for (int64_t k = i; k < cw; k += (int64_t)gridDim.x * blockDim.x) c[k] = 0u;
    for (int64_t k = i; k < lb_words; k += (int64_t)gridDim.x * blockDim.x) lb[k] = 0ull;
}

__global__ void clear_status_kernel(Ctrl* ctrl) { ctrl->status = 0u; }

__global__ void zero_words_kernel(uint32_t* p, int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = 0u;
}

hipError_t launch_zero_words(uint32_t* p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_words_kernel, dim3(256), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_clear_ctrl(Ctrl* ctrl, uint64_t* lb, int64_t lb_words, hipStream_t st) {
    hipLaunchKernelGGL(clear_ctrl_kernel, dim3(256), dim3(256), 0, st, ctrl, lb, lb_words);
    return hipGetLastError();
}

hipError_t launch_clear_status(Ctrl* ctrl, hipStream_t st) {
    hipLaunchKernelGGL(clear_status_kernel, dim3(1), dim3(1), 0, st, ctrl);
    return hipGetLastError();
}

template hipError_t launch_project_bin<float>(const Frame<float>&, const float*, const int32_t*, hipStream_t);
template hipError_t launch_project_bin<double>(const Frame<double>&, const double*, const int32_t*, hipStream_t);
template hipError_t launch_project_backward<float>(const Frame<float>&, const float*, float*, hipStream_t);
template hipError_t launch_project_backward<double>(const Frame<double>&, const double*, double*, hipStream_t);
template hipError_t launch_pose_backward<float>(const Frame<float>&, const float*, double*, hipStream_t);
template hipError_t launch_pose_backward<double>(const Frame<double>&, const double*, double*, hipStream_t);
template hipError_t launch_project_backward_adam<float>(const Frame<float>&, float*, float*, float*, float*,
                                                        const dqo_adam&, int64_t*, hipStream_t);
template hipError_t launch_project_backward_adam<double>(const Frame<double>&, double*, double*, double*, double*,
                                                         const dqo_adam&, int64_t*, hipStream_t);

}  // namespace dqo
