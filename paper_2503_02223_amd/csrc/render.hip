// Tile rasterization: forward alpha blending and its adjoint.
//
// One workgroup per (view, pixel tile), one thread per pixel; the tile's sorted
// pair range is streamed through LDS in batches of one record per thread, and
// every thread then walks the batch from LDS (broadcast reads).  Blending is a
// per-pixel recurrence, not a dense contraction, so this path is VALU and
// transcendental bound and uses no matrix cores.
//
// The inner loops are written without divergent branches: every lane computes
// the contribution test, non-contributing lanes carry a zero weight, and whole
// steps are skipped only when the entire wavefront agrees (ballots), so the
// per-pair cost is a straight line of VALU work instead of exec-mask juggling.
//
// The forward keeps only T_final and the position of the last blended
// Gaussian per pixel.  The backward walks each pixel from that position back to
// the front of its tile's range, recomputing alpha exactly as the forward did
// and the transmittance by division (T_i = T_{i+1} / (1 - alpha_i)), and
// reduces the per-pixel gradients of each Gaussian over the workgroup: six
// Gaussians x ten values are transposed-and-summed across the 64 lanes of a
// wave (each lane ends up owning one value), then summed over the waves in
// LDS, and written once per (tile, Gaussian) pair to its own slot, which is
// marked written (pairs left unwritten count as zero); the per-Gaussian
// totals are formed later in a fixed order, so no atomics are needed and the
// result is deterministic.
#include "dqo_device.hpp"

namespace dqo {

template <typename T>
__device__ __forceinline__ T fmadd(T a, T b, T c) { return fma(a, b, c); }

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

// Walk records: what the render kernels keep in LDS for each pair of a batch,
// the splat restated in the coordinates of the pair's tile.  With (du, dv) a
// pixel centre's offset from the splat's mean, the pixel's alpha before the
// clamp is 2^E with E = a du^2 + 2b du dv + c dv^2 + log2(o): the conic of
// Eq. (12)'s Gaussian scaled by -log2(e)/2 and the opacity folded in.  A
// pair contributes at a pixel exactly when E reaches the record's threshold,
// max(log2 o - q_max log2(e)/2, log2 alpha_min), which is Q <= q_max and
// alpha >= alpha_min at once.  Forward and backward evaluate E with the same
// code from the same record, so both take the same decisions.
//   [0, 1] mean relative to the tile's corner (mu, mv); [2, 3, 4] a, b, c;
//   [5] log2 o; [6] threshold; [7] the pair's position; [8] depth; [9] object
//   id; [10, 11, 12] colour; [13..15] unused.
constexpr int kWalkWords = 16;
enum WalkWord { kWMu = 0, kWMv = 1, kWA = 2, kWM = 3, kWC = 4, kWLop = 5, kWThr = 6, kWPos = 7, kWZ = 8,
                kWId = 9, kWR = 10, kWG = 11, kWB = 12 };
template <typename T>
__device__ __forceinline__ T neg_half_log2e() { return T(-0.72134752044448170368); }

template <typename T>
__device__ __forceinline__ T log2_of(T x);
template <>
__device__ __forceinline__ float log2_of<float>(float x) { return log2f(x); }
template <>
__device__ __forceinline__ double log2_of<double>(double x) { return log2(x); }
template <typename T>
__device__ __forceinline__ T exp2_of(T x);
template <>
__device__ __forceinline__ float exp2_of<float>(float x) { return __builtin_amdgcn_exp2f(x); }
template <>
__device__ __forceinline__ double exp2_of<double>(double x) { return exp2(x); }

// Walk record of splat record r (mx, my, A, B, C, o, z, id, r, g, b) for the
// tile whose first pixel's corner is (ox, oy), stored at dst (LDS).
template <typename T>
__device__ __forceinline__ void store_walk_record(T* dst, const T (&r)[kRecWords], T ox, T oy, int pos,
                                                  const Consts<T>& cs) {
    const T kq = neg_half_log2e<T>();
    const T lop = log2_of<T>(r[5]);
    T w[kWalkWords];
    w[kWMu] = r[0] - ox;
    w[kWMv] = r[1] - oy;
    w[kWA] = kq * r[2];
    w[kWM] = kq * r[3];
    w[kWC] = kq * r[4];
    w[kWLop] = lop;
    w[kWThr] = max(fmadd(kq, cs.q_max, lop), log2_of<T>(cs.alpha_min));
    w[kWPos] = id_to_word<T>(pos);
    w[kWZ] = r[6];
    w[kWId] = r[7];
    w[kWR] = r[8];
    w[kWG] = r[9];
    w[kWB] = r[10];
    w[13] = w[14] = w[15] = T(0);
    if constexpr (sizeof(T) == 4) {
        float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
        for (int q = 0; q < 4; ++q) d4[q] = make_float4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < kWalkWords; ++k) dst[k] = w[k];
    }
}

// The exponent E at the pixel centre (u, v) of the tile (offsets from its
// corner), as du p + dv r + log2 o with (du, dv) its offset from the mean and
// (p, r) = (a du + b dv, b du + c dv), the scaled conic times (du, dv): half
// the gradient of E with respect to (du, dv), which the backward reuses.
template <typename T>
__device__ __forceinline__ T walk_exponent(const T* w, T u, T v, T& du, T& dv, T& p, T& r) {
    du = u - w[kWMu];
    dv = v - w[kWMv];
    p = fmadd(w[kWA], du, w[kWM] * dv);
    r = fmadd(w[kWC], dv, w[kWM] * du);
    return fmadd(du, p, fmadd(dv, r, w[kWLop]));
}

// The first kRecWords values of a splat record from global memory into
// registers; the pad value (word 11) is not loaded (set to zero).  Loading it
// into a register the compiler counts as free would make the next write of
// that register wait for the load, and with it for every load before.
template <typename T>
__device__ __forceinline__ void load_splat_global(T (&r)[kRecWords], const T* src) {
#pragma unroll
    for (int k = 0; k < kRecWords - 1; ++k) r[k] = src[k];
    r[kRecWords - 1] = T(0);
}
template <>
__device__ __forceinline__ void load_splat_global<float>(float (&r)[kRecWords], const float* src) {
    const float4* s4 = reinterpret_cast<const float4*>(src);
    const float4 a = s4[0], b = s4[1];
    const float3 c = *reinterpret_cast<const float3*>(src + 8);
    r[0] = a.x; r[1] = a.y; r[2] = a.z; r[3] = a.w;
    r[4] = b.x; r[5] = b.y; r[6] = b.z; r[7] = b.w;
    r[8] = c.x; r[9] = c.y; r[10] = c.z;
    r[11] = 0.0f;
}
// The walked values of a splat record and the slot of its (tile tx, ty) pair:
// the item's first slot plus the tile's place in its rectangle, row-major
// (the record's last four values, the same 64-byte line in FP32).
template <typename T>
__device__ __forceinline__ uint32_t load_splat_slot(T (&r)[kRecWords], const T* src, int tx, int ty) {
    load_splat_global<T>(r, src);
    const uint32_t base = (uint32_t)word_to_id<T>(src[kSpSlot]);
    const uint32_t xy = (uint32_t)word_to_id<T>(src[kSpRect]);
    const uint32_t w = (uint32_t)word_to_id<T>(src[kSpRectW]);
    return base + (uint32_t)(ty - (int)(xy >> 16)) * w + (uint32_t)(tx - (int)(xy & 0xFFFFu));
}
template <>
__device__ __forceinline__ uint32_t load_splat_slot<float>(float (&r)[kRecWords], const float* src, int tx, int ty) {
    load_splat_global<float>(r, src);
    const float3 t = *reinterpret_cast<const float3*>(src + kSpSlot);  // the pad after them is not loaded either
    const uint32_t base = __float_as_uint(t.x), xy = __float_as_uint(t.y), w = __float_as_uint(t.z);
    return base + (uint32_t)(ty - (int)(xy >> 16)) * w + (uint32_t)(tx - (int)(xy & 0xFFFFu));
}

// Whether a splat can contribute at any rendered pixel centre of a tile,
// whose centres lie in the box [bx0, bx1] x [by0, by1]: the smallest
// Mahalanobis form Q over the box (Q is convex: 0 where the mean lies in the
// box, else the least of the four edge minima, each edge's at its clamped
// stationary point) against q_max, and the largest alpha, o exp(-Q_min / 2),
// against alpha_min.  About a quarter of the (tile, Gaussian) pairs that the
// 3-sigma box puts in a tile fail it.  Both bounds keep a margin, so the
// per-pixel tests, evaluated in other arithmetic, can never accept a splat
// this rejects: skipping the rejected ones leaves every result bitwise the
// same (a rejected splat would carry zero weight at every pixel).
template <typename T>
__device__ __forceinline__ bool tile_may_contribute(const T (&sp)[kRecWords], int px0, int px1, int py0, int py1,
                                                    const Consts<T>& cs) {
    if (px0 > px1 || py0 > py1) return false;
    const T bx0 = T(px0) + T(0.5), bx1 = T(px1) + T(0.5), by0 = T(py0) + T(0.5), by1 = T(py1) + T(0.5);
    const T mx = sp[0], my = sp[1], A = sp[2], B = sp[3], C = sp[4];
    auto qf = [&](T dx, T dy) { return fmadd(A * dx, dx, fmadd(T(2) * B * dx, dy, C * dy * dy)); };
    // approximate reciprocals: they only move the clamped stationary points,
    // where Q is flat to first order, far inside the bounds' margins
    const T iA = fast_rcp<T>(A), iC = fast_rcp<T>(C);
    T q = T(0);
    if (!(mx >= bx0 && mx <= bx1 && my >= by0 && my <= by1)) {
        const T ex0 = bx0 - mx, ex1 = bx1 - mx, ey0 = by0 - my, ey1 = by1 - my;
        q = min(min(qf(ex0, min(max(-B * ex0 * iC, ey0), ey1)), qf(ex1, min(max(-B * ex1 * iC, ey0), ey1))),
                min(qf(min(max(-B * ey0 * iA, ex0), ex1), ey0), qf(min(max(-B * ey1 * iA, ex0), ex1), ey1)));
    }
    return q <= cs.q_max * T(1.001) + T(1e-3) && sp[5] * fast_exp<T>(T(-0.5) * q) >= cs.alpha_min * T(0.999);
}

// The pixels of a tile that are rendered (inside the image and the view's
// window): columns [px0, px1], rows [py0, py1] (empty when px0 > px1 or
// py0 > py1).  Wave-uniform integers.
template <typename T>
__device__ __forceinline__ void tile_pixel_box(const Views<T>& V, int view, int tx, int ty, int TW, int TH, int& px0,
                                               int& px1, int& py0, int& py1) {
    const DevCam<T>& c = V.cam[view];
    px0 = max(tx * TW, c.win_x0);
    px1 = min(tx * TW + TW, c.win_x1) - 1;
    py0 = max(ty * TH, c.win_y0);
    py1 = min(ty * TH + TH, c.win_y1) - 1;
}

// Number of set bits of a wave-wide ballot below this lane.
__device__ __forceinline__ int rank_below(uint64_t bal) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
}

// Records whose contribution tests are evaluated together (FP32; FP64 keeps 4
// to bound register use).
#ifndef DQO_FWD_GROUP
#define DQO_FWD_GROUP 8
#endif
template <typename T>
constexpr int fwd_group() { return (sizeof(T) == 8 && DQO_FWD_GROUP > 4) ? 4 : DQO_FWD_GROUP; }

// PROBS: with the instance channels; NB: with the per-pixel blend count.
template <typename T, int TW, int TH, bool PROBS, bool NB = true>
__global__ __launch_bounds__(TW* TH) void render_forward_kernel(
    Views<T> V, Consts<T> cs, int K, const T* __restrict__ splats, uint32_t* __restrict__ pvals,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ schedule, T* __restrict__ color, T* __restrict__ depth, T* __restrict__ tfinal,
    int32_t* __restrict__ last, T* __restrict__ probs, int32_t* __restrict__ idmap,
    const int32_t* __restrict__ target, T* __restrict__ ptarget, int32_t* __restrict__ nblend, uint32_t cap,
    uint32_t M, T* __restrict__ ckpt, uint32_t ckpt_cap,
    int32_t* __restrict__ tile_last, const uint32_t* __restrict__ seg_base, uint4* __restrict__ seg_list,
    uint32_t seg_cap, Ctrl* __restrict__ ctrl) {
    constexpr int BLOCK = TW * TH;
    constexpr int NW = BLOCK / kWave;
    __shared__ __align__(16) T s_sp[BLOCK * kWalkWords];
    __shared__ int s_wc[NW];
    extern __shared__ unsigned char s_dyn[];
    T* s_P = reinterpret_cast<T*>(s_dyn);  // [K][BLOCK] when PROBS

    const int tid = threadIdx.x;
    const int tile = (int)min(schedule[blockIdx.x], (uint32_t)(gridDim.x - 1));
    const int view = tile / V.tiles_per_view;
    const int t = tile - view * V.tiles_per_view;
    const int ty = t / V.tiles_x, tx = t - ty * V.tiles_x;
    const int px = tx * TW + (tid % TW), py = ty * TH + (tid / TW);
    // pixels of the image outside the view's window are written as empty
    const bool in_img = px < V.W && py < V.H;
    const bool inside = in_img && in_window(V.cam[view], px, py);
    const int64_t HW = (int64_t)V.W * V.H;
    const int64_t pix = (int64_t)py * V.W + px;
    // the pixel centre relative to the tile's corner
    const T u = T(tid % TW) + T(0.5), v = T(tid / TW) + T(0.5);
    const T ox = T(tx * TW), oy = T(ty * TH);
    const uint32_t re = min(ranges[2 * tile + 1], cap), rs = min(ranges[2 * tile], re);
    const uint32_t sbase = (BLOCK == kWave && ckpt) ? seg_base[tile] : 0u;  // used at the end
#ifndef DQO_FWD_PRIO
#define DQO_FWD_PRIO 0
#endif
    if constexpr (DQO_FWD_PRIO == 1) {
        if (blockIdx.x < gridDim.x / 8u) __builtin_amdgcn_s_setprio(3);
    } else if constexpr (DQO_FWD_PRIO == 2) {
        const uint32_t len = re - rs;
        if (len > 512u) __builtin_amdgcn_s_setprio(3);
        else if (len > 256u) __builtin_amdgcn_s_setprio(2);
        else if (len > 128u) __builtin_amdgcn_s_setprio(1);
    } else if constexpr (DQO_FWD_PRIO == 3) {
        const uint32_t q = blockIdx.x * 4u / gridDim.x;
        if (q == 0u) __builtin_amdgcn_s_setprio(3);
        else if (q == 1u) __builtin_amdgcn_s_setprio(2);
        else if (q == 2u) __builtin_amdgcn_s_setprio(1);
    }
    int tgt = -2;
    if (target && in_img) tgt = job_target(V.cam[view].job, target[view * HW + pix]);
    if (PROBS)
        for (int k = 0; k < K; ++k) s_P[k * BLOCK + tid] = T(0);

    T Tt = T(1), c0 = T(0), c1 = T(0), c2 = T(0), dd = T(0), pt = T(0);
    int lastpos = -1, nb_count = 0;
    bool done = !inside;
    int bx0, bx1, by0, by1;
    tile_pixel_box<T>(V, view, tx, ty, TW, TH, bx0, bx1, by0, by1);
    const int lane = tid & (kWave - 1), wave = tid / kWave;
    // Software prefetch: this lane's record of the next batch is loaded into
    // registers while the current batch is walked; the pair index one batch
    // further ahead is loaded one step earlier still.
    T pf[kRecWords];
    uint32_t pv = (rs + tid < re) ? pvals[rs + tid] : 0u, rec2 = 0u;
    if (rs + tid < re) load_splat_global<T>(pf, splats + (size_t)min(pv & kPairItem, M - 1) * kSplatWords);
    // (the index is masked and clamped where it is used: doing it here would
    // wait for the load, and with it for every load issued before)
    if (rs + BLOCK + tid < re) rec2 = pvals[rs + BLOCK + tid];
    for (uint32_t b0 = rs; b0 < re; b0 += BLOCK) {
        if (__syncthreads_count(!done) == 0) break;
        if constexpr (BLOCK == kWave) {
            // State before each segment boundary of the pair range, for the
            // segmented backward (which restarts there).
            const uint32_t rel = b0 - rs;
            if (ckpt && rel > 0 && rel % kSegLen == 0 && rel / kSegLen < (uint32_t)kSegMax) {
                const uint32_t e = boundary_record(rs, rel / kSegLen);
                if (e < ckpt_cap) {
                    T* c = ckpt + (size_t)e * 6 * kWave + tid;
                    c[0 * kWave] = Tt;
                    c[1 * kWave] = c0;
                    c[2 * kWave] = c1;
                    c[3 * kWave] = c2;
                    c[4 * kWave] = dd;
                    c[5 * kWave] = pt;
                }
            }
        }
        // The batch's records that may contribute somewhere in the tile, in
        // order, compacted into LDS with their positions in the pad word.
        const bool cand = (b0 + tid < re) && tile_may_contribute<T>(pf, bx0, bx1, by0, by1, cs);
        // the others are marked for the backward, which then skips them
        if (b0 + tid < re && !cand && !(pv & kPairSkip)) pvals[b0 + tid] = pv | kPairSkip;
        const uint64_t bal = __ballot(cand);
        int nb = __popcll(bal), off = 0;
        if constexpr (NW > 1) {
            if (lane == 0) s_wc[wave] = nb;
            __syncthreads();
            nb = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                off += (w < wave) ? s_wc[w] : 0;
                nb += s_wc[w];
            }
        }
        if (cand) {
            store_walk_record<T>(s_sp + (off + rank_below(bal)) * kWalkWords, pf, ox, oy, (int)(b0 + tid), cs);
        }
        __syncthreads();
        pv = rec2;
        if (b0 + BLOCK + tid < re) load_splat_global<T>(pf, splats + (size_t)min(pv & kPairItem, M - 1) * kSplatWords);
        if (b0 + 2 * BLOCK + tid < re) rec2 = pvals[b0 + 2 * BLOCK + tid];
        if (!wave_any(!done)) continue;
        // Groups of fwd_group<T>() records: their contribution tests (exponent,
        // exponential, threshold) are independent and evaluated side
        // by side, which hides the VALU and LDS latency that one wavefront
        // per SIMD would otherwise expose; only the transmittance recurrence
        // then runs serially, in depth order, with the same arithmetic as a
        // one-by-one walk.
        constexpr int kFwdGroup = fwd_group<T>();
        for (int j0 = 0; j0 < nb; j0 += kFwdGroup) {
            // the test words (and positions) of the group first; the blending
            // words are read only where the group has a contribution
            T rec[kFwdGroup][kWPos + 1];
            T a0[kFwdGroup];
            bool c0k[kFwdGroup];
            bool any = false;
#pragma unroll
            for (int k = 0; k < kFwdGroup; ++k) {
                const T* w = s_sp + min(j0 + k, nb - 1) * kWalkWords;
#pragma unroll
                for (int q = 0; q <= kWPos; ++q) rec[k][q] = w[q];
            }
#pragma unroll
            for (int k = 0; k < kFwdGroup; ++k) {
                T dx, dy, pp, rr;
                const T E = walk_exponent(rec[k], u, v, dx, dy, pp, rr);
                a0[k] = min(exp2_of<T>(E), cs.alpha_max);
                c0k[k] = (j0 + k < nb) && (E >= rec[k][kWThr]);
                any = any || c0k[k];
            }
            if (!wave_any(any && !done)) continue;
            T bl[kFwdGroup][kWB - kWZ + 1];  // depth, id, colour of each record
#pragma unroll
            for (int k = 0; k < kFwdGroup; ++k) {
                const T* w = s_sp + min(j0 + k, nb - 1) * kWalkWords;
#pragma unroll
                for (int q = kWZ; q <= kWB; ++q) bl[k][q - kWZ] = w[q];
            }
            // (taken as written here: the reads are issued together and
            // waited for once, not one record at a time inside the recurrence)
#pragma unroll
            for (int k = 0; k < kFwdGroup; ++k)
#pragma unroll
                for (int q = 0; q <= kWB - kWZ; ++q) asm volatile("" : "+v"(bl[k][q]));
#pragma unroll
            for (int k = 0; k < kFwdGroup; ++k) {
                const T* bw = bl[k] - kWZ;
                const bool contrib = c0k[k] && !done;
                const T a = contrib ? a0[k] : T(0);
                const T Tn = Tt * (T(1) - a);
                const bool stop = contrib && (Tn < cs.t_min);
                const T w = stop ? T(0) : a * Tt;
                c0 = fmadd(w, bw[kWR], c0);
                c1 = fmadd(w, bw[kWG], c1);
                c2 = fmadd(w, bw[kWB], c2);
                dd = fmadd(w, bw[kWZ], dd);
                const int id = word_to_id<T>(bw[kWId]);
                pt += (id == tgt) ? w : T(0);
                const bool blended = w != T(0);
                lastpos = blended ? word_to_id<T>(rec[k][kWPos]) : lastpos;
                if constexpr (NB) nb_count += blended ? 1 : 0;
                if (PROBS && blended && id >= 0 && id < K) s_P[id * BLOCK + tid] += w;
                Tt = stop ? Tt : Tn;
                done = done || stop;
            }
            if (!wave_any(!done)) break;
        }
    }
    if constexpr (BLOCK == kWave) {
        if (ckpt) {
            // The tile's last blended position: how far its backward has work.
            int m = lastpos;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) m = max(m, __shfl_xor(m, d));
            if (tid == 0) tile_last[tile] = m;
            // The tile's entries of the backward's segment list, at the place
            // the sort reserved for its segments: every 64-pair segment up to
            // the last blended position, with the end of its walk (one past
            // that position when it lies in the segment) and the boundary
            // record at its end (none where no pixel blends past it: the
            // segment holding the last blended position and the range's
            // last); the segments behind are marked empty (no walk).
            const uint32_t nseg = tile_segments(re - rs);
            const uint32_t k = (m >= (int)rs && m < (int)re) ? min(((uint32_t)m - rs) / (uint32_t)kSegLen + 1u, nseg) : 0u;
            const uint32_t last_end = (uint32_t)m + 1u;
            for (uint32_t j = (uint32_t)tid; j < nseg; j += kWave) {
                const uint32_t pos = sbase + j;
                if (pos >= seg_cap) break;
                const uint32_t s0 = rs + j * (uint32_t)kSegLen;
                const bool tail = j + 1u >= nseg;  // the last segment takes the rest of the range
                const uint32_t s1 = tail ? re : s0 + (uint32_t)kSegLen;
                const bool past = !tail && last_end > s1;
                seg_list[pos] = j < k ? make_uint4((uint32_t)tile, s0, min(last_end, s1), past ? boundary_record(rs, j + 1u) : kNoBoundary)
                                      : make_uint4((uint32_t)tile, 0u, 0u, kNoBoundary);
            }
            if (blockIdx.x == 0 && tid == 0) {
                // the forward these states belong to (checked by the backward)
                ctrl->seg_stamp[0] = ctrl->epoch;
                ctrl->seg_stamp[1] = (uint64_t)(uintptr_t)last;
                ctrl->seg_stamp[2] = (uint64_t)(uintptr_t)target;
            }
        }
    }
    if (!in_img) return;
    const int64_t o = view * HW + pix;
    color[(view * 3 + 0) * HW + pix] = c0 + Tt * cs.bg[0];
    color[(view * 3 + 1) * HW + pix] = c1 + Tt * cs.bg[1];
    color[(view * 3 + 2) * HW + pix] = c2 + Tt * cs.bg[2];
    depth[o] = dd;
    tfinal[o] = Tt;
    last[o] = lastpos;
    if (NB && nblend) nblend[o] = nb_count;
    if (ptarget && target) ptarget[o] = (tgt == -1) ? Tt : pt;
    if (PROBS) {
        int best = K;
        T bv = Tt;
        for (int k = K - 1; k >= 0; --k) {
            const T pk = s_P[k * BLOCK + tid];
            probs[((int64_t)view * K + k) * HW + pix] = pk;
            if (pk >= bv) {
                bv = pk;
                best = k;
            }
        }
        if (idmap) idmap[o] = (best == K) ? -1 : best;
    }
}

// ---------------------------------------------------------------- backward
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;  // pair slot of a record that is not loaded
constexpr int kChunk = 6;  // Gaussians per transposed reduction (6 x 10 = 60 of 64 lanes)

template <typename T, int D, int M>
__device__ __forceinline__ void butterfly_step(T (&v)[64], int lane) {
    const bool up = (lane & D) != 0;
#pragma unroll
    for (int i = 0; i < M / 2; ++i) {
        const T send = up ? v[i] : v[i + M / 2];
        const T keep = up ? v[i + M / 2] : v[i];
        v[i] = keep + __shfl_xor(send, D);
    }
}

// After the call, v[0] of lane L holds the sum over the wave of value L.
template <typename T>
__device__ __forceinline__ void wave_transpose_sum(T (&v)[64], int lane) {
    butterfly_step<T, 32, 64>(v, lane);
    butterfly_step<T, 16, 32>(v, lane);
    butterfly_step<T, 8, 16>(v, lane);
    butterfly_step<T, 4, 8>(v, lane);
    butterfly_step<T, 2, 4>(v, lane);
    butterfly_step<T, 1, 2>(v, lane);
}

// FP32 on gfx950.  The two cross-row levels use v_permlane32_swap /
// v_permlane16_swap: swapping the upper half of x = v[i] with the lower half of
// y = v[i + M/2] and adding the two results leaves, in every lane, the pair sum
// of exactly the value that lane keeps (one swap and one add per value pair).
// The in-row levels pair lanes with DPP row_mirror (lane ^ 15), row_half_mirror
// (lane ^ 7) and quad_perm (lane ^ 2, lane ^ 1); with 32 and 16 these masks are
// linearly independent, so each lane still sums all 64 lanes once, and the lane
// bit that selects the kept half is the same as in the XOR butterfly.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

template <int CTRL, int D, int M>
__device__ __forceinline__ void dpp_step(float (&v)[64], int lane) {
    const bool up = (lane & D) != 0;
#pragma unroll
    for (int i = 0; i < M / 2; ++i) {
        const float send = up ? v[i] : v[i + M / 2];
        const float keep = up ? v[i + M / 2] : v[i];
        v[i] = keep + dpp_mov<CTRL>(send);
    }
}

template <>
__device__ __forceinline__ void wave_transpose_sum<float>(float (&v)[64], int lane) {
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 32]), false,
                                                        false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 16]), false,
                                                        false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    dpp_step<0x140, 8, 16>(v, lane);  // row_mirror: lane ^ 15
    dpp_step<0x141, 4, 8>(v, lane);   // row_half_mirror: lane ^ 7
    dpp_step<0x4E, 2, 4>(v, lane);    // quad_perm [2,3,0,1]: lane ^ 2
    dpp_step<0xB1, 1, 2>(v, lane);    // quad_perm [1,0,3,2]: lane ^ 1
}


template <typename T, int TW, int TH>
__global__ __launch_bounds__(TW* TH) void render_backward_kernel(
    Views<T> V, Consts<T> cs, int K, const T* __restrict__ splats,
    const uint32_t* __restrict__ pvals, const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ schedule,
    const T* __restrict__ tfinal, const int32_t* __restrict__ last, const int32_t* __restrict__ target,
    const T* __restrict__ dC, const T* __restrict__ dD, const T* __restrict__ dT, const T* __restrict__ dP,
    const T* __restrict__ dPt, T* __restrict__ partials, uint8_t* __restrict__ written, uint32_t cap, uint32_t M) {
    constexpr int BLOCK = TW * TH;
    constexpr int NW = BLOCK / kWave;
    __shared__ __align__(16) T s_sp[BLOCK * kWalkWords];
    __shared__ uint32_t s_slot[BLOCK];
    __shared__ T s_red[2][NW][kWave];
    __shared__ int s_maxlast;
    __shared__ int s_wc[NW];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid >> 6;
    const int tile = (int)min(schedule[blockIdx.x], (uint32_t)(gridDim.x - 1));
    const int view = tile / V.tiles_per_view;
    const int t = tile - view * V.tiles_per_view;
    const int ty = t / V.tiles_x, tx = t - ty * V.tiles_x;
    const int px = tx * TW + (tid % TW), py = ty * TH + (tid / TW);
    const bool inside = px < V.W && py < V.H && in_window(V.cam[view], px, py);
    const int64_t HW = (int64_t)V.W * V.H;
    const int64_t pix = (int64_t)py * V.W + px;
    const int64_t o = view * HW + pix;
    // the pixel centre relative to the tile's corner
    const T u = T(tid % TW) + T(0.5), v_px = T(tid / TW) + T(0.5);
    const T ox = T(tx * TW), oy = T(ty * TH);
    const uint32_t re = min(ranges[2 * tile + 1], cap), rs = min(ranges[2 * tile], re);

    int lastp = -1;
    T Tcur = T(1), gc0 = T(0), gc1 = T(0), gc2 = T(0), gd = T(0), gt = T(0), gpt = T(0);
    int tgt = -2;
    if (inside) {
        lastp = last[o];
        if (lastp < (int)rs || lastp >= (int)re) lastp = -1;  // not from this frame's forward: no work
        Tcur = tfinal[o];
        gc0 = dC[(view * 3 + 0) * HW + pix];
        gc1 = dC[(view * 3 + 1) * HW + pix];
        gc2 = dC[(view * 3 + 2) * HW + pix];
        gd = dD ? dD[o] : T(0);
        gt = dT ? dT[o] : T(0);
        if (dPt && target) {
            tgt = job_target(V.cam[view].job, target[o]);
            gpt = dPt[o];
            if (tgt == -1) gt += gpt;
        }
    }
    if (tid == 0) s_maxlast = -1;
    __syncthreads();
    if (lastp >= 0) atomicMax(&s_maxlast, lastp);
    __syncthreads();
    const int maxlast = __builtin_amdgcn_readfirstlane(s_maxlast);  // uniform: scalar walk bounds
    // Pairs behind every pixel's last blended Gaussian are not written and
    // stay unmarked (their partials count as zero).
    const uint32_t hi = (maxlast >= (int)rs) ? (uint32_t)(maxlast + 1) : rs;
    T S = Tcur * (gc0 * cs.bg[0] + gc1 * cs.bg[1] + gc2 * cs.bg[2] + gt);
    int buf = 0;
    for (uint32_t bend = hi; bend > rs;) {
        const uint32_t bstart = (bend - rs > (uint32_t)BLOCK) ? bend - BLOCK : rs;
        const int nbr = (int)(bend - bstart);
        __syncthreads();
        // the batch's records that may contribute in the tile (those the
        // forward did not mark), compacted in order
        T r[kRecWords];
        uint32_t slot = 0u;
        bool cand = false;
        if (tid < nbr) {
            const uint32_t pv = pvals[bstart + tid];
            if (!(pv & kPairSkip)) {
                slot = load_splat_slot<T>(r, splats + (size_t)min(pv, M - 1) * kSplatWords, tx, ty);
                cand = true;
            }
        }
        const uint64_t bal = __ballot(cand);
        if (lane == 0) s_wc[wave] = __popcll(bal);
        __syncthreads();
        int nb = 0, off = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            off += (w < wave) ? s_wc[w] : 0;
            nb += s_wc[w];
        }
        if (cand) {
            const int q = off + rank_below(bal);
            store_walk_record<T>(s_sp + q * kWalkWords, r, ox, oy, (int)(bstart + tid), cs);
            s_slot[q] = slot;
        }
        __syncthreads();
        for (int c0 = nb - 1; c0 >= 0; c0 -= kChunk) {
            T v[64];
#pragma unroll
            for (int k = 0; k < 64; ++k) v[k] = T(0);
            bool any = false;
#pragma unroll
            for (int c = 0; c < kChunk; ++c) {
                const int jl = c0 - c;
                if (jl < 0) break;
                const T* sp = s_sp + jl * kWalkWords;
                T dx, dy, pp, rr;
                const T E = walk_exponent(sp, u, v_px, dx, dy, pp, rr);
                const bool contrib = (E >= sp[kWThr]) && (word_to_id<T>(sp[kWPos]) <= lastp);
                if (!wave_any(contrib)) continue;
                const T araw = exp2_of<T>(E);
                const bool clamped = !(araw < cs.alpha_max);
                const T a0 = clamped ? cs.alpha_max : araw;
                any = true;
                const T a = contrib ? a0 : T(0);
                const T roma = fast_rcp<T>(T(1) - a);
                const T Ti = Tcur * roma;
                const T w = a * Ti;
                const int id = word_to_id<T>(sp[kWId]);
                T vv = fmadd(gc0, sp[kWR], fmadd(gc1, sp[kWG], fmadd(gc2, sp[kWB], gd * sp[kWZ])));
                vv += (tgt >= 0 && id == tgt) ? gpt : T(0);
                if (dP && contrib && id >= 0 && id < K) vv += dP[((int64_t)view * K + id) * HW + pix];
                const T dalpha = contrib ? (Ti * vv - S * roma) : T(0);
                S = fmadd(w, vv, S);
                Tcur = Ti;
                v[c * kGradWords + 6] = gc0 * w;
                v[c * kGradWords + 7] = gc1 * w;
                v[c * kGradWords + 8] = gc2 * w;
                v[c * kGradWords + 9] = gd * w;
                // dq = -2 dL/dQ; the conic rows from the exponent's (p, r)
                const T dq = clamped ? T(0) : dalpha * a;
                const T iq = T(1) / neg_half_log2e<T>();
                v[c * kGradWords + 5] = dq;  // o dL/do (the opacity's sum is divided by o)
                v[c * kGradWords + 0] = dq * iq * pp;
                v[c * kGradWords + 1] = dq * iq * rr;
                v[c * kGradWords + 2] = T(-0.5) * dq * dx * dx;
                v[c * kGradWords + 3] = -dq * dx * dy;
                v[c * kGradWords + 4] = T(-0.5) * dq * dy * dy;
            }
            if (wave_any(any)) wave_transpose_sum<T>(v, lane);
            if constexpr (NW == 1) {
                // one wavefront per tile: the transposed sums are the block sums
                const int c = lane / kGradWords;
                const int jl = c0 - c;
                if (lane < kChunk * kGradWords && jl >= 0) {
                    const uint32_t slot = s_slot[jl];
                    if (slot < cap) {
                        partials[(size_t)slot * kGradWords + (lane - c * kGradWords)] = v[0];
                        if (lane == c * kGradWords) written[slot] = 1;
                    }
                }
                continue;
            }
            s_red[buf][wave][lane] = v[0];
            __syncthreads();
            if (tid < kChunk * kGradWords) {
                const int c = tid / kGradWords;
                const int jl = c0 - c;
                if (jl >= 0) {
                    T sum = T(0);
#pragma unroll
                    for (int w2 = 0; w2 < NW; ++w2) sum += s_red[buf][w2][tid];
                    const uint32_t slot = s_slot[jl];
                    if (slot < cap) {
                        partials[(size_t)slot * kGradWords + (tid - c * kGradWords)] = sum;
                        if (tid == c * kGradWords) written[slot] = 1;
                    }
                }
            }
            buf ^= 1;
        }
        bend = bstart;
    }
}

// Backward for 64-pixel tiles: the workgroup is one wavefront, so the
// transposed wave sums are already the tile sums and no barrier is needed
// between chunks.  The conic words are summed without their constant factors
// (-1/2 on the two diagonal words, -1 on the mixed one), which the lane that
// stores a word's sum applies once.  Only Gaussians that contribute somewhere in the tile take a
// reduction slot: the walk finds the next contributing Gaussian, fills slot c
// (c = 0..5, a separate statically indexed code section each, so the slot
// values stay in fixed registers), and after six slots the wave transposes and
// sums them.  Pairs that take no slot are not written (unmarked: zero
// partials).  Every take writes all
// ten values of its slot, so nothing is cleared between chunks: the values
// past the NS filled slots are set to zero here, as constants.
template <int NS, typename T>
__device__ __forceinline__ void flush_slots(T (&v)[64], uint32_t chunk, T* __restrict__ partials,
                                            uint8_t* __restrict__ written, uint32_t cap) {
    // The lane's place in the transposed sums, derived here at each flush (an
    // opaque copy of the lane index keeps the compiler from hoisting it out
    // of the walk, where these values would only occupy registers).
    int lane = (int)__lane_id();
    asm volatile("" : "+v"(lane));
    const int lane_slot = (lane * 205) >> 11;  // lane / kGradWords for lane < 64
    const int word = lane - lane_slot * kGradWords;
#pragma unroll
    for (int k = NS * kGradWords; k < 64; ++k) v[k] = T(0);
    wave_transpose_sum<T>(v, lane);
    const uint32_t slot = (uint32_t)__shfl((int)chunk, lane_slot);
    if (lane < NS * kGradWords) {
        if (slot < cap) {
            const T factor = (word <= 1) ? T(1) / neg_half_log2e<T>()
                             : (word == 2 || word == 4) ? T(-0.5) : (word == 3) ? T(-1) : T(1);
            partials[(size_t)slot * kGradWords + word] = v[0] * factor;
            if (word == 0) written[slot] = 1;
        }
    }
}

template <int C>
struct SlotIdx {
    static constexpr int value = C;
};

template <typename T, int TW, int TH, bool PROBS, bool PREFETCH>
__device__ __forceinline__ void backward_unit(
    const Views<T>& V, const Consts<T>& cs, int K, const T* __restrict__ splats,
    const uint32_t* __restrict__ pvals, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ schedule, const T* __restrict__ tfinal, const int32_t* __restrict__ last,
    const int32_t* __restrict__ target, const T* __restrict__ dC, const T* __restrict__ dD, const T* __restrict__ dT,
    const T* __restrict__ dP, const T* __restrict__ dPt, T* __restrict__ partials, uint8_t* __restrict__ written,
    uint32_t cap, uint32_t M, const uint4* __restrict__ seg_list, const T* __restrict__ ckpt, uint32_t ckpt_cap,
    const T* __restrict__ color, const T* __restrict__ depth, const T* __restrict__ ptarget, T* s_sp,
    uint32_t* s_slot, uint32_t unit) {
    const int lane = threadIdx.x;
    const uint32_t n_tiles = (uint32_t)(V.n_views * V.tiles_per_view);
    // A listed segment comes with its walk [s0, hi) and the boundary record
    // at its end (pixels blending past s1 restart from it); a whole tile
    // walks its range up to its pixels' last blended position.
    int tile;
    uint32_t s0, s1, hi_seg = 0u, bnd = kNoBoundary;
    if (seg_list) {
        const uint4 en = seg_list[unit];
        if (en.z <= en.y) return;  // a segment behind its tile's last blended position (uniform)
        tile = (int)min(en.x, n_tiles - 1u);
        s0 = min(en.y, cap);
        hi_seg = min(max(en.z, s0), cap);
        bnd = en.w;
        s1 = (bnd == kNoBoundary) ? 0xFFFFFFFFu : s0 + (uint32_t)kSegLen;
    } else {
        tile = (int)min(schedule[unit], n_tiles - 1u);
        s0 = min(ranges[2 * tile], cap);
        s1 = min(ranges[2 * tile + 1], cap);
    }
    const int view = tile / V.tiles_per_view;
    const int t = tile - view * V.tiles_per_view;
    const int ty = t / V.tiles_x, tx = t - ty * V.tiles_x;
    const int px = tx * TW + (lane % TW), py = ty * TH + (lane / TW);
    const bool inside = px < V.W && py < V.H && in_window(V.cam[view], px, py);
    const int64_t HW = (int64_t)V.W * V.H;
    const int64_t pix = (int64_t)py * V.W + px;
    const int64_t o = view * HW + pix;
    // the pixel centre relative to the tile's corner
    const T u = T(lane % TW) + T(0.5), v_px = T(lane / TW) + T(0.5);
    const T ox = T(tx * TW), oy = T(ty * TH);

    // Batches of up to 64 pairs, from the walk's end down.  A listed
    // segment knows where its walk ends, so the first batch's pair indices
    // are loaded before the pixels' values, and its records (which need the
    // indices) right after them; the pixel values are used only then.
    auto batch_lo = [&](uint32_t e) { return (e - s0 > (uint32_t)kWave) ? e - kWave : s0; };
    uint32_t rec_first = 0u;
    if (seg_list && lane < (int)(hi_seg - batch_lo(hi_seg))) rec_first = pvals[batch_lo(hi_seg) + lane];

    int lastp = -1;
    T Tcur = T(1), gc0 = T(0), gc1 = T(0), gc2 = T(0), gd = T(0), gt = T(0), gpt = T(0);
    int tgt = -2, tgt_raw = -1;
    T ck[6] = {}, col0 = T(0), col1 = T(0), col2 = T(0), dep = T(0), ptg = T(0);
    if (inside) {
        lastp = last[o];
        Tcur = tfinal[o];
        gc0 = dC[(view * 3 + 0) * HW + pix];
        gc1 = dC[(view * 3 + 1) * HW + pix];
        gc2 = dC[(view * 3 + 2) * HW + pix];
        gd = dD ? dD[o] : T(0);
        gt = dT ? dT[o] : T(0);
        if (dPt && target) {
            tgt_raw = target[o];
            gpt = dPt[o];
        }
        if (bnd != kNoBoundary) {
            // Some pixels blend past this segment: they restart at its end
            // from the state the forward stored there (loaded for every
            // pixel, beside the values above).
            const T* c = ckpt + (size_t)min(bnd, ckpt_cap - 1u) * 6 * kWave + lane;
#pragma unroll
            for (int q = 0; q < 6; ++q) ck[q] = c[q * kWave];
            col0 = color[(view * 3 + 0) * HW + pix];
            col1 = color[(view * 3 + 1) * HW + pix];
            col2 = color[(view * 3 + 2) * HW + pix];
            dep = depth[o];
            ptg = ptarget ? ptarget[o] : T(0);
        }
    }
    // A lane's record of a batch and its pair slot (kNoSlot: a pair the
    // forward marked as contributing nowhere in the tile, not loaded).
    T pf[kRecWords];
    uint32_t pf_slot = kNoSlot;
    auto load_pair = [&](uint32_t pv) {
        if (pv & kPairSkip) pf_slot = kNoSlot;
        else pf_slot = load_splat_slot<T>(pf, splats + (size_t)min(pv, M - 1) * kSplatWords, tx, ty);
    };
    if (seg_list && lane < (int)(hi_seg - batch_lo(hi_seg))) load_pair(rec_first);

    bool restart = false;
    T S_restart = T(0);
    if (inside) {
        // nothing in this segment (whole tiles: nothing of this frame's)
        if (lastp < (int)s0 || (!seg_list && lastp >= (int)s1)) lastp = -1;
        if (dPt && target) {
            tgt = job_target(V.cam[view].job, tgt_raw);
            if (tgt == -1) gt += gpt;
        }
        if (bnd != kNoBoundary) {
            // The sum behind the boundary is the total minus the part in front
            // of it (colour without the background term, depth, target
            // probability).
            if (lastp >= (int)s1) {
                const T Tf = Tcur;
                const T behind = gc0 * ((col0 - Tf * cs.bg[0]) - ck[1]) + gc1 * ((col1 - Tf * cs.bg[1]) - ck[2]) +
                                 gc2 * ((col2 - Tf * cs.bg[2]) - ck[3]) + gd * (dep - ck[4]) +
                                 (tgt >= 0 ? gpt * (ptg - ck[5]) : T(0));
                S_restart = behind + Tf * (gc0 * cs.bg[0] + gc1 * cs.bg[1] + gc2 * cs.bg[2] + gt);
                Tcur = ck[0];
                lastp = (int)s1 - 1;
                restart = true;
            }
        }
    }
    // Pairs behind every pixel's last blended Gaussian, and pairs that
    // contribute nowhere in the tile, are not written and stay unmarked
    // (their partials count as zero).
    uint32_t hi = hi_seg;
    if (!seg_list) {
        int maxlast = lastp;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) maxlast = max(maxlast, __shfl_xor(maxlast, d));
        // Equal in every lane; said so, the walk state derived from it lives
        // in scalar registers and the loop control is scalar branches
        // (measured 10% faster than the same walk with its state in vector
        // registers).
        maxlast = __builtin_amdgcn_readfirstlane(maxlast);
        hi = (maxlast >= (int)s0) ? (uint32_t)(maxlast + 1) : s0;
    }
    T S = restart ? S_restart : Tcur * (gc0 * cs.bg[0] + gc1 * cs.bg[1] + gc2 * cs.bg[2] + gt);
    T v[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) v[k] = T(0);
    uint32_t chunk = 0u;  // lane c < kChunk: the pair slot of the Gaussian in reduction slot c
    // the target-probability gradient joins a Gaussian's colour sum where its
    // object is the pixel's target (tgt -1: T_final's gradient carries it)
    const T gpt_obj = tgt >= 0 ? gpt : T(0);
    // walk state (wave-uniform): the LDS batch holds positions [bstart, bend)
    uint32_t bend = hi, bstart = hi;
    int jl = -1;
    // contribution state of the Gaussian found by `next`, zero in the lanes
    // it does not blend: alpha, and alpha where it is not clamped (the factor
    // of alpha's derivatives)
    const T* sp = s_sp;
    T dx = T(0), dy = T(0), a = T(0), a_free = T(0), pp = T(0), rr = T(0);

    // The first batch is A = [a_s, a_e) (already loaded for a listed
    // segment).  With PREFETCH (whole tiles: many batches) the next batch's
    // records are held in registers while the current one is walked, and the
    // pair indices of the batch after it (B) are loaded one step earlier
    // still; without it (segments: mostly one batch) later batches are
    // loaded when reached, and the record registers are free during the walk.
    uint32_t a_e = hi, a_s = batch_lo(hi);
    if (!seg_list && lane < (int)(a_e - a_s)) load_pair(pvals[a_s + lane]);
    uint32_t b_e = a_s, b_s = batch_lo(a_s), rec_b = 0u;
    // (clamped where used, so that nothing waits for this load early)
    if constexpr (PREFETCH) rec_b = (lane < (int)(b_e - b_s)) ? pvals[b_s + lane] : 0u;
    bool first_batch = true;

    // The walk record of the Gaussian being tested, read from LDS (16-byte
    // broadcast reads at a 24-bit multiply of its index; the compiler issues
    // each where its values are first used).
    T cur[kWPos + 1];
    auto lds_rec = [&](int j) {
        if constexpr (sizeof(T) == 4) {
            const float4* s4 = reinterpret_cast<const float4*>(reinterpret_cast<const char*>(s_sp) +
                                                               __mul24(j, (int)(kWalkWords * sizeof(T))));
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const float4 a = s4[q];
                cur[4 * q] = a.x;
                cur[4 * q + 1] = a.y;
                cur[4 * q + 2] = a.z;
                cur[4 * q + 3] = a.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k <= kWPos; ++k) cur[k] = s_sp[j * kWalkWords + k];
        }
    };
    // Advances to the next Gaussian (descending) that contributes at some pixel
    // of the tile; false at the end of the range.  The two wave-wide tests are
    // ballots of single comparisons combined as masks, which keeps them in
    // scalar instructions.
    auto next = [&]() -> bool {
        for (;;) {
            if (jl < 0) {
                if (a_e <= a_s) return false;
                bend = a_e;
                bstart = a_s;
                const int nbr = (int)(bend - bstart);
                if constexpr (!PREFETCH) {
                    if (!first_batch && lane < nbr) load_pair(pvals[bstart + lane]);
                    first_batch = false;
                }
                __syncthreads();
                // the records that may contribute in the tile (those the
                // forward did not mark), compacted in order
                const bool cand = lane < nbr && pf_slot != kNoSlot;
                const uint64_t bal = __builtin_amdgcn_ballot_w64(cand);
                if (cand) {
                    const int q = rank_below(bal);
                    store_walk_record<T>(s_sp + q * kWalkWords, pf, ox, oy, (int)(bstart + lane), cs);
                    s_slot[q] = pf_slot;
                }
                __syncthreads();
                jl = __popcll(bal) - 1;
                a_e = b_e;
                a_s = b_s;
                b_e = a_s;
                b_s = batch_lo(a_s);
                if constexpr (PREFETCH) {
                    if (lane < (int)(a_e - a_s)) load_pair(rec_b);
                    rec_b = (lane < (int)(b_e - b_s)) ? pvals[b_s + lane] : 0u;
                }
                if (jl < 0) continue;  // nothing in this batch can contribute
            }
            lds_rec(jl);
            sp = cur;
            const T E = walk_exponent(sp, u, v_px, dx, dy, pp, rr);
            const T araw = exp2_of<T>(E);
            const bool clamped = !(araw < cs.alpha_max);
            const T a0 = clamped ? cs.alpha_max : araw;  // min(araw, alpha_max), one select
            const bool contrib = (E >= sp[kWThr]) & (word_to_id<T>(sp[kWPos]) <= lastp);
            a = contrib ? a0 : T(0);
            if (__builtin_amdgcn_ballot_w64(a != T(0)) == 0ull) {
                --jl;
                continue;
            }
            a_free = clamped ? T(0) : a;
            return true;
        }
    };
    // Gradient of the found Gaussian into slot C; advances the walk.
    // In the lanes the Gaussian does not blend, a = 0 leaves T and S as they
    // are and zeroes every word (w = 0, a_free = 0).
    auto take = [&](auto cidx) {
        constexpr int C = decltype(cidx)::value;
        const T roma = fast_rcp<T>(T(1) - a);
        const T Ti = Tcur * roma;
        const T w = a * Ti;
        const T* bw = s_sp + jl * kWalkWords;  // the blending words
        const int id = word_to_id<T>(bw[kWId]);
        T vv = fmadd(gc0, bw[kWR], fmadd(gc1, bw[kWG], fmadd(gc2, bw[kWB], gd * bw[kWZ])));
        vv += (id == tgt) ? gpt_obj : T(0);
        if constexpr (PROBS) {
            if (a != T(0) && id >= 0 && id < K) vv += dP[((int64_t)view * K + id) * HW + pix];
        }
        const T dalpha = fmadd(Ti, vv, -(S * roma));
        S = fmadd(w, vv, S);
        Tcur = Ti;
        // dq = -2 dL/dQ: the mean words are dq (p, r) (the scaled conic
        // times the offset), the conic words dq dx^2, dq dx dy, dq dy^2, each
        // before its constant factor; the opacity word is dq = o dL/do
        const T dq = dalpha * a_free;
        const T t1 = dq * dx, t2 = dq * dy;
        v[C * kGradWords + 0] = dq * pp;
        v[C * kGradWords + 1] = dq * rr;
        v[C * kGradWords + 2] = t1 * dx;
        v[C * kGradWords + 3] = t1 * dy;
        v[C * kGradWords + 4] = t2 * dy;
        v[C * kGradWords + 5] = dq;
        v[C * kGradWords + 6] = gc0 * w;
        v[C * kGradWords + 7] = gc1 * w;
        v[C * kGradWords + 8] = gc2 * w;
        v[C * kGradWords + 9] = gd * w;
        const uint32_t pslot = s_slot[jl];
        chunk = (lane == C) ? pslot : chunk;
        --jl;
    };
    // Six slots: four and five (fewer registers, five waves per SIMD with
    // four) measured slower, the transposed sums then costing more per slot.
    constexpr int NS = kChunk;
    static_assert(NS >= 2 && NS <= 6, "reduction slots");
    for (;;) {
        if (!next()) break;
        take(SlotIdx<0>{});
        if (!next()) { flush_slots<1>(v, chunk, partials, written, cap); break; }
        take(SlotIdx<1>{});
        if constexpr (NS > 2) {
            if (!next()) { flush_slots<2>(v, chunk, partials, written, cap); break; }
            take(SlotIdx<2>{});
        }
        if constexpr (NS > 3) {
            if (!next()) { flush_slots<3>(v, chunk, partials, written, cap); break; }
            take(SlotIdx<3>{});
        }
        if constexpr (NS > 4) {
            if (!next()) { flush_slots<4>(v, chunk, partials, written, cap); break; }
            take(SlotIdx<4>{});
        }
        if constexpr (NS > 5) {
            if (!next()) { flush_slots<5>(v, chunk, partials, written, cap); break; }
            take(SlotIdx<5>{});
        }
        flush_slots<NS>(v, chunk, partials, written, cap);
    }
}

// PROBS: with gradients of the instance channels; SEG: a launch over the
// segment list (instantiations of their own)
template <typename T, int TW, int TH, bool PROBS, bool SEG>
__global__ __launch_bounds__(kWave, 4) void render_backward_wave_kernel(
    Views<T> V, Consts<T> cs, int K, const T* __restrict__ splats,
    const uint32_t* __restrict__ pvals, const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ schedule,
    const T* __restrict__ tfinal, const int32_t* __restrict__ last, const int32_t* __restrict__ target,
    const T* __restrict__ dC, const T* __restrict__ dD, const T* __restrict__ dT, const T* __restrict__ dP,
    const T* __restrict__ dPt, T* __restrict__ partials, uint8_t* __restrict__ written, uint32_t cap, uint32_t M,
    const uint4* __restrict__ seg_list, const T* __restrict__ ckpt, uint32_t ckpt_cap, const T* __restrict__ color,
    const T* __restrict__ depth, const T* __restrict__ ptarget, const Ctrl* __restrict__ ctrl) {
    static_assert(TW * TH == kWave, "one wavefront per tile");
    __shared__ __align__(16) T s_sp[kWave * kWalkWords];
    __shared__ uint32_t s_slot[kWave];

    const int lane = threadIdx.x;
    // One wavefront per tile, or (with a segment list) per listed segment of
    // a tile's pair range, [s0, s1) of [rs, re); the list is built after the
    // forward, so its length is read here and the rest of the grid, sized for
    // the longest possible list, exits at once.  (A resident grid drawing
    // entries from a work counter was measured slower: the loop around the
    // walk raised its register demand past the budget and spilled.)
    // The segments restart from states stored by one particular forward; if
    // the frame was binned again since, or the images are another forward's,
    // those states are not this backward's and every tile is walked whole
    // instead (the grid holds at least one workgroup per tile).
    const uint32_t n_tiles = (uint32_t)(V.n_views * V.tiles_per_view);
    if (seg_list && (ctrl->seg_stamp[0] != (uint64_t)ctrl->epoch || ctrl->seg_stamp[1] != (uint64_t)(uintptr_t)last ||
                     ctrl->seg_stamp[2] != (uint64_t)(uintptr_t)target))
        seg_list = nullptr;
    const uint32_t n_units = seg_list ? ctrl->counters[kCounterSegTotal] : n_tiles;
    // Segment units in chunks of 16 consecutive list entries (a tile's
    // segments, which read the same pixel inputs) on one XCD: workgroup b runs
    // on XCD b % 8, and the chunks are dealt to the XCDs round-robin, so the
    // heavy tiles at the head of the list still spread over the device.  Each
    // XCD has its own L2; at the 200k view this cut the backward's HBM reads
    // from 148 to 103 MB (chunks of 4: 116 MB, of 64: 99 MB but slower).
#ifndef DQO_BWD_XCD_CHUNK
#define DQO_BWD_XCD_CHUNK 16
#endif
    uint32_t unit = blockIdx.x;
    if constexpr (SEG && DQO_BWD_XCD_CHUNK > 0) {
        constexpr uint32_t c = DQO_BWD_XCD_CHUNK;
        if (seg_list) {
            const uint32_t x = blockIdx.x % 8u, r = blockIdx.x / 8u;
            unit = ((r / c) * 8u + x) * c + r % c;
        }
    }
    if (unit >= n_units) return;
    // (a segmented launch walks a stale frame's whole tiles without prefetch)
    backward_unit<T, TW, TH, PROBS, !SEG>(V, cs, K, splats, pvals, ranges, schedule, tfinal, last, target, dC, dD, dT,
                                          dP, dPt, partials, written, cap, M, seg_list, ckpt, ckpt_cap, color, depth,
                                          ptarget, s_sp, s_slot, unit);
}

// ---------------------------------------------------------------- launchers
template <typename T, int TW, int TH>
static hipError_t fwd_tile(const Frame<T>& f, const dqo_images& img, hipStream_t st) {
    const int blocks = f.views.n_views * f.views.tiles_per_view;
    if (blocks == 0) return hipSuccess;
    const StatePtrs& s = f.s;
    // Boundary states, tile ends and the backward's segment list, for a
    // backward that can run segmented (no instance channels: their sums behind
    // a boundary would need every object's prefix).
    const bool seg = segmented_backward(s, blocks) && !img.probs;
    if (img.probs && f.K > 0) {
        const size_t dyn = (size_t)f.K * TW * TH * sizeof(T);
        hipLaunchKernelGGL((render_forward_kernel<T, TW, TH, true>), dim3(blocks), dim3(TW * TH), dyn, st, f.views,
                           f.consts, f.K, (const T*)s.splats, s.pair_vals[0], s.ranges, s.schedule, (T*)img.color,
                           (T*)img.depth, (T*)img.t_final, img.last, (T*)img.probs, img.id_map, img.target,
                           (T*)img.p_target, img.n_blend, (uint32_t)s.capacity, (uint32_t)s.items,
                           (T*)(seg ? s.ckpt : nullptr), (uint32_t)s.ckpt_cap, s.tile_last, s.seg_base, s.seg_list,
                           (uint32_t)s.seg_cap, s.ctrl);
    } else {
        auto kern = img.n_blend ? render_forward_kernel<T, TW, TH, false, true> : render_forward_kernel<T, TW, TH, false, false>;
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(TW * TH), 0, st, f.views,
                           f.consts, f.K, (const T*)s.splats, s.pair_vals[0], s.ranges, s.schedule, (T*)img.color,
                           (T*)img.depth, (T*)img.t_final, img.last, (T*)nullptr, (int32_t*)nullptr, img.target,
                           (T*)img.p_target, img.n_blend, (uint32_t)s.capacity, (uint32_t)s.items,
                           (T*)(seg ? s.ckpt : nullptr), (uint32_t)s.ckpt_cap, s.tile_last, s.seg_base, s.seg_list,
                           (uint32_t)s.seg_cap, s.ctrl);
    }
    return hipGetLastError();
}

template <typename T, int TW, int TH>
static hipError_t bwd_tile(const Frame<T>& f, const dqo_images& img, const dqo_image_grads& g, hipStream_t st) {
    const int blocks = f.views.n_views * f.views.tiles_per_view;
    if (blocks == 0) return hipSuccess;
    const StatePtrs& s = f.s;
    if constexpr (TW * TH == kWave) {
        // Segments of the pair ranges, each restarted from the forward's
        // boundary states (stored by a forward without instance channels,
        // which also built the segment list).
        const bool seg = segmented_backward(s, blocks) && !img.probs && !g.d_probs && img.color && img.depth &&
                         (img.p_target || !g.d_p_target);
        // units = segments up to each tile's end <= tiles + pairs / kSegLen = seg_cap
        const int64_t gq = 8 * std::max(1, DQO_BWD_XCD_CHUNK);  // whole XCD chunks
        const unsigned grid = seg ? (unsigned)((std::max<int64_t>(s.seg_cap, blocks) + gq - 1) / gq * gq)
                                  : (unsigned)blocks;
        auto kern = g.d_probs ? (seg ? render_backward_wave_kernel<T, TW, TH, true, true>
                                     : render_backward_wave_kernel<T, TW, TH, true, false>)
                              : (seg ? render_backward_wave_kernel<T, TW, TH, false, true>
                                     : render_backward_wave_kernel<T, TW, TH, false, false>);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kWave), 0, st, f.views, f.consts, f.K, (const T*)s.splats,
                           s.pair_vals[0], s.ranges, s.schedule, (const T*)img.t_final, img.last, img.target,
                           (const T*)g.d_color, (const T*)g.d_depth, (const T*)g.d_t_final, (const T*)g.d_probs,
                           (const T*)g.d_p_target, (T*)s.partials, s.written, (uint32_t)s.capacity,
                           (uint32_t)s.items, seg ? s.seg_list : nullptr, (const T*)s.ckpt, (uint32_t)s.ckpt_cap,
                           (const T*)img.color, (const T*)img.depth, (const T*)img.p_target, s.ctrl);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((render_backward_kernel<T, TW, TH>), dim3(blocks), dim3(TW * TH), 0, st, f.views, f.consts,
                       f.K, (const T*)s.splats, s.pair_vals[0], s.ranges, s.schedule,
                       (const T*)img.t_final, img.last, img.target, (const T*)g.d_color, (const T*)g.d_depth,
                       (const T*)g.d_t_final, (const T*)g.d_probs, (const T*)g.d_p_target, (T*)s.partials, s.written,
                       (uint32_t)s.capacity, (uint32_t)s.items);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_render_forward(const Frame<T>& f, const dqo_images& img, hipStream_t st) {
    const int tw = f.views.tile_w, th = f.views.tile_h;
    if (tw == 16 && th == 16) return fwd_tile<T, 16, 16>(f, img, st);
    if (tw == 8 && th == 8) return fwd_tile<T, 8, 8>(f, img, st);
    if (tw == 16 && th == 8) return fwd_tile<T, 16, 8>(f, img, st);
    if (tw == 32 && th == 8) return fwd_tile<T, 32, 8>(f, img, st);
    if (tw == 8 && th == 32) return fwd_tile<T, 8, 32>(f, img, st);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_render_backward(const Frame<T>& f, const dqo_images& img, const dqo_image_grads& g,
                                  hipStream_t st) {
    const int tw = f.views.tile_w, th = f.views.tile_h;
    if (tw == 16 && th == 16) return bwd_tile<T, 16, 16>(f, img, g, st);
    if (tw == 8 && th == 8) return bwd_tile<T, 8, 8>(f, img, g, st);
    if (tw == 16 && th == 8) return bwd_tile<T, 16, 8>(f, img, g, st);
    if (tw == 32 && th == 8) return bwd_tile<T, 32, 8>(f, img, g, st);
    if (tw == 8 && th == 32) return bwd_tile<T, 8, 32>(f, img, g, st);
    return hipErrorInvalidValue;
}

template hipError_t launch_render_forward<float>(const Frame<float>&, const dqo_images&, hipStream_t);
template hipError_t launch_render_forward<double>(const Frame<double>&, const dqo_images&, hipStream_t);
template hipError_t launch_render_backward<float>(const Frame<float>&, const dqo_images&, const dqo_image_grads&,
                                                  hipStream_t);
template hipError_t launch_render_backward<double>(const Frame<double>&, const dqo_images&,
                                                   const dqo_image_grads&, hipStream_t);

}  // namespace dqo
