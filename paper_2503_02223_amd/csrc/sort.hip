// Stable LSD radix sort passes (8-bit digits, one kernel per pass) and tile ranges.
//
// A pass reads 256 x IPT (key, value) items per block, ranks them stably inside the
// block with wave-wide match ballots, obtains the block's global offset per
// digit by decoupled look-back over the preceding blocks, then writes the
// items out digit-sorted through LDS so stores are coalesced.  Block order is
// the workgroup index when the whole grid fits on the device at once (every
// block it waits on is then running); otherwise it is taken from an atomic
// ticket, so that every block waited on has started.  The ticket costs a
// contended global atomic per block (2.5 us at 383 blocks, measured).
// Digit histograms of every pass are accumulated before the first pass by the
// kernel that produced the keys.
#include <algorithm>

#include "dqo_device.hpp"
#include "sort_common.hpp"

namespace dqo {

template <int NT, int IPT, bool REL>
__global__ __launch_bounds__(NT) void radix_pass_kernel(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* __restrict__ n_dev, uint32_t n_host, int shift,
    const uint32_t* __restrict__ ghist, int hist_stride, int hist_copies, uint64_t* lb, uint32_t* counter,
    int resident, Ctrl* ctrl, DepthRel rel) {
    static_assert(NT >= kRadixBins && NT % kWave == 0, "one thread per digit at least");
    constexpr int kTile = NT * IPT;
    constexpr int kWaves = NT / kWave;
    __shared__ uint32_t s_keys[kTile];
    __shared__ uint32_t s_vals[kTile];
    __shared__ uint32_t s_wcnt[kWaves][kRadixBins];
    __shared__ uint32_t s_dstart[kRadixBins];
    __shared__ uint32_t s_gbase[kRadixBins];
    __shared__ uint32_t s_tmp[kWaves];
    __shared__ uint32_t s_bid, s_epoch, s_grouped;
    __shared__ uint32_t s_next[REL ? kRadixBins : 1];  // REL: counts of the next pass's digit

    const int tid = threadIdx.x;
    // REL: the digits of key - base (clamped to 2^24 - 1 when three passes
    // suffice), from the key range the projection left in copies
    __shared__ uint32_t s_krange[2];
    if (REL && tid < kWave) {
        uint32_t v = tid < 2 * kHistCopies ? (&ctrl->dkey_range[0][0])[tid] : 0u;
        // lanes of even index hold max(~key) copies, odd ones max(key)
#pragma unroll
        for (int d = 2; d < 2 * kHistCopies; d <<= 1) v = max(v, (uint32_t)__shfl_xor(v, d));
        if (tid < 2) s_krange[tid] = v;
    }
    const int lane = tid & (kWave - 1);
    const int wave = tid >> 6;
    // Every load that does not depend on another is issued before the first
    // wait: the item count, the block's keys at its workgroup index (the order
    // in force unless a ticket is drawn; bounded by the buffer's size n_host,
    // the tail past the count is masked below), the digit totals and the
    // control words.
    const uint32_t n_read = n_dev ? *n_dev : n_host;
    uint32_t key[IPT], val[IPT], rank[IPT];
    auto load_block = [&](uint32_t b) {
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const uint32_t pos = b * (uint32_t)kTile + wave * (kWave * IPT) + i * kWave + lane;
            key[i] = pos < n_host ? kin[pos] : 0u;
            val[i] = pos < n_host ? vin[pos] : 0u;
        }
    };
    if (resident) load_block(blockIdx.x);
    const int t = tid;
    const bool owner = t < kRadixBins;
    uint32_t gcount = 0;
    if (owner) {
        // the digit's count over all keys: the sum of the histogram copies
        for (int c = 0; c < hist_copies; ++c) gcount += ghist[c * hist_stride + t];
    }
    if (tid == 0) {
        // Workgroup-index order needs the whole grid on the device at once;
        // once a bounded wait has given up (status bit, kept until the caller
        // clears it) the order comes from the ticket instead, every frame.
        // A resident grid, whose blocks all start together, sums its
        // predecessors in groups; ticket order (blocks staggered in time)
        // walks the chain.
        const bool ticket = !resident || (ctrl->status & (uint32_t)DQO_STATUS_TIMEOUT) != 0u;
        s_bid = ticket ? atomicAdd(counter, 1u) : blockIdx.x;
        s_grouped = (ticket || !DQO_LB_GROUPED) ? 0u : 1u;
        s_epoch = ctrl->epoch;
    }
    for (int i = tid; i < kWaves * kRadixBins; i += NT) (&s_wcnt[0][0])[i] = 0;
    if (REL && tid < kRadixBins) s_next[tid] = 0u;
    __syncthreads();
    uint32_t kbase = 0u, clamp = 0xFFFFFFFFu;
    if constexpr (REL) {
        const uint32_t kmin = ~s_krange[0], kmax = s_krange[1];
        const bool any = kmax >= kmin;
        kbase = any ? (kmin & ~(uint32_t)(kRadixBins - 1)) : 0u;
        const bool three = any && kmax - kbase < 0xFFFFFFu;
        if (three) clamp = 0xFFFFFFu;
        if (rel.pass == 3 && three) return;  // uniform: nothing left to sort
        if (rel.pass == 2 && three) {
            kout = rel.kout_final;
            vout = rel.vout_final;
            rel.next_hist = nullptr;  // no fourth pass to count for
        }
    }
    auto digit = [&](uint32_t k, int sh) -> uint32_t {
        if constexpr (REL) k = min(k - kbase, clamp);
        return (k >> sh) & (kRadixBins - 1);
    };
    const uint32_t bid = s_bid;
    const uint32_t n = min(n_read, n_host);
    const uint32_t base = bid * (uint32_t)kTile;
    if (base >= n) return;  // uniform over the block; no later block waits on this one
    const uint32_t epoch = s_epoch;
    // ticket order, or a grid not resident: the block's keys now
    if (!resident || bid != blockIdx.x) load_block(bid);

    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const uint32_t pos = base + wave * (kWave * IPT) + i * kWave + lane;
        const bool valid = pos < n;
        const uint32_t d = digit(key[i], shift);
        if (REL && rel.next_hist && valid) atomicAdd(&s_next[digit(key[i], shift + kRadixBits)], 1u);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
        uint32_t old = 0;
        if (valid) old = s_wcnt[wave][d];
        const bool leader = valid && ((peers >> lane) == 1ull);
        if (leader) s_wcnt[wave][d] = old + (uint32_t)__popcll(peers);
        rank[i] = old + below;
    }
    __syncthreads();

    // Thread t < 256 owns digit t: per-wave exclusive offsets and the block total.
    uint32_t total = 0;
    if (owner) {
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t c = s_wcnt[w][t];
            s_wcnt[w][t] = total;
            total += c;
        }
    }
    const uint32_t dstart = block_exclusive_scan<NT>(total, s_tmp);
    const uint32_t gdig = block_exclusive_scan<NT>(gcount, s_tmp);
    if (owner) {
        s_dstart[t] = dstart;
        // A digit that no key has anywhere needs no chain: every block skips it.
        uint32_t excl = 0u;
        if (gcount) {
            excl = s_grouped ? lookback_grouped(lb + t, lb + (size_t)gridDim.x * kRadixBins + t, kRadixBins, (int)bid,
                                                total, epoch, &ctrl->status)
                             : lookback_exclusive(lb + t, kRadixBins, (int)bid, total, epoch, &ctrl->status);
        }
        s_gbase[t] = gdig + excl;
    }
    __syncthreads();

#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const uint32_t pos = base + wave * (kWave * IPT) + i * kWave + lane;
        if (pos < n) {
            const uint32_t d = digit(key[i], shift);
            const uint32_t p = s_dstart[d] + s_wcnt[wave][d] + rank[i];
            if (p < (uint32_t)kTile) {
                s_keys[p] = key[i];
                s_vals[p] = val[i];
            }
        }
    }
    __syncthreads();
    const uint32_t cnt = min((uint32_t)kTile, n - base);
    for (uint32_t q = tid; q < cnt; q += NT) {
        const uint32_t k = s_keys[q];
        const uint32_t d = digit(k, shift);
        const uint32_t o = s_gbase[d] + (q - s_dstart[d]);
        if (o < n) {  // always true unless a bounded wait gave up (status bit set)
            kout[o] = k;
            vout[o] = s_vals[q];
        }
    }
    if constexpr (REL) {
        if (rel.next_hist && owner) {
            const uint32_t c = s_next[t];
            if (c) atomicAdd(&rel.next_hist[(size_t)(blockIdx.x % hist_copies) * hist_stride + t], c);
        }
    }
}

// [start, end) of every tile that holds pairs, from the boundaries of the
// sorted pair keys (tiles without pairs keep the empty range written when the
// frame was projected).  The same pass clears the written marks of the pairs
// (four one-byte marks per word), which the render backward sets.
__global__ __launch_bounds__(256) void tile_bounds_kernel(const uint32_t* __restrict__ keys,
                                                          const uint32_t* __restrict__ n_dev, uint32_t n_host,
                                                          uint32_t* __restrict__ ranges,
                                                          uint32_t* __restrict__ written_words) {
    const uint32_t n = min(*n_dev, n_host);
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
        const uint32_t t = keys[i];
        if (i == 0 || keys[i - 1] != t) ranges[2 * t] = i;
        if (i + 1 == n || keys[i + 1] != t) ranges[2 * t + 1] = i + 1;
    }
    const uint32_t nw = (n + 3u) / 4u;
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < nw; i += gridDim.x * 256u) written_words[i] = 0u;
}

// Launch order of the render workgroups: tiles by decreasing pair count.
// Workgroups are dispatched in index order and spread round-robin over the
// XCDs and CUs, so the heaviest tiles, which are spatially clustered, start
// first and on different compute units instead of queueing on the same ones,
// and the launch ends with the lightest.  Counts are exact up to 4095 (larger
// ones share the top bin).  Against power-of-two classes of the count (tiles
// of a class in index order), the exact order made the backward replayed on
// its own at the 200k view 5% faster and the forward 6%; inside the whole
// training step the difference was within run-to-run noise.  Order among
// equal counts is arbitrary; results do not depend on the order (every tile
// writes only its own pixels and pair slots).
constexpr int kSchedThreads = 1024;
constexpr int kSchedBins = 4096;

// Up to kSchedRegs tiles per thread are loaded once, all at once, and kept in
// registers (their ranges are read by two dependent phases: the count
// histogram and the scatter); more tiles loop over global memory.
constexpr int kSchedRegs = 8;
__global__ __launch_bounds__(kSchedThreads) void tile_schedule_kernel(const uint32_t* __restrict__ ranges,
                                                                     int tiles, uint32_t* __restrict__ schedule,
                                                                     int seg, uint32_t* __restrict__ seg_base,
                                                                     Ctrl* __restrict__ ctrl) {
    __shared__ uint32_t s_cnt[kSchedBins];  // bin b holds count kSchedBins - 1 - b (descending order)
    // segmented backward: the segments of each bin's tiles, then the bin's
    // cursor in the segment list
    __shared__ uint32_t s_seg[kSchedBins];
    __shared__ uint32_t s_tmp[kSchedThreads / kWave];
    constexpr int kPer = kSchedBins / kSchedThreads;
    const int tid = threadIdx.x;
    auto bin_of_w = [](uint32_t w) { return kSchedBins - 1 - (int)min(w, (uint32_t)(kSchedBins - 1)); };
    auto width = [&](int t) {
        const uint2 r = reinterpret_cast<const uint2*>(ranges)[t];
        return r.y - r.x;
    };
    // thread tid holds tiles tid + k * kSchedThreads (coalesced loads)
    const bool regs = tiles <= kSchedRegs * kSchedThreads;
    uint32_t w[kSchedRegs];
    if (regs) {
#pragma unroll
        for (int k = 0; k < kSchedRegs; ++k) {
            const int t = tid + k * kSchedThreads;
            w[k] = t < tiles ? width(t) : 0u;
        }
    }
    for (int b = tid; b < kSchedBins; b += kSchedThreads) s_cnt[b] = s_seg[b] = 0u;
    __syncthreads();
    auto count = [&](uint32_t wt) {
        atomicAdd(&s_cnt[bin_of_w(wt)], 1u);
        if (seg) atomicAdd(&s_seg[bin_of_w(wt)], tile_segments(wt));
    };
    if (regs) {
#pragma unroll
        for (int k = 0; k < kSchedRegs; ++k)
            if (tid + k * kSchedThreads < tiles) count(w[k]);
    } else {
        for (int t = tid; t < tiles; t += kSchedThreads) count(width(t));
    }
    __syncthreads();
    uint32_t c[kPer], g[kPer], sum = 0, gsum = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        c[k] = s_cnt[tid * kPer + k];
        g[k] = s_seg[tid * kPer + k];
        sum += c[k];
        gsum += g[k];
    }
    uint32_t off = block_exclusive_scan<kSchedThreads>(sum, s_tmp);
    uint32_t goff = seg ? block_exclusive_scan<kSchedThreads>(gsum, s_tmp) : 0u;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        s_cnt[tid * kPer + k] = off;
        s_seg[tid * kPer + k] = goff;
        off += c[k];
        goff += g[k];
    }
    // The backward's segment list holds every 64-pair segment of every tile,
    // tiles by bin (heaviest first); the forward fills in each tile's entries
    // once it knows how far its pixels blend (the rest it marks empty).
    if (seg && tid == kSchedThreads - 1) ctrl->counters[kCounterSegTotal] = goff;
    __syncthreads();
    auto place = [&](int t, uint32_t wt) {
        schedule[atomicAdd(&s_cnt[bin_of_w(wt)], 1u)] = (uint32_t)t;
        if (seg) seg_base[t] = atomicAdd(&s_seg[bin_of_w(wt)], tile_segments(wt));
    };
    if (regs) {
#pragma unroll
        for (int k = 0; k < kSchedRegs; ++k)
            if (tid + k * kSchedThreads < tiles) place(tid + k * kSchedThreads, w[k]);
    } else {
        for (int t = tid; t < tiles; t += kSchedThreads) place(t, width(t));
    }
}

template <int NT, int IPT>
static hipError_t radix_launch(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                               const uint32_t* n_dev, uint32_t n_host, int shift, const uint32_t* ghist,
                               int hist_stride, int hist_copies, uint64_t* lb, uint32_t* counter, Ctrl* ctrl,
                               hipStream_t st, const DepthRel* rel) {
    const int blocks = (int)((n_host + NT * IPT - 1) / (NT * IPT));
    // the whole grid is resident: workgroup index order (unless a wait has timed out)
    const DepthRel r = rel ? *rel : DepthRel{0, nullptr, nullptr, nullptr};
    if (rel) {
        const int res = blocks <= resident_blocks<radix_pass_kernel<NT, IPT, true>, NT>() ? 1 : 0;
        hipLaunchKernelGGL((radix_pass_kernel<NT, IPT, true>), dim3(blocks), dim3(NT), 0, st, kin, vin, kout, vout,
                           n_dev, n_host, shift, ghist, hist_stride, hist_copies, lb, counter, res, ctrl, r);
    } else {
        const int res = blocks <= resident_blocks<radix_pass_kernel<NT, IPT, false>, NT>() ? 1 : 0;
        hipLaunchKernelGGL((radix_pass_kernel<NT, IPT, false>), dim3(blocks), dim3(NT), 0, st, kin, vin, kout, vout,
                           n_dev, n_host, shift, ghist, hist_stride, hist_copies, lb, counter, res, ctrl, r);
    }
    return hipGetLastError();
}

bool radix_resident(int nt, int ipt, int64_t items) {
    const int64_t blocks = (items + (int64_t)nt * ipt - 1) / ((int64_t)nt * ipt);
    int res = 0;
#define DQO_RADIX_RES(NT_, IPT_) \
    if (nt == NT_ && ipt == IPT_) res = resident_blocks<radix_pass_kernel<NT_, IPT_, false>, NT_>();
    DQO_RADIX_RES(256, 8)
    DQO_RADIX_RES(256, 16)
    DQO_RADIX_RES(256, 32)
    DQO_RADIX_RES(512, 4)
    DQO_RADIX_RES(512, 9)
    DQO_RADIX_RES(512, 18)
    DQO_RADIX_RES(1024, 2)
    DQO_RADIX_RES(1024, 4)
    DQO_RADIX_RES(1024, 8)
    DQO_RADIX_RES(1024, 16)
#undef DQO_RADIX_RES
    return blocks <= res;
}

hipError_t launch_radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                             const uint32_t* n_dev, uint32_t n_host, int shift, const uint32_t* ghist,
                             int hist_stride, int hist_copies, uint64_t* lb, uint32_t* counter, Ctrl* ctrl,
                             hipStream_t st, int nt, int ipt, const DepthRel* rel) {
    if (n_host == 0) return hipSuccess;
#define DQO_RADIX_CASE(NT_, IPT_)                                                                            \
    if (nt == NT_ && ipt == IPT_)                                                                            \
        return radix_launch<NT_, IPT_>(kin, vin, kout, vout, n_dev, n_host, shift, ghist, hist_stride, hist_copies, \
                                       lb, counter, ctrl, st, rel);
    DQO_RADIX_CASE(256, 8)
    DQO_RADIX_CASE(256, 16)
    DQO_RADIX_CASE(256, 32)
    DQO_RADIX_CASE(512, 4)
    DQO_RADIX_CASE(512, 9)
    DQO_RADIX_CASE(512, 18)
    DQO_RADIX_CASE(1024, 2)
    DQO_RADIX_CASE(1024, 4)
    DQO_RADIX_CASE(1024, 8)
    DQO_RADIX_CASE(1024, 16)
#undef DQO_RADIX_CASE
    return hipErrorInvalidValue;
}

// Per-tile depth order.  The pairs were emitted in item order and stably
// sorted by tile, so each tile's range holds its items in index order; one
// workgroup per tile sorts them by the item's depth key, ties by item index:
// the order a stable sort of every item by depth followed by the stable tile
// sort gives.  Up to kTileSortLds pairs: a bitonic network over the 64-bit
// values key << 32 | item, padded to P = 256 E (E = 1..16 values per thread,
// held in registers in blocked order: value e = thread E + r).  Its stages
// with a partner distance j < E run inside a thread, those with j < 64 E
// across the lanes of a wavefront (shuffles), and only those with j >= 64 E
// (three at P = 4096) through LDS with barriers.  Longer ranges: four stable
// 8-bit passes over global memory by the workgroup, through tmp (slow; meant
// for rare long tiles).  Tiles are taken in the launch order of the render
// (longest first), so the longest sorts start first.
constexpr int kTileSortThreads = 256;
constexpr int kTileSortLds = 4096;

__device__ __forceinline__ uint64_t keep_lo_hi(uint64_t mine, uint64_t other, bool keep_min) {
    const bool lt = mine < other;
    return (lt == keep_min) ? mine : other;
}

template <int E>
__device__ __forceinline__ void tile_bitonic(uint64_t (&x)[16], uint64_t* s_x, int tid, uint32_t P) {
    const int lane = tid & (kWave - 1);
    for (uint32_t k = 2u; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0u; j >>= 1) {
            if (j < (uint32_t)E) {
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    if ((r & (int)j) == 0) {
                        const uint32_t e = (uint32_t)tid * E + r;
                        const bool up = (e & k) == 0u;
                        const uint64_t a = x[r], b = x[r | (int)j];
                        const bool swap = (a > b) == up;
                        x[r] = swap ? b : a;
                        x[r | (int)j] = swap ? a : b;
                    }
                }
            } else if (j < (uint32_t)(kWave * E)) {
                const int d = (int)(j / (uint32_t)E);
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    const uint64_t y = (uint64_t)__shfl_xor((unsigned long long)x[r], d);
                    const uint32_t e = (uint32_t)tid * E + r;
                    x[r] = keep_lo_hi(x[r], y, ((e & j) == 0u) == ((e & k) == 0u));
                }
            } else {
#pragma unroll
                for (int r = 0; r < E; ++r) s_x[tid * E + r] = x[r];
                __syncthreads();
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    const uint32_t e = (uint32_t)tid * E + r;
                    x[r] = keep_lo_hi(x[r], s_x[e ^ j], ((e & j) == 0u) == ((e & k) == 0u));
                }
                __syncthreads();
            }
        }
    }
    (void)lane;
}

__global__ __launch_bounds__(kTileSortThreads) void tile_sort_kernel(const uint32_t* __restrict__ ranges,
                                                                    const uint32_t* __restrict__ schedule,
                                                                    const uint32_t* __restrict__ dkeys, uint32_t M,
                                                                    uint32_t cap, uint32_t lds_max, int tiles,
                                                                    uint32_t* __restrict__ pvals,
                                                                    uint32_t* __restrict__ tmp) {
    __shared__ uint64_t s_k[kTileSortLds];
    __shared__ uint32_t s_off[kRadixBins];
    __shared__ uint32_t s_wcnt[kTileSortThreads / kWave][kRadixBins];
    __shared__ uint32_t s_scan[kTileSortThreads / kWave];
    const int tid = threadIdx.x;
    const uint32_t tile = min(schedule[blockIdx.x], (uint32_t)(tiles - 1));
    const uint32_t re = min(ranges[2 * tile + 1], cap), rs = min(ranges[2 * tile], re);
    const uint32_t n = re - rs;
    if (n <= 1u) return;
    if (n <= min(lds_max, (uint32_t)kTileSortLds)) {
        int E = 1;
        while ((uint32_t)(kTileSortThreads * E) < n) E <<= 1;
        const uint32_t P = (uint32_t)(kTileSortThreads * E);
        uint64_t x[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const uint32_t e = (uint32_t)tid * E + r;
            x[r] = ~0ull;  // padding sorts last
            if (r < E && e < n) {
                const uint32_t item = min(pvals[rs + e], M - 1);
                x[r] = ((uint64_t)dkeys[item] << 32) | item;
            }
        }
        switch (E) {
            case 1: tile_bitonic<1>(x, s_k, tid, P); break;
            case 2: tile_bitonic<2>(x, s_k, tid, P); break;
            case 4: tile_bitonic<4>(x, s_k, tid, P); break;
            case 8: tile_bitonic<8>(x, s_k, tid, P); break;
            default: tile_bitonic<16>(x, s_k, tid, P); break;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const uint32_t e = (uint32_t)tid * E + r;
            if (r < E && e < n) pvals[rs + e] = (uint32_t)x[r];
        }
        return;
    }
    // Long range: stable LSD passes, 256 items per round in index order,
    // ranked inside each wavefront by match ballots.
    const int lane = tid & (kWave - 1), wave = tid >> 6;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t* src = pvals + rs;
    uint32_t* dst = tmp + rs;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = pass * kRadixBits;
        for (int w = 0; w < kTileSortThreads / kWave; ++w)
            if (tid < kRadixBins) s_wcnt[w][tid] = 0u;
        if (tid < kRadixBins) s_off[tid] = 0u;
        __syncthreads();
        for (uint32_t i = tid; i < n; i += kTileSortThreads)
            atomicAdd(&s_off[(dkeys[min(src[i], M - 1)] >> shift) & (kRadixBins - 1)], 1u);
        __syncthreads();
        {
            const uint32_t c = tid < kRadixBins ? s_off[tid] : 0u;
            const uint32_t ex = block_exclusive_scan<kTileSortThreads>(c, s_scan);
            __syncthreads();
            if (tid < kRadixBins) s_off[tid] = ex;
            __syncthreads();
        }
        for (uint32_t c0 = 0; c0 < n; c0 += kTileSortThreads) {
            const uint32_t i = c0 + (uint32_t)tid;
            const bool valid = i < n;
            const uint32_t item = valid ? src[i] : 0u;
            const uint32_t d = valid ? (dkeys[min(item, M - 1)] >> shift) & (kRadixBins - 1) : 0u;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < kRadixBits; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                peers &= bit ? bb : ~bb;
            }
            const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
            if (valid && (peers >> lane) == 1ull) s_wcnt[wave][d] = (uint32_t)__popcll(peers);
            __syncthreads();
            if (valid) {
                uint32_t before = 0;
                for (int w = 0; w < wave; ++w) before += s_wcnt[w][d];
                dst[s_off[d] + before + below] = item;
            }
            __syncthreads();
            if (tid < kRadixBins) {
                uint32_t total = 0;
                for (int w = 0; w < kTileSortThreads / kWave; ++w) {
                    total += s_wcnt[w][tid];
                    s_wcnt[w][tid] = 0u;
                }
                s_off[tid] += total;
            }
            __syncthreads();
        }
        uint32_t* t = src;
        src = dst;
        dst = t;
    }
    // four passes: the result is back in pvals
}

hipError_t launch_pair_sort(const StatePtrs& s, int tiles_total, hipStream_t st) {
    const uint32_t cap = (uint32_t)s.capacity;
    const uint32_t* n_dev = &s.ctrl->num_pairs;
    // short blocks while that grid is resident at once, else long ones
    const bool short_ok = radix_resident(kPairNt, kPairIptShort, cap);
    const int nt = short_ok ? kPairNt : kPairNtLong, ipt = short_ok ? kPairIptShort : kPairIptLong;
    // the fused emission has done pass 0 (its output is in the other buffer)
    const int p0 = s.fused_emit ? 1 : 0;
    int src = s.pair_first_buf ^ p0;
    for (int p = p0; p < s.pair_passes; ++p) {
        hipError_t e = launch_radix_pass(s.pair_keys[src], s.pair_vals[src], s.pair_keys[src ^ 1],
                                         s.pair_vals[src ^ 1], n_dev, cap, p * kRadixBits,
                                         &s.ctrl->hist_pair[0][p][0], kMaxPairPasses * kRadixBins, s.hist_copies_pair, s.lb_pair + (size_t)p * lb_blocks(s.pair_blocks) * kRadixBins,
                                         &s.ctrl->counters[kCounterPair + p], s.ctrl, st, nt, ipt);
        if (e != hipSuccess) return e;
        src ^= 1;
    }
    if (tiles_total > 0) {
        // one pair per thread, every key load in flight at once
        const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1 << 20, ((int64_t)cap + 255) / 256));
        hipLaunchKernelGGL(tile_bounds_kernel, dim3(grid), dim3(256), 0, st, s.pair_keys[0], n_dev, cap, s.ranges,
                           (uint32_t*)s.written);
        hipLaunchKernelGGL(tile_schedule_kernel, dim3(1), dim3(kSchedThreads), 0, st, s.ranges, tiles_total,
                           s.schedule, segmented_backward(s, tiles_total) ? 1 : 0, s.seg_base, s.ctrl);
        if (s.tile_sort)
            hipLaunchKernelGGL(tile_sort_kernel, dim3((unsigned)tiles_total), dim3(kTileSortThreads), 0, st, s.ranges,
                               s.schedule, s.depth_keys[0], (uint32_t)s.items, cap, (uint32_t)s.tile_sort_lds,
                               tiles_total, s.pair_vals[0], s.pair_vals[1]);
        return hipGetLastError();
    }
    return launch_clear_written(s, st);
}

}  // namespace dqo
