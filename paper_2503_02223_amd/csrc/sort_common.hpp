// Wave- and block-level scans used by the radix passes and the pair emission.
#pragma once
#include "dqo_device.hpp"

namespace dqo {

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t t = __shfl_up(v, d);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive scan over a block of NT threads; s_tmp holds NT / 64 words.
// Contains two barriers: every thread of the block must call it.
template <int NT>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_tmp) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    const uint32_t incl = wave_inclusive_scan(v, lane);
    if (lane == kWave - 1) s_tmp[wave] = incl;
    __syncthreads();
    uint32_t off = 0;
    for (int w = 0; w < wave; ++w) off += s_tmp[w];
    __syncthreads();
    return off + incl - v;
}
__device__ __forceinline__ uint32_t block_exclusive_scan_256(uint32_t v, uint32_t* s_tmp) {
    return block_exclusive_scan<256>(v, s_tmp);
}

// Depth passes sort the digits of key - base, base = the frame's smallest
// visible key rounded down to a multiple of 256 (the low digit is the key's
// own).  When every visible key lies below base + 2^24 - 1, three passes
// suffice: the digits of min(key - base, 2^24 - 1) (the culled key
// 0xffffffff maps to 2^24 - 1, behind every visible one); the third pass then
// writes the final buffer and the fourth does nothing.  Each pass counts the
// next pass's digits (the projection counts the first).
struct DepthRel {
    int pass;             // 0..3
    uint32_t* kout_final;  // third pass: the final buffers, taken when three passes suffice
    uint32_t* vout_final;
    uint32_t* next_hist;   // digit counts of the next pass (copy c at c * hist_stride), nullptr after the last
};

hipError_t launch_radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                             const uint32_t* n_dev, uint32_t n_host, int shift, const uint32_t* ghist,
                             int hist_stride, int hist_copies, uint64_t* lb, uint32_t* counter, Ctrl* ctrl,
                             hipStream_t st, int nt, int ipt, const DepthRel* rel = nullptr);
// Whether a radix pass of nt threads x ipt items per block over `items` keys
// fits on the device at once (resident-grid block order).
bool radix_resident(int nt, int ipt, int64_t items);

}  // namespace dqo
