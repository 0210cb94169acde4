// Device-side helpers and launch interfaces shared by the libdqo translation
// units.  gfx950 (CDNA4) only: wave64, 160 KiB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dqo.h"

namespace dqo {

constexpr int kWave = 64;
constexpr int kParams = DQO_NUM_PARAMS;
// Splat record (one 64-byte line in FP32): mx,my,A,B,C,o,z,id,r,g,b,pad, then
// the item's first pair slot, its tile rectangle's x0 | y0 << 16 and width,
// pad.  The render kernels read the first kRecWords and build their walk
// records from them.
constexpr int kSplatWords = 16;
constexpr int kRecWords = 12;
constexpr int kSpSlot = 12, kSpRect = 13, kSpRectW = 14;
constexpr int kGradWords = 10;    // dmx,dmy,dA,dB,dC, o*do, dr,dg,db,dz
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kSortThreads = 256;
// Items per thread of a radix pass.  The decoupled look-back costs one memory
// latency per window of preceding blocks, so longer blocks shorten the chain
// but lengthen each block's own ranking and scatter.  Measured on one MI355X:
// the pair passes take short blocks (then 4096 items; 4608 now, below) while
// that grid fits on the device at once (1.5M pairs of the 640x480 view: 1761 -> 1788 it/s against 8192) and
// 8192-item blocks beyond (49M pairs of eight keyframes: 163 -> 175 it/s); the
// depth passes are fastest with 2048-item blocks at 200k items (4096: 1700 ->
// 1672 it/s, 8192 slower still) and with 8192-item blocks from about a
// million (175 -> 180 it/s at 9.6M); 4096 in between.
// Workgroup sizes of the depth and pair passes (256 or 1024 threads).
#ifndef DQO_DEPTH_NT
#define DQO_DEPTH_NT 256
#endif
#ifndef DQO_PAIR_NT
#define DQO_PAIR_NT 512
#endif
#ifndef DQO_PAIR_IPT_SHORT
#define DQO_PAIR_IPT_SHORT (DQO_PAIR_NT == 512 ? 9 : DQO_PAIR_NT == 256 ? 16 : 8)
#endif
#ifndef DQO_DEPTH_IPT_SMALL
#define DQO_DEPTH_IPT_SMALL (DQO_DEPTH_NT == 256 ? 8 : 4)
#endif
// Pair passes whose grid fits on the device at once: 512 threads x 9 pairs
// (4608-pair blocks, two per CU; 22.7 -> 21.3 us per pass at 1.5M pairs
// against 256 x 16); longer grids: 256 x 32.
constexpr int kDepthNt = DQO_DEPTH_NT, kPairNt = DQO_PAIR_NT, kPairNtLong = 256;
constexpr int kPairIptShort = DQO_PAIR_IPT_SHORT, kPairIptLong = 32;
constexpr int kPairTileMin = kPairNt * kPairIptShort < kPairNtLong * kPairIptLong ? kPairNt * kPairIptShort
                                                                                   : kPairNtLong * kPairIptLong;  // sizes the pair look-back arrays
inline int depth_ipt(int64_t items) {
    constexpr int s = DQO_DEPTH_IPT_SMALL;
    return items < (int64_t(1) << 18) ? s : items < (int64_t(1) << 19) ? 2 * s : 4 * s;
}
// Scan + emission: one record per thread, 512 per block, so that each of the
// 8 wavefronts emits the pairs of its own 64 records (with the first pair
// pass fused, two blocks share a CU: 35.8 -> 34.4 us at the 200k view against
// 1024; 256 per block: 46.5 us).
constexpr int kSegLen = 64;        // pairs per backward segment of a 64-pixel tile
constexpr int kSegMax = 255;       // segments per tile (the last one takes the rest of the range)
constexpr uint32_t kNoBoundary = 0xFFFFFFFFu;  // segment-list entry of a tile's last segment: no restart
// Pair values are item indices; the render forward sets this bit on the pairs
// whose Gaussian cannot contribute at any pixel of their tile, and the render
// backward skips those pairs without loading their records.
constexpr uint32_t kPairSkip = 0x80000000u;
constexpr uint32_t kPairItem = 0x7FFFFFFFu;
#ifndef DQO_SCAN_THREADS
#define DQO_SCAN_THREADS 512
#endif
constexpr int kScanThreads = DQO_SCAN_THREADS;
constexpr int kScanIpt = 1;  // 2 and 4 measured slower at 200k items (1646 -> 1627 / 1573 it/s)
constexpr int kScanTile = kScanThreads * kScanIpt;
constexpr int kMaxDepthPasses = 4;
constexpr int kMaxPairPasses = 4;
constexpr int kLossBlocks = 512;
constexpr int kLossParts = 8;      // partial sums per loss workgroup (6 used)
// Scratch of the allocation-free object loss: kLossBlocks - 1 rows of
// kLossParts partial sums and the valid-depth count (32 KiB per device).
constexpr int kNoAllocScratchDoubles = kLossParts * (kLossBlocks - 1) + 1;
constexpr int kNoAllocMaxDevices = 64;

// Counter slots in the control block (dynamic block index per look-back chain).
constexpr int kCounterDepth = 0;   // + pass
constexpr int kCounterScan = 4;    // scan + emission blocks (ticket order after a timeout)
constexpr int kCounterPair = 5;    // + pass
constexpr int kCounterAdam = 12;   // workgroups done in the fused project-backward + Adam
constexpr int kCounterSegTotal = 13;  // entries in the backward's segment list
constexpr int kNumCounters = 16;
constexpr int kHistCopies = 16;
constexpr int kProjItems = 4;      // items per thread of the projection kernel

// Control block at the start of DQO_BUF_CONTROL.
struct Ctrl {
    uint32_t status;
    uint32_t epoch;
    uint32_t num_pairs;   // total pairs requested (may exceed the capacity)
    uint32_t n_valid;     // valid-depth pixel count of the last loss
    uint32_t counters[kNumCounters];
    // Which forward the segmented backward's boundary states, tile ends and
    // segment list belong to: the binning epoch and the addresses of that
    // forward's `last` and `target` images.  A backward whose frame or images
    // differ walks the whole tiles instead (the stored states are not its own).
    uint64_t seg_stamp[3];
    // Digit histograms of every radix pass, in kHistCopies copies: a workgroup
    // adds its counts to copy (block index mod kHistCopies), which spreads the
    // atomics over more addresses; a radix pass sums the copies of its digit.
    uint32_t hist_depth[kHistCopies][kMaxDepthPasses][kRadixBins];
    uint32_t hist_pair[kHistCopies][kMaxPairPasses][kRadixBins];
    double loss_partials[kLossBlocks][kLossParts];
    // The frame's visible depth keys in kHistCopies copies (projection
    // workgroup w adds to copy w mod kHistCopies): max of ~key (so that the
    // cleared word is neutral) and max of key.
    uint32_t dkey_range[kHistCopies][2];
};

template <typename T>
struct DevCam {
    T R[9];
    T t[3];
    T fx, fy, cx, cy;
    T limx, limy;  // |x/z|, |y/z| limits of the projection Jacobian (1.3 x half field of view)
    int32_t seg_lo, seg_hi;  // Gaussians [seg_lo, seg_hi) are seen by this view
    int32_t win_x0, win_y0, win_x1, win_y1;    // pixels rendered: x0 <= u < x1, y0 <= v < y1
    int32_t tile_x0, tile_y0, tile_x1, tile_y1;  // tiles overlapping the window (inclusive; empty if x1 < x0)
    int32_t job;  // -1 whole-scene view, else the object of a per-object job
};

// Whether pixel (u, v) of a view is rendered (inside the image and the window).
template <typename T>
__device__ __forceinline__ bool in_window(const DevCam<T>& c, int u, int v) {
    return u >= c.win_x0 && u < c.win_x1 && v >= c.win_y0 && v < c.win_y1;
}

// The target id a view's pixel is rendered against: the observed id t in a
// whole-scene view; in a per-object job of object k, k where t == k and -1
// ("not this object", probability T_final) elsewhere.
__device__ __forceinline__ int job_target(int job, int t) { return job < 0 ? t : (t == job ? job : -1); }

// Everything a kernel needs to know about the views (passed by value).
template <typename T>
struct Views {
    DevCam<T> cam[DQO_MAX_VIEWS];
    int n_views;
    int W, H;
    int tile_w, tile_h;
    int tiles_x, tiles_y;
    int tiles_per_view;
};

template <typename T>
struct Consts {
    T z_near, dilation, q_max, alpha_min, alpha_max, t_min;
    T bg[3];
};

// Segments of a tile's pair range for the segmented backward (0 for an empty
// tile); the last one takes the rest of the range when a tile has more than
// kSegMax.
// Segmenting the backward pays where there are few tiles for the machine (the
// longest ranges then finish last); with more tiles than this the grid is
// balanced by tiles alone and the boundary states, the list and the restarts
// only add work (measured: 1M Gaussians at 1200x680, 12750 tiles, backward
// 11% slower segmented).
constexpr int kSegTilesMax = 8192;
// The boundary state at pair position b (a multiple of kSegLen past its
// tile's first position rs) is record rs / kSegLen + (b - rs) / kSegLen: the
// records of different tiles never meet (a tile of n pairs has fewer than
// n / kSegLen boundaries and the next starts n positions later), and they
// stay below capacity / kSegLen + 1.
__host__ __device__ constexpr uint32_t boundary_record(uint32_t rs, uint32_t k) { return rs / kSegLen + k; }
__device__ __forceinline__ uint32_t tile_segments(uint32_t range) {
    return min((range + kSegLen - 1) / (uint32_t)kSegLen, (uint32_t)kSegMax);
}

// Look-back words: [flag:2 | epoch:30 | value:32].
constexpr uint64_t kFlagAggregate = 1ull;
constexpr uint64_t kFlagInclusive = 2ull;
constexpr uint32_t kSpinLimit = 1u << 22;

__device__ __forceinline__ uint64_t lb_pack(uint64_t flag, uint32_t epoch, uint32_t value) {
    return (flag << 62) | ((uint64_t)(epoch & 0x3fffffffu) << 32) | value;
}
__device__ __forceinline__ uint32_t lb_flag(uint64_t w, uint32_t epoch) {
    return ((uint32_t)(w >> 32) & 0x3fffffffu) == (epoch & 0x3fffffffu) ? (uint32_t)(w >> 62) : 0u;
}
__device__ __forceinline__ void lb_store(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t lb_load(const uint64_t* p) {
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix of `slot` over the chain 0..slot-1 (decoupled look-back).
// Publishes the aggregate first, then the inclusive value.  Every wait is
// bounded: on timeout the status bit is set and the partial sum is used.
#ifndef DQO_LB_WINDOW
#define DQO_LB_WINDOW 8
#endif
__device__ __forceinline__ uint32_t lookback_exclusive(uint64_t* words, int stride, int slot, uint32_t agg,
                                                       uint32_t epoch, uint32_t* status) {
    if (slot == 0) {
        lb_store(words, lb_pack(kFlagInclusive, epoch, agg));
        return 0u;
    }
    lb_store(words + (size_t)slot * stride, lb_pack(kFlagAggregate, epoch, agg));
    uint32_t excl = 0;
    int j = slot - 1;
    uint32_t spins = 0;
    // Look back over a window of predecessors per round trip: the loads are
    // independent, so the walk costs one memory latency per kLbWindow blocks
    // (when every block starts at once, the inclusive prefix advances by one
    // window per round trip).  A stalled block re-reads its whole window, so
    // wide windows cost bandwidth: 8 measured fastest of 8, 16, 32 and 64
    // (49 and 367 blocks of 256 digit chains).
    constexpr int kLbWindow = DQO_LB_WINDOW;
    while (j >= 0) {
        uint64_t w[kLbWindow];
#pragma unroll
        for (int k = 0; k < kLbWindow; ++k)
            w[k] = (j - k >= 0) ? lb_load(words + (size_t)(j - k) * stride) : lb_pack(kFlagInclusive, epoch, 0u);
        bool finished = false, stalled = false;
        int used = 0;
#pragma unroll
        for (int k = 0; k < kLbWindow; ++k) {
            if (finished || stalled) continue;
            const uint32_t f = lb_flag(w[k], epoch);
            if (f == 0) {
                stalled = true;
                continue;
            }
            excl += (uint32_t)w[k];
            ++used;
            if (f == kFlagInclusive) finished = true;
        }
        if (finished) break;
        j -= used;
        if (stalled) {
            if (++spins > kSpinLimit) {
                atomicOr(status, (uint32_t)DQO_STATUS_TIMEOUT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    lb_store(words + (size_t)slot * stride, lb_pack(kFlagInclusive, epoch, excl + agg));
    return excl;
}

// Sum of the values published at words[j * stride], j in [lo, hi), waiting
// for each to carry this epoch; the loads of up to 8 entries are in flight at
// once and only the entries not yet published are read again.
__device__ __forceinline__ uint32_t lb_sum_published(const uint64_t* words, int stride, int lo, int hi,
                                                     uint32_t epoch, uint32_t* status) {
    uint32_t sum = 0, spins = 0;
    for (int j0 = lo; j0 < hi; j0 += 8) {
        uint32_t pending = (hi - j0 >= 8) ? 0xFFu : ((1u << (hi - j0)) - 1u);
        while (pending) {
            uint64_t w[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) w[k] = ((pending >> k) & 1u) ? lb_load(words + (size_t)(j0 + k) * stride) : 0ull;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (((pending >> k) & 1u) && lb_flag(w[k], epoch) != 0u) {
                    sum += (uint32_t)w[k];
                    pending &= ~(1u << k);
                }
            }
            if (pending) {
                if (++spins > kSpinLimit) {
                    atomicOr(status, (uint32_t)DQO_STATUS_TIMEOUT);
                    return sum;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
    }
    return sum;
}

// Exclusive prefix of `slot` over 0..slot-1 when every block of the grid
// starts at once.  The chained walk above then reads every predecessor's
// aggregate, a window per round trip (slot / 16 round trips in all, as the
// inclusive values spread).  Here blocks form groups of kLbGroup: each block
// publishes its aggregate, the last block of a group sums the group and
// publishes the group's total at gwords, and a block adds the totals of the
// groups before its own to the aggregates of the blocks before it in its
// group: three round trips, and far fewer loads.  Blocks wait only on blocks
// of lower index.
constexpr int kLbGroup = 16;
#ifndef DQO_LB_GROUPED
#define DQO_LB_GROUPED 1
#endif
__host__ __device__ constexpr int lb_groups(int blocks) { return (blocks + kLbGroup - 1) / kLbGroup; }
__host__ __device__ constexpr int lb_blocks(int blocks) { return blocks + lb_groups(blocks); }  // words per digit
__device__ __forceinline__ uint32_t lookback_grouped(uint64_t* words, uint64_t* gwords, int stride, int slot,
                                                     uint32_t agg, uint32_t epoch, uint32_t* status) {
    lb_store(words + (size_t)slot * stride, lb_pack(kFlagAggregate, epoch, agg));
    const int g = slot / kLbGroup, first = g * kLbGroup;
    const uint32_t in_group = lb_sum_published(words, stride, first, slot, epoch, status);
    if (slot == first + kLbGroup - 1)
        lb_store(gwords + (size_t)g * stride, lb_pack(kFlagAggregate, epoch, in_group + agg));
    return in_group + lb_sum_published(gwords, stride, 0, g, epoch, status);
}

template <typename T>
__device__ __forceinline__ T fast_exp(T x);
template <>
__device__ __forceinline__ float fast_exp<float>(float x) { return __expf(x); }
template <>
__device__ __forceinline__ double fast_exp<double>(double x) { return exp(x); }

// Reciprocal: the hardware v_rcp_f32 (1 ulp) in FP32, exact division in FP64.
template <typename T>
__device__ __forceinline__ T fast_rcp(T x);
template <>
__device__ __forceinline__ float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <>
__device__ __forceinline__ double fast_rcp<double>(double x) { return 1.0 / x; }

template <typename T>
__device__ __forceinline__ T id_to_word(int id);
template <>
__device__ __forceinline__ float id_to_word<float>(int id) { return __int_as_float(id); }
template <>
__device__ __forceinline__ double id_to_word<double>(int id) { return (double)id; }

template <typename T>
__device__ __forceinline__ int word_to_id(T w);
template <>
__device__ __forceinline__ int word_to_id<float>(float w) { return __float_as_int(w); }
template <>
__device__ __forceinline__ int word_to_id<double>(double w) { return (int)w; }

// Quaternion (normalised, w,x,y,z) to rotation matrix, row-major.
template <typename T>
__device__ __forceinline__ void quat_rot(T w, T x, T y, T z, T R[9]) {
    R[0] = T(1) - T(2) * (y * y + z * z);
    R[1] = T(2) * (x * y - w * z);
    R[2] = T(2) * (x * z + w * y);
    R[3] = T(2) * (x * y + w * z);
    R[4] = T(1) - T(2) * (x * x + z * z);
    R[5] = T(2) * (y * z - w * x);
    R[6] = T(2) * (x * z - w * y);
    R[7] = T(2) * (y * z + w * x);
    R[8] = T(1) - T(2) * (x * x + y * y);
}

}  // namespace dqo

// ---- launchers (host functions defined in the .hip files) -------------------
namespace dqo {

struct StatePtrs {
    void* splats;
    short4* rects;
    uint32_t* counts;
    uint32_t* offsets;
    uint32_t* depth_keys[3];  // [0]: the state buffer; [1], [2]: scratch of the depth passes
    uint32_t* depth_vals[3];
    uint32_t* pair_keys[2];
    uint32_t* pair_vals[2];
    uint32_t* ranges;
    uint32_t* schedule;   // [V*tiles] launch order of the render workgroups
    // Segmented backward of 64-pixel tiles: a tile's pair range is walked in
    // segments of kSegLen pairs, one wavefront each, restarted from
    // per-pixel states the forward stores at the segment boundaries.
    uint4* seg_list;      // [seg_cap] (tile, first position, walk end, boundary record) in launch order (after the forward)
    uint32_t* seg_base;   // [V*tiles] first entry of each tile's segments in the backward's list
    int32_t* tile_last;   // [V*tiles] last blended position in each tile (forward)
    void* ckpt;           // [ckpt_cap][6][64] T, colour (3), depth, target probability before each boundary
    int64_t seg_cap, ckpt_cap;
    void* partials;
    void* sums;           // [V*n][kGradWords] per-item totals of the pair partials
    double* pose_partials;  // [V][ceil(n/256)][6] per-block camera-pose gradient sums
    uint8_t* written;     // [cap] 1 where the render backward wrote the pair's partials
    uint32_t* scan_base;  // [scan blocks] pair offset of each scan block (two-level scan)
    Ctrl* ctrl;
    uint64_t* lb_depth;   // [kMaxDepthPasses][blocks][256]
    uint64_t* lb_scan;    // [blocks][257]: 256 digits of the fused first pair pass, then the pair count
    uint64_t* lb_pair;    // [kMaxPairPasses][blocks][256]
    int64_t items;        // V * n
    int64_t capacity;
    int depth_blocks;     // radix blocks over items
    int scan_blocks;
    int pair_blocks;      // radix blocks over capacity
    int pair_passes;
    int pair_first_buf;   // buffer emission writes into so the sort ends in buffer 0
    // Per-tile depth order: items are not sorted by depth; pairs are emitted
    // in item order (order = identity) and each tile's pairs sorted after the
    // tile sort.
    bool tile_sort;
    bool fused_emit;      // the emission performs the first pair pass (resident scan grid)
    int tile_sort_lds;    // longest tile range sorted in LDS (longer ones: global-memory passes)
    int hist_copies_depth;  // histogram copies in use (1..kHistCopies), by producer workgroup count
    int hist_copies_pair;
};

template <typename T>
struct Frame {
    Views<T> views;
    Consts<T> consts;
    int64_t n;
    int K;
    StatePtrs s;
};

template <typename T>
hipError_t launch_project_bin(const Frame<T>& f, const T* params, const int32_t* ids, hipStream_t st);
hipError_t launch_pair_sort(const StatePtrs& s, int tiles_total, hipStream_t st);
// Workgroups of the scan + emission (fused with the first pair pass or not)
// that the device holds at once.
int scan_emit_resident(bool fused);
template <typename T>
hipError_t launch_render_forward(const Frame<T>& f, const dqo_images& img, hipStream_t st);
template <typename T>
hipError_t launch_render_backward(const Frame<T>& f, const dqo_images& img, const dqo_image_grads& g,
                                  hipStream_t st);
template <typename T>
hipError_t launch_project_backward(const Frame<T>& f, const T* params, T* grads, hipStream_t st);
// Object loss over V images of HW pixels; per-workgroup partial sums in
// partials[loss_partial_blocks(V * HW)][kLossParts] (at most kLossBlocks - 1
// rows), the valid-depth pixel count in *n_valid.  views: each view's pixel
// window and job (-1 whole scene).
struct LossViewsHost {
    int32_t win[DQO_MAX_VIEWS][4];
    int32_t job[DQO_MAX_VIEWS];
    int32_t W;
};
int loss_partial_blocks(int64_t npix);
template <typename T>
hipError_t launch_object_loss(int64_t HW, int V, const dqo_images& img, const dqo_targets& tgt,
                              const dqo_loss_weights& w, double* loss, const dqo_image_grads& g,
                              const LossViewsHost& views, double* partials, uint32_t* n_valid, hipStream_t st);
template <typename T>
hipError_t launch_adam(T* p, const T* g, T* m, T* v, int64_t n, const dqo_adam& hp, int64_t step, int64_t* d_step,
                       hipStream_t st, int rows = kParams);
hipError_t launch_id_boxes(const int32_t* id_map, int n_views, int W, int H, int K, double* boxes, int32_t* box_obj,
                           int32_t* box_view, hipStream_t st);
hipError_t launch_fit_quadric(int n_obj, int64_t n_boxes, const double* boxes, const int32_t* box_obj,
                              const int32_t* box_view, int n_views, const double* P, const int32_t* img_wh,
                              double border, double* Q, double* mu, double* R, double* axes,
                              int32_t* status, hipStream_t st);
hipError_t launch_clear_ctrl(Ctrl* ctrl, uint64_t* lb, int64_t lb_words, hipStream_t st);
hipError_t launch_clear_status(Ctrl* ctrl, hipStream_t st);
hipError_t launch_zero_words(uint32_t* p, int64_t n, hipStream_t st);

// The order in which items emit their pairs (and own consecutive pair
// slots): the depth order, or item order (nullptr) under per-tile depth order.
inline const uint32_t* item_order(const StatePtrs& s) { return s.tile_sort ? nullptr : s.depth_vals[0]; }

// Workgroups of Kernel (at Threads per group, no dynamic LDS) that the
// current device holds at once, computed once per kernel; 0 if unknown.
template <auto Kernel, int Threads>
inline int resident_blocks() {
    static const int n = [] {
        int dev = 0, per_cu = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, Kernel, Threads, 0) != hipSuccess) return 0;
        return per_cu * prop.multiProcessorCount;
    }();
    return n;
}
hipError_t launch_clear_written(const StatePtrs& s, hipStream_t st);
// Whether the 64-pixel-tile backward of a frame with these tiles runs
// segmented (the forward then stores boundary states and the sort their
// offsets).
inline bool segmented_backward(const StatePtrs& s, int tiles_total) {
    return s.ckpt_cap > 0 && tiles_total > 0 && tiles_total <= kSegTilesMax;
}
hipError_t launch_associate(int n_obj, const double* mu, const double* R, const double* ax, int64_t n_det,
                            const double* boxes, const int32_t* det_frame, int n_frames, const double* P,
                            const int32_t* img_wh, double iou_min, double* iou, int32_t* match, double* occ,
                            hipStream_t st);
hipError_t launch_quadric_distance(int na, const double* mu_a, const double* R_a, const double* ax_a, int nb,
                                   const double* mu_b, const double* R_b, const double* ax_b, double tau, double* qd,
                                   hipStream_t st);
hipError_t launch_associate_decide(int64_t n_det, int n_obj, const int32_t* match, const double* qd_obs,
                                   const double* occ, const double* qd_det, const int32_t* label, double qd_min,
                                   double t_occ, double qd_occ, int32_t* fine, int32_t* parent, int32_t* root,
                                   int32_t* obj, hipStream_t st);
hipError_t launch_quadric_iou_grad(int n_obj, int n_views, int64_t n_boxes, const double* boxes,
                                   const int32_t* box_obj, const int32_t* box_view, const double* P,
                                   const int32_t* img_wh, const double* theta, double* loss, double* grad,
                                   double* box_iou, hipStream_t st);
hipError_t launch_refine_quadrics(int n_obj, int n_views, int64_t n_boxes, const double* boxes,
                                  const int32_t* box_obj, const int32_t* box_view, const double* P,
                                  const int32_t* img_wh, const int32_t* status, const dqo_refine_cfg& c, double* mu,
                                  double* R, double* axes, double* Q, double* loss, double* box_iou, hipStream_t st);
template <typename T>
hipError_t launch_pose_backward(const Frame<T>& f, const T* params, double* pose, hipStream_t st);
template <typename T>
hipError_t launch_project_backward_adam(const Frame<T>& f, T* params, T* grads, T* m, T* v, const dqo_adam& hp,
                                        int64_t* d_step, hipStream_t st);
template <typename T>
hipError_t launch_incremental_masks(const Frame<T>& f, const dqo_images& img, const dqo_targets& tgt,
                                    const dqo_increment_cfg& cfg, uint8_t* masks, int32_t* counts, hipStream_t st);
template <typename T>
hipError_t launch_densify(const Frame<T>& f, const dqo_targets& tgt, const uint8_t* masks,
                          const dqo_increment_cfg& cfg, int64_t n_old, int64_t n_cap, T* params, int32_t* ids,
                          int64_t* counts, hipStream_t st);

}  // namespace dqo
