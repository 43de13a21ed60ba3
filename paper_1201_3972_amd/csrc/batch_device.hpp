// batch_device.hpp -- one persistent launch over a batch of frames of uneven
// size, pixel type and window (the FNR filter of fnr_device.hpp, one pass).
//
// The host lists every frame's tiles in one index space per window class and
// uploads, per batch: a descriptor per frame, a tile -> frame map and a queue
// {next, total, base} per class.
// Workgroups take tiles from the queue with one atomic each; the atomic for the
// next tile is issued before the current tile's loads, so its latency hides
// behind them.  Per tile the workgroup switches (uniformly) to the device code
// of the frame's pixel type and window; LDS is sized for the largest window of
// the kernel's class.  Tiles of all frames interleave in the queue, so large
// and small frames, cheap and expensive windows share the device evenly.
#pragma once

#include "fnr_device.hpp"

namespace irf {

struct FrameDesc {
    const uint8_t *src;
    uint8_t *dst;
    uint64_t src_pitch, dst_pitch;
    unsigned long long *count;  // nullable: += noisy pixels of this frame
    int width, height;
    int tiles_x, tiles;  // tiles of this frame
    int tile_begin;      // first tile of this frame in the class's index space
    int kind;            // batch_kind(dtype bytes, window)
    int aligned;
    int pad;
};

struct BatchQueue {
    unsigned int next;   // next tile to hand out
    unsigned int total;  // tiles in the class
    unsigned int base;   // the class's first entry in the tile -> frame map
    unsigned int pad;
};

// Window classes, one kernel each: 3..9 (selection networks; 4 waves per SIMD),
// 11..15 (networks; 2 waves), and one class per window above 15x15 (group
// bisection; their code does not share one kernel without spilling).  LDS and
// registers are sized for the class's largest window, so a batch whose windows
// all lie in one class (the usual video mixes of 3..9) runs as one persistent
// launch.
constexpr int kBatchClasses = 10;
constexpr int kBatchClassMin[kBatchClasses] = {3, 11, 17, 19, 21, 23, 25, 27, 29, 31};
constexpr int kBatchClassMax[kBatchClasses] = {9, 15, 17, 19, 21, 23, 25, 27, 29, 31};
// Occupancy targets: every window's code sits in its class's kernel, whose
// register count is the worst case over them; these targets keep each kernel at
// the occupancy of its largest window's own kernel without spilling.
constexpr int kBatchClassWaves[kBatchClasses] = {4, 2, 2, 2, 2, 2, 2, 2, 2, 2};

__host__ __device__ constexpr int batch_kind(int bytes, int window) {
    return (bytes == 1 ? 0 : 16) + (window - 3) / 2;
}
__host__ __device__ constexpr int batch_class(int window) {
    return window <= kBatchClassMax[0] ? 0 : (window <= kBatchClassMax[1] ? 1 : 2 + (window - 17) / 2);
}

// One tile of the queue, with the stack kernel's issue order: the tile's global
// loads go out before the barrier that frees the LDS of the previous tile
// (inside load_tile), and wave priorities favour every phase but detection.
template <typename T, int K, int NT>
__device__ __forceinline__ uint32_t batch_tile(const FrameDesc &d, int local, unsigned char *smem,
                                               uint32_t ticket, unsigned int *s_next, uint32_t pk_one) {
    using G = Geometry<K, NT>;
    TileSmem<K, NT> &sm = *reinterpret_cast<TileSmem<K, NT> *>(smem);
    StackArgs a = {};
    a.src = d.src;
    a.dst = d.dst;
    a.src_pitch = d.src_pitch;
    a.dst_pitch = d.dst_pitch;
    a.width = d.width;
    a.height = d.height;
    a.tiles_x = d.tiles_x;
    a.tiles_per_frame = d.tiles;
    a.total_tiles = d.tiles;
    a.aligned = d.aligned;
    a.pk_one = pk_one;
    int f, x0, y0;
    tile_origin(a, local, G::TH, f, x0, y0);
    const bool small = load_tile<T, K, NT, false, true>(a.src, a.src_pitch, a.width, a.height, x0, y0,
                                                        a.aligned != 0, sm.tile);
    post_small(sm.large, small);
    if (threadIdx.x == 0) {
        sm.count = 0;
        *s_next = ticket;  // the loads were waited for, so the atomic has returned too
    }
    __syncthreads();
    return process_tile<T, K, MODE_FNR, NT, default_select(K), true>(a, local, sm, tile_small<NT>(sm.large));
}

// The tile's device code by (pixel type, window) among the class's windows:
// a uniform branch over the kinds, each an inlined filter body.
template <int CLASS, int NT, int K = kBatchClassMin[CLASS]>
__device__ __forceinline__ uint32_t batch_dispatch(const FrameDesc &d, int local, unsigned char *smem,
                                                   uint32_t ticket, unsigned int *slot, uint32_t pk_one) {
    if constexpr (K > kBatchClassMax[CLASS]) {
        // no such kind (the host admits only windows of the class): hand the
        // next ticket on so the loop still advances
        if (threadIdx.x == 0) *slot = ticket;
        __syncthreads();
        return 0;
    } else {
        if (d.kind == batch_kind(1, K)) return batch_tile<uint8_t, K, NT>(d, local, smem, ticket, slot, pk_one);
        if (d.kind == batch_kind(2, K)) return batch_tile<uint16_t, K, NT>(d, local, smem, ticket, slot, pk_one);
        return batch_dispatch<CLASS, NT, K + 2>(d, local, smem, ticket, slot, pk_one);
    }
}

template <int CLASS, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(kBatchClassWaves[CLASS], 8))) void fnr_batch_kernel(const FrameDesc *descs,
                                                             const uint32_t *tile_frame,
                                                             BatchQueue *queue, uint32_t pk_one) {
    constexpr int KMAX = kBatchClassMax[CLASS];
    __shared__ __attribute__((aligned(16))) unsigned char smem[sizeof(TileSmem<KMAX, NT>)];
    // next-tile slots alternate by iteration: thread 0 fills slot i&1 of
    // iteration i before the barrier that follows the tile's load, and every
    // thread reads it at the end of the iteration; the next write to that slot
    // (iteration i+2) lies behind the barriers of iteration i+1
    __shared__ unsigned int s_next[2];
    const unsigned int total = queue->total;
    tile_frame += queue->base;
    if (threadIdx.x == 0) s_next[0] = atomicAdd(&queue->next, 1u);
    __syncthreads();
    unsigned int t = s_next[0];
    for (unsigned int it = 1; t < total; ++it) {
        unsigned int *slot = &s_next[it & 1];
        t = __builtin_amdgcn_readfirstlane(t);  // uniform: descriptor reads become scalar
        const FrameDesc d = descs[tile_frame[t]];
        const int local = (int)t - d.tile_begin;
        uint32_t ticket = 0;
        if (threadIdx.x == 0) ticket = atomicAdd(&queue->next, 1u);
        const uint32_t flagged = batch_dispatch<CLASS, NT>(d, local, smem, ticket, slot, pk_one);
        if (d.count != nullptr && (threadIdx.x & 63) == 0 && flagged != 0)
            atomicAdd(d.count, (unsigned long long)flagged);
        t = *slot;  // the barrier inside the next load_tile frees this tile's LDS
    }
}

}  // namespace irf
