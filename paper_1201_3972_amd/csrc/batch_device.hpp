// batch_device.hpp -- one persistent launch over a batch of frames of uneven
// size, pixel type and window (the FNR filter of fnr_device.hpp, one pass).
//
// The host lists every frame's tiles in one index space and uploads, per
// batch: a descriptor per frame, a tile -> frame map and a queue {next, total}.
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
    unsigned int pad[2];
};

// Window classes, one kernel each: 3..7, 9..11 and 13..15 (LDS and registers
// sized for the class's largest window).
constexpr int kBatchClasses = 3;
constexpr int kBatchClassMax[kBatchClasses] = {7, 11, 15};
// Occupancy targets: every window's code sits in its class's kernel, whose
// register count is the worst case over them; these targets keep each kernel at
// the occupancy of its largest window's own kernel without spilling.
constexpr int kBatchClassWaves[kBatchClasses] = {4, 3, 2};

__host__ __device__ constexpr int batch_kind(int bytes, int window) {
    return (bytes == 1 ? 0 : 8) + (window - 3) / 2;
}
__host__ __device__ constexpr int batch_class(int window) {
    return window <= kBatchClassMax[0] ? 0 : (window <= kBatchClassMax[1] ? 1 : 2);
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
    load_tile<T, K, NT, false, true>(a.src, a.src_pitch, a.width, a.height, x0, y0, a.aligned != 0, sm.tile);
    if (threadIdx.x == 0) {
        sm.count = 0;
        *s_next = ticket;  // the loads were waited for, so the atomic has returned too
    }
    __syncthreads();
    return process_tile<T, K, MODE_FNR, NT, default_select(K), true>(a, local, sm);
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
        uint32_t flagged = 0;
        if constexpr (CLASS == 0) {
            switch (d.kind) {
                case batch_kind(1, 3): flagged = batch_tile<uint8_t, 3, NT>(d, local, smem, ticket, slot, pk_one); break;
                case batch_kind(1, 5): flagged = batch_tile<uint8_t, 5, NT>(d, local, smem, ticket, slot, pk_one); break;
                case batch_kind(1, 7): flagged = batch_tile<uint8_t, 7, NT>(d, local, smem, ticket, slot, pk_one); break;
                case batch_kind(2, 3): flagged = batch_tile<uint16_t, 3, NT>(d, local, smem, ticket, slot, pk_one); break;
                case batch_kind(2, 5): flagged = batch_tile<uint16_t, 5, NT>(d, local, smem, ticket, slot, pk_one); break;
                default: flagged = batch_tile<uint16_t, 7, NT>(d, local, smem, ticket, slot, pk_one); break;
            }
        } else if constexpr (CLASS == 1) {
            switch (d.kind) {
                case batch_kind(1, 9): flagged = batch_tile<uint8_t, 9, NT>(d, local, smem, ticket, slot, pk_one); break;
                case batch_kind(1, 11): flagged = batch_tile<uint8_t, 11, NT>(d, local, smem, ticket, slot, pk_one); break;
                case batch_kind(2, 9): flagged = batch_tile<uint16_t, 9, NT>(d, local, smem, ticket, slot, pk_one); break;
                default: flagged = batch_tile<uint16_t, 11, NT>(d, local, smem, ticket, slot, pk_one); break;
            }
        } else {
            switch (d.kind) {
                case batch_kind(1, 13): flagged = batch_tile<uint8_t, 13, NT>(d, local, smem, ticket, slot, pk_one); break;
                case batch_kind(1, 15): flagged = batch_tile<uint8_t, 15, NT>(d, local, smem, ticket, slot, pk_one); break;
                case batch_kind(2, 13): flagged = batch_tile<uint16_t, 13, NT>(d, local, smem, ticket, slot, pk_one); break;
                default: flagged = batch_tile<uint16_t, 15, NT>(d, local, smem, ticket, slot, pk_one); break;
            }
        }
        if (d.count != nullptr && (threadIdx.x & 63) == 0 && flagged != 0)
            atomicAdd(d.count, (unsigned long long)flagged);
        t = *slot;  // the barrier inside the next load_tile frees this tile's LDS
    }
}

}  // namespace irf
