// fused_device.hpp -- two passes of the FNR filter in one launch.
//
// The iterative use of the method (the filter applied to its own output, the
// procedure behind Figs. 5-6 of Section 4) reads and writes every frame once per
// pass when the passes run as separate launches.  Here one tile runs both: the
// staged input block gets pass 1 (detection, medians of the flagged pixels)
// in LDS, and pass 2 then reads those results straight from LDS.  Pass 2 of an
// output pixel needs pass-1 results within r of it, so a tile's pass-2 output
// is its 128-column block less 4 columns on each side (enough for r <= 4) and
// less r rows at the top and bottom: tiles overlap, and the overlap is computed
// twice.  Each pass reads an unchanged copy of the previous pass's frame, as in
// the separate launches, so the result equals two single passes exactly,
// borders included: before pass 2, block pixels outside the frame take the
// pass-1 result of the nearest frame pixel (the replicated border of the
// pass-1 frame).
#pragma once

#include "fnr_device.hpp"

namespace irf {

// Output columns of a fused tile, and the largest window it serves.
constexpr int kFusedTileW = kTileW - 8;
constexpr int kFusedMaxWindow = 9;

template <int K, int NT>
struct FusedGeometry {
    using G = Geometry<K, NT>;
    static constexpr int out_rows = G::TH - 2 * G::r;  // pass-2 output rows per tile
    static_assert(K <= kFusedMaxWindow && G::r <= 4, "pass-1 ring of 4 columns covers r <= 4");
    static_assert(G::halo >= 2 * G::r, "the input halo covers both passes");
};

// Persistent kernel over fused tiles.  Tile t of frame f has its output origin
// (ox, oy) = (kFusedTileW * (t % tiles_x), out_rows * (t / tiles_x)) and its
// block at (ox - 4, oy - r).  Counts: a.count[0] += pass-1 flags and
// a.count[1] += pass-2 flags, each over the output pixels only, so that every
// pixel of the frame is counted once per pass.  Issue order as in the stack
// kernel: the block's loads go out before the barrier that frees the previous
// block's LDS, and both detections run at the lowest wave priority, every
// other phase at the highest.
template <typename T, int K, int NT, int SEL>
__global__ __launch_bounds__(NT) void fnr_fused2_kernel(StackArgs a) {
    using G = Geometry<K, NT>;
    constexpr int R = G::R, r = G::r, TH = G::TH;
    constexpr int OH = FusedGeometry<K, NT>::out_rows;
    __shared__ __attribute__((aligned(16))) TileSmem<K, NT> sm;
    const TileRange rg = xcd_range(blockIdx.x, gridDim.x, a.total_tiles);
    const bool aligned = a.aligned != 0;
    const int W = a.width, H = a.height;
    const int tid = threadIdx.x;
    const int tx = tid % kThreadsX, strip = tid / kThreadsX;
    const int centre0 = (strip * R + r) * G::pitch + G::halo + 4 * tx;
    uint32_t n1 = 0, n2 = 0;  // this thread's output pixels flagged by pass 1 and pass 2
    for (int t = rg.first; t < rg.end; t += rg.stride) {
        const int f = t / a.tiles_per_frame;
        const int rem = t - f * a.tiles_per_frame;
        const int ty = rem / a.tiles_x;
        const int ox = (rem - ty * a.tiles_x) * kFusedTileW, oy = ty * OH;
        const int x0 = ox - 4, y0 = oy - r;
        const bool small = load_tile<T, K, NT, true, true>(a.src + (uint64_t)f * a.src_stride, a.src_pitch, W, H,
                                                           x0, y0, aligned, sm.tile);
        post_small(sm.large, small);
        if (tid == 0) sm.count = 0;
        __syncthreads();
        // pass 2 reads pass-1 results, which are values of the staged block, so
        // the staged values decide both passes' detection path
        const bool f16 = tile_small<NT>(sm.large);
        const int px = x0 + 4 * tx, py = y0 + strip * R;
        const uint32_t in_frame = box_bits(R, px, py, 0, W, 0, H);
        const uint32_t out = box_bits(R, px, py, ox, min(ox + kFusedTileW, W), oy, min(oy + OH, H));

        // pass 1 on every frame pixel of the block
        const uint32_t f1 = (f16 ? detect_block<K, true>(sm.tile, strip, tx, a.pk_one)
                                 : detect_block<K, false>(sm.tile, strip, tx, a.pk_one)) &
                            in_frame;
        n1 += __builtin_popcount(f1 & out);
        if constexpr (K == 3) {
            // dense 3 x 3 path: the whole block in registers, written back once
            // every thread has read the input tile
            uint32_t o1[R][2];
            dense3_block<R>(sm.tile, strip, tx, f1, o1);
            __syncthreads();
#pragma unroll
            for (int q = 0; q < R; ++q)
                *reinterpret_cast<uint2 *>(sm.tile + centre0 + q * G::pitch) = make_uint2(o1[q][0], o1[q][1]);
        } else {
            median_into_tile<K, NT, SEL, G::tile_px, true>(sm, f1, centre0, t, a.pk_one);
        }
        if (tid == 0) sm.count = 0;  // every thread read the pass-1 list length before its selection
        __syncthreads();

        // block pixels outside the frame: the pass-1 result of the nearest frame
        // pixel (those are never written here, so one barrier suffices)
        if (x0 < 0 || y0 < 0 || x0 + kTileW > W || y0 + TH > H) {  // uniform
            uint32_t m = ~in_frame;
            while (m) {
                const int b = __builtin_ctz(m);
                m &= m - 1;
                const int col = bit_col(b), row = bit_row(b);
                const int cx = min(max(px + col, 0), W - 1), cy = min(max(py + row, 0), H - 1);
                sm.tile[centre0 + row * G::pitch + col] = sm.tile[centre0 + (cy - py) * G::pitch + (cx - px)];
            }
            __syncthreads();
        }

        // pass 2 on the output pixels
        __builtin_amdgcn_s_setprio(0);
        const uint32_t f2 = (f16 ? detect_block<K, true>(sm.tile, strip, tx, a.pk_one)
                                 : detect_block<K, false>(sm.tile, strip, tx, a.pk_one)) &
                            out;
        n2 += __builtin_popcount(f2);
        uint32_t o2[R][2];
        if constexpr (K == 3) {
            dense3_block<R>(sm.tile, strip, tx, f2, o2);
        } else {
            median_into_tile<K, NT, SEL, G::tile_px, true>(sm, f2, centre0, t, a.pk_one);
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const uint2 c = *reinterpret_cast<const uint2 *>(sm.tile + centre0 + q * G::pitch);
                o2[q][0] = c.x;
                o2[q][1] = c.y;
            }
        }

        // store the thread's output pixels (a thread holds whole 4-column groups
        // of the output, or none; the last tile of a row may end inside one)
        __builtin_amdgcn_s_setprio(3);
        if (out != 0) {
            uint8_t *dst = a.dst + (uint64_t)f * a.dst_stride;
            const int xend = min(ox + kFusedTileW, W);
#pragma unroll
            for (int q = 0; q < R; ++q) {
                if (((out >> q) & 1u) == 0) continue;
                const uint32_t ro = __umul24((uint32_t)(py + q), (uint32_t)a.dst_pitch);
                store4<T>(dst, ro, px, xend, aligned, o2[q][0], o2[q][1]);
            }
        }
        __builtin_amdgcn_s_setprio(0);
    }
    if (a.count != nullptr) {
        const uint32_t s1 = __builtin_amdgcn_readlane(wave_inclusive_sum(n1), 63);
        const uint32_t s2 = __builtin_amdgcn_readlane(wave_inclusive_sum(n2), 63);
        if ((tid & 63) == 0) {
            if (s1 != 0) atomicAdd(a.count, (unsigned long long)s1);
            if (s2 != 0) atomicAdd(a.count + 1, (unsigned long long)s2);
        }
    }
}

}  // namespace irf
