// fnr_device.hpp -- device code of the FNR impulse filter for gfx950.
//
// The method (Gupta, Beg, Niranjan, "A Novel Approach to Fast Image Filtering
// Algorithm of Infrared Images based on Intro Sort Algorithm"):
//   * S_xy is the k x k window around (x, y), centre included (Section 3.3);
//   * a pixel is noisy when its grey level equals the window's minimum or
//     maximum (Eq. 3a/3b and Step 2 of Section 3.3);
//   * a noisy pixel takes the window median, every other pixel keeps its value
//     (Section 3.4); the frame may be filtered several times (Section 4).
// Border windows replicate the edge pixels; each pass reads an unchanged input.
//
// A persistent workgroup of 128 threads (two waves) walks a range of tiles of
// kTileW x (4*R) output pixels.  Each tile and an r-pixel halo (rounded out to
// 8 columns) are staged in LDS as 16-bit values, whatever the pixel type.  The
// steps:
//   1. load:    coalesced 8-pixel chunks, rows and columns clamped at the border;
//   2. detect:  every thread owns 4 columns x R rows; window min and max are
//               separable: per input row a packed-u16 horizontal min/max over k
//               columns (two pixels per VGPR), then a van Herk / Gil-Werman
//               sliding min/max down the R+k-1 rows;
//   3. compact: flagged pixels of the tile go to an LDS list (wave prefix scan);
//   4. select:  networks: each lane takes two list entries and
//               computes both medians in packed u16 registers by forgetful
//               selection over sorted blocks merged into a sorted run whose
//               provably-non-median ends are dropped (window rows are read as
//               whole 32-bit words); bisection:
//               each lane holds one window in registers (two values per VGPR)
//               and bisects on grey level, counting the values above the probe
//               (bit-by-bit value search).  Which one, and the workgroup size,
//               come from the host's per-window tuning table;
//   5. store:   results replace the flagged pixels in LDS, then the tile is
//               written out with vector stores.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "netgen.hpp"

namespace irf {

constexpr int kThreads = 128;                // workgroup of the batch kernels
constexpr int kTileW = 128;                  // output columns per tile
constexpr int kThreadsX = kTileW / 4;        // 32 threads across, 4 columns each
constexpr int kStrips = kThreads / kThreadsX;  // 4 strips of R rows
// Selection algorithm: forgetful selection networks on two windows per lane,
// grey-level bisection on one window per lane, grey-level bisection on one
// window per group of 4 to 32 lanes, or a two-pass radix select over LDS
// histograms on one window per group of 16 lanes (the last two for windows
// above 15x15, whose values no longer fit one lane's registers; the radix
// select up to 31x31).
enum Select : int { kSelectNetwork = 1, kSelectBisect = 2, kSelectGroup = 3, kSelectHist = 4 };
constexpr int kNetworkMaxWindow = 15;
constexpr int kHistLanes = 16;  // lanes per window of the histogram radix select
constexpr int kHistBins = 256;  // bins of one radix pass
constexpr int kLargeMaxWindow = 31;  // windows of the radix select, the batch kernels and 256-thread tiles
// Untuned choices of the stack kernels: 5x5 and 7x7 take 256-thread workgroups
// on tiles of twice the height, which fill their selection waves better (a
// 128x32 tile holds about 80 window pairs at 7x7 at the usual impulse rates,
// just over one wave's worth); the other windows up to 15x15 run faster with
// the smaller tile, those from 17x17 to 31x31 (group bisection) with the
// larger one; above 31x31 only 128-thread tiles exist.  Networks beat bisection
// at every window (by 2.4x at 15x15).  The host's tuning table starts from
// these and an autotuner may replace them.
constexpr int default_threads(int K) {
    return (K == 5 || K == 7 || (K > kNetworkMaxWindow && K <= kLargeMaxWindow)) ? 256 : 128;
}
constexpr int default_select(int K) { return K <= kNetworkMaxWindow ? kSelectNetwork : kSelectGroup; }
constexpr int kMaxWindow = 63;

enum Mode : int {
    MODE_DETECT = 0,       // write the noise mask (and count)
    MODE_FNR = 1,          // detect, then median at the noisy pixels
    MODE_MEDIAN_MASK = 2,  // median where a caller mask is non-zero
    MODE_MEDIAN_ALL = 3,   // median everywhere (the standard median filter)
    MODE_DETECT_DIR = 4,   // write the mask of the opt-in directional detector (3x3 only)
};

// One launch covers a stack of equally sized frames laid out with fixed strides.
struct StackArgs {
    const uint8_t *src;
    uint8_t *dst;            // MODE_FNR / MODE_MEDIAN_*
    const uint8_t *mask_in;  // MODE_MEDIAN_MASK
    uint8_t *mask_out;       // MODE_DETECT
    uint64_t src_pitch, dst_pitch, mask_pitch;     // bytes between rows (< 2^24)
    uint64_t src_stride, dst_stride, mask_stride;  // bytes between frames
    int width, height;
    int tiles_x, tiles_per_frame;
    int total_tiles;
    int aligned;  // every base address and pitch is a multiple of 16 bytes
    unsigned long long *count;  // nullable: += flagged pixels
    // 0x00010001, passed in so the compiler keeps the packed min with it as one
    // v_pk_min_u16 instead of expanding it into per-half compares and selects
    uint32_t pk_one;
};

template <int K, int NT = kThreads>
struct Geometry {
    static constexpr int r = K / 2;
    static constexpr int R = 8;  // output rows per thread
    static constexpr int TH = NT / kThreadsX * R;
    static constexpr int rows = TH + 2 * r;  // LDS rows
    static constexpr int tile_px = kTileW * TH;
    // LDS columns staged left and right of the tile (8 up to 17x17, 16 up to
    // 33x33, 32 above), 8-pixel load chunks per LDS row, and the LDS row pitch
    // in 16-bit values: 8 values of padding make it 76 (84, 100) dwords, so
    // rows 8 apart (the two 32-lane halves of a wave during detection) fall on
    // opposite halves of the 64 banks.
    static constexpr int halo = r <= 8 ? 8 : r <= 16 ? 16 : 32;
    static constexpr int chunks = (kTileW + 2 * halo) / 8;
    static constexpr int pitch = kTileW + 2 * halo + 8;
    static_assert(K >= 3 && K <= kMaxWindow && (K & 1), "odd window 3..63");
    static_assert(NT % 64 == 0 && NT % kThreadsX == 0, "whole waves of whole thread rows");
    static_assert(r <= halo, "halo must cover the window radius");
    static_assert(rows * pitch <= 65536, "LDS offsets are 16-bit");
};

// ---------------------------------------------------------------------------
// packed 16-bit helpers (two pixels per 32-bit register)
// ---------------------------------------------------------------------------
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk_min(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, a),
                                                                  __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ uint32_t pk_max(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                  __builtin_bit_cast(u16x2, b)));
}
// max(a - b, 0) per half
__device__ __forceinline__ uint32_t pk_subsat(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, a),
                                                                      __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ uint32_t pk_add(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) + __builtin_bit_cast(u16x2, b));
}
// (hi half of lo_word, lo half of hi_word): the pair one pixel to the right of lo_word
__device__ __forceinline__ uint32_t shift_pair(uint32_t hi_word, uint32_t lo_word) {
    return __builtin_amdgcn_alignbyte(hi_word, lo_word, 2);
}

// Three-input min / max of packed pairs for tiles whose values are all below
// 0x4000 (every 8-bit frame, and 14-bit data).  Read as IEEE half-precision
// bit patterns such values are positive and finite (normal or subnormal) and
// order exactly like the integers, and the packed half-precision minimum3 /
// maximum3 of gfx950 returns one of its inputs bit for bit (the kernels keep
// half-precision subnormals: no flushing), so one instruction does the work of
// two packed integer min / max.  Each is written as the one instruction (an
// ALU operation on registers): built from two-input minimum intrinsics, the
// compiler shares common sub-minima between neighbouring groups and emits
// three-input instructions with a repeated operand, which saves nothing.
__device__ __forceinline__ uint32_t h_min3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_pk_minimum3_f16 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
__device__ __forceinline__ uint32_t h_max3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_pk_maximum3_f16 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
// (min(a.lo, a.hi, p.lo), min(a.lo, a.hi, p.hi)), and the same for max: the
// second operand is a with its halves swapped (op_sel)
__device__ __forceinline__ uint32_t h_min_both(uint32_t a, uint32_t p) {
    uint32_t r;
    asm("v_pk_minimum3_f16 %0, %1, %1, %2 op_sel:[0,1,0] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(a), "v"(p));
    return r;
}
__device__ __forceinline__ uint32_t h_max_both(uint32_t a, uint32_t p) {
    uint32_t r;
    asm("v_pk_maximum3_f16 %0, %1, %1, %2 op_sel:[0,1,0] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(a), "v"(p));
    return r;
}
// Largest value the three-input path takes (exclusive): a tile qualifies when
// no staged value has either of the top two bits set.
constexpr uint32_t kF16SafeMask = 0xC000C000u;

// ---------------------------------------------------------------------------
// 1. tile load
// ---------------------------------------------------------------------------
// Addresses inside a frame are 32-bit byte offsets from the frame's base (the
// host keeps every frame's span below 4 GiB and its pitch below 2^24 bytes), so
// the base stays in scalar registers and a row offset is one 24-bit multiply.
template <typename T>
__device__ __forceinline__ uint32_t load_px(const uint8_t *frame, uint32_t row_off, int x) {
    if constexpr (sizeof(T) == 1)
        return frame[row_off + (uint32_t)x];
    else
        return *reinterpret_cast<const uint16_t *>(frame + (row_off + 2u * (uint32_t)x));
}

__device__ __forceinline__ uint4 widen8(uint2 b) {
    uint4 v;
    v.x = (b.x & 0xffu) | ((b.x & 0xff00u) << 8);
    v.y = ((b.x >> 16) & 0xffu) | ((b.x >> 8) & 0xff0000u);
    v.z = (b.y & 0xffu) | ((b.y & 0xff00u) << 8);
    v.w = ((b.y >> 16) & 0xffu) | ((b.y >> 8) & 0xff0000u);
    return v;
}

__device__ __forceinline__ uint4 splat8(uint32_t v) {
    uint32_t p = v | (v << 16);
    return make_uint4(p, p, p, p);
}

// One 8-pixel chunk of the frame row at byte offset row_off, starting at column
// gx, columns clamped to the frame: a vector load when the chunk lies inside
// (and the layout is 16-byte aligned), one pixel repeated when it lies wholly
// left or right of the frame, per-pixel clamped loads when it straddles an edge.
// HALF: gx is 4 more than a multiple of 8, so the chunk is loaded as two halves
// (each then aligned to its own size).
template <typename T, bool HALF = false>
__device__ __forceinline__ uint4 load_chunk(const uint8_t *frame, uint32_t row_off, int gx, int W,
                                            bool aligned) {
    if (aligned && gx >= 0 && gx + 8 <= W) {
        const uint32_t off = row_off + (uint32_t)gx * (uint32_t)sizeof(T);
        if constexpr (HALF) {
            if constexpr (sizeof(T) == 2) {
                const uint2 lo = *reinterpret_cast<const uint2 *>(frame + off);
                const uint2 hi = *reinterpret_cast<const uint2 *>(frame + off + 8u);
                return make_uint4(lo.x, lo.y, hi.x, hi.y);
            } else {
                const uint32_t lo = *reinterpret_cast<const uint32_t *>(frame + off);
                const uint32_t hi = *reinterpret_cast<const uint32_t *>(frame + off + 4u);
                return widen8(make_uint2(lo, hi));
            }
        } else if constexpr (sizeof(T) == 2) {
            return *reinterpret_cast<const uint4 *>(frame + off);
        } else {
            return widen8(*reinterpret_cast<const uint2 *>(frame + off));
        }
    }
    if (gx + 8 <= 0) return splat8(load_px<T>(frame, row_off, 0));
    if (gx >= W) return splat8(load_px<T>(frame, row_off, W - 1));
    // chunks that cross an edge are rare: an empty asm makes gx opaque here,
    // so the compiler does not compute the eight clamped columns for every
    // tile ahead of the branch
    asm volatile("" : "+v"(gx));
    uint32_t e[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) e[i] = load_px<T>(frame, row_off, min(max(gx + i, 0), W - 1));
    return make_uint4(e[0] | (e[1] << 16), e[2] | (e[3] << 16), e[4] | (e[5] << 16), e[6] | (e[7] << 16));
}

// A raw buffer resource over a frame (no range limit beyond 4 GiB; the host
// keeps every frame's span below that): loads through it take a per-thread
// 32-bit offset and a wave-uniform 32-bit offset in a scalar register, so a
// row offset that is the same for the whole wave costs no vector instruction.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t frame_rsrc(const uint8_t *frame) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(frame), (short)0, -1, 0x00020000);
}

// One 8-pixel chunk that lies wholly inside the frame on a 16-byte-aligned
// layout, at byte offset voff + soff (soff wave-uniform) from the frame base.
template <typename T, bool HALF>
__device__ __forceinline__ uint4 load_inside(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
    if constexpr (HALF) {
        if constexpr (sizeof(T) == 2) {
            const auto lo = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0);
            const auto hi = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)(voff + 8u), (int)soff, 0);
            return make_uint4(lo[0], lo[1], hi[0], hi[1]);
        } else {
            const uint32_t lo = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff, (int)soff, 0);
            const uint32_t hi = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)(voff + 4u), (int)soff, 0);
            return widen8(make_uint2(lo, hi));
        }
    } else if constexpr (sizeof(T) == 2) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voff, (int)soff, 0);
        return make_uint4(v[0], v[1], v[2], v[3]);
    } else {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0);
        return widen8(make_uint2(v[0], v[1]));
    }
}

// Stage rows y0-r .. y0+TH+r-1 and columns x0-halo .. x0+kTileW+halo-1 of a
// frame in LDS (row-major, G::pitch values apart), coordinates outside the
// frame clamped to the nearest edge pixel.  Each row is 16 interior chunks and
// 2 * HC halo chunks (HC = halo / 8 on each side): thread t loads interior
// chunk t % 16 of rows t / 16, t / 16 + NT / 16, ... and halo chunks t,
// t + NT, ... (chunk h is number h % (2 HC) of row h / (2 HC), the left ones
// first), so a thread's column is the same on every tile.  All loads are
// issued before the first LDS write.
//
// Addressing: within a round, a thread's chunk sits at a fixed offset from
// the wave's first row and the tile's first column, which are wave-uniform.
// When the rows a wave loads in a round lie inside the frame and the tile's
// columns (interior, or halo) do too (every round of most tiles), the load is
// a buffer load at that fixed offset plus a scalar one; only the other rounds
// clamp rows and columns per thread.
//
// EARLY (the persistent stack, batch and fused kernels): the workgroup
// barrier that frees the previous tile's LDS is taken here, after this
// thread's global loads are issued and before its LDS writes, so the wait at
// the barrier overlaps the loads' latency; the loads are issued at the highest
// wave priority.
// The chunks of one tile held in registers between their loads and their LDS
// writes, and the geometry of the load rounds.
template <int K, int NT>
struct TileChunks {
    using G = Geometry<K, NT>;
    static constexpr int kStep = NT / 16;
    static constexpr int kRounds = (G::rows + kStep - 1) / kStep;
    static constexpr int HC = G::halo / 8;                    // halo chunks on each side
    static constexpr int kHalos = 2 * HC * G::rows;           // halo chunks of the tile
    static constexpr int kHRounds = (kHalos + NT - 1) / NT;
    static constexpr int kHStep = NT / (2 * HC);              // halo rows per round
    static constexpr int kHWave = 64 / (2 * HC);              // halo rows of a wave in a round
    static_assert(kTileW == 16 * 8 && G::chunks == 16 + 2 * HC, "16 interior chunks per row");
    uint4 v[kRounds], h[kHRounds];
};

// The thread's halo chunk column (fixed for the whole kernel).
template <int K, int NT>
__device__ __forceinline__ int halo_column(int tid) {
    using C = TileChunks<K, NT>;
    const int which = tid % (2 * C::HC);
    return C::HC == 1 ? (which ? Geometry<K, NT>::chunks - 1 : 0) : (which < C::HC ? which : 16 + which);
}

// Issue the global loads of the tile at (x0, y0) into registers.
template <typename T, int K, int NT, bool HALF>
__device__ __forceinline__ void issue_tile(const uint8_t *src, uint64_t pitch, int W, int H, int x0, int y0,
                                           bool aligned, TileChunks<K, NT> &c) {
    using G = Geometry<K, NT>;
    using C = TileChunks<K, NT>;
    constexpr uint32_t b = sizeof(T);
    const int tid = threadIdx.x;
    const int cx = tid & 15, row0 = tid >> 4;
    const int ytop = y0 - G::r;
    const uint32_t p32 = (uint32_t)pitch;
    const __amdgpu_buffer_rsrc_t rs = frame_rsrc(src);
    // wave-uniform: the wave's first interior and halo row within a round, and
    // whether the tile's interior and halo columns lie inside the frame
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wrow = wave * 4, whrow = wave * C::kHWave;
    const bool in_x = aligned && x0 >= 0 && x0 + kTileW <= W;
    const bool in_xh = aligned && x0 - G::halo >= 0 && x0 + kTileW + G::halo <= W;
    // per thread: column and offset from the wave's first row
    const int gx = x0 + 8 * cx;
    const uint32_t voff = (uint32_t)(row0 & 3) * p32 + 8u * b * (uint32_t)cx;
    const int hrow0 = tid / (2 * C::HC);
    const int hcol = halo_column<K, NT>(tid);
    const int gxh = x0 - G::halo + 8 * hcol;
    const uint32_t voffh = (uint32_t)(hrow0 - whrow) * p32 + 8u * b * (uint32_t)hcol;
#pragma unroll
    for (int j = 0; j < C::kRounds; ++j) {
        const int row = row0 + j * C::kStep;
        const int first = ytop + j * C::kStep + wrow;  // the wave's rows: first .. first + 3
        if (in_x && first >= 0 && first + 3 < H) {
            if (j < C::kRounds - 1 || row < G::rows)
                c.v[j] = load_inside<T, HALF>(rs, voff, (uint32_t)first * p32 + (uint32_t)x0 * b);
        } else if (j < C::kRounds - 1 || row < G::rows) {
            const int gy = min(max(ytop + row, 0), H - 1);
            c.v[j] = load_chunk<T, HALF>(src, __umul24((uint32_t)gy, p32), gx, W, aligned);
        }
    }
#pragma unroll
    for (int j = 0; j < C::kHRounds; ++j) {
        const int hc = tid + j * NT;
        const int hrow = hrow0 + j * C::kHStep;
        const int first = ytop + j * C::kHStep + whrow;  // the wave's halo rows: first .. first + kHWave - 1
        if (in_xh && first >= 0 && first + C::kHWave - 1 < H) {
            if (hc < C::kHalos)
                c.h[j] = load_inside<T, HALF>(rs, voffh, (uint32_t)first * p32 + (uint32_t)(x0 - G::halo) * b);
        } else if (hc < C::kHalos) {
            const int gy = min(max(ytop + hrow, 0), H - 1);
            c.h[j] = load_chunk<T, HALF>(src, __umul24((uint32_t)gy, p32), gxh, W, aligned);
        }
    }
}

// Write the chunks into the LDS tile.
template <int K, int NT>
__device__ __forceinline__ void commit_tile(const TileChunks<K, NT> &c, uint16_t *tile) {
    using G = Geometry<K, NT>;
    using C = TileChunks<K, NT>;
    const int tid = threadIdx.x;
    const int cx = tid & 15, row0 = tid >> 4;
    const int hrow0 = tid / (2 * C::HC);
    const int hcol = halo_column<K, NT>(tid);
#pragma unroll
    for (int j = 0; j < C::kRounds; ++j) {
        const int row = row0 + j * C::kStep;
        if (j < C::kRounds - 1 || row < G::rows)
            *reinterpret_cast<uint4 *>(tile + row * G::pitch + 8 * (cx + C::HC)) = c.v[j];
    }
#pragma unroll
    for (int j = 0; j < C::kHRounds; ++j) {
        const int hc = tid + j * NT;
        if (hc < C::kHalos) {
            const int hrow = hrow0 + j * C::kHStep;
            *reinterpret_cast<uint4 *>(tile + hrow * G::pitch + 8 * hcol) = c.h[j];
        }
    }
}

// Whether every value of the thread's chunks lies below 0x4000 (the range of
// the three-input half-precision detection path).
template <int K, int NT>
__device__ __forceinline__ bool chunks_small(const TileChunks<K, NT> &c) {
    using G = Geometry<K, NT>;
    using C = TileChunks<K, NT>;
    const int tid = threadIdx.x;
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < C::kRounds; ++j) {
        const uint32_t w = c.v[j].x | c.v[j].y | c.v[j].z | c.v[j].w;
        if (j < C::kRounds - 1 || (tid >> 4) + j * C::kStep < G::rows) acc |= w;
    }
#pragma unroll
    for (int j = 0; j < C::kHRounds; ++j) {
        const uint32_t w = c.h[j].x | c.h[j].y | c.h[j].z | c.h[j].w;
        if (tid + j * NT < C::kHalos) acc |= w;
    }
    return (acc & kF16SafeMask) == 0;
}

// Stage the tile; returns whether the values this thread staged all lie below
// 0x4000 (always for 8-bit frames; callers that do not use it drop the test).
template <typename T, int K, int NT = kThreads, bool HALF = false, bool EARLY = false>
__device__ __forceinline__ bool load_tile(const uint8_t *src, uint64_t pitch, int W, int H, int x0,
                                          int y0, bool aligned, uint16_t *tile) {
    TileChunks<K, NT> c;
    if constexpr (EARLY) __builtin_amdgcn_s_setprio(3);
    issue_tile<T, K, NT, HALF>(src, pitch, W, H, x0, y0, aligned, c);
    if constexpr (EARLY) {
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
    }
    commit_tile<K, NT>(c, tile);
    if constexpr (sizeof(T) == 1)
        return true;
    else
        return chunks_small<K, NT>(c);
}

// ---------------------------------------------------------------------------
// 2. detection: separable window min / max on packed pairs
// ---------------------------------------------------------------------------
// Half swaps and broadcasts fold into the op_sel fields of the packed min/max.
__device__ __forceinline__ u16x2 as_pair(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ uint32_t both_min(uint32_t x) {  // min of the halves, in both halves
    const u16x2 v = as_pair(x);
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(v, __builtin_shufflevector(v, v, 1, 0)));
}
__device__ __forceinline__ uint32_t both_max(uint32_t x) {
    const u16x2 v = as_pair(x);
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(v, __builtin_shufflevector(v, v, 1, 0)));
}
__device__ __forceinline__ uint32_t hi_lo(uint32_t a, uint32_t b) {  // (a.hi, b.lo)
    return __builtin_bit_cast(uint32_t, __builtin_shufflevector(as_pair(a), as_pair(b), 1, 2));
}

// One aligned 8-byte LDS word as two dwords.  The empty asm takes the word
// whole, so the read stays a 64-bit LDS read: left alone, the compiler splits
// such a word into dword reads and pairs them again in its own order, and the
// dword pairs' 8-bit offsets reach only three tile rows from one address (a new
// address per few rows), while lanes two dwords apart collide in the LDS banks.
// In the detection rows the 64-bit reads measured 1.6-3% faster at 7x7 on the
// 640x512 stack, and most kernels hold fewer VGPRs.
__device__ __forceinline__ void lds_word2(const void *p, uint32_t &lo, uint32_t &hi) {
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    u32x2 w = *reinterpret_cast<const u32x2 *>(p);
    asm("" : "+v"(w));
    lo = w.x;
    hi = w.y;
}

// Horizontal min/max over k columns for the thread's 4 output columns of one
// LDS row.  `p` points at the thread's first output column.  Outputs: packed
// pair 0 = columns (0,1), pair 1 = columns (2,3); c0, c1 = the centre pairs.
//
// Odd radius r = 2m+1: with E_j the aligned pair (columns 2j, 2j+1), output
// column 0 takes columns -r..r and column 1 takes -r+1..r+1.  Both contain the
// r whole pairs E_-m..E_m; their min over both halves (a packed min with the
// halves swapped) plus the one column each still lacks, -r for column 0 and
// r+1 for column 1, packed into one pair, gives pair 0.  Pair 1 is the same two
// columns further right, and shares E_-m+1..E_m with pair 0.  No odd-aligned
// pair is ever formed.
template <int r, bool F16 = false>
__device__ __forceinline__ void row_minmax_odd(const uint16_t *p, uint32_t &mn0, uint32_t &mn1,
                                               uint32_t &mx0, uint32_t &mx1, uint32_t &c0, uint32_t &c1) {
    constexpr int m = (r - 1) / 2;
    constexpr int JLO = (-m - 1) & ~1, JHI = (m + 2) | 1;  // whole aligned 8-byte words
    constexpr int NJ = JHI - JLO + 1;
    const uint2 *q = reinterpret_cast<const uint2 *>(p);
    uint32_t D[NJ];
#pragma unroll
    for (int j = 0; j < NJ; j += 2) lds_word2(q + (j + JLO) / 2, D[j], D[j + 1]);
    auto E = [&](int j) -> uint32_t { return D[j - JLO]; };
    const uint32_t p0 = hi_lo(E(-m - 1), E(m + 1)), p1 = hi_lo(E(-m), E(m + 2));
    c0 = E(0);
    c1 = E(1);
    if constexpr (F16) {
        // E_-m+1 .. E_m-1 (an odd count) folded in threes, then E_m with each
        // output pair's own end pair
        uint32_t smn = E(1 - m), smx = smn;
#pragma unroll
        for (int j = 2 - m; j + 1 <= m - 1; j += 2) {
            smn = h_min3(smn, E(j), E(j + 1));
            smx = h_max3(smx, E(j), E(j + 1));
        }
        const uint32_t a_mn = h_min3(smn, E(m), E(-m)), a_mx = h_max3(smx, E(m), E(-m));
        const uint32_t b_mn = h_min3(smn, E(m), E(m + 1)), b_mx = h_max3(smx, E(m), E(m + 1));
        mn0 = h_min_both(a_mn, p0);
        mx0 = h_max_both(a_mx, p0);
        mn1 = h_min_both(b_mn, p1);
        mx1 = h_max_both(b_mx, p1);
        return;
    }
    uint32_t a_mn = E(0), a_mx = E(0), b_mn = E(1), b_mx = E(1);
    if constexpr (m > 0) {
        uint32_t smn = E(1 - m), smx = smn;  // E_-m+1 .. E_m, shared by both pairs
#pragma unroll
        for (int j = 2 - m; j <= m; ++j) {
            smn = pk_min(smn, E(j));
            smx = pk_max(smx, E(j));
        }
        a_mn = pk_min(smn, E(-m));
        a_mx = pk_max(smx, E(-m));
        b_mn = pk_min(smn, E(m + 1));
        b_mx = pk_max(smx, E(m + 1));
    }
    mn0 = pk_min(both_min(a_mn), p0);
    mx0 = pk_max(both_max(a_mx), p0);
    mn1 = pk_min(both_min(b_mn), p1);
    mx1 = pk_max(both_max(b_mx), p1);
}

// Even radius and 3x3: the shared middle offsets with odd-aligned pairs built by
// byte alignment (at 3x3 this measured faster than the odd-radius form).
template <int r, bool F16 = false>
__device__ __forceinline__ void row_minmax(const uint16_t *p, uint32_t &mn0, uint32_t &mn1,
                                           uint32_t &mx0, uint32_t &mx1, uint32_t &c0, uint32_t &c1) {
    if constexpr ((r & 1) && r >= 3) {
        row_minmax_odd<r, F16>(p, mn0, mn1, mx0, mx1, c0, c1);
        return;
    }
    // pairs JLO..JHI cover columns -r .. 3+r; the range is widened to whole
    // 8-byte words so every LDS read is aligned
    constexpr int JLO = (-((r + 1) / 2)) & ~1;
    constexpr int JHI = ((3 + r) / 2) | 1;
    constexpr int NJ = JHI - JLO + 1;
    const uint2 *q = reinterpret_cast<const uint2 *>(p);
    uint32_t D[NJ];
#pragma unroll
    for (int j = 0; j < NJ; j += 2) lds_word2(q + (j + JLO) / 2, D[j], D[j + 1]);
    // V(o) = packed (pixel o, pixel o+1) relative to output column 0
    auto V = [&](int o) -> uint32_t {
        if ((o & 1) == 0) return D[o / 2 - JLO];
        return shift_pair(D[(o + 1) / 2 - JLO], D[(o - 1) / 2 - JLO]);
    };
    // pair 0 needs offsets -r..r, pair 1 needs 2-r..r+2; share 2-r..r
    uint32_t smin = V(2 - r), smax = smin;
    uint32_t a = V(-r), b = V(1 - r), c = V(r + 1), d = V(r + 2);
    c0 = D[0 - JLO];
    c1 = D[1 - JLO];
    if constexpr (F16) {
        // 2r - 2 shared offsets after the first, folded in threes
#pragma unroll
        for (int o = 3 - r; o + 1 <= r; o += 2) {
            const uint32_t v = V(o), w = V(o + 1);
            smin = h_min3(smin, v, w);
            smax = h_max3(smax, v, w);
        }
        mn0 = h_min3(smin, a, b);
        mx0 = h_max3(smax, a, b);
        mn1 = h_min3(smin, c, d);
        mx1 = h_max3(smax, c, d);
        return;
    }
#pragma unroll
    for (int o = 3 - r; o <= r; ++o) {
        uint32_t v = V(o);
        smin = pk_min(smin, v);
        smax = pk_max(smax, v);
    }
    mn0 = pk_min(smin, pk_min(a, b));
    mx0 = pk_max(smax, pk_max(a, b));
    mn1 = pk_min(smin, pk_min(c, d));
    mx1 = pk_max(smax, pk_max(c, d));
}

// Flag bit layout inside a thread's 32-bit mask: bit q (+0, +16, +8, +24) is
// column 0 (1, 2, 3) of output row q.
__device__ __forceinline__ int bit_col(int b) { return (((b >> 3) & 1) << 1) | (b >> 4); }
__device__ __forceinline__ int bit_row(int b) { return b & 7; }

// Flags of the thread's 4 x R block (bit set = noisy).
//
// Rows are consumed in order.  The vertical window min/max of output row o is
// op(suffix of the K-row block holding row o, from o; prefix of the next block,
// up to o+K-1) -- van Herk / Gil-Werman with blocks of K rows.  A block's
// suffixes are formed when its last row arrives, prefixes run as rows arrive,
// and every output row is turned into flag bits as soon as both parts exist, so
// only about one block of horizontal results is live at a time.
template <int K, bool F16 = false>
__device__ __forceinline__ uint32_t detect_block_blocks(const uint16_t *tile, int strip, int tx,
                                                        uint32_t pk_one) {
    using G = Geometry<K>;
    constexpr int R = G::R, L = R + K - 1;
    const uint16_t *base = tile + strip * R * G::pitch + G::halo + 4 * tx;
    uint32_t mn0[L], mn1[L], mx0[L], mx1[L];  // horizontal results, then block suffixes
    uint32_t pmn0[L], pmn1[L], pmx0[L], pmx1[L];  // running prefixes within a block
    uint32_t c0[R], c1[R];
    uint32_t flags = 0;
    auto emit = [&](int o, uint32_t vmn0, uint32_t vmn1, uint32_t vmx0, uint32_t vmx1) {
        // a half is zero exactly when the centre equals the window min or max;
        // 1 - min(z, 1) turns that into one flag bit per half
        const uint32_t z0 = pk_min(pk_subsat(c0[o], vmn0), pk_subsat(vmx0, c0[o]));
        const uint32_t z1 = pk_min(pk_subsat(c1[o], vmn1), pk_subsat(vmx1, c1[o]));
        const uint32_t f0 = pk_subsat(pk_one, z0);
        const uint32_t f1 = pk_subsat(pk_one, z1);
        flags |= (f0 | (f1 << 8)) << o;
    };
    static_for(std::make_integer_sequence<int, L>{}, [&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int blk = i / K, first = blk * K;
        uint32_t a, b;
        row_minmax<G::r, F16>(base + i * G::pitch, mn0[i], mn1[i], mx0[i], mx1[i], a, b);
        if constexpr (i >= G::r && i < G::r + R) {
            c0[i - G::r] = a;
            c1[i - G::r] = b;
        }
        // running prefix of this block
        if constexpr (i == first) {
            pmn0[i] = mn0[i]; pmn1[i] = mn1[i]; pmx0[i] = mx0[i]; pmx1[i] = mx1[i];
        } else {
            pmn0[i] = pk_min(pmn0[i - 1], mn0[i]); pmn1[i] = pk_min(pmn1[i - 1], mn1[i]);
            pmx0[i] = pk_max(pmx0[i - 1], mx0[i]); pmx1[i] = pk_max(pmx1[i - 1], mx1[i]);
        }
        // output o = i-K+1 straddling two blocks: suffix of its block + this prefix
        constexpr int o = i - K + 1;
        if constexpr (o >= 0 && o < R && o % K != 0)
            emit(o, pk_min(mn0[o], pmn0[i]), pk_min(mn1[o], pmn1[i]), pk_max(mx0[o], pmx0[i]),
                 pk_max(mx1[o], pmx1[i]));
        // block complete: suffixes in place, and the output that starts the
        // block.  The last block has no block after it, so no output straddles
        // out of it: its one output (when it starts one) takes the running
        // prefix, which already spans the whole block.
        if constexpr (i == L - 1 && i - first == K - 1) {
            if constexpr (first < R) emit(first, pmn0[i], pmn1[i], pmx0[i], pmx1[i]);
        } else if constexpr (i % K == K - 1 || i == L - 1) {
            static_for(std::make_integer_sequence<int, i - first>{}, [&](auto jc) {
                constexpr int j = i - 1 - decltype(jc)::value;
                mn0[j] = pk_min(mn0[j], mn0[j + 1]); mn1[j] = pk_min(mn1[j], mn1[j + 1]);
                mx0[j] = pk_max(mx0[j], mx0[j + 1]); mx1[j] = pk_max(mx1[j], mx1[j + 1]);
            });
            if constexpr (first < R && i - first == K - 1)
                emit(first, mn0[first], mn1[first], mx0[first], mx1[first]);
        }
    });
    return flags;
}

// The same flags for windows taller than the thread's block (K > R): rows
// [R-1, K) lie in every output row's window (the core, reduced as it streams
// by); output row o also needs the suffix of rows [o, R-1) and the prefix of
// rows [K, o+K).  Only the R-1 rows before the core are held.
template <int K, bool F16 = false>
__device__ __forceinline__ uint32_t detect_block_core(const uint16_t *tile, int strip, int tx,
                                                      uint32_t pk_one) {
    using G = Geometry<K>;
    constexpr int R = G::R, L = R + K - 1, A = R - 1;
    static_assert(K > R && A > 0, "core split needs windows taller than the block");
    const uint16_t *base = tile + strip * R * G::pitch + G::halo + 4 * tx;
    uint32_t mn0[A], mn1[A], mx0[A], mx1[A];          // rows before the core, then suffixes
    uint32_t cmn0 = 0, cmn1 = 0, cmx0 = 0, cmx1 = 0;  // core
    uint32_t pmn0 = 0, pmn1 = 0, pmx0 = 0, pmx1 = 0;  // prefix of the rows after the core
    uint32_t c0[R], c1[R];
    uint32_t flags = 0;
    auto emit = [&](int o, uint32_t vmn0, uint32_t vmn1, uint32_t vmx0, uint32_t vmx1) {
        const uint32_t z0 = pk_min(pk_subsat(c0[o], vmn0), pk_subsat(vmx0, c0[o]));
        const uint32_t z1 = pk_min(pk_subsat(c1[o], vmn1), pk_subsat(vmx1, c1[o]));
        const uint32_t f0 = pk_subsat(pk_one, z0);
        const uint32_t f1 = pk_subsat(pk_one, z1);
        flags |= (f0 | (f1 << 8)) << o;
    };
    static_for(std::make_integer_sequence<int, L>{}, [&](auto ic) {
        constexpr int i = decltype(ic)::value;
        uint32_t a0, a1, b0, b1, ca, cb;
        row_minmax<G::r, F16>(base + i * G::pitch, a0, a1, b0, b1, ca, cb);
        if constexpr (i >= G::r && i < G::r + R) {
            c0[i - G::r] = ca;
            c1[i - G::r] = cb;
        }
        if constexpr (i < A) {
            mn0[i] = a0; mn1[i] = a1; mx0[i] = b0; mx1[i] = b1;
        } else if constexpr (i < K) {
            if constexpr (i == A) {
                cmn0 = a0; cmn1 = a1; cmx0 = b0; cmx1 = b1;
            } else {
                cmn0 = pk_min(cmn0, a0); cmn1 = pk_min(cmn1, a1);
                cmx0 = pk_max(cmx0, b0); cmx1 = pk_max(cmx1, b1);
            }
            if constexpr (i == K - 1) {
                // suffixes of the rows before the core, each folded with the core
                mn0[A - 1] = pk_min(mn0[A - 1], cmn0); mn1[A - 1] = pk_min(mn1[A - 1], cmn1);
                mx0[A - 1] = pk_max(mx0[A - 1], cmx0); mx1[A - 1] = pk_max(mx1[A - 1], cmx1);
                static_for(std::make_integer_sequence<int, A - 1>{}, [&](auto jc) {
                    constexpr int j = A - 2 - decltype(jc)::value;
                    mn0[j] = pk_min(mn0[j], mn0[j + 1]); mn1[j] = pk_min(mn1[j], mn1[j + 1]);
                    mx0[j] = pk_max(mx0[j], mx0[j + 1]); mx1[j] = pk_max(mx1[j], mx1[j + 1]);
                });
                emit(0, mn0[0], mn1[0], mx0[0], mx1[0]);
            }
        } else {
            if constexpr (i == K) {
                pmn0 = a0; pmn1 = a1; pmx0 = b0; pmx1 = b1;
            } else {
                pmn0 = pk_min(pmn0, a0); pmn1 = pk_min(pmn1, a1);
                pmx0 = pk_max(pmx0, b0); pmx1 = pk_max(pmx1, b1);
            }
            constexpr int o = i - K + 1;  // rows [o, o+K) are now all seen
            if constexpr (o < A)
                emit(o, pk_min(mn0[o], pmn0), pk_min(mn1[o], pmn1), pk_max(mx0[o], pmx0),
                     pk_max(mx1[o], pmx1));
            else
                emit(o, pk_min(cmn0, pmn0), pk_min(cmn1, pmn1), pk_max(cmx0, pmx0), pk_max(cmx1, pmx1));
        }
    });
    return flags;
}

template <int K, bool F16 = false>
__device__ __forceinline__ uint32_t detect_block(const uint16_t *tile, int strip, int tx,
                                                 uint32_t pk_one) {
    if constexpr (K > Geometry<K>::R)
        return detect_block_core<K, F16>(tile, strip, tx, pk_one);
    else
        return detect_block_blocks<K, F16>(tile, strip, tx, pk_one);
}

// Flags of the opt-in directional detector for the thread's 4 x R block (not
// the paper's detector; a reading of Fig. 1's caption): a pixel is flagged when,
// on each of the four lines through it in its 3 x 3 window (row, column, both
// diagonals), its grey level lies outside the range of its two neighbours,
// ties counting as inside.  Per LDS row the thread holds the aligned pairs
// (0,1), (2,3) and the odd pairs (-1,0), (1,2), (3,4); "outside" is nonzero
// per half exactly when the centre is below the line's minimum or above its
// maximum.
template <int K>
__device__ __forceinline__ uint32_t directional_block(const uint16_t *tile, int strip, int tx,
                                                      uint32_t pk_one) {
    using G = Geometry<K>;
    static_assert(K == 3, "the directional test is defined on the 3 x 3 window");
    constexpr int R = G::R;
    const uint16_t *base = tile + strip * R * G::pitch + G::halo + 4 * tx;
    uint32_t C0[R + 2], C1[R + 2], L0[R + 2], M[R + 2], R1[R + 2];
#pragma unroll
    for (int i = 0; i < R + 2; ++i) {
        const uint2 *q = reinterpret_cast<const uint2 *>(base + i * G::pitch);
        const uint2 w0 = q[-1], w1 = q[0], w2 = q[1];  // columns -4..-1, 0..3, 4..7
        C0[i] = w1.x;
        C1[i] = w1.y;
        L0[i] = shift_pair(w1.x, w0.y);
        M[i] = shift_pair(w1.y, w1.x);
        R1[i] = shift_pair(w2.x, w1.y);
    }
    auto outside = [](uint32_t c, uint32_t a, uint32_t b) {
        return pk_subsat(pk_min(a, b), c) | pk_subsat(c, pk_max(a, b));
    };
    uint32_t flags = 0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int i = q + 1;
        // row, column, diagonal (top-left to bottom-right), anti-diagonal
        const uint32_t z0 = pk_min(pk_min(outside(C0[i], L0[i], M[i]), outside(C0[i], C0[i - 1], C0[i + 1])),
                                   pk_min(outside(C0[i], L0[i - 1], M[i + 1]), outside(C0[i], M[i - 1], L0[i + 1])));
        const uint32_t z1 = pk_min(pk_min(outside(C1[i], M[i], R1[i]), outside(C1[i], C1[i - 1], C1[i + 1])),
                                   pk_min(outside(C1[i], M[i - 1], R1[i + 1]), outside(C1[i], R1[i - 1], M[i + 1])));
        flags |= (pk_min(z0, pk_one) | (pk_min(z1, pk_one) << 8)) << q;
    }
    return flags;
}

// Bits of the thread's block that lie inside the frame.
__device__ __forceinline__ uint32_t valid_bits(int R, int W, int H, int px, int py) {
    int rows = min(max(H - py, 0), R);
    uint32_t rb = (rows >= 8) ? 0xffu : ((1u << rows) - 1u);
    uint32_t m = 0;
    if (px + 0 < W) m |= rb;
    if (px + 1 < W) m |= rb << 16;
    if (px + 2 < W) m |= rb << 8;
    if (px + 3 < W) m |= rb << 24;
    return m;
}

// Bits of the thread's block (columns px..px+3, rows py..py+R-1, any of them
// possibly negative) whose pixel lies in columns [xlo, xhi) and rows [ylo, yhi).
__device__ __forceinline__ uint32_t box_bits(int R, int px, int py, int xlo, int xhi, int ylo, int yhi) {
    const int r0 = min(max(ylo - py, 0), R), r1 = min(max(yhi - py, 0), R);
    const uint32_t rb = r1 > r0 ? (((r1 - r0) >= 32 ? 0xffffffffu : ((1u << (r1 - r0)) - 1u)) << r0) : 0u;
    uint32_t m = 0;
    if (px + 0 >= xlo && px + 0 < xhi) m |= rb;
    if (px + 1 >= xlo && px + 1 < xhi) m |= rb << 16;
    if (px + 2 >= xlo && px + 2 < xhi) m |= rb << 8;
    if (px + 3 >= xlo && px + 3 < xhi) m |= rb << 24;
    return m;
}

// ---------------------------------------------------------------------------
// 4. median selection on two windows at once (packed u16)
// ---------------------------------------------------------------------------
template <int... I, typename F>
__device__ __forceinline__ void static_for(std::integer_sequence<int, I...>, F &&f) {
    (f(std::integral_constant<int, I>{}), ...);
}

// Compare-exchange of two packed pairs (both halves at once).
__device__ __forceinline__ void cex(uint32_t &a, uint32_t &b) {
    const uint32_t lo = pk_min(a, b);
    b = pk_max(a, b);
    a = lo;
}

// Sort a[0..N) with the odd-even merge network (indices are compile-time).
template <int N>
__device__ __forceinline__ void sort_block(uint32_t *a) {
    static_for(std::make_integer_sequence<int, net::Network<N>::size>{}, [&](auto c) {
        constexpr int i = net::network<N>.lo[decltype(c)::value];
        constexpr int j = net::network<N>.hi[decltype(c)::value];
        cex(a[i], a[j]);
    });
}

// Merge sorted a[0..L) and sorted b[0..S) into out[0..L+S).  Both halves of the
// merge network are padded with 0xffff (+infinity for 16-bit values); the
// compiler folds every comparison against the padding constant.
template <int L, int S>
__device__ __forceinline__ void merge_sorted(const uint32_t *a, const uint32_t *b, uint32_t *out) {
    constexpr int P = net::pow2_at_least(L > S ? L : S);
    uint32_t x[2 * P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        x[i] = i < L ? a[i] : 0xffffffffu;
        x[P + i] = i < S ? b[i] : 0xffffffffu;
    }
    static_for(std::make_integer_sequence<int, net::MergeNetwork<P>::size>{}, [&](auto c) {
        constexpr int i = net::merge_network<P>.lo[decltype(c)::value];
        constexpr int j = net::merge_network<P>.hi[decltype(c)::value];
        cex(x[i], x[j]);
    });
#pragma unroll
    for (int i = 0; i < L + S; ++i) out[i] = x[i];
}

// Block sizes of the forgetful selection (first block, later blocks).
template <int K>
struct BlockPlan {
    static constexpr int N = K * K;
    static constexpr int block = K <= 3 ? 4 : (K <= 5 ? 8 : 16);
    static constexpr int size_at(int pos) { return block < N - pos ? block : N - pos; }
    static constexpr int max_run = 64;
};

// One row of two K x K windows, packed: out[i] holds a value of window 0 in its
// low half and one of window 1 in its high half.  q0 and q1 point at the 32-bit
// LDS words holding the rows' first values, p0 and p1 are the parities of the
// rows' first columns.  A row is read as the (K+1)/2 whole words that cover it,
// so no LDS access straddles a word: with even parity the row runs from the low
// half of word 0 to the low half of word K/2, with odd parity from the high
// half of word 0 to the high half of word K/2.  Only that one value differs
// between the parities; the values come out in a fixed order that is not the
// column order, which the median ignores.
// 3 x 3 rows are read value by value instead (three 16-bit reads per window and
// row cost less than the word reads and the byte permutes).
struct PairRow {
    const uint16_t *w0, *w1;  // first values of the windows' top rows
    const uint32_t *q0, *q1;  // the words holding them
    uint32_t s0, s1;          // byte selectors of the parity-dependent values
};

__device__ __forceinline__ PairRow pair_row(const uint16_t *tile, uint32_t o0, uint32_t o1) {
    const uint32_t *t32 = reinterpret_cast<const uint32_t *>(tile);
    // the parity-dependent value of window 0 goes to bytes 0-1, that of window 1
    // to bytes 2-3 (source bytes 0-3 = word 0, 4-7 = word K/2)
    return {tile + o0, tile + o1, t32 + (o0 >> 1), t32 + (o1 >> 1), 0x0100u + (o0 & 1) * 0x0606u,
            (0x0100u + (o1 & 1) * 0x0606u) << 16};
}

template <int K>
__device__ __forceinline__ void load_pair_row(const PairRow &w, int row, uint32_t *out) {
    if constexpr (K == 3) {
#pragma unroll
        for (int i = 0; i < K; ++i) {
            u16x2 v;  // element-wise build lets the compiler load straight into each half
            v.x = w.w0[row * Geometry<K>::pitch + i];
            v.y = w.w1[row * Geometry<K>::pitch + i];
            out[i] = __builtin_bit_cast(uint32_t, v);
        }
        return;
    }
    constexpr int D = (K + 1) / 2;
    constexpr uint32_t kLoLo = 0x05040100u, kHiHi = 0x07060302u, kLoHi = 0x07060100u;
    uint32_t a[D], b[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        a[j] = w.q0[row * (Geometry<K>::pitch / 2) + j];
        b[j] = w.q1[row * (Geometry<K>::pitch / 2) + j];
    }
    int n = 0;
    out[n++] = __builtin_amdgcn_perm(b[0], a[0], kHiHi);
#pragma unroll
    for (int j = 1; j < D - 1; ++j) {
        out[n++] = __builtin_amdgcn_perm(b[j], a[j], kLoLo);
        out[n++] = __builtin_amdgcn_perm(b[j], a[j], kHiHi);
    }
    out[n++] = __builtin_amdgcn_perm(b[D - 1], a[D - 1], kLoLo);
    const uint32_t x0 = __builtin_amdgcn_perm(a[D - 1], a[0], w.s0);
    const uint32_t x1 = __builtin_amdgcn_perm(b[D - 1], b[0], w.s1);
    out[n++] = __builtin_amdgcn_perm(x1, x0, kLoHi);
}

// Forgetful selection over sorted blocks.  State: a sorted run of L values, the
// rank T (0-based) that the median has among the run plus the N-POS values not
// yet read.  Each step sorts the next block, merges it into the run and drops
// every value that cannot have rank T: the DLOW smallest (even if all unread
// values were smaller they would still rank below T) and the DHIGH largest
// (more than T run values lie below them).  When every value has been read the
// run holds exactly one value, the median.
template <int K, int POS, int L, int T>
__device__ __forceinline__ uint32_t select_blocks(const uint32_t *run, const PairRow &w, uint32_t *win) {
    constexpr int N = K * K;
    if constexpr (POS == N) {
        static_assert(L == 1, "forgetful selection must end with one value");
        return run[0];
    } else {
        constexpr int S = BlockPlan<K>::size_at(POS);
        constexpr int M = L + S;
        constexpr int U = N - POS - S;
        constexpr int DLOW = T - U > 0 ? T - U : 0;
        constexpr int DHIGH = M - 1 - T > 0 ? M - 1 - T : 0;
        constexpr int NL = M - DLOW - DHIGH;
        static_assert(M <= 2 * BlockPlan<K>::max_run, "run too long");
        // rows are read when the block that reaches their first value starts
#pragma unroll
        for (int row = (POS + K - 1) / K; row * K < POS + S; ++row) load_pair_row<K>(w, row, win + row * K);
        uint32_t blk[S];
#pragma unroll
        for (int i = 0; i < S; ++i) blk[i] = win[POS + i];
        sort_block<S>(blk);
        uint32_t merged[M];
        if constexpr (L == 0) {
#pragma unroll
            for (int i = 0; i < S; ++i) merged[i] = blk[i];
        } else {
            merge_sorted<L, S>(run, blk, merged);
        }
        return select_blocks<K, POS + S, NL, T - DLOW>(merged + DLOW, w, win);
    }
}

template <int K>
__device__ __forceinline__ uint32_t median_pair(const uint16_t *tile, uint32_t o0, uint32_t o1) {
    static_assert(Geometry<K>::pitch % 2 == 0, "window rows must keep their parity");
    uint32_t win[K * K];
    return select_blocks<K, 0, 0, (K * K - 1) / 2>(nullptr, pair_row(tile, o0, o1), win);
}

// One window per lane held in registers (the default for 13x13 and 15x15), two
// window values per VGPR: a bisection on grey level over [g_min, g_max] counts
// the values above the probe with three packed operations per register and
// round (the window is read from LDS once).  pk_one = 0x00010001 from the host
// (a literal lets the compiler split the packed count into per-half compares).
template <int K>
__device__ __forceinline__ uint32_t median_registers(const uint16_t *w, uint32_t pk_one) {
    constexpr int N = K * K, NP = (N + 1) / 2;
    constexpr uint32_t rank = (N - 1) / 2;
    uint32_t v[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int e0 = 2 * j, e1 = 2 * j + 1;
        const uint32_t lo = w[(e0 / K) * Geometry<K>::pitch + e0 % K];
        // an odd element count leaves the last high half empty: it repeats the
        // last element, whose second copy is taken out of the count below
        const uint32_t hi = e1 < N ? w[(e1 / K) * Geometry<K>::pitch + e1 % K] : lo;
        v[j] = lo | (hi << 16);
    }
    uint32_t mn = 0xffffffffu, mx = 0u;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        mn = pk_min(mn, v[j]);
        mx = pk_max(mx, v[j]);
    }
    uint32_t lo = min(mn & 0xffffu, mn >> 16), hi = max(mx & 0xffffu, mx >> 16);
    const uint32_t pad = (N & 1) ? (v[NP - 1] >> 16) : 0u;  // duplicated value (odd N)
    while (lo < hi) {
        const uint32_t t = (lo + hi) >> 1;
        const uint32_t tt = t | (t << 16);
        uint32_t above = 0;
#pragma unroll
        for (int j = 0; j < NP; ++j) above = pk_add(above, pk_min(pk_subsat(v[j], tt), pk_one));
        uint32_t gt = (above & 0xffffu) + (above >> 16);
        if ((N & 1) && pad > t) gt -= 1;
        if (N - gt > rank)
            hi = t;
        else
            lo = t + 1;
    }
    return lo;
}

// One window per group of lanes (windows above 15x15).  The group's L lanes
// (aligned inside a 16-lane DPP row, or a 32-lane half of the wave) hold the
// window's values g, g + L, g + 2L, ... (S_xy order), two per VGPR, and run the
// same grey-level bisection as median_registers with counts summed over the
// group by DPP butterflies (and one lane swizzle across the two rows of a
// 32-lane group).  Registers past the window's end repeat its first value,
// taken back out of every count.  L is the smallest group whose share fits 48
// registers (4 lanes at 17x17 and 19x19, 8 up to 27x27, 16 up to 39x39); the
// windows above take 32 lanes and up to 63 registers each (63x63).  Each round
// costs every lane three packed operations per register plus log2(L) butterfly
// steps, so fewer lanes waste fewer steps, while larger shares cost the kernel
// occupancy.
template <int K>
struct GroupPlan {
    static constexpr int N = K * K;
    static constexpr int regs_for(int l) { return (N + 2 * l - 1) / (2 * l); }
    static constexpr int lanes = regs_for(4) <= 48 ? 4 : regs_for(8) <= 48 ? 8 : regs_for(16) <= 48 ? 16 : 32;
    static constexpr int regs = regs_for(lanes);  // packed registers per lane
    static constexpr int pad = 2 * lanes * regs - N;                // repeated values in the group
    static_assert(K > lanes, "a lane's next value is at most one window row further");
    static_assert(regs <= 64, "a lane's share of the window fits 64 registers");
};

// op over the aligned group of L lanes (L = 4, 8, 16 or 32), result in every
// lane.
template <int L, typename Op>
__device__ __forceinline__ uint32_t group_reduce(uint32_t v, Op op) {
    static_assert(L == 4 || L == 8 || L == 16 || L == 32, "groups of 4, 8, 16 or 32 lanes");
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xf, 0xf, false));   // lane ^ 1
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xf, 0xf, false));   // lane ^ 2
    if constexpr (L >= 8)
        v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, false));  // 7 - lane in 8
    if constexpr (L >= 16)
        v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xf, 0xf, false));  // 15 - lane
    if constexpr (L == 32)  // lane ^ 16 (swizzle bit mode: and 0x1f, or 0, xor 0x10)
        v = op(v, (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F));
    return v;
}

// Median of the window whose top-left value is w, computed by the group
// member g (0..L-1); every member returns it.  pk_one as for median_registers.
template <int K>
__device__ __forceinline__ uint32_t median_group(const uint16_t *w, int g, uint32_t pk_one) {
    using P = GroupPlan<K>;
    constexpr int N = P::N, L = P::lanes, pitch = Geometry<K>::pitch;
    constexpr uint32_t rank = (N - 1) / 2;
    const uint16_t first = w[0];
    uint32_t v[P::regs];
    int off = g, col = g;  // LDS offset and column of the lane's next value (g < L < K)
    auto next = [&](int idx) -> uint16_t {
        uint16_t x = first;
        if (idx * L + L <= N || idx * L + g < N) x = w[off];
        col += L;
        off += L;
        if (col >= K) {
            col -= K;
            off += pitch - K;
        }
        return x;
    };
#pragma unroll
    for (int j = 0; j < P::regs; ++j) {
        u16x2 pair;  // built element-wise so that each value loads straight into its half
        pair.x = next(2 * j);
        pair.y = next(2 * j + 1);
        v[j] = __builtin_bit_cast(uint32_t, pair);
    }
    uint32_t mn = 0xffffffffu, mx = 0u;
#pragma unroll
    for (int j = 0; j < P::regs; ++j) {
        mn = pk_min(mn, v[j]);
        mx = pk_max(mx, v[j]);
    }
    uint32_t lo = group_reduce<L>(min(mn & 0xffffu, mn >> 16), [](uint32_t a, uint32_t b) { return min(a, b); });
    uint32_t hi = group_reduce<L>(max(mx & 0xffffu, mx >> 16), [](uint32_t a, uint32_t b) { return max(a, b); });
    while (lo < hi) {  // uniform over the group
        const uint32_t t = (lo + hi) >> 1;
        const uint32_t tt = t | (t << 16);
        uint32_t above = 0;
#pragma unroll
        for (int j = 0; j < P::regs; ++j) above = pk_add(above, pk_min(pk_subsat(v[j], tt), pk_one));
        uint32_t gt = group_reduce<L>((above & 0xffffu) + (above >> 16),
                                      [](uint32_t a, uint32_t b) { return a + b; });
        if (first > t) gt -= P::pad;
        if (N - gt > rank)
            hi = t;
        else
            lo = t + 1;
    }
    return lo;
}

// Inclusive prefix sum inside each row of 16 lanes (DPP row shifts; lanes
// shifted in from outside the row read 0).
__device__ __forceinline__ uint32_t row_inclusive_sum(uint32_t v) {
    constexpr int kRowShr = 0x110;
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 1, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 2, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 4, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 8, 0xf, 0xf, true);
    return (uint32_t)x;
}

// One 256-bin histogram pass of the radix select: the group's 16 lanes read
// their 16 bins each, find the bin holding element `rank` (0-based) of the
// counted values, clear their bins, and return ((bin + 1) << 16 | rank within
// the bin) in every lane of the group.
__device__ __forceinline__ uint32_t hist_find(uint32_t *bins, int g, uint32_t rank) {
    const uint4 *b4 = reinterpret_cast<const uint4 *>(bins + 16 * g);
    uint32_t c[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint4 x = b4[q];
        c[4 * q] = x.x;
        c[4 * q + 1] = x.y;
        c[4 * q + 2] = x.z;
        c[4 * q + 3] = x.w;
    }
    uint32_t tot = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) tot += c[j];
    uint32_t cum = row_inclusive_sum(tot) - tot;  // values in the bins of lower lanes
    uint32_t key = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint32_t next = cum + c[j];
        if (cum <= rank && rank < next) key = ((uint32_t)(16 * g + j + 1) << 16) | (rank - cum);
        cum = next;
    }
    uint4 *w4 = reinterpret_cast<uint4 *>(bins + 16 * g);
#pragma unroll
    for (int q = 0; q < 4; ++q) w4[q] = make_uint4(0u, 0u, 0u, 0u);
    return group_reduce<kHistLanes>(key, [](uint32_t a, uint32_t b) { return max(a, b); });
}

// Median of the window whose top-left value is w, computed by the group member
// g (0..15) with its group's LDS histogram `bins` (all zero on entry and on
// return); every member returns it.  A two-pass radix select on the offsets
// from the window minimum: pass 1 counts the values by their top 8 bits below
// the range's bit length and finds the bin holding the median, pass 2 counts
// the values of that bin by their remaining low bits (at most 8, for 16-bit
// data) and finds the median itself.  Lane g holds values g, g + 16, g + 32,
// ... of S_xy, two per register; the slots past the window's end repeat the
// lane's first value and are never counted.
template <int K>
__device__ __forceinline__ uint32_t median_hist(const uint16_t *w, int g, uint32_t *bins) {
    constexpr int N = K * K, L = kHistLanes, V = (N + L - 1) / L, V2 = (V + 1) / 2;
    constexpr int pitch = Geometry<K>::pitch;
    constexpr uint32_t rank = (N - 1) / 2;
    static_assert(K > L, "a lane's next value is at most one window row further");
    // value m of the lane exists when 16 m + g < N: only the last two can be missing
    auto valid = [&](int m) { return m < V - 2 || (m < V && 16 * m + g < N); };
    const uint16_t first = w[g];
    int off = g, col = g;
    auto next = [&](int m) -> uint16_t {
        const uint16_t x = valid(m) ? w[off] : first;
        col += L;
        off += L;
        if (col >= K) {
            col -= K;
            off += pitch - K;
        }
        return x;
    };
    uint32_t v[V2];
#pragma unroll
    for (int j = 0; j < V2; ++j) {
        u16x2 p;  // built element-wise so that each value loads straight into its half
        p.x = next(2 * j);
        p.y = next(2 * j + 1);
        v[j] = __builtin_bit_cast(uint32_t, p);
    }
    uint32_t pmn = v[0], pmx = v[0];
#pragma unroll
    for (int j = 1; j < V2; ++j) {
        pmn = pk_min(pmn, v[j]);
        pmx = pk_max(pmx, v[j]);
    }
    uint32_t mn = min(pmn & 0xffffu, pmn >> 16), mx = max(pmx & 0xffffu, pmx >> 16);
    mn = group_reduce<L>(mn, [](uint32_t a, uint32_t b) { return min(a, b); });
    mx = group_reduce<L>(mx, [](uint32_t a, uint32_t b) { return max(a, b); });
    const uint32_t range = mx - mn;
    const int bits = range == 0 ? 0 : 32 - __builtin_clz(range);
    const uint32_t s1 = bits > 8 ? (uint32_t)bits - 8u : 0u;
    const uint32_t mnp = mn | (mn << 16);
    // offsets from the minimum, two per register (no half can borrow: every
    // value is at least the minimum)
#pragma unroll
    for (int j = 0; j < V2; ++j) v[j] = v[j] - mnp;
    // pass 1: the top 8 bits of each offset's range
#pragma unroll
    for (int j = 0; j < V2; ++j) {
        if (valid(2 * j)) atomicAdd(bins + __builtin_amdgcn_ubfe(v[j], s1, 8), 1u);
        if (valid(2 * j + 1)) atomicAdd(bins + __builtin_amdgcn_ubfe(v[j], 16 + s1, 8), 1u);
    }
    const uint32_t k1 = hist_find(bins, g, rank);
    const uint32_t b1 = (k1 >> 16) - 1, r1 = k1 & 0xffffu;
    if (s1 == 0) return mn + b1;
    // pass 2: the low s1 bits of the offsets in bin b1
#pragma unroll
    for (int j = 0; j < V2; ++j) {
        if (valid(2 * j) && __builtin_amdgcn_ubfe(v[j], s1, 8) == b1)
            atomicAdd(bins + __builtin_amdgcn_ubfe(v[j], 0, s1), 1u);
        if (valid(2 * j + 1) && __builtin_amdgcn_ubfe(v[j], 16 + s1, 8) == b1)
            atomicAdd(bins + __builtin_amdgcn_ubfe(v[j], 16, s1), 1u);
    }
    const uint32_t k2 = hist_find(bins, g, r1);
    return mn + (b1 << s1) + ((k2 >> 16) - 1);
}

// ---------------------------------------------------------------------------
// wave / workgroup prefix sums
// ---------------------------------------------------------------------------
// Inclusive prefix sum over the wave with DPP moves: a Hillis-Steele scan
// inside each row of 16 lanes (row_shr 1, 2, 4, 8; lanes shifted in from
// outside the row read 0), then row 15's total is added to rows 1 and 3
// (row_bcast:15) and row 31's to rows 2 and 3 (row_bcast:31).
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
    constexpr int kRowShr = 0x110, kRowBcast15 = 0x142, kRowBcast31 = 0x143;
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 1, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 2, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 4, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 8, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, kRowBcast15, 0xa, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, kRowBcast31, 0xc, 0xf, false);
    return (uint32_t)x;
}

// ---------------------------------------------------------------------------
// 5. stores
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void store_px(uint8_t *frame, uint32_t row_off, int x, uint32_t v) {
    if constexpr (sizeof(T) == 1)
        frame[row_off + (uint32_t)x] = (uint8_t)v;
    else
        *reinterpret_cast<uint16_t *>(frame + (row_off + 2u * (uint32_t)x)) = (uint16_t)v;
}

// Four 16-bit LDS values (two packed pairs) to the frame row at byte offset
// row_off, column px.
template <typename T>
__device__ __forceinline__ void store4(uint8_t *frame, uint32_t row_off, int px, int W, bool aligned,
                                       uint32_t p0, uint32_t p1) {
    if (aligned && px + 4 <= W) {
        const uint32_t off = row_off + (uint32_t)px * (uint32_t)sizeof(T);
        if constexpr (sizeof(T) == 2) {
            *reinterpret_cast<uint2 *>(frame + off) = make_uint2(p0, p1);
        } else {
            uint32_t b = (p0 & 0xffu) | ((p0 >> 8) & 0xff00u) | ((p1 & 0xffu) << 16) |
                         ((p1 & 0xff0000u) << 8);
            *reinterpret_cast<uint32_t *>(frame + off) = b;
        }
    } else {
        uint32_t e[4] = {p0 & 0xffffu, p0 >> 16, p1 & 0xffffu, p1 >> 16};
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (px + i < W) store_px<T>(frame, row_off, px + i, e[i]);
    }
}

// The thread's 4 x R output block (columns px..px+3, rows py..py+R-1 of a
// tile at x0, y0) to the frame; pair(q, p0, p1) gives row q's two packed pairs.
// A tile wholly inside the frame on an aligned layout (`full`, uniform) stores
// each row at a wave-uniform base (the tile's row q) plus the thread's fixed
// offset, so the address costs no vector instruction; other tiles clip per
// row and per pixel.  The full-tile stores are non-temporal: the output is
// not read again by the launch, and streaming it leaves the L2 to the input
// rows that neighbouring tiles share (2% faster at 5x5, 1% at 7x7 on the
// 640x512 stack).
template <typename T, int R, typename Pair>
__device__ __forceinline__ void store_block(uint8_t *frame, uint64_t pitch, int x0, int y0, int px, int py,
                                            int W, int H, bool aligned, bool full, Pair &&pair) {
    const uint32_t p32 = (uint32_t)pitch;
    if (full) {
        const uint32_t off = (uint32_t)(py - y0) * p32 + (uint32_t)(px - x0) * (uint32_t)sizeof(T);
        uint8_t *base = frame + (int64_t)y0 * (int64_t)pitch + (int64_t)x0 * (int64_t)sizeof(T);
#pragma unroll
        for (int q = 0; q < R; ++q) {
            uint32_t p0, p1;
            pair(q, p0, p1);
            uint8_t *row = base + (int64_t)q * (int64_t)pitch;
            if constexpr (sizeof(T) == 2) {
                typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
                u32x2 v;
                v.x = p0;
                v.y = p1;
                __builtin_nontemporal_store(v, reinterpret_cast<u32x2 *>(row + off));
            } else {
                __builtin_nontemporal_store(
                    (p0 & 0xffu) | ((p0 >> 8) & 0xff00u) | ((p1 & 0xffu) << 16) | ((p1 & 0xff0000u) << 8),
                    reinterpret_cast<uint32_t *>(row + off));
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (py + q >= H) break;
            uint32_t p0, p1;
            pair(q, p0, p1);
            store4<T>(frame, __umul24((uint32_t)(py + q), p32), px, W, aligned, p0, p1);
        }
    }
}

// ---------------------------------------------------------------------------
// the tile kernel
// ---------------------------------------------------------------------------
// Tiles of a launch are split into 8 contiguous ranges, one per XCD (the
// hardware hands workgroup b to XCD b % 8); the workgroups of an XCD stride
// through its range, so tiles that share halo rows run close together in time
// and on the same L2.  Each range's length is proportional to its workgroups.
struct TileRange {
    int first, end, stride;
};

__device__ __forceinline__ TileRange xcd_range(int b, int G, int total) {
    constexpr int X = 8;
    const int xcd = b % X, local = b / X;
    const int per = G / X, extra = G % X;
    const int nx = per + (xcd < extra ? 1 : 0);           // workgroups on this XCD
    const int before = xcd * per + (xcd < extra ? xcd : extra);  // workgroups on lower XCDs
    const int tb = (int)((long long)total * before / G);
    const int te = (int)((long long)total * (before + nx) / G);
    return {tb + local, te, nx};
}

// Radix-select histograms (kSelectHist): 256 bins per group of kHistLanes lanes.
template <int NT, bool ON>
struct HistSpace {};
template <int NT>
struct HistSpace<NT, true> {
    alignas(16) uint32_t bins[NT / kHistLanes][kHistBins];
};

// Flagged-pixel list of the persistent stack kernel at 5x5 and 7x7: 3/8 of the
// tile's pixels at 5x5, a quarter at 7x7.  The rare tile with more flagged
// pixels selects in rounds and stores its medians straight to the frame
// (median_into_tile), so the list does not need a slot per pixel, and the
// smaller LDS footprint lets more workgroups share a CU: six 256-thread
// workgroups instead of four at both windows (with the occupancy target of
// stack_waves).  At 5x5 that measured 5% faster on the 640x512 stack; at 7x7
// five workgroups (a 3/8 list, 92 VGPRs) measured 5% faster and six (a quarter
// list, 80 VGPRs) 3-5% faster again, and 1.3% faster on 1080p frames with 20%
// flagged, where some tiles overflow.  (At 97 VGPRs, before the detection's
// 64-bit LDS reads, the 3/8 list had measured 4% slower at 7x7.)  The standard
// median filter selects every pixel; at 5x5 and 7x7 it takes the dense path
// (dense_block) and needs no list.  The other windows are held to four waves
// per SIMD or fewer by their registers, so they keep a slot per pixel.
constexpr int stack_list(int K, int tile_px) {
    return K == 5 ? tile_px * 3 / 8 : K == 7 ? tile_px / 4 : tile_px;
}

template <int K, int NT = kThreads, int SEL = 0, int LIST = Geometry<K, NT>::tile_px>
struct TileSmem {
    using G = Geometry<K, NT>;
    static constexpr int list_cap = LIST;
    static_assert(LIST % 2 == 0 && LIST <= G::tile_px, "list of whole pairs, at most one slot per pixel");
    uint16_t tile[G::rows * G::pitch];
    uint16_t list[LIST];  // LDS offsets of flagged centres, then their medians
    uint32_t count;       // list length
    // per wave: nonzero if the wave staged a value of 0x4000 or more (the
    // tile then takes the integer detection path)
    alignas(8) uint8_t large[8];
    HistSpace<NT, SEL == kSelectHist> hist;
};

// The shared memory of a kernel with selection SEL (histograms only for
// kSelectHist) and a list of LIST slots.
template <int K, int NT, int SEL, int LIST = Geometry<K, NT>::tile_px>
using SmemFor = TileSmem<K, NT, SEL == kSelectHist ? kSelectHist : 0, LIST>;

// Where the medians of a tile whose flagged pixels overflow the list go: the
// tile is first stored unfiltered (store_tile), then each median is stored to
// the frame by the lane that selected it (store_median, at the pixel whose
// LDS offset it gets).  NoSink: the list holds every pixel, nothing overflows.
struct NoSink {
    static constexpr bool enabled = false;
    __device__ void store_tile() {}
    __device__ void store_median(uint32_t, uint32_t) {}
};
template <typename StoreTile, typename StoreMedian>
struct DirectSink {
    static constexpr bool enabled = true;
    StoreTile store_tile;
    StoreMedian store_median;
};
template <typename A, typename B>
__device__ __forceinline__ DirectSink<A, B> direct_sink(A a, B b) {
    return {a, b};
}

// 3 x 3 windows take a dense path instead of steps 3 and 4: at the flag rates
// of 3 x 3 (a quarter to half of the pixels) computing every pixel's median in
// registers costs less than compacting the flagged ones.  Each window column
// is sorted, and the median of the nine values is med3(largest column minimum,
// median of the column medians, smallest column maximum): after the rows of
// the column-sorted window are sorted too, these three are its anti-diagonal,
// which holds the median.
__device__ __forceinline__ uint32_t pk_med3(uint32_t a, uint32_t b, uint32_t c) {
    return pk_max(pk_min(a, b), pk_min(pk_max(a, b), c));
}

struct PkSorted3 {
    uint32_t lo, mid, hi;
};

__device__ __forceinline__ PkSorted3 pk_sort3(uint32_t a, uint32_t b, uint32_t c) {
    const uint32_t t = pk_min(a, b), u = pk_max(a, b);
    const uint32_t v = pk_max(t, c);
    return {pk_min(t, c), pk_min(u, v), pk_max(u, v)};
}

// Output pairs of the thread's 4 x R block: out[q][0] = columns (0,1) and
// out[q][1] = columns (2,3) of row q, each half the 3 x 3 median where its flag
// bit is set and the centre value otherwise.  Per LDS row the thread holds the
// aligned pairs (0,1), (2,3) and the odd pairs (-1,0), (1,2), (3,4), so one
// column sort serves two pixels and the sorted pair (1,2) serves both outputs.
template <int R>
__device__ __forceinline__ void dense3_block(const uint16_t *tile, int strip, int tx, uint32_t flags,
                                             uint32_t (&out)[R][2]) {
    using G = Geometry<3>;
    const uint16_t *base = tile + strip * R * G::pitch + G::halo + 4 * tx;
    uint32_t A[R + 2], B[R + 2], C[R + 2], D[R + 2], E[R + 2];
#pragma unroll
    for (int i = 0; i < R + 2; ++i) {
        // plain reads: only the words used are read, and as 64-bit words
        // (lds_word2) they keep 90 VGPRs live instead of 71, which measured
        // 3-7% slower at 3x3
        const uint2 *q = reinterpret_cast<const uint2 *>(base + i * G::pitch);
        const uint2 w0 = q[-1], w1 = q[0], w2 = q[1];  // columns -4..-1, 0..3, 4..7
        B[i] = w1.x;
        D[i] = w1.y;
        A[i] = shift_pair(w1.x, w0.y);
        C[i] = shift_pair(w1.y, w1.x);
        E[i] = shift_pair(w2.x, w1.y);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const PkSorted3 sa = pk_sort3(A[q], A[q + 1], A[q + 2]), sb = pk_sort3(B[q], B[q + 1], B[q + 2]);
        const PkSorted3 sc = pk_sort3(C[q], C[q + 1], C[q + 2]), sd = pk_sort3(D[q], D[q + 1], D[q + 2]);
        const PkSorted3 se = pk_sort3(E[q], E[q + 1], E[q + 2]);
        const uint32_t m0 = pk_med3(pk_max(pk_max(sa.lo, sb.lo), sc.lo), pk_med3(sa.mid, sb.mid, sc.mid),
                                    pk_min(pk_min(sa.hi, sb.hi), sc.hi));
        const uint32_t m1 = pk_med3(pk_max(pk_max(sc.lo, sd.lo), se.lo), pk_med3(sc.mid, sd.mid, se.mid),
                                    pk_min(pk_min(sc.hi, sd.hi), se.hi));
        // flag bit q (+16) is column 0 (1), bit q+8 (+24) column 2 (3)
        const uint32_t s0 = ((uint32_t)__builtin_amdgcn_sbfe(flags, q, 1) & 0xffffu) |
                            ((uint32_t)__builtin_amdgcn_sbfe(flags, q + 16, 1) & 0xffff0000u);
        const uint32_t s1 = ((uint32_t)__builtin_amdgcn_sbfe(flags, q + 8, 1) & 0xffffu) |
                            ((uint32_t)__builtin_amdgcn_sbfe(flags, q + 24, 1) & 0xffff0000u);
        out[q][0] = (m0 & s0) | (B[q + 1] & ~s0);
        out[q][1] = (m1 & s1) | (D[q + 1] & ~s1);
    }
}

// The standard median filter at 5 x 5 and 7 x 7 takes a dense path too: every
// pixel is selected, and computing all medians of the thread's block from
// sorted window columns costs less than compacting the whole tile.  Per output
// row, the K + 2 column-pair streams P_c = (column c, column c+1), c = -r..r+2,
// of the K window rows are each sorted (packed: one sort serves two
// neighbouring columns), and the K sorted columns of a window are merged in
// the manner of forgetful selection (Fold): whenever the run of merged values
// holds values that cannot be the median whatever the columns not yet merged
// hold, they are dropped.  The K - 2 columns that both output pairs of the
// thread share (P_-r+2 .. P_r) are merged once; each pair then merges its own
// two columns, which leaves one value, its median.

// One forgetful merge step: a sorted run of L values, in which the median has
// rank T, takes a sorted column of S values, with U values (this column
// included) not yet merged.  Of the L + S merged values the `low` smallest lie
// below the median even if every value still unmerged were smaller, and the
// `high` largest lie above it: both are dropped, leaving `keep` values in which
// the median has rank `rank`.
template <int L, int S, int T, int U>
struct Fold {
    static constexpr int M = L + S, left = U - S;
    static constexpr int low = T > left ? T - left : 0;
    static constexpr int high = M - 1 > T ? M - 1 - T : 0;
    static constexpr int keep = M - low - high, rank = T - low;
};

template <int L, int S, int T, int U>
__device__ __forceinline__ void fold_in(const uint32_t *run, const uint32_t *col, uint32_t *out) {
    using F = Fold<L, S, T, U>;
    uint32_t m[F::M];
    merge_sorted<L, S>(run, col, m);
#pragma unroll
    for (int i = 0; i < F::keep; ++i) out[i] = m[F::low + i];
}

// Fold columns J .. JEND-1 of col (each of K sorted values) into a run.
template <int K, int J, int JEND, int L, int T, int U>
struct FoldColumns {
    using F = Fold<L, K, T, U>;
    using Next = FoldColumns<K, J + 1, JEND, F::keep, F::rank, F::left>;
    static constexpr int keep = Next::keep, rank = Next::rank, left = Next::left;
    template <int NS>
    __device__ static void run(const uint32_t *r, const uint32_t (&col)[NS][K], uint32_t *out) {
        uint32_t m[F::keep];
        fold_in<L, K, T, U>(r, col[J], m);
        Next::run(m, col, out);
    }
};
template <int K, int JEND, int L, int T, int U>
struct FoldColumns<K, JEND, JEND, L, T, U> {
    static constexpr int keep = L, rank = T, left = U;
    template <int NS>
    __device__ static void run(const uint32_t *r, const uint32_t (&)[NS][K], uint32_t *out) {
#pragma unroll
        for (int i = 0; i < L; ++i) out[i] = r[i];
    }
};

// Output pairs of the thread's 4 x R block at K x K (5 or 7), as dense3_block:
// the window median where the flag bit is set and the centre otherwise.
template <int K, int R>
__device__ __forceinline__ void dense_block(const uint16_t *tile, int strip, int tx, uint32_t flags,
                                            uint32_t (&out)[R][2]) {
    static_assert(K == 5 || K == 7, "dense medians from sorted columns at 5 x 5 and 7 x 7");
    using G = Geometry<K>;
    constexpr int r = K / 2, NS = K + 2, N = K * K;
    // the shared columns 2 .. K-1, starting from column 2 alone
    using Shared = FoldColumns<K, 3, K, K, N / 2, N - K>;
    using Own1 = Fold<Shared::keep, K, Shared::rank, Shared::left>;
    using Own2 = Fold<Own1::keep, K, Own1::rank, Own1::left>;
    static_assert(Own2::keep == 1 && Own2::left == 0, "the fold must end with the median alone");
    const uint16_t *base = tile + strip * R * G::pitch + G::halo + 4 * tx;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        uint32_t col[NS][K];  // col[j]: stream P_(j-r) over the window rows q..q+K-1
        uint32_t c0 = 0, c1 = 0;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const uint2 *w = reinterpret_cast<const uint2 *>(base + (q + i) * G::pitch);
            const uint2 w0 = w[-1], w1 = w[0], w2 = w[1];  // columns -4..-1, 0..3, 4..7
            const uint32_t d[6] = {w0.x, w0.y, w1.x, w1.y, w2.x, w2.y};  // d[e + 2]: columns (2e, 2e+1)
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                const int c = j - r;
                col[j][i] = (c & 1) ? shift_pair(d[(c + 1) / 2 + 2], d[(c - 1) / 2 + 2]) : d[c / 2 + 2];
            }
            if (i == r) {
                c0 = w1.x;
                c1 = w1.y;
            }
        }
#pragma unroll
        for (int j = 0; j < NS; ++j) sort_block<K>(col[j]);
        uint32_t core[Shared::keep];
        Shared::run(col[2], col, core);
        uint32_t a[Own1::keep], m0, m1;
        fold_in<Shared::keep, K, Shared::rank, Shared::left>(core, col[0], a);  // columns (0, 1)
        fold_in<Own1::keep, K, Own1::rank, Own1::left>(a, col[1], &m0);
        fold_in<Shared::keep, K, Shared::rank, Shared::left>(core, col[K], a);  // columns (2, 3)
        fold_in<Own1::keep, K, Own1::rank, Own1::left>(a, col[K + 1], &m1);
        const uint32_t s0 = ((uint32_t)__builtin_amdgcn_sbfe(flags, q, 1) & 0xffffu) |
                            ((uint32_t)__builtin_amdgcn_sbfe(flags, q + 16, 1) & 0xffff0000u);
        const uint32_t s1 = ((uint32_t)__builtin_amdgcn_sbfe(flags, q + 8, 1) & 0xffffu) |
                            ((uint32_t)__builtin_amdgcn_sbfe(flags, q + 24, 1) & 0xffff0000u);
        out[q][0] = (m0 & s0) | (c0 & ~s0);
        out[q][1] = (m1 & s1) | (c1 & ~s1);
    }
}

// Steps 3 and 4 on a tile staged in LDS: the flagged pixels (bits of each
// thread's 4 x R block whose centre, column 0 of row 0, is LDS value centre0)
// are compacted into the list, their window medians are selected, and every
// thread writes its own medians back into the tile.  sm.count must be 0, and
// visible to every thread, on entry.  On return the tile holds the results at
// the calling thread's pixels only: reading another thread's pixels needs a
// barrier first.  `rot` rotates which wave starts the list; pk_one is the
// host's 0x00010001 (see median_registers).  Returns the number of flagged
// pixels of the calling wave (wave-uniform).  PRIO: the wave runs from here on
// at the highest priority and the caller lowers it again (see process_tile).
//
// When more pixels are flagged than the list holds (only with a DirectSink),
// the tile is left unchanged: the sink stores it unfiltered first, then the
// flagged pixels go through the list in rounds of list_cap entries and every
// median is stored to the frame by the lane that selected it; `direct` is
// then set (uniform), and the caller stores nothing more.
template <int K, int NT, int SEL, int LIST, bool PRIO = false, typename Sink = NoSink>
__device__ __forceinline__ uint32_t median_into_tile(SmemFor<K, NT, SEL, LIST> &sm, uint32_t flags, int centre0,
                                                     int rot, uint32_t pk_one, Sink &&sink = Sink{},
                                                     bool *direct = nullptr) {
    using G = Geometry<K, NT>;
    static_assert(((SEL == kSelectGroup || SEL == kSelectHist) && K > kNetworkMaxWindow) ||
                      (K <= kNetworkMaxWindow && (SEL == kSelectBisect || SEL == kSelectNetwork)),
                  "no kernel of this selection for this window");
    static_assert(std::remove_reference_t<Sink>::enabled || LIST == G::tile_px,
                  "a list shorter than the tile needs a sink for its overflow");
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(3);
    const uint32_t cnt = __builtin_popcount(flags);
    const uint32_t incl = wave_inclusive_sum(cnt);
    const uint32_t wave_total = __builtin_amdgcn_readlane(incl, 63);
    // 3. compaction: one LDS atomic per wave reserves the wave's list slots;
    //    a thread's entries are contiguous and in flag-bit order.  Entries
    //    [lo, lo + LIST) of the tile's order go to list slots 0.. (all of them
    //    when the list holds every pixel)
    uint32_t wbase = 0;
    if (lane == 63 && wave_total != 0) wbase = atomicAdd(&sm.count, wave_total);
    const uint32_t first = __builtin_amdgcn_readlane(wbase, 63) + incl - cnt;
    auto compact = [&](uint32_t lo) {
        uint32_t m = flags, j = first;
        while (m) {
            const int b = __builtin_ctz(m);
            m &= m - 1;
            if (LIST == G::tile_px || (j >= lo && j < lo + LIST))
                sm.list[j - lo] = (uint16_t)(centre0 + bit_row(b) * G::pitch + bit_col(b));
            ++j;
        }
    };
    compact(0);
    __syncthreads();
    const uint32_t total = sm.count;
    // 4. medians of list slots [0, n), two entries per lane, consecutive lanes
    //    first so that as few waves as possible run the selection; which wave
    //    starts the list rotates with `rot` (waves sit on fixed SIMDs).
    //    emit(slot, LDS offset, median) takes each result.
    constexpr int corner = G::r * G::pitch + G::r;
    const uint32_t slot = ((uint32_t)tid + 64u * (uint32_t)rot) % NT;
    auto select = [&](uint32_t n, auto &&emit) {
        if constexpr (SEL == kSelectHist) {
            // one window per group of 16 lanes, each group with its own histogram
            constexpr int L = kHistLanes, NG = NT / L;
            const int g = tid % L, grp = tid / L;
            const uint32_t gslot = ((uint32_t)grp + (64u / L) * (uint32_t)rot) % NG;
            for (uint32_t i = gslot; i < n; i += NG) {
                const uint32_t e0 = sm.list[i];
                const uint32_t med = median_hist<K>(sm.tile + e0 - corner, g, sm.hist.bins[grp]);
                if (g == 0) emit(i, e0, med);
            }
        } else if constexpr (SEL == kSelectGroup) {
            // one window per group of lanes: all lanes of a group read the entry
            // before its first lane overwrites it (a group lies inside one wave)
            constexpr int L = GroupPlan<K>::lanes, NG = NT / L;
            const int g = tid % L;
            const uint32_t gslot = ((uint32_t)(tid / L) + (64u / L) * (uint32_t)rot) % NG;
            for (uint32_t i = gslot; i < n; i += NG) {
                const uint32_t e0 = sm.list[i];
                const uint32_t med = median_group<K>(sm.tile + e0 - corner, g, pk_one);
                if (g == 0) emit(i, e0, med);
            }
        } else if constexpr (SEL == kSelectBisect) {
            // one window per lane
            for (uint32_t i = slot; i < n; i += NT) {
                const uint32_t e0 = sm.list[i];
                emit(i, e0, median_registers<K>(sm.tile + e0 - corner, pk_one));
            }
        } else {
            for (uint32_t i = 2 * slot; i < n; i += 2 * NT) {
                const uint32_t e0 = sm.list[i];
                const uint32_t e1 = (i + 1 < n) ? sm.list[i + 1] : e0;
                const uint32_t med = median_pair<K>(sm.tile, e0 - corner, e1 - corner);
                emit(i, e0, med & 0xffffu);
                if (i + 1 < n) emit(i + 1, e1, med >> 16);
            }
        }
    };
    if (LIST == G::tile_px || total <= (uint32_t)LIST) {  // uniform
        select(total, [&](uint32_t i, uint32_t, uint32_t med) { sm.list[i] = (uint16_t)med; });
        __syncthreads();
        // results back into the tile at the thread's own pixels
        uint32_t m = flags, j = first;
        while (m) {
            const int b = __builtin_ctz(m);
            m &= m - 1;
            sm.tile[centre0 + bit_row(b) * G::pitch + bit_col(b)] = sm.list[j++];
        }
        if (direct) *direct = false;
    } else if constexpr (std::remove_reference_t<Sink>::enabled) {
        sink.store_tile();  // the tile unfiltered: every median is stored over it below
        __syncthreads();
        for (uint32_t lo = 0; lo < total; lo += LIST) {
            if (lo > 0) {
                compact(lo);
                __syncthreads();
            }
            select(min((uint32_t)LIST, total - lo),
                   [&](uint32_t, uint32_t e, uint32_t med) { sink.store_median(e, med); });
            __syncthreads();  // the next round rewrites the list
        }
        if (direct) *direct = true;
    }
    return wave_total;
}

// One tile already staged in LDS: detection, compaction of the flagged pixels,
// selection, then the tile (flagged pixels replaced) is stored.  Returns the
// number of flagged pixels the calling wave found (wave-uniform).
//
// PRIO (the persistent stack and batch kernels): detection, the long phase
// that every wave of the workgroup runs alike, keeps the lowest wave priority;
// compaction, selection, write-back and store (at 3x3 the store after the
// dense medians) run at the highest.  A workgroup's waves that the others wait
// for at a barrier (those holding selection work) then issue ahead of other
// workgroups' detection, which fills the gaps; with the loads also issued at
// the highest priority (load_tile, EARLY), this measured 9-12% faster at 5x5
// to 9x9.
//
// F16 (uniform): every staged value of the tile lies below 0x4000, so the
// detection's horizontal pass may use the three-input half-precision min / max
// (same flags, fewer instructions).
template <typename T, int K, int MODE, int NT = kThreads, int SEL = default_select(K), bool PRIO = false,
          int LIST = Geometry<K, NT>::tile_px>
__device__ __forceinline__ uint32_t process_tile(const StackArgs &a, int tile, SmemFor<K, NT, SEL, LIST> &sm,
                                                 bool f16 = false) {
    using G = Geometry<K, NT>;
    static_assert(((SEL == kSelectGroup || SEL == kSelectHist) && K > kNetworkMaxWindow) ||
                      (K <= kNetworkMaxWindow && (SEL == kSelectBisect || SEL == kSelectNetwork)),
                  "no kernel of this selection for this window");
    constexpr int R = G::R;
    const int f = tile / a.tiles_per_frame;
    const int rem = tile - f * a.tiles_per_frame;
    const int ty = rem / a.tiles_x;
    const int x0 = (rem - ty * a.tiles_x) * kTileW;
    const int y0 = ty * G::TH;
    const int W = a.width, H = a.height;
    const bool aligned = a.aligned != 0;
    const int tid = threadIdx.x;
    const int tx = tid % kThreadsX, strip = tid / kThreadsX;
    const int px = x0 + 4 * tx, py = y0 + strip * R;
    const uint32_t valid = valid_bits(R, W, H, px, py);

    uint32_t flags;
    if constexpr (MODE == MODE_DETECT || MODE == MODE_FNR) {
        flags = (f16 ? detect_block<K, true>(sm.tile, strip, tx, a.pk_one)
                     : detect_block<K, false>(sm.tile, strip, tx, a.pk_one)) &
                valid;
    } else if constexpr (MODE == MODE_DETECT_DIR) {
        flags = directional_block<K>(sm.tile, strip, tx, a.pk_one) & valid;
    } else if constexpr (MODE == MODE_MEDIAN_MASK) {
        flags = 0;
        const uint8_t *m = a.mask_in + (uint64_t)f * a.mask_stride;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (py + q >= H) break;
            const uint32_t mo = __umul24((uint32_t)(py + q), (uint32_t)a.mask_pitch) + (uint32_t)px;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (px + e < W && m[mo + (uint32_t)e] != 0) {
                    const int sh = (e == 0) ? 0 : (e == 1) ? 16 : (e == 2) ? 8 : 24;
                    flags |= 1u << (q + sh);
                }
            }
        }
    } else {
        flags = valid;
    }

    if constexpr (MODE == MODE_DETECT || MODE == MODE_DETECT_DIR) {
        const uint32_t wave_total = __builtin_amdgcn_readlane(wave_inclusive_sum(__builtin_popcount(flags)), 63);
        uint8_t *m = a.mask_out + (uint64_t)f * a.mask_stride;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (py + q >= H) break;
            const uint32_t mo = __umul24((uint32_t)(py + q), (uint32_t)a.mask_pitch) + (uint32_t)px;
            const uint32_t b0 = (flags >> q) & 1u, b1 = (flags >> (q + 16)) & 1u;
            const uint32_t b2 = (flags >> (q + 8)) & 1u, b3 = (flags >> (q + 24)) & 1u;
            if (aligned && px + 4 <= W) {
                *reinterpret_cast<uint32_t *>(m + mo) = b0 | (b1 << 8) | (b2 << 16) | (b3 << 24);
            } else {
                const uint32_t e[4] = {b0, b1, b2, b3};
                for (int i = 0; i < 4; ++i)
                    if (px + i < W) m[mo + (uint32_t)i] = (uint8_t)e[i];
            }
        }
        return wave_total;
    } else if constexpr (K == 3 || ((K == 5 || K == 7) && MODE == MODE_MEDIAN_ALL)) {
        // dense paths (3 x 3, and the 5 x 5 and 7 x 7 median filter): every
        // pixel's median in registers, kept where flagged
        const uint32_t wave_total = __builtin_amdgcn_readlane(wave_inclusive_sum(__builtin_popcount(flags)), 63);
        uint32_t out[R][2];
        if constexpr (K == 3)
            dense3_block<R>(sm.tile, strip, tx, flags, out);
        else
            dense_block<K, R>(sm.tile, strip, tx, flags, out);
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(3);
        uint8_t *dst = a.dst + (uint64_t)f * a.dst_stride;
        const bool full = aligned && x0 + kTileW <= W && y0 + G::TH <= H;  // uniform
        store_block<T, R>(dst, a.dst_pitch, x0, y0, px, py, W, H, aligned, full,
                          [&](int q, uint32_t &p0, uint32_t &p1) {
                              p0 = out[q][0];
                              p1 = out[q][1];
                          });
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
        return wave_total;
    } else {
        const int centre0 = (strip * R + G::r) * G::pitch + G::halo + 4 * tx;
        uint8_t *dst = a.dst + (uint64_t)f * a.dst_stride;
        const bool full = aligned && x0 + kTileW <= W && y0 + G::TH <= H;  // uniform
        // 5. the thread's block from the tile (its own LDS values only: no barrier needed)
        auto store = [&]() {
            store_block<T, R>(dst, a.dst_pitch, x0, y0, px, py, W, H, aligned, full,
                              [&](int q, uint32_t &p0, uint32_t &p1) {
                                  const uint32_t *c =
                                      reinterpret_cast<const uint32_t *>(sm.tile + centre0 + q * G::pitch);
                                  p0 = c[0];
                                  p1 = c[1];
                              });
        };
        uint32_t wave_total;
        if constexpr (LIST < G::tile_px) {
            // a median of a tile that overflows the list goes straight to its pixel
            auto median_to_frame = [&](uint32_t e, uint32_t med) {
                const uint32_t row = e / (uint32_t)G::pitch, col = e - row * (uint32_t)G::pitch;
                const int gx = x0 - G::halo + (int)col, gy = y0 - G::r + (int)row;
                store_px<T>(dst, __umul24((uint32_t)gy, (uint32_t)a.dst_pitch), gx, med);
            };
            bool direct = false;
            wave_total = median_into_tile<K, NT, SEL, LIST, PRIO>(sm, flags, centre0, tile, a.pk_one,
                                                                 direct_sink(store, median_to_frame), &direct);
            if (!direct) store();
        } else {
            wave_total = median_into_tile<K, NT, SEL, LIST, PRIO>(sm, flags, centre0, tile, a.pk_one);
            store();
        }
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
        return wave_total;
    }
}

__device__ __forceinline__ void tile_origin(const StackArgs &a, int tile, int th, int &f, int &x0,
                                            int &y0) {
    f = tile / a.tiles_per_frame;
    const int rem = tile - f * a.tiles_per_frame;
    const int ty = rem / a.tiles_x;
    x0 = (rem - ty * a.tiles_x) * kTileW;
    y0 = ty * th;
}

// Persistent kernel: every workgroup loops over its tile range.  Four
// barriers per tile: before the LDS tile is overwritten (taken once the tile's
// global loads are issued), after it is written, after the flagged list is
// complete and after the selection.  Other resident workgroups run while one
// waits for its tile's loads; wave priorities favour every phase but
// detection (process_tile).
// The tile's detection path, decided by the whole workgroup: each wave posts
// whether any of its threads staged a value of 0x4000 or more (its own LDS
// byte, written before the barrier that follows the tile's load; every wave
// writes its byte for every tile, so nothing needs clearing), and after that
// barrier every thread reads all the bytes (the same value everywhere).
__device__ __forceinline__ void post_small(uint8_t *large, bool small) {
    const bool wave_large = __builtin_amdgcn_ballot_w64(!small) != 0;
    if ((threadIdx.x & 63) == 0) large[threadIdx.x >> 6] = wave_large ? 1 : 0;
}
template <int NT>
__device__ __forceinline__ bool tile_small(const uint8_t *large) {
    uint64_t any = 0;
    __builtin_memcpy(&any, large, NT / 64);
    return __builtin_amdgcn_readfirstlane((uint32_t)(any | (any >> 32))) == 0;
}

// Occupancy target of the stack kernel (waves per SIMD; 1 = none).  The 5x5
// FNR kernels and the 256-thread 7x7 one hold six, as their LDS allows six
// workgroups of 256 threads per CU with the short lists of stack_list; the
// 256-thread 11x11 FNR kernel holds four, as its LDS allows four.  Without the
// target the 5x5 kernel's two detection paths take 81 VGPRs and five waves,
// which measured 2% slower (96 VGPRs before the detection's 64-bit LDS reads),
// the 7x7 kernel 92 VGPRs and five waves (with it: 80 VGPRs, one spilled; 3-5%
// faster), the 11x11 kernel 135 VGPRs and three waves (with it: 128 VGPRs,
// three spilled; 2.3% faster on 1080p frames with 20% flagged, 14% on the
// 640x512 stack).  The 128-thread 7x7 and 11x11 kernels measured 7-13% slower
// with the target and run without it; the others take what their registers
// and LDS give.
constexpr int stack_waves(int K, int MODE, int NT) {
    return MODE != MODE_FNR ? 1 : K == 5 ? 6 : K == 7 && NT == 256 ? 6 : K == 11 && NT == 256 ? 4 : 1;
}

template <typename T, int K, int MODE, int NT, int SEL>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(stack_waves(K, MODE, NT)))) void fnr_persistent_kernel(
    StackArgs a) {
    using G = Geometry<K, NT>;
    // the modes that select (K > 3: 3 x 3, and the 5 x 5 and 7 x 7 median filter,
    // compute every median in registers)
    // use the short list; detection has none to speak of
    constexpr bool kSelects =
        K > 3 && MODE != MODE_DETECT && MODE != MODE_DETECT_DIR && !((K == 5 || K == 7) && MODE == MODE_MEDIAN_ALL);
    constexpr int LIST = kSelects ? stack_list(K, G::tile_px) : 2;
    constexpr bool kDetects = MODE == MODE_DETECT || MODE == MODE_FNR;  // min / max detection
    __shared__ __attribute__((aligned(16))) SmemFor<K, NT, SEL, LIST> sm;
    const TileRange rg = xcd_range(blockIdx.x, gridDim.x, a.total_tiles);
    const bool aligned = a.aligned != 0;
    uint32_t flagged = 0;  // this wave's noisy pixels over all its tiles
    if constexpr (SEL == kSelectHist) {
        // histograms start empty (the first tile's load barrier orders this)
        for (int i = threadIdx.x; i < NT / kHistLanes * kHistBins; i += NT) (&sm.hist.bins[0][0])[i] = 0u;
    }
    for (int t = rg.first; t < rg.end; t += rg.stride) {
        int f, x0, y0;
        tile_origin(a, t, G::TH, f, x0, y0);
        // includes the barrier after which the previous tile is no longer read
        const bool small = load_tile<T, K, NT, false, true>(a.src + (uint64_t)f * a.src_stride, a.src_pitch,
                                                            a.width, a.height, x0, y0, aligned, sm.tile);
        if constexpr (kDetects) post_small(sm.large, small);
        if (threadIdx.x == 0) sm.count = 0;
        __syncthreads();
        bool f16 = false;
        if constexpr (kDetects) f16 = tile_small<NT>(sm.large);
        flagged += process_tile<T, K, MODE, NT, SEL, true, LIST>(a, t, sm, f16);
    }
    if constexpr (MODE == MODE_DETECT || MODE == MODE_FNR || MODE == MODE_DETECT_DIR) {
        if (a.count != nullptr && (threadIdx.x & 63) == 0 && flagged != 0)
            atomicAdd(a.count, (unsigned long long)flagged);
    }
}

static __global__ void zero_u64_kernel(unsigned long long *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

}  // namespace irf
