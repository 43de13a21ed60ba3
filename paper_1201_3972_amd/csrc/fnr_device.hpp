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
// One workgroup of 256 threads filters one tile of kTileW x (8*R) output
// pixels.  The tile and an r-pixel halo (rounded out to 8 columns) are staged in
// LDS as 16-bit values, whatever the pixel type.  The steps:
//   1. load:    coalesced 8-pixel chunks, rows and columns clamped at the border;
//   2. detect:  every thread owns 4 columns x R rows; window min and max are
//               separable: per input row a packed-u16 horizontal min/max over k
//               columns (two pixels per VGPR), then a van Herk / Gil-Werman
//               sliding min/max down the R+k-1 rows;
//   3. compact: flagged pixels of the tile go to an LDS list (wave prefix scan);
//   4. select:  each lane takes two list entries and computes both medians in
//               packed u16 registers: k <= 7 by forgetful selection over a sorted
//               working set, k >= 9 by a bisection on grey level that counts the
//               window values at or below the probe (bit-by-bit value search);
//   5. store:   results replace the flagged pixels in LDS, then the tile is
//               written out with vector stores.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "netgen.hpp"

namespace irf {

constexpr int kThreads = 256;
constexpr int kTileW = 128;                  // output columns per tile
constexpr int kThreadsX = kTileW / 4;        // 32 threads across, 4 columns each
constexpr int kStrips = kThreads / kThreadsX;  // 8 strips of R rows
constexpr int kHalo = 8;                     // LDS columns kept left and right of the tile
constexpr int kLdsW = kTileW + 2 * kHalo;    // 144 16-bit values per LDS row
constexpr int kChunks = kLdsW / 8;           // 8-pixel load chunks per LDS row
constexpr int kMaxWindow = 15;

enum Mode : int {
    MODE_DETECT = 0,       // write the noise mask (and count)
    MODE_FNR = 1,          // detect, then median at the noisy pixels
    MODE_MEDIAN_MASK = 2,  // median where a caller mask is non-zero
    MODE_MEDIAN_ALL = 3,   // median everywhere (the standard median filter)
};

// One launch covers a stack of equally sized frames laid out with fixed strides.
struct StackArgs {
    const uint8_t *src;
    uint8_t *dst;            // MODE_FNR / MODE_MEDIAN_*
    const uint8_t *mask_in;  // MODE_MEDIAN_MASK
    uint8_t *mask_out;       // MODE_DETECT
    uint64_t src_pitch, dst_pitch, mask_pitch;     // bytes between rows
    uint64_t src_stride, dst_stride, mask_stride;  // bytes between frames
    int width, height;
    int tiles_x, tiles_per_frame;
    int total_tiles;
    int aligned;  // every base address and pitch is a multiple of 16 bytes
    unsigned long long *count;  // nullable: += flagged pixels
};

template <int K>
struct Geometry {
    static constexpr int r = K / 2;
    static constexpr int R = 8;  // output rows per thread
    static constexpr int TH = kStrips * R;
    static constexpr int rows = TH + 2 * r;  // LDS rows
    static constexpr int tile_px = kTileW * TH;
    static_assert(K >= 3 && K <= kMaxWindow && (K & 1), "odd window 3..15");
    static_assert(r <= kHalo, "halo must cover the window radius");
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

// ---------------------------------------------------------------------------
// 1. tile load
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ uint32_t load_px(const uint8_t *row, int x) {
    if constexpr (sizeof(T) == 1)
        return row[x];
    else
        return reinterpret_cast<const uint16_t *>(row)[x];
}

__device__ __forceinline__ uint4 widen8(uint2 b) {
    uint4 v;
    v.x = (b.x & 0xffu) | ((b.x & 0xff00u) << 8);
    v.y = ((b.x >> 16) & 0xffu) | ((b.x >> 8) & 0xff0000u);
    v.z = (b.y & 0xffu) | ((b.y & 0xff00u) << 8);
    v.w = ((b.y >> 16) & 0xffu) | ((b.y >> 8) & 0xff0000u);
    return v;
}

// Stage rows y0-r .. y0+TH+r-1 and columns x0-kHalo .. x0+kTileW+kHalo-1 of the
// frame in LDS (row-major, kLdsW values per row).  Coordinates outside the
// frame are clamped to the nearest edge pixel.
template <typename T, int K>
__device__ __forceinline__ void load_tile(const uint8_t *src, uint64_t pitch, int W, int H, int x0,
                                          int y0, bool aligned, uint16_t *tile) {
    using G = Geometry<K>;
    for (int idx = threadIdx.x; idx < G::rows * kChunks; idx += kThreads) {
        int row = idx / kChunks;
        int c = idx - row * kChunks;
        int gy = min(max(y0 - G::r + row, 0), H - 1);
        int gx = x0 - kHalo + 8 * c;
        const uint8_t *rp = src + (uint64_t)gy * pitch;
        uint4 v;
        if (aligned && gx >= 0 && gx + 8 <= W) {
            if constexpr (sizeof(T) == 2)
                v = *reinterpret_cast<const uint4 *>(rp + 2 * (uint64_t)gx);
            else
                v = widen8(*reinterpret_cast<const uint2 *>(rp + gx));
        } else {
            uint32_t e[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) e[i] = load_px<T>(rp, min(max(gx + i, 0), W - 1));
            v.x = e[0] | (e[1] << 16);
            v.y = e[2] | (e[3] << 16);
            v.z = e[4] | (e[5] << 16);
            v.w = e[6] | (e[7] << 16);
        }
        *reinterpret_cast<uint4 *>(tile + row * kLdsW + 8 * c) = v;
    }
}

// ---------------------------------------------------------------------------
// 2. detection: separable window min / max on packed pairs
// ---------------------------------------------------------------------------
// Horizontal min/max over k columns for the thread's 4 output columns of one
// LDS row.  `p` points at the thread's first output column.  Outputs: packed
// pair 0 = columns (0,1), pair 1 = columns (2,3).
template <int r>
__device__ __forceinline__ void row_minmax(const uint16_t *p, uint32_t &mn0, uint32_t &mn1,
                                           uint32_t &mx0, uint32_t &mx1, uint32_t &c0, uint32_t &c1) {
    constexpr int JLO = -((r + 1) / 2);  // first pair needed
    constexpr int JHI = (3 + r) / 2;     // last pair needed
    constexpr int NJ = JHI - JLO + 1;
    const uint32_t *q = reinterpret_cast<const uint32_t *>(p);
    uint32_t D[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) D[j] = q[j + JLO];
    // V(o) = packed (pixel o, pixel o+1) relative to output column 0
    auto V = [&](int o) -> uint32_t {
        if ((o & 1) == 0) return D[o / 2 - JLO];
        return shift_pair(D[(o + 1) / 2 - JLO], D[(o - 1) / 2 - JLO]);
    };
    // pair 0 needs offsets -r..r, pair 1 needs 2-r..r+2; share 2-r..r
    uint32_t smin = V(2 - r), smax = smin;
#pragma unroll
    for (int o = 3 - r; o <= r; ++o) {
        uint32_t v = V(o);
        smin = pk_min(smin, v);
        smax = pk_max(smax, v);
    }
    uint32_t a = V(-r), b = V(1 - r), c = V(r + 1), d = V(r + 2);
    mn0 = pk_min(smin, pk_min(a, b));
    mx0 = pk_max(smax, pk_max(a, b));
    mn1 = pk_min(smin, pk_min(c, d));
    mx1 = pk_max(smax, pk_max(c, d));
    c0 = D[0 - JLO];
    c1 = D[1 - JLO];
}

// out[i] = op(h[i .. i+K-1]) for i < R by van Herk / Gil-Werman: block suffix
// and prefix scans of length K, one combine per output.  Unused scan entries are
// removed by the compiler.
template <int K, int R, bool IS_MIN>
__device__ __forceinline__ void sliding(const uint32_t (&h)[R + K - 1], uint32_t (&out)[R]) {
    constexpr int L = R + K - 1;
    auto op = [](uint32_t a, uint32_t b) { return IS_MIN ? pk_min(a, b) : pk_max(a, b); };
    uint32_t suf[L], pre[L];
#pragma unroll
    for (int i = L - 1; i >= 0; --i)
        suf[i] = (i % K == K - 1 || i == L - 1) ? h[i] : op(h[i], suf[i + 1]);
#pragma unroll
    for (int i = 0; i < L; ++i) pre[i] = (i % K == 0) ? h[i] : op(pre[i - 1], h[i]);
#pragma unroll
    for (int i = 0; i < R; ++i) out[i] = (i % K == 0) ? suf[i] : op(suf[i], pre[i + K - 1]);
}

// Flag bit layout inside a thread's 32-bit mask: bit q (+0, +16, +8, +24) is
// column 0 (1, 2, 3) of output row q.
__device__ __forceinline__ int bit_col(int b) { return (((b >> 3) & 1) << 1) | (b >> 4); }
__device__ __forceinline__ int bit_row(int b) { return b & 7; }

// Flags of the thread's 4 x R block (bit set = noisy).
template <int K>
__device__ __forceinline__ uint32_t detect_block(const uint16_t *tile, int strip, int tx) {
    using G = Geometry<K>;
    constexpr int R = G::R, L = R + K - 1;
    const uint16_t *base = tile + strip * R * kLdsW + kHalo + 4 * tx;
    uint32_t hmn0[L], hmn1[L], hmx0[L], hmx1[L], c0[R], c1[R];
#pragma unroll
    for (int i = 0; i < L; ++i) {
        uint32_t a, b;
        row_minmax<G::r>(base + i * kLdsW, hmn0[i], hmn1[i], hmx0[i], hmx1[i], a, b);
        if (i >= G::r && i < G::r + R) {
            c0[i - G::r] = a;
            c1[i - G::r] = b;
        }
    }
    uint32_t vmn0[R], vmn1[R], vmx0[R], vmx1[R];
    sliding<K, R, true>(hmn0, vmn0);
    sliding<K, R, true>(hmn1, vmn1);
    sliding<K, R, false>(hmx0, vmx0);
    sliding<K, R, false>(hmx1, vmx1);
    uint32_t keep = 0;  // bit set = signal pixel
#pragma unroll
    for (int q = 0; q < R; ++q) {
        // a half is zero exactly when the centre equals the window min or max
        uint32_t z0 = pk_min(pk_subsat(c0[q], vmn0[q]), pk_subsat(vmx0[q], c0[q]));
        uint32_t z1 = pk_min(pk_subsat(c1[q], vmn1[q]), pk_subsat(vmx1[q], c1[q]));
        keep |= pk_min(z0, 0x00010001u) << q;
        keep |= pk_min(z1, 0x00010001u) << (q + 8);
    }
    return ~keep;
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

// ---------------------------------------------------------------------------
// 4. median selection on two windows at once (packed u16)
// ---------------------------------------------------------------------------
// Window element i (row-major) of the window whose top-left LDS value is w.
template <int K>
__device__ __forceinline__ uint32_t win_pair(const uint16_t *w0, const uint16_t *w1, int i) {
    int off = (i / K) * kLdsW + (i % K);
    return (uint32_t)w0[off] | ((uint32_t)w1[off] << 16);
}

template <int... I, typename F>
__device__ __forceinline__ void static_for(std::integer_sequence<int, I...>, F &&f) {
    (f(std::integral_constant<int, I>{}), ...);
}

// Forgetful selection: sort the first M = (n+3)/2 values (odd-even merge
// network), drop the two ends (neither can be the median of n), then for each
// remaining value insert it into the sorted run and drop both ends again.  After
// the last value the run holds one element: the median.  Insertion of x into a
// sorted run s, ends dropped, is s'[i] = max(s[i], min(s[i+1], x)).
template <int K>
__device__ __forceinline__ uint32_t median_forgetful(const uint16_t *w0, const uint16_t *w1) {
    constexpr int N = K * K;
    constexpr int M = (N + 3) / 2;
    uint32_t a[M];
#pragma unroll
    for (int i = 0; i < M; ++i) a[i] = win_pair<K>(w0, w1, i);
    static_for(std::make_integer_sequence<int, net::Network<M>::size>{}, [&](auto c) {
        constexpr int i = net::network<M>.lo[decltype(c)::value];
        constexpr int j = net::network<M>.hi[decltype(c)::value];
        uint32_t lo = pk_min(a[i], a[j]);
        uint32_t hi = pk_max(a[i], a[j]);
        a[i] = lo;
        a[j] = hi;
    });
    // run = a[1 .. M-2]
#pragma unroll
    for (int t = 0; t < N - M; ++t) {
        uint32_t x = win_pair<K>(w0, w1, M + t);
        int L = M - 2 - t;  // current run length, run at a[1 .. L]
#pragma unroll
        for (int i = 1; i < M - 1; ++i)
            if (i < L) a[i] = pk_max(a[i], pk_min(a[i + 1], x));
    }
    return a[1];
}

// Bisection on grey level: the median is the smallest value t with more than
// (n-1)/2 window values <= t.  Works on [g_min, g_max] of each window, two
// windows per lane; count of values above t uses saturating subtraction.
template <int K>
__device__ __forceinline__ uint32_t median_bisect(const uint16_t *w0, const uint16_t *w1) {
    constexpr int N = K * K;
    constexpr uint32_t rank = (N - 1) / 2;
    uint32_t mn = 0xffffffffu, mx = 0u;
    for (int i = 0; i < N; ++i) {
        uint32_t v = win_pair<K>(w0, w1, i);
        mn = pk_min(mn, v);
        mx = pk_max(mx, v);
    }
    uint32_t lo0 = mn & 0xffffu, lo1 = mn >> 16, hi0 = mx & 0xffffu, hi1 = mx >> 16;
    while (lo0 < hi0 || lo1 < hi1) {
        uint32_t t0 = (lo0 + hi0) >> 1, t1 = (lo1 + hi1) >> 1;
        uint32_t t = t0 | (t1 << 16);
        uint32_t above = 0;  // packed count of values > t
        for (int i = 0; i < N; ++i) {
            uint32_t v = win_pair<K>(w0, w1, i);
            above = pk_add(above, pk_min(pk_subsat(v, t), 0x00010001u));
        }
        uint32_t le0 = N - (above & 0xffffu), le1 = N - (above >> 16);
        if (lo0 < hi0) {
            if (le0 > rank) hi0 = t0;
            else lo0 = t0 + 1;
        }
        if (lo1 < hi1) {
            if (le1 > rank) hi1 = t1;
            else lo1 = t1 + 1;
        }
    }
    return lo0 | (lo1 << 16);
}

template <int K>
__device__ __forceinline__ uint32_t median_pair(const uint16_t *w0, const uint16_t *w1) {
    if constexpr (K <= 7)
        return median_forgetful<K>(w0, w1);
    else
        return median_bisect<K>(w0, w1);
}

// ---------------------------------------------------------------------------
// wave / workgroup prefix sums
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// ---------------------------------------------------------------------------
// 5. stores
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void store_px(uint8_t *row, int x, uint32_t v) {
    if constexpr (sizeof(T) == 1)
        row[x] = (uint8_t)v;
    else
        reinterpret_cast<uint16_t *>(row)[x] = (uint16_t)v;
}

// Four 16-bit LDS values (two packed pairs) to the frame row at column px.
template <typename T>
__device__ __forceinline__ void store4(uint8_t *row, int px, int W, bool aligned, uint32_t p0,
                                       uint32_t p1) {
    if (aligned && px + 4 <= W) {
        if constexpr (sizeof(T) == 2) {
            *reinterpret_cast<uint2 *>(row + 2 * (uint64_t)px) = make_uint2(p0, p1);
        } else {
            uint32_t b = (p0 & 0xffu) | ((p0 >> 8) & 0xff00u) | ((p1 & 0xffu) << 16) |
                         ((p1 & 0xff0000u) << 8);
            *reinterpret_cast<uint32_t *>(row + px) = b;
        }
    } else {
        uint32_t e[4] = {p0 & 0xffffu, p0 >> 16, p1 & 0xffffu, p1 >> 16};
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (px + i < W) store_px<T>(row, px + i, e[i]);
    }
}

// ---------------------------------------------------------------------------
// the tile kernel
// ---------------------------------------------------------------------------
// Workgroups are handed to the 8 XCDs round-robin; renumber them so each XCD
// walks a contiguous range of tiles (neighbouring tiles share halo rows in the
// XCD's L2).
__device__ __forceinline__ int xcd_tile(int b, int n) {
    constexpr int X = 8;
    int per = (n + X - 1) / X;
    int tall = n % X == 0 ? X : n % X;
    int xcd = b % X, local = b / X;
    return xcd < tall ? xcd * per + local : tall * per + (xcd - tall) * (per - 1) + local;
}

template <typename T, int K, int MODE>
__device__ __forceinline__ void filter_tile(const StackArgs &a, int tile) {
    using G = Geometry<K>;
    constexpr int R = G::R;
    __shared__ __attribute__((aligned(16))) uint16_t lds_tile[G::rows * kLdsW];
    __shared__ uint16_t lds_list[G::tile_px];
    __shared__ uint32_t lds_wave[kThreads / 64];

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

    const uint8_t *src = a.src + (uint64_t)f * a.src_stride;
    load_tile<T, K>(src, a.src_pitch, W, H, x0, y0, aligned, lds_tile);
    __syncthreads();

    uint32_t flags;
    if constexpr (MODE == MODE_DETECT || MODE == MODE_FNR) {
        flags = detect_block<K>(lds_tile, strip, tx) & valid;
    } else if constexpr (MODE == MODE_MEDIAN_MASK) {
        flags = 0;
        const uint8_t *m = a.mask_in + (uint64_t)f * a.mask_stride;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (py + q >= H) break;
            const uint8_t *mr = m + (uint64_t)(py + q) * a.mask_pitch;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (px + e < W && mr[px + e] != 0) {
                    int sh = (e == 0) ? 0 : (e == 1) ? 16 : (e == 2) ? 8 : 24;
                    flags |= 1u << (q + sh);
                }
            }
        }
    } else {
        flags = valid;
    }

    const int lane = tid & 63, wave = tid >> 6;
    const uint32_t cnt = __builtin_popcount(flags);
    const uint32_t incl = wave_inclusive_sum(cnt);
    if (lane == 63) lds_wave[wave] = incl;
    __syncthreads();
    uint32_t base = incl - cnt, total = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        uint32_t t = lds_wave[w];
        if (w < wave) base += t;
        total += t;
    }

    if constexpr (MODE == MODE_DETECT || MODE == MODE_FNR) {
        if (a.count != nullptr && tid == 0 && total != 0) atomicAdd(a.count, (unsigned long long)total);
    }

    if constexpr (MODE == MODE_DETECT) {
        uint8_t *m = a.mask_out + (uint64_t)f * a.mask_stride;
        for (int q = 0; q < R; ++q) {
            if (py + q >= H) break;
            uint8_t *mr = m + (uint64_t)(py + q) * a.mask_pitch;
            uint32_t b0 = (flags >> q) & 1u, b1 = (flags >> (q + 16)) & 1u;
            uint32_t b2 = (flags >> (q + 8)) & 1u, b3 = (flags >> (q + 24)) & 1u;
            if (aligned && px + 4 <= W) {
                *reinterpret_cast<uint32_t *>(mr + px) = b0 | (b1 << 8) | (b2 << 16) | (b3 << 24);
            } else {
                uint32_t e[4] = {b0, b1, b2, b3};
                for (int i = 0; i < 4; ++i)
                    if (px + i < W) mr[px + i] = (uint8_t)e[i];
            }
        }
        return;
    } else {
        // 3. compaction: LDS offsets of the flagged pixels' centres
        const int centre0 = (strip * R + G::r) * kLdsW + kHalo + 4 * tx;
        {
            uint32_t m = flags, j = base;
            while (m) {
                int b = __builtin_ctz(m);
                m &= m - 1;
                lds_list[j++] = (uint16_t)(centre0 + bit_row(b) * kLdsW + bit_col(b));
            }
        }
        __syncthreads();
        // 4. medians, two list entries per lane
        const int corner = G::r * kLdsW + G::r;
        for (uint32_t i = 2 * tid; i < total; i += 2 * kThreads) {
            uint32_t e0 = lds_list[i];
            uint32_t e1 = (i + 1 < total) ? lds_list[i + 1] : e0;
            uint32_t med = median_pair<K>(lds_tile + e0 - corner, lds_tile + e1 - corner);
            lds_list[i] = (uint16_t)(med & 0xffffu);
            if (i + 1 < total) lds_list[i + 1] = (uint16_t)(med >> 16);
        }
        __syncthreads();
        // results back into the tile at the thread's own pixels
        {
            uint32_t m = flags, j = base;
            while (m) {
                int b = __builtin_ctz(m);
                m &= m - 1;
                lds_tile[centre0 + bit_row(b) * kLdsW + bit_col(b)] = lds_list[j++];
            }
        }
        // 5. store the thread's block (its own LDS values only: no barrier needed)
        uint8_t *dst = a.dst + (uint64_t)f * a.dst_stride;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (py + q >= H) break;
            const uint32_t *c = reinterpret_cast<const uint32_t *>(lds_tile + centre0 + q * kLdsW);
            store4<T>(dst + (uint64_t)(py + q) * a.dst_pitch, px, W, aligned, c[0], c[1]);
        }
    }
}

template <typename T, int K, int MODE>
__global__ __launch_bounds__(kThreads) void fnr_stack_kernel(StackArgs a) {
    filter_tile<T, K, MODE>(a, xcd_tile(blockIdx.x, a.total_tiles));
}

__global__ void zero_u64_kernel(unsigned long long *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

}  // namespace irf
