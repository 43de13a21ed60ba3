// stack_launch.hpp -- host launch of the single-size (frame and stack) kernels
// by window, mode, workgroup size and selection algorithm.  The kernels of each
// pixel type are instantiated in their own translation unit (stack_u8.hip,
// stack_u16.hip), so the two compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include "fnr_device.hpp"
#include "fused_device.hpp"
#include "host_common.hpp"

namespace irf {

// One tuning-table entry: workgroup size (128 or 256 threads, i.e. tiles of
// 128x32 or 128x64 pixels) and selection algorithm (Select).
struct Tuning {
    int threads;
    int select;
};

inline Tuning default_tuning(int window) { return {default_threads(window), default_select(window)}; }

// Whether a kernel exists for (window, tuning): 128 or 256 threads; networks
// and one-lane bisection up to 15x15, group bisection and the histogram radix
// select up to 31x31; above that group bisection on 128 threads only.
inline bool tuning_available(int window, Tuning t) {
    if (t.threads != 128 && t.threads != 256) return false;
    if (window <= kNetworkMaxWindow) return t.select == kSelectNetwork || t.select == kSelectBisect;
    if (window <= kLargeMaxWindow) return t.select == kSelectGroup || t.select == kSelectHist;
    return t.threads == 128 && t.select == kSelectGroup;
}

// Launch the stack kernel of the pixel type for a.total_tiles tiles; false if
// the combination has no kernel (nothing is launched then).  Windows above
// 15x15 go to launch_stack_large_*, and those above 31x31 on to
// launch_stack_huge_*, each instantiated in translation units of their own
// (stack_large_u8.hip, stack_large_u16.hip, stack_huge_u8.hip,
// stack_huge_u16.hip) so the build stays parallel.
bool launch_stack_u8(int window, int mode, Tuning t, const StackArgs &a, hipStream_t s);
bool launch_stack_u16(int window, int mode, Tuning t, const StackArgs &a, hipStream_t s);
bool launch_stack_large_u8(int window, int mode, Tuning t, const StackArgs &a, hipStream_t s);
bool launch_stack_large_u16(int window, int mode, Tuning t, const StackArgs &a, hipStream_t s);
bool launch_stack_huge_u8(int window, int mode, Tuning t, const StackArgs &a, hipStream_t s);
bool launch_stack_huge_u16(int window, int mode, Tuning t, const StackArgs &a, hipStream_t s);

// Two passes in one launch (fused.hip): windows up to 9x9, workgroups of 256 or
// 512 threads (blocks of 128 x 64 or 128 x 128 pixels).
inline bool fused_available(int window, int threads) {
    return window >= 3 && window <= kFusedMaxWindow && (window & 1) && (threads == 256 || threads == 512);
}
// Pass-2 output rows of a fused tile.
inline int fused_tile_rows(int window, int threads) {
    return threads / kThreadsX * Geometry<3>::R - 2 * (window / 2);
}
// Fusion setting that picks per frame size (the untuned default).
constexpr int kFusionAuto = -1;
// The automatic choice (the default): separate passes.  Both kernels are
// bound by vector ALU work per covered pixel, and a fused block outputs only
// 120 x (TH - k + 1) of its 128 x TH pixels, so its tiling never covers fewer
// pixels than the tiles of two single passes (6 fused tiles cover a 640-pixel
// row that 5 plain tiles cover, for one); at equal coverage separate passes
// measured faster at 3x3 to 7x7 (320x240 u8 and 640x512 u16 stacks).  The
// exception is 8-bit 9x9, where the 512-thread fused kernel measured 1.22x
// faster on 320x240 frames and 1.1x on 640x512 ones: that choice is left to
// the autotuner's table, which takes it from its own measurement.  The fused
// kernels run when set explicitly, or when the autotuner finds one faster on
// the caller's frames.
inline int auto_fusion(int /*width*/, int /*height*/, int /*window*/, int /*plain_threads*/) { return 0; }
// Launch the fused kernel for a.total_tiles fused tiles (the caller sets the
// tile counts from kFusedTileW and fused_tile_rows); false if no kernel exists.
bool launch_fused2(int bytes, int window, int threads, const StackArgs &a, hipStream_t s);

namespace stack_impl {

// Persistent grid: as many workgroups as fit on the device at once (never more
// than there are tiles).
template <typename T, int K, int MODE, int NT, int SEL>
int persistent_grid(int total_tiles) {
    static const int per_cu = [] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fnr_persistent_kernel<T, K, MODE, NT, SEL>, NT,
                                                         0) != hipSuccess ||
            n < 1)
            n = 1;
        return n;
    }();
    const long long g = (long long)per_cu * host::device_cus();
    return (int)(g < total_tiles ? g : total_tiles);
}

template <typename T, int K, int MODE, int NT, int SEL>
void launch_variant(const StackArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((fnr_persistent_kernel<T, K, MODE, NT, SEL>),
                       dim3(persistent_grid<T, K, MODE, NT, SEL>(a.total_tiles)), dim3(NT), 0, s, a);
}

// Detection selects nothing: its kernels exist per workgroup size only.
template <typename T, int K, int MODE, int NT>
bool launch_threads(int select, const StackArgs &a, hipStream_t s) {
    if constexpr (MODE == MODE_DETECT || MODE == MODE_DETECT_DIR) {
        launch_variant<T, K, MODE, NT, default_select(K)>(a, s);
        return true;
    } else if constexpr (K > kNetworkMaxWindow) {
        if constexpr (K <= kLargeMaxWindow) {
            if (select == kSelectHist) {
                launch_variant<T, K, MODE, NT, kSelectHist>(a, s);
                return true;
            }
        }
        if (select != kSelectGroup) return false;
        launch_variant<T, K, MODE, NT, kSelectGroup>(a, s);
        return true;
    } else {
        if (select == kSelectBisect) {
            launch_variant<T, K, MODE, NT, kSelectBisect>(a, s);
            return true;
        }
        if constexpr (K <= kNetworkMaxWindow) {
            if (select == kSelectNetwork) {
                launch_variant<T, K, MODE, NT, kSelectNetwork>(a, s);
                return true;
            }
        }
        return false;
    }
}

template <typename T, int K, int MODE>
bool launch_tuned(Tuning t, const StackArgs &a, hipStream_t s) {
    if (t.threads == 128) return launch_threads<T, K, MODE, 128>(t.select, a, s);
    if constexpr (K <= kLargeMaxWindow) {
        if (t.threads == 256) return launch_threads<T, K, MODE, 256>(t.select, a, s);
    }
    return false;
}

// The window ranges of the translation units: up to 15x15, 17x17 .. 31x31,
// 33x33 .. 63x63.
enum WindowRange : int { kSmallWindows = 0, kLargeWindows = 1, kHugeWindows = 2 };

template <typename T, int MODE, int RANGE>
bool launch_window(int window, Tuning t, const StackArgs &a, hipStream_t s) {
    if constexpr (RANGE == kSmallWindows) {
        switch (window) {
            case 3: return launch_tuned<T, 3, MODE>(t, a, s);
            case 5: return launch_tuned<T, 5, MODE>(t, a, s);
            case 7: return launch_tuned<T, 7, MODE>(t, a, s);
            case 9: return launch_tuned<T, 9, MODE>(t, a, s);
            case 11: return launch_tuned<T, 11, MODE>(t, a, s);
            case 13: return launch_tuned<T, 13, MODE>(t, a, s);
            case 15: return launch_tuned<T, 15, MODE>(t, a, s);
            default: return false;
        }
    } else if constexpr (RANGE == kLargeWindows) {
        switch (window) {
            case 17: return launch_tuned<T, 17, MODE>(t, a, s);
            case 19: return launch_tuned<T, 19, MODE>(t, a, s);
            case 21: return launch_tuned<T, 21, MODE>(t, a, s);
            case 23: return launch_tuned<T, 23, MODE>(t, a, s);
            case 25: return launch_tuned<T, 25, MODE>(t, a, s);
            case 27: return launch_tuned<T, 27, MODE>(t, a, s);
            case 29: return launch_tuned<T, 29, MODE>(t, a, s);
            case 31: return launch_tuned<T, 31, MODE>(t, a, s);
            default: return false;
        }
    } else {
        switch (window) {
            case 33: return launch_tuned<T, 33, MODE>(t, a, s);
            case 35: return launch_tuned<T, 35, MODE>(t, a, s);
            case 37: return launch_tuned<T, 37, MODE>(t, a, s);
            case 39: return launch_tuned<T, 39, MODE>(t, a, s);
            case 41: return launch_tuned<T, 41, MODE>(t, a, s);
            case 43: return launch_tuned<T, 43, MODE>(t, a, s);
            case 45: return launch_tuned<T, 45, MODE>(t, a, s);
            case 47: return launch_tuned<T, 47, MODE>(t, a, s);
            case 49: return launch_tuned<T, 49, MODE>(t, a, s);
            case 51: return launch_tuned<T, 51, MODE>(t, a, s);
            case 53: return launch_tuned<T, 53, MODE>(t, a, s);
            case 55: return launch_tuned<T, 55, MODE>(t, a, s);
            case 57: return launch_tuned<T, 57, MODE>(t, a, s);
            case 59: return launch_tuned<T, 59, MODE>(t, a, s);
            case 61: return launch_tuned<T, 61, MODE>(t, a, s);
            case 63: return launch_tuned<T, 63, MODE>(t, a, s);
            default: return false;
        }
    }
}

template <typename T, int RANGE>
bool launch_stack(int window, int mode, Tuning t, const StackArgs &a, hipStream_t s) {
    switch (mode) {
        case MODE_DETECT: return launch_window<T, MODE_DETECT, RANGE>(window, t, a, s);
        case MODE_FNR: return launch_window<T, MODE_FNR, RANGE>(window, t, a, s);
        case MODE_MEDIAN_MASK: return launch_window<T, MODE_MEDIAN_MASK, RANGE>(window, t, a, s);
        case MODE_MEDIAN_ALL: return launch_window<T, MODE_MEDIAN_ALL, RANGE>(window, t, a, s);
        case MODE_DETECT_DIR:  // the 3 x 3 directional test only
            if constexpr (RANGE == kSmallWindows)
                return window == 3 && launch_tuned<T, 3, MODE_DETECT_DIR>(t, a, s);
            return false;
        default: return false;
    }
}

}  // namespace stack_impl
}  // namespace irf
