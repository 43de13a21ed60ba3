// irfilter.hip -- host runtime and C ABI of the FNR filter (see include/irfilter.h).
//
// Validation runs on the host before any HIP call, so argument errors are
// reported without touching the device.  Launches go to the caller's stream;
// nothing here allocates device memory.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <atomic>
#include <mutex>

#include "../../include/irfilter.h"
#include "fnr_device.hpp"
#include "host_common.hpp"
#include "stack_launch.hpp"

namespace irf {
namespace {

using namespace host;

constexpr int kVersion = (1 << 16) | 2;  // 1.2: windows up to 63x63 (1.1: pass fusion, directional detector)

// Tuning table of the single-size kernels, per pixel type and window: 0 means
// the untuned default, otherwise threads | select << 16.  Entries change only
// through ir_filter_set_tuning; a launch reads its entry once.
constexpr int kWindowSlots = (IRF_MAX_WINDOW - 3) / 2 + 1;
std::atomic<uint32_t> g_tuning[2][kWindowSlots];

// Fusion of pass pairs, per pixel type and window: 0 means automatic (the
// default), 1 runs every pass as its own launch, otherwise the fused kernel's
// workgroup size.
std::atomic<uint32_t> g_fusion[2][kWindowSlots];

int window_slot(int window) { return (window - 3) / 2; }

int fusion_of(irf_dtype dtype, int window) {
    const uint32_t v = g_fusion[dtype == IRF_U8 ? 0 : 1][window_slot(window)].load(std::memory_order_relaxed);
    if (v == 0) return kFusionAuto;
    return v == 1 ? 0 : (int)v;
}

Tuning tuning_of(irf_dtype dtype, int window) {
    const uint32_t v = g_tuning[dtype == IRF_U8 ? 0 : 1][window_slot(window)].load(std::memory_order_relaxed);
    if (v == 0) return default_tuning(window);
    return {(int)(v & 0xffffu), (int)(v >> 16)};
}

int tile_rows(int threads) { return threads / kThreadsX * Geometry<3>::R; }

template <int MODE>
irf_status launch(irf_dtype dtype, int window, int nframes, StackArgs a, hipStream_t s) {
    const Tuning t = tuning_of(dtype, window);
    const int th = tile_rows(t.threads);
    a.tiles_x = (a.width + kTileW - 1) / kTileW;
    const int tiles_y = (a.height + th - 1) / th;
    const uint64_t per_frame = (uint64_t)a.tiles_x * (uint64_t)tiles_y;
    const uint64_t total = per_frame * (uint64_t)nframes;
    if (total > 0x7fffffffull) return IRF_ERR_DIMS;
    a.tiles_per_frame = (int)per_frame;
    a.total_tiles = (int)total;
    a.pk_one = 0x00010001u;
    (void)hipGetLastError();
    const bool ok = dtype == IRF_U8 ? launch_stack_u8(window, MODE, t, a, s)
                                    : launch_stack_u16(window, MODE, t, a, s);
    if (!ok) return IRF_ERR_WINDOW;
    if (hipGetLastError() != hipSuccess) return IRF_ERR_HIP;
    return IRF_OK;
}

// Fused workgroup size for pairs of passes over width x height frames, 0 for
// separate passes.
int resolved_fusion(irf_dtype dtype, int window, int width, int height) {
    const int f = fusion_of(dtype, window);
    return f == kFusionAuto ? auto_fusion(width, height, window, tuning_of(dtype, window).threads) : f;
}

// Two passes of the filter in one launch; a.count (if set) receives both
// passes' counts, in two consecutive entries.
irf_status launch_fused(irf_dtype dtype, int window, int threads, int nframes, StackArgs a, hipStream_t s) {
    const int oh = fused_tile_rows(window, threads);
    a.tiles_x = (a.width + kFusedTileW - 1) / kFusedTileW;
    const int tiles_y = (a.height + oh - 1) / oh;
    const uint64_t per_frame = (uint64_t)a.tiles_x * (uint64_t)tiles_y;
    const uint64_t total = per_frame * (uint64_t)nframes;
    if (total > 0x7fffffffull) return IRF_ERR_DIMS;
    a.tiles_per_frame = (int)per_frame;
    a.total_tiles = (int)total;
    a.pk_one = 0x00010001u;
    (void)hipGetLastError();
    if (!launch_fused2(bytes_of(dtype), window, threads, a, s)) return IRF_ERR_WINDOW;
    if (hipGetLastError() != hipSuccess) return IRF_ERR_HIP;
    return IRF_OK;
}

irf_status zero_counts(uint64_t *p, int n, hipStream_t s) {
    if (!p) return IRF_OK;
    (void)hipGetLastError();
    hipLaunchKernelGGL(zero_u64_kernel, dim3((n + 63) / 64), dim3(64), 0, s,
                       reinterpret_cast<unsigned long long *>(p), n);
    return hipGetLastError() == hipSuccess ? IRF_OK : IRF_ERR_HIP;
}

irf_status run_frames(const void *src, size_t src_pitch, size_t src_stride, void *dst,
                      size_t dst_pitch, size_t dst_stride, int width, int height, int nframes,
                      irf_dtype dtype, int window, int passes, void *scratch, size_t scratch_pitch,
                      size_t scratch_stride, uint64_t *counts, hipStream_t stream) {
    if (!src || !dst) return IRF_ERR_NULL;
    irf_status st = check_common(width, height, nframes, dtype, window);
    if (st) return st;
    if (passes < 1 || passes > IRF_MAX_PASSES) return IRF_ERR_PASSES;
    if (passes >= 2 && !scratch) return IRF_ERR_PASSES;
    const int b = bytes_of(dtype);
    if ((st = check_layout(src_pitch, src_stride, width, height, nframes, b))) return st;
    if ((st = check_layout(dst_pitch, dst_stride, width, height, nframes, b))) return st;
    const Span ss = span_of(src, src_pitch, src_stride, width, height, nframes, b);
    const Span ds = span_of(dst, dst_pitch, dst_stride, width, height, nframes, b);
    if (overlap(ss, ds)) return IRF_ERR_ALIAS;
    if (passes >= 2) {
        if ((st = check_layout(scratch_pitch, scratch_stride, width, height, nframes, b))) return st;
        const Span xs = span_of(scratch, scratch_pitch, scratch_stride, width, height, nframes, b);
        if (overlap(xs, ss) || overlap(xs, ds)) return IRF_ERR_ALIAS;
    }
    if (counts) {
        // the counts are zeroed and accumulated while the passes read src and
        // write dst and scratch: they may share memory with none of them
        const Span cs = {reinterpret_cast<uintptr_t>(counts),
                         reinterpret_cast<uintptr_t>(counts) + sizeof(uint64_t) * (size_t)passes};
        if (overlap(cs, ss) || overlap(cs, ds)) return IRF_ERR_ALIAS;
        if (passes >= 2 &&
            overlap(cs, span_of(scratch, scratch_pitch, scratch_stride, width, height, nframes, b)))
            return IRF_ERR_ALIAS;
    }
    if ((st = zero_counts(counts, passes, stream))) return st;
    // Pairs of passes run fused where a fused kernel is enabled, an odd last
    // pass on its own.  Launch l reads the frame launch l-1 wrote (src for the
    // first) and writes dst when an even number of launches follow it, else
    // scratch, so no launch reads the frame it writes.
    const int fuse = passes >= 2 ? resolved_fusion(dtype, window, width, height) : 0;
    const int launches = fuse ? (passes + 1) / 2 : passes;
    const void *in = src;
    size_t in_pitch = src_pitch, in_stride = src_stride;
    for (int l = 1, p = 1; l <= launches; ++l) {
        const int np = (fuse && p < passes) ? 2 : 1;  // passes in this launch, p being the first
        const bool to_dst = ((launches - l) & 1) == 0;
        void *out = to_dst ? dst : scratch;
        const size_t out_pitch = to_dst ? dst_pitch : scratch_pitch;
        const size_t out_stride = to_dst ? dst_stride : scratch_stride;
        StackArgs a = {};
        a.src = static_cast<const uint8_t *>(in);
        a.dst = static_cast<uint8_t *>(out);
        a.src_pitch = in_pitch;
        a.dst_pitch = out_pitch;
        a.src_stride = in_stride;
        a.dst_stride = out_stride;
        a.width = width;
        a.height = height;
        a.aligned = is16(in) && is16(out) && is16(in_pitch) && is16(out_pitch) &&
                    (nframes == 1 || (is16(in_stride) && is16(out_stride)));
        a.count = counts ? reinterpret_cast<unsigned long long *>(counts + (p - 1)) : nullptr;
        st = np == 2 ? launch_fused(dtype, window, fuse, nframes, a, stream)
                     : launch<MODE_FNR>(dtype, window, nframes, a, stream);
        if (st) return st;
        p += np;
        in = out;
        in_pitch = out_pitch;
        in_stride = out_stride;
    }
    return IRF_OK;
}

// ir_filter_run_noalloc: the intermediate passes of a call live in this
// file-scope device array instead of a caller's scratch frame.  Every GPU the
// library runs on holds its own copy until the process ends; all calls on one
// GPU share it, so calls that overlap on one GPU race.  In host code the
// array's name is only a stand-in: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
namespace noalloc {

constexpr size_t kScratchBytes = (size_t)32 << 20;  // one 4096 x 4096 u16 frame
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of `scratch`, per device

// Address of this device's `scratch`, looked up with the device current on
// the first call that needs it.
irf_status device_scratch(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return IRF_ERR_HIP;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return IRF_ERR_HIP;
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return IRF_OK;
}

// Row pitch of the intermediate frames: whole 256-byte lines.
size_t scratch_pitch(int width, irf_dtype dtype) {
    return ((size_t)width * (size_t)bytes_of(dtype) + 255) / 256 * 256;
}

}  // namespace noalloc

}  // namespace
}  // namespace irf

using namespace irf;

extern "C" {

irf_status ir_filter_detect(const void *src, size_t src_pitch, uint8_t *mask, size_t mask_pitch,
                            int width, int height, irf_dtype dtype, int window,
                            uint64_t *flagged_count, hipStream_t stream) {
    try {
        if (!src || !mask) return IRF_ERR_NULL;
        irf_status st = check_common(width, height, 1, dtype, window);
        if (st) return st;
        const int b = bytes_of(dtype);
        if ((st = check_layout(src_pitch, 0, width, height, 1, b))) return st;
        if ((st = check_layout(mask_pitch, 0, width, height, 1, 1))) return st;
        const Span ss = span_of(src, src_pitch, 0, width, height, 1, b);
        const Span ms = span_of(mask, mask_pitch, 0, width, height, 1, 1);
        if (overlap(ss, ms)) return IRF_ERR_ALIAS;
        if (flagged_count) {
            const Span cs = {reinterpret_cast<uintptr_t>(flagged_count),
                             reinterpret_cast<uintptr_t>(flagged_count) + sizeof(uint64_t)};
            if (overlap(cs, ss) || overlap(cs, ms)) return IRF_ERR_ALIAS;
        }
        if ((st = zero_counts(flagged_count, 1, stream))) return st;
        StackArgs a = {};
        a.src = static_cast<const uint8_t *>(src);
        a.mask_out = mask;
        a.src_pitch = src_pitch;
        a.mask_pitch = mask_pitch;
        a.width = width;
        a.height = height;
        a.aligned = is16(src) && is16(src_pitch) && is16(mask) && is16(mask_pitch);
        a.count = reinterpret_cast<unsigned long long *>(flagged_count);
        return launch<MODE_DETECT>(dtype, window, 1, a, stream);
    } catch (...) {
        return IRF_ERR_HIP;
    }
}

irf_status ir_filter_detect_directional(const void *src, size_t src_pitch, uint8_t *mask, size_t mask_pitch,
                                        int width, int height, irf_dtype dtype, uint64_t *flagged_count,
                                        hipStream_t stream) {
    try {
        if (!src || !mask) return IRF_ERR_NULL;
        irf_status st = check_common(width, height, 1, dtype, 3);
        if (st) return st;
        const int b = bytes_of(dtype);
        if ((st = check_layout(src_pitch, 0, width, height, 1, b))) return st;
        if ((st = check_layout(mask_pitch, 0, width, height, 1, 1))) return st;
        const Span ss = span_of(src, src_pitch, 0, width, height, 1, b);
        const Span ms = span_of(mask, mask_pitch, 0, width, height, 1, 1);
        if (overlap(ss, ms)) return IRF_ERR_ALIAS;
        if (flagged_count) {
            const Span cs = {reinterpret_cast<uintptr_t>(flagged_count),
                             reinterpret_cast<uintptr_t>(flagged_count) + sizeof(uint64_t)};
            if (overlap(cs, ss) || overlap(cs, ms)) return IRF_ERR_ALIAS;
        }
        if ((st = zero_counts(flagged_count, 1, stream))) return st;
        StackArgs a = {};
        a.src = static_cast<const uint8_t *>(src);
        a.mask_out = mask;
        a.src_pitch = src_pitch;
        a.mask_pitch = mask_pitch;
        a.width = width;
        a.height = height;
        a.aligned = is16(src) && is16(src_pitch) && is16(mask) && is16(mask_pitch);
        a.count = reinterpret_cast<unsigned long long *>(flagged_count);
        return launch<MODE_DETECT_DIR>(dtype, 3, 1, a, stream);
    } catch (...) {
        return IRF_ERR_HIP;
    }
}

irf_status ir_filter_median(const void *src, size_t src_pitch, const uint8_t *mask,
                            size_t mask_pitch, void *dst, size_t dst_pitch, int width, int height,
                            irf_dtype dtype, int window, hipStream_t stream) {
    try {
        if (!src || !dst) return IRF_ERR_NULL;
        irf_status st = check_common(width, height, 1, dtype, window);
        if (st) return st;
        const int b = bytes_of(dtype);
        if ((st = check_layout(src_pitch, 0, width, height, 1, b))) return st;
        if ((st = check_layout(dst_pitch, 0, width, height, 1, b))) return st;
        if (mask && (st = check_layout(mask_pitch, 0, width, height, 1, 1))) return st;
        const Span ss = span_of(src, src_pitch, 0, width, height, 1, b);
        const Span ds = span_of(dst, dst_pitch, 0, width, height, 1, b);
        if (overlap(ss, ds)) return IRF_ERR_ALIAS;
        if (mask && overlap(span_of(mask, mask_pitch, 0, width, height, 1, 1), ds)) return IRF_ERR_ALIAS;
        StackArgs a = {};
        a.src = static_cast<const uint8_t *>(src);
        a.dst = static_cast<uint8_t *>(dst);
        a.mask_in = mask;
        a.src_pitch = src_pitch;
        a.dst_pitch = dst_pitch;
        a.mask_pitch = mask_pitch;
        a.width = width;
        a.height = height;
        a.aligned = is16(src) && is16(src_pitch) && is16(dst) && is16(dst_pitch) &&
                    (!mask || (is16(mask) && is16(mask_pitch)));
        return mask ? launch<MODE_MEDIAN_MASK>(dtype, window, 1, a, stream)
                    : launch<MODE_MEDIAN_ALL>(dtype, window, 1, a, stream);
    } catch (...) {
        return IRF_ERR_HIP;
    }
}

irf_status ir_filter_run(const void *src, size_t src_pitch, void *dst, size_t dst_pitch, int width,
                         int height, irf_dtype dtype, int window, int passes, void *scratch,
                         size_t scratch_pitch, uint64_t *flagged_count, hipStream_t stream) {
    try {
        return run_frames(src, src_pitch, 0, dst, dst_pitch, 0, width, height, 1, dtype, window,
                          passes, scratch, scratch_pitch, 0, flagged_count, stream);
    } catch (...) {
        return IRF_ERR_HIP;
    }
}

irf_status ir_filter_run_noalloc(const void *src, size_t src_pitch, void *dst, size_t dst_pitch, int width,
                                 int height, irf_dtype dtype, int window, int passes, uint64_t *flagged_count,
                                 hipStream_t stream) {
    try {
        if (!src || !dst) return IRF_ERR_NULL;
        irf_status st = check_common(width, height, 1, dtype, window);
        if (st) return st;
        if (passes < 1 || passes > IRF_MAX_PASSES) return IRF_ERR_PASSES;
        const size_t pitch = noalloc::scratch_pitch(width, dtype);
        if (passes >= 2 && pitch * (size_t)height > noalloc::kScratchBytes) return IRF_ERR_CAPACITY;
        void *scr = nullptr;
        if (passes >= 2 && (st = noalloc::device_scratch(&scr))) return st;
        return run_frames(src, src_pitch, 0, dst, dst_pitch, 0, width, height, 1, dtype, window, passes, scr,
                          pitch, 0, flagged_count, stream);
    } catch (...) {
        return IRF_ERR_HIP;
    }
}

irf_status ir_filter_run_frames(const void *src, size_t src_pitch, size_t src_stride, void *dst,
                                size_t dst_pitch, size_t dst_stride, int width, int height,
                                int nframes, irf_dtype dtype, int window, int passes, void *scratch,
                                size_t scratch_pitch, size_t scratch_stride,
                                uint64_t *flagged_count, hipStream_t stream) {
    try {
        return run_frames(src, src_pitch, src_stride, dst, dst_pitch, dst_stride, width, height,
                          nframes, dtype, window, passes, scratch, scratch_pitch, scratch_stride,
                          flagged_count, stream);
    } catch (...) {
        return IRF_ERR_HIP;
    }
}

const char *ir_filter_status_string(irf_status s) {
    switch (s) {
        case IRF_OK: return "ok";
        case IRF_ERR_NULL: return "null pointer";
        case IRF_ERR_DIMS: return "invalid dimensions";
        case IRF_ERR_PITCH: return "pitch or stride too small";
        case IRF_ERR_DTYPE: return "unsupported pixel type";
        case IRF_ERR_WINDOW: return "window must be odd and within 3..63 (3..31 for batch plans and the server)";
        case IRF_ERR_PASSES: return "invalid pass count or missing scratch";
        case IRF_ERR_ALIAS: return "output overlaps an input";
        case IRF_ERR_HIP: return "HIP error";
        case IRF_ERR_NOMEM: return "out of memory";
        case IRF_ERR_CAPACITY: return "batch exceeds plan capacity";
        case IRF_ERR_TUNING: return "no kernel for that workgroup size and selection algorithm";
    }
    return "unknown status";
}

int ir_filter_version(void) { return kVersion; }

irf_status ir_filter_get_tuning(irf_dtype dtype, int window, int *threads, int *select) {
    if (!threads || !select) return IRF_ERR_NULL;
    if (dtype != IRF_U8 && dtype != IRF_U16) return IRF_ERR_DTYPE;
    if (window < 3 || window > IRF_MAX_WINDOW || (window & 1) == 0) return IRF_ERR_WINDOW;
    const Tuning t = tuning_of(dtype, window);
    *threads = t.threads;
    *select = t.select;
    return IRF_OK;
}

irf_status ir_filter_get_fusion(irf_dtype dtype, int window, int *threads) {
    if (!threads) return IRF_ERR_NULL;
    if (dtype != IRF_U8 && dtype != IRF_U16) return IRF_ERR_DTYPE;
    if (window < 3 || window > IRF_MAX_WINDOW || (window & 1) == 0) return IRF_ERR_WINDOW;
    *threads = fusion_of(dtype, window);
    return IRF_OK;
}

irf_status ir_filter_resolve_fusion(irf_dtype dtype, int window, int width, int height, int *threads) {
    if (!threads) return IRF_ERR_NULL;
    const irf_status st = check_common(width, height, 1, dtype, window);
    if (st) return st;
    *threads = resolved_fusion(dtype, window, width, height);
    return IRF_OK;
}

irf_status ir_filter_set_fusion(irf_dtype dtype, int window, int threads) {
    if (dtype != IRF_U8 && dtype != IRF_U16) return IRF_ERR_DTYPE;
    if (window < 3 || window > IRF_MAX_WINDOW || (window & 1) == 0) return IRF_ERR_WINDOW;
    uint32_t v;
    if (threads == -1)
        v = 0;
    else if (threads == 0)
        v = 1;
    else if (fused_available(window, threads))
        v = (uint32_t)threads;
    else
        return IRF_ERR_TUNING;
    g_fusion[dtype == IRF_U8 ? 0 : 1][window_slot(window)].store(v, std::memory_order_relaxed);
    return IRF_OK;
}

irf_status ir_filter_set_tuning(irf_dtype dtype, int window, int threads, int select) {
    if (dtype != IRF_U8 && dtype != IRF_U16) return IRF_ERR_DTYPE;
    if (window < 3 || window > IRF_MAX_WINDOW || (window & 1) == 0) return IRF_ERR_WINDOW;
    uint32_t v = 0;  // threads = select = 0 restores the default
    if (threads != 0 || select != 0) {
        if (!tuning_available(window, {threads, select})) return IRF_ERR_TUNING;
        v = (uint32_t)threads | ((uint32_t)select << 16);
    }
    g_tuning[dtype == IRF_U8 ? 0 : 1][window_slot(window)].store(v, std::memory_order_relaxed);
    return IRF_OK;
}

}  // extern "C"
