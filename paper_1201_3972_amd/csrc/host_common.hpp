// host_common.hpp -- argument checks shared by the host entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/irfilter.h"

namespace irf {
namespace host {

inline int bytes_of(irf_dtype d) { return d == IRF_U8 ? 1 : (d == IRF_U16 ? 2 : 0); }

// One frame stack as seen by validation: [base, base + extent) must not overlap
// another output or input.
struct Span {
    uintptr_t lo, hi;
};

inline Span span_of(const void *p, size_t pitch, size_t stride, int width, int height, int nframes,
             int bytes) {
    uintptr_t lo = reinterpret_cast<uintptr_t>(p);
    uint64_t ext = (uint64_t)stride * (uint64_t)(nframes - 1) + (uint64_t)pitch * (uint64_t)(height - 1) +
                   (uint64_t)width * (uint64_t)bytes;
    return {lo, lo + (uintptr_t)ext};
}

inline bool overlap(Span a, Span b) { return a.lo < b.hi && b.lo < a.hi; }

inline bool is16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
inline bool is16(size_t v) { return (v & 15u) == 0; }

inline irf_status check_common(int width, int height, int nframes, irf_dtype dtype, int window) {
    if (width < 1 || height < 1 || width > IRF_MAX_DIM || height > IRF_MAX_DIM || nframes < 1)
        return IRF_ERR_DIMS;
    if (bytes_of(dtype) == 0) return IRF_ERR_DTYPE;
    if (window < 3 || window > IRF_MAX_WINDOW || (window & 1) == 0) return IRF_ERR_WINDOW;
    return IRF_OK;
}

// Batch plans and the server run windows up to IRF_MAX_BATCH_WINDOW.
inline irf_status check_batch_frame(int width, int height, irf_dtype dtype, int window) {
    const irf_status st = check_common(width, height, 1, dtype, window);
    if (st) return st;
    return window > IRF_MAX_BATCH_WINDOW ? IRF_ERR_WINDOW : IRF_OK;
}

// Device code addresses a frame with 32-bit byte offsets from its base and
// 24-bit row multiplies: a pitch must stay below 2^24 bytes and a frame's span
// below 4 GiB.
constexpr size_t kMaxPitch = ((size_t)1 << 24) - 1;
constexpr uint64_t kMaxFrameSpan = ((uint64_t)1 << 32) - 1;

inline irf_status check_layout(size_t pitch, size_t stride, int width, int height, int nframes, int bytes) {
    if (pitch < (size_t)width * (size_t)bytes) return IRF_ERR_PITCH;
    if (pitch > kMaxPitch) return IRF_ERR_PITCH;
    if ((uint64_t)pitch * (uint64_t)(height - 1) + (uint64_t)width * (uint64_t)bytes > kMaxFrameSpan)
        return IRF_ERR_PITCH;
    if (nframes > 1 && stride < pitch * (size_t)height) return IRF_ERR_PITCH;
    return IRF_OK;
}

inline int device_cus() {
    static const int cus = [] {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
            n = 256;
        return n;
    }();
    return cus;
}


}  // namespace host
}  // namespace irf
