// fused.hip -- host launch of the fused two-pass kernels (fused_device.hpp).
#include <hip/hip_runtime.h>

#include "fused_device.hpp"
#include "host_common.hpp"
#include "stack_launch.hpp"

namespace irf {
namespace {

template <typename T, int K, int NT>
bool launch_k(const StackArgs &a, hipStream_t s) {
    static const int per_cu = [] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fnr_fused2_kernel<T, K, NT, kSelectNetwork>, NT,
                                                         0) != hipSuccess ||
            n < 1)
            n = 1;
        return n;
    }();
    const long long g = (long long)per_cu * host::device_cus();
    const int grid = (int)(g < a.total_tiles ? g : a.total_tiles);
    hipLaunchKernelGGL((fnr_fused2_kernel<T, K, NT, kSelectNetwork>), dim3(grid), dim3(NT), 0, s, a);
    return true;
}

template <typename T, int NT>
bool launch_nt(int window, const StackArgs &a, hipStream_t s) {
    switch (window) {
        case 3: return launch_k<T, 3, NT>(a, s);
        case 5: return launch_k<T, 5, NT>(a, s);
        case 7: return launch_k<T, 7, NT>(a, s);
        case 9: return launch_k<T, 9, NT>(a, s);
        default: return false;
    }
}

template <typename T>
bool launch_t(int window, int threads, const StackArgs &a, hipStream_t s) {
    if (threads == 256) return launch_nt<T, 256>(window, a, s);
    if (threads == 512) return launch_nt<T, 512>(window, a, s);
    return false;
}

}  // namespace

bool launch_fused2(int bytes, int window, int threads, const StackArgs &a, hipStream_t s) {
    if (!fused_available(window, threads)) return false;
    return bytes == 1 ? launch_t<uint8_t>(window, threads, a, s) : launch_t<uint16_t>(window, threads, a, s);
}

}  // namespace irf
