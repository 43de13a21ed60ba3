// batch_kernels.hpp -- host launch of the batch class kernels.  Each class's
// kernels (workgroups of 128 and 256 threads) are instantiated in a
// translation unit of their own (batch_c0.hip, batch_c1.hip, batch_cl_a.hip,
// batch_cl_b.hip) so that they compile in parallel; batch.hip reaches them
// through BatchClass<CLASS>.
#pragma once

#include <hip/hip_runtime.h>

#include "batch_device.hpp"

namespace irf {

template <int CLASS>
struct BatchClass {
    // Workgroups of the class kernel with `threads` threads resident per CU.
    static int blocks_per_cu(int threads);
    // Launch it with `grid` workgroups over the tables of one plan set.
    static void launch(int threads, int grid, const FrameDesc *descs, const uint32_t *tile_frame,
                       BatchQueue *queue, hipStream_t stream);
};

#ifdef IRF_BATCH_CLASS_DEFINITIONS
template <int CLASS>
int BatchClass<CLASS>::blocks_per_cu(int threads) {
    int n = 0;
    const hipError_t e = threads == 256
                             ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fnr_batch_kernel<CLASS, 256>, 256, 0)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fnr_batch_kernel<CLASS, 128>, 128, 0);
    return (e != hipSuccess || n < 1) ? 1 : n;
}

template <int CLASS>
void BatchClass<CLASS>::launch(int threads, int grid, const FrameDesc *descs, const uint32_t *tile_frame,
                               BatchQueue *queue, hipStream_t stream) {
    if (threads == 256)
        hipLaunchKernelGGL((fnr_batch_kernel<CLASS, 256>), dim3(grid), dim3(256), 0, stream, descs, tile_frame,
                           queue, 0x00010001u);
    else
        hipLaunchKernelGGL((fnr_batch_kernel<CLASS, 128>), dim3(grid), dim3(128), 0, stream, descs, tile_frame,
                           queue, 0x00010001u);
}
#else
extern template struct BatchClass<0>;
extern template struct BatchClass<1>;
extern template struct BatchClass<2>;
extern template struct BatchClass<3>;
extern template struct BatchClass<4>;
extern template struct BatchClass<5>;
extern template struct BatchClass<6>;
extern template struct BatchClass<7>;
extern template struct BatchClass<8>;
extern template struct BatchClass<9>;
#endif

}  // namespace irf
