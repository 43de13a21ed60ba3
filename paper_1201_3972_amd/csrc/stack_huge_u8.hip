// stack_huge_u8.hip -- the 8-bit instantiations of the single-size kernels
// for windows 33x33 to 63x63 (group bisection, 128-thread workgroups).
#include "stack_launch.hpp"

namespace irf {
bool launch_stack_huge_u8(int window, int mode, Tuning t, const StackArgs &a, hipStream_t s) {
    return stack_impl::launch_stack<uint8_t, stack_impl::kHugeWindows>(window, mode, t, a, s);
}
}  // namespace irf
