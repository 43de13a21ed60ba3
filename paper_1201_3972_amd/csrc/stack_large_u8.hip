// stack_large_u8.hip -- the 8-bit instantiations of the single-size kernels
// for windows 17x17 to 31x31 (group bisection and the radix select).
#include "stack_launch.hpp"

namespace irf {
bool launch_stack_large_u8(int window, int mode, Tuning t, const StackArgs &a, hipStream_t s) {
    if (window > kLargeMaxWindow) return launch_stack_huge_u8(window, mode, t, a, s);
    return stack_impl::launch_stack<uint8_t, stack_impl::kLargeWindows>(window, mode, t, a, s);
}
}  // namespace irf
