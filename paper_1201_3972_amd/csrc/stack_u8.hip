// stack_u8.hip -- the 8-bit instantiations of the single-size kernels up to 15x15.
#include "stack_launch.hpp"

namespace irf {
bool launch_stack_u8(int window, int mode, Tuning t, const StackArgs &a, hipStream_t s) {
    if (window > kNetworkMaxWindow) return launch_stack_large_u8(window, mode, t, a, s);
    return stack_impl::launch_stack<uint8_t, stack_impl::kSmallWindows>(window, mode, t, a, s);
}
}  // namespace irf
