// batch_cl_a.hip -- the batch class kernels of windows 17, 19, 21 and 23 (see batch_kernels.hpp).
#define IRF_BATCH_CLASS_DEFINITIONS
#include "batch_kernels.hpp"

namespace irf {
template struct BatchClass<2>;
template struct BatchClass<3>;
template struct BatchClass<4>;
template struct BatchClass<5>;
}  // namespace irf
