// batch_cl_b.hip -- the batch class kernels of windows 25, 27, 29 and 31 (see batch_kernels.hpp).
#define IRF_BATCH_CLASS_DEFINITIONS
#include "batch_kernels.hpp"

namespace irf {
template struct BatchClass<6>;
template struct BatchClass<7>;
template struct BatchClass<8>;
template struct BatchClass<9>;
}  // namespace irf
