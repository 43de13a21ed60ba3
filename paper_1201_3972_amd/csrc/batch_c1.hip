// batch_c1.hip -- the batch class kernel of windows 11..15 (see batch_kernels.hpp).
#define IRF_BATCH_CLASS_DEFINITIONS
#include "batch_kernels.hpp"

namespace irf {
template struct BatchClass<1>;
}  // namespace irf
