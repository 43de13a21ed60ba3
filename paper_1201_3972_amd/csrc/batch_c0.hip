// batch_c0.hip -- the batch class kernel of windows 3..9 (see batch_kernels.hpp).
#define IRF_BATCH_CLASS_DEFINITIONS
#include "batch_kernels.hpp"

namespace irf {
template struct BatchClass<0>;
}  // namespace irf
