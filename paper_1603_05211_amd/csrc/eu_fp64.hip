// FP64 kernels.  Built with -ffp-contract=off: every floating-point result
// follows the reference expression tree operation for operation.
#include "eu_kset_impl.hpp"

namespace eu {
const KSet kset_f64 = impl::make<double>();
}
