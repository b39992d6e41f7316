// FP32 kernels (state, reconstruction and flux in FP32; the CFL reduction,
// totals and details stay FP64).
#include "eu_kset_impl.hpp"

namespace eu {
const KSet kset_f32 = impl::make<float>();
}
