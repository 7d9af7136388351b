// L2P kernels for orders 12.
#include "l2p_impl.hpp"

namespace fmm {

FMM_INSTANTIATE_L2P(12)

}  // namespace fmm
