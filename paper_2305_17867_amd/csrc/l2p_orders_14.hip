// L2P kernels for orders 14.
#include "l2p_impl.hpp"

namespace fmm {

FMM_INSTANTIATE_L2P(14)

}  // namespace fmm
