// L2P kernels for orders 16.
#include "l2p_impl.hpp"

namespace fmm {

FMM_INSTANTIATE_L2P(16)

}  // namespace fmm
