// L2P kernels for orders 8, 9.
#include "l2p_impl.hpp"

namespace fmm {

FMM_INSTANTIATE_L2P(8)
FMM_INSTANTIATE_L2P(9)

}  // namespace fmm
