// L2P kernels for orders 15.
#include "l2p_impl.hpp"

namespace fmm {

FMM_INSTANTIATE_L2P(15)

}  // namespace fmm
