// L2P kernels for orders 10.
#include "l2p_impl.hpp"

namespace fmm {

FMM_INSTANTIATE_L2P(10)

}  // namespace fmm
