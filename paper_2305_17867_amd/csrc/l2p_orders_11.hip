// L2P kernels for orders 11.
#include "l2p_impl.hpp"

namespace fmm {

FMM_INSTANTIATE_L2P(11)

}  // namespace fmm
