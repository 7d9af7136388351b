// L2P kernels for orders 13.
#include "l2p_impl.hpp"

namespace fmm {

FMM_INSTANTIATE_L2P(13)

}  // namespace fmm
