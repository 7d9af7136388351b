// P2M kernels for orders 14.
#include "p2m_impl.hpp"

namespace fmm {

FMM_INSTANTIATE_P2M(14)

}  // namespace fmm
