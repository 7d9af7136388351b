// P2M kernels for orders 8, 9.
#include "p2m_impl.hpp"

namespace fmm {

FMM_INSTANTIATE_P2M(8)
FMM_INSTANTIATE_P2M(9)

}  // namespace fmm
