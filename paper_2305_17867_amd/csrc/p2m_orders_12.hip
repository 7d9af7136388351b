// P2M kernels for orders 12.
#include "p2m_impl.hpp"

namespace fmm {

FMM_INSTANTIATE_P2M(12)

}  // namespace fmm
