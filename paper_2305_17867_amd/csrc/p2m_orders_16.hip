// P2M kernels for orders 16.
#include "p2m_impl.hpp"

namespace fmm {

FMM_INSTANTIATE_P2M(16)

}  // namespace fmm
