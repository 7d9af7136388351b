// P2M kernels for orders 10.
#include "p2m_impl.hpp"

namespace fmm {

FMM_INSTANTIATE_P2M(10)

}  // namespace fmm
