// P2M kernels for orders 15.
#include "p2m_impl.hpp"

namespace fmm {

FMM_INSTANTIATE_P2M(15)

}  // namespace fmm
