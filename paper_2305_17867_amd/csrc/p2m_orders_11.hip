// P2M kernels for orders 11.
#include "p2m_impl.hpp"

namespace fmm {

FMM_INSTANTIATE_P2M(11)

}  // namespace fmm
