// P2M kernels for orders 13.
#include "p2m_impl.hpp"

namespace fmm {

FMM_INSTANTIATE_P2M(13)

}  // namespace fmm
