// Order dispatch of the M2M and L2L launches (kernels in translate_impl.hpp).
#include "../../include/fmm.h"
#include "common.hpp"
#include "kernels.hpp"

namespace fmm {

int launch_trans_order_0(const TransArgs& a, int dtype, bool l2l, hipStream_t s);
int launch_trans_order_1(const TransArgs& a, int dtype, bool l2l, hipStream_t s);
int launch_trans_order_2(const TransArgs& a, int dtype, bool l2l, hipStream_t s);
int launch_trans_order_3(const TransArgs& a, int dtype, bool l2l, hipStream_t s);
int launch_trans_order_4(const TransArgs& a, int dtype, bool l2l, hipStream_t s);
int launch_trans_order_5(const TransArgs& a, int dtype, bool l2l, hipStream_t s);
int launch_trans_order_6(const TransArgs& a, int dtype, bool l2l, hipStream_t s);
int launch_trans_order_7(const TransArgs& a, int dtype, bool l2l, hipStream_t s);
int launch_trans_order_8(const TransArgs& a, int dtype, bool l2l, hipStream_t s);
int launch_trans_order_9(const TransArgs& a, int dtype, bool l2l, hipStream_t s);
int launch_trans_order_10(const TransArgs& a, int dtype, bool l2l, hipStream_t s);
int launch_trans_order_11(const TransArgs& a, int dtype, bool l2l, hipStream_t s);
int launch_trans_order_12(const TransArgs& a, int dtype, bool l2l, hipStream_t s);
int launch_trans_order_13(const TransArgs& a, int dtype, bool l2l, hipStream_t s);
int launch_trans_order_14(const TransArgs& a, int dtype, bool l2l, hipStream_t s);
int launch_trans_order_15(const TransArgs& a, int dtype, bool l2l, hipStream_t s);
int launch_trans_order_16(const TransArgs& a, int dtype, bool l2l, hipStream_t s);

namespace {

int launch_trans(const TransArgs& a, int p, int dtype, bool l2l, hipStream_t s) {
  if (a.n_parent == 0) return FMM_OK;
  switch (p) {
    case 0: return launch_trans_order_0(a, dtype, l2l, s);
    case 1: return launch_trans_order_1(a, dtype, l2l, s);
    case 2: return launch_trans_order_2(a, dtype, l2l, s);
    case 3: return launch_trans_order_3(a, dtype, l2l, s);
    case 4: return launch_trans_order_4(a, dtype, l2l, s);
    case 5: return launch_trans_order_5(a, dtype, l2l, s);
    case 6: return launch_trans_order_6(a, dtype, l2l, s);
    case 7: return launch_trans_order_7(a, dtype, l2l, s);
    case 8: return launch_trans_order_8(a, dtype, l2l, s);
    case 9: return launch_trans_order_9(a, dtype, l2l, s);
    case 10: return launch_trans_order_10(a, dtype, l2l, s);
    case 11: return launch_trans_order_11(a, dtype, l2l, s);
    case 12: return launch_trans_order_12(a, dtype, l2l, s);
    case 13: return launch_trans_order_13(a, dtype, l2l, s);
    case 14: return launch_trans_order_14(a, dtype, l2l, s);
    case 15: return launch_trans_order_15(a, dtype, l2l, s);
    case 16: return launch_trans_order_16(a, dtype, l2l, s);
    default: return fail(FMM_EUNSUPPORTED, "order out of range");
  }
}

}  // namespace

int launch_m2m(const TransArgs& a, int p, int dtype, hipStream_t s) { return launch_trans(a, p, dtype, false, s); }
int launch_l2l(const TransArgs& a, int p, int dtype, hipStream_t s) { return launch_trans(a, p, dtype, true, s); }

}  // namespace fmm
