// INT8-slice form (precision form): digit split and integer matrix-core GEMM.
#include "internal.h"

namespace mp {

template <int C>
hipError_t launch_split_int8(const SplitOperand<double> &, const SplitOperand<double> &, int, hipStream_t) {
  return hipErrorNotSupported;
}
template <int C>
hipError_t launch_gemm_int8(const void *, const void *, const int *, const int *, int64_t, int64_t, int64_t, int, int,
                            int, int, double *, int, int64_t, int, int64_t *, int, hipStream_t) {
  return hipErrorNotSupported;
}

#define MP_INST(C)                                                                                                \
  template hipError_t launch_split_int8<C>(const SplitOperand<double> &, const SplitOperand<double> &, int,       \
                                           hipStream_t);                                                          \
  template hipError_t launch_gemm_int8<C>(const void *, const void *, const int *, const int *, int64_t, int64_t, \
                                          int64_t, int, int, int, int, double *, int, int64_t, int, int64_t *, int, \
                                          hipStream_t);
MP_INST(2)
MP_INST(3)
MP_INST(4)
#undef MP_INST

}  // namespace mp
