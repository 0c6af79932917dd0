// FP32 instantiations of the NumericSolve sweep with four lanes per segment.
#include "numeric_quad_impl.h"

namespace top {

template <>
hipError_t launch_numeric_quad<float>(const Variant& v, const SweepArgs<float>& a, int n_tiles, hipStream_t st) {
  return dispatch_numeric_quad<float>(v, a, n_tiles, st);
}

}  // namespace top
