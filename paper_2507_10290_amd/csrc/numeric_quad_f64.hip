// FP64 instantiations of the NumericSolve sweep with four lanes per segment.
#include "numeric_quad_impl.h"

namespace top {

template <>
hipError_t launch_numeric_quad<double>(const Variant& v, const SweepArgs<double>& a, int n_tiles, hipStream_t st) {
  return dispatch_numeric_quad<double>(v, a, n_tiles, st);
}

}  // namespace top
