// FP32 instantiations of the NumericSolve sweep kernel (64-lane tiles).
#include "numeric_impl.h"

namespace top {

template <>
hipError_t launch_numeric_sweep<float>(const Variant& v, const SweepArgs<float>& a, int n_tiles, hipStream_t st) {
  return dispatch_numeric_sweep<float>(v, a, n_tiles, st);
}

}  // namespace top
