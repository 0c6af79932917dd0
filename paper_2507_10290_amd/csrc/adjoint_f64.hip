// FP64 instantiations of the adjoint kernel: tiles of up to 64 segments, run as 192 lanes (one per
// segment and axis).
#include "adjoint_impl.h"

namespace top {

template <>
hipError_t launch_adjoint<double>(const Variant& v, const AdjArgs<double>& a, int n_tiles, hipStream_t st) {
  return dispatch_adjoint<double, 64>(v, a, n_tiles, st);
}

}  // namespace top
