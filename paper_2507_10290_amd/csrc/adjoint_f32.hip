// FP32 instantiations of the adjoint kernel: tiles of up to 128 segments, run as 384 lanes (one per
// segment and axis) at two waves per SIMD.
#include "adjoint_impl.h"

namespace top {

template <>
hipError_t launch_adjoint<float>(const Variant& v, const AdjArgs<float>& a, int n_tiles, hipStream_t st) {
  return dispatch_adjoint<float, 128>(v, a, n_tiles, st);
}

}  // namespace top
