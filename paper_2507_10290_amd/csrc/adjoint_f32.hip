// FP32 instantiations of the adjoint kernel (tiles of up to 256 lanes: one wave per SIMD, room
// for forward and adjoint state together).
#include "adjoint_impl.h"

namespace top {

template <>
hipError_t launch_adjoint<float>(const Variant& v, const AdjArgs<float>& a, int n_tiles, hipStream_t st) {
  return dispatch_adjoint<float, 256, 256>(v, a, n_tiles, st);
}

}  // namespace top
