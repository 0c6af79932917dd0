// FP64 instantiations of the adjoint kernel (tiles of up to 256 lanes).
#include "adjoint_impl.h"

namespace top {

template <>
hipError_t launch_adjoint<double>(const Variant& v, const AdjArgs<double>& a, int n_tiles, hipStream_t st) {
  return dispatch_adjoint<double, 256, 256>(v, a, n_tiles, st);
}

}  // namespace top
