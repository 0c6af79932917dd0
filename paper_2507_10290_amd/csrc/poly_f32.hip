// FP32 instantiations of the polytope-corridor sweep kernel (tiles of up to 256 lanes).
#include "poly_impl.h"

namespace top {

template <>
hipError_t launch_poly_sweep<float>(const Variant& v, const SweepArgs<float>& a, int n_tiles, hipStream_t st) {
  return dispatch_poly_sweep<float>(v, a, n_tiles, st);
}

template <>
int poly_resident<float>(const Variant& v, int W) {
  return resident_poly<float>(v, W);
}

}  // namespace top
