// FP64 instantiations of the polytope-corridor sweep kernel (tiles of up to 256 lanes).
#include "poly_impl.h"

namespace top {

template <>
hipError_t launch_poly_sweep<double>(const Variant& v, const SweepArgs<double>& a, int n_tiles, hipStream_t st) {
  return dispatch_poly_sweep<double>(v, a, n_tiles, st);
}

template <>
int poly_resident<double>(const Variant& v, int W) {
  return resident_poly<double>(v, W);
}

}  // namespace top
