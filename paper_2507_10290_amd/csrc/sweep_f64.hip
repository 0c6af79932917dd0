// FP64 instantiations of the resident sweep kernel (tiles of up to 256 lanes: one wave per SIMD,
// so the doubled register state fits without spilling to memory).
#include "sweep_impl.h"

namespace top {

template <>
hipError_t launch_sweep<double>(const Variant& v, const SweepArgs<double>& a, int n_tiles, hipStream_t st) {
  return dispatch_sweep<double, 256, 256>(v, a, n_tiles, st);
}

template <>
int sweep_resident<double>(const Variant& v, int W) {
  return resident_sweep<double, 256, 256>(v, W);
}

}  // namespace top
