// FP32 instantiations of the resident sweep kernel: quintic tiles of up to 512 lanes (two waves
// per SIMD), septic tiles of up to 256 lanes (the box + velocity instance is compiled for two waves
// per SIMD as well, sweep_min_waves; the other septic instances for one).
#include "sweep_impl.h"

namespace top {

template <>
hipError_t launch_sweep<float>(const Variant& v, const SweepArgs<float>& a, int n_tiles, hipStream_t st) {
  return dispatch_sweep<float, 512, 256>(v, a, n_tiles, st);
}

template <>
int sweep_resident<float>(const Variant& v, int W) {
  return resident_sweep<float, 512, 256>(v, W);
}

}  // namespace top
