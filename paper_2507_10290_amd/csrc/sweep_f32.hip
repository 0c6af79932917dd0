// FP32 instantiations of the resident sweep kernel: quintic tiles of up to 512 lanes (two waves
// per SIMD), septic tiles of up to 256 lanes (one wave per SIMD, room for its larger state).
#include "sweep_impl.h"

namespace top {

template <>
hipError_t launch_sweep<float>(const Variant& v, const SweepArgs<float>& a, int n_tiles, hipStream_t st) {
  return dispatch_sweep<float, 512, 256>(v, a, n_tiles, st);
}

}  // namespace top
