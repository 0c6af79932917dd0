// Instantiations of the sweep with one lane per segment and axis (float32 and float64).
#include "sweep_axis_impl.h"

namespace top {

template <>
hipError_t launch_sweep_axis<float>(const Variant& v, const SweepArgs<float>& a, int n_tiles, hipStream_t st) {
  return dispatch_sweep_axis<float, kAxisMaxTile>(v, a, n_tiles, st);
}

template <>
hipError_t launch_sweep_axis<double>(const Variant& v, const SweepArgs<double>& a, int n_tiles, hipStream_t st) {
  return dispatch_sweep_axis<double, 128>(v, a, n_tiles, st);
}

}  // namespace top
