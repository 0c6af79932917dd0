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

template <>
int sweep_axis_resident<float>(const Variant& v, int W) {
  return resident_sweep_axis<float, kAxisMaxTile>(v, W);
}

template <>
int sweep_axis_resident<double>(const Variant& v, int W) {
  return resident_sweep_axis<double, 128>(v, W);
}

__global__ void zero_u64_kernel(unsigned long long* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace top
