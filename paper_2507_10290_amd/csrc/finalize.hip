// Outputs of a run, in float64: monomial coefficients, and per-segment
// partial sums of the objective and of the squared stopping residuals
// (Sec. III-D.3), reduced per trajectory in a fixed order.
#include "common.h"

namespace top {

template <typename R, int P, int S>
__device__ void finalize_segment(const FinalArgs<R>& a, int64_t i) {
  constexpr int N = 2 * P;
  const int64_t ld = a.ld;
  const double T = a.T[i];
  const double iT = 1.0 / T;
  const uint8_t fl = a.flags[i];
  const bool first = fl & kFirst, last = fl & kLast;
  double iTp[N], Tp[N];
  iTp[0] = 1.0;
  Tp[0] = 1.0;
  for (int o = 1; o < N; ++o) { iTp[o] = iTp[o - 1] * iT; Tp[o] = Tp[o - 1] * T; }
  double c[3][N];
  for (int ax = 0; ax < 3; ++ax)
#pragma unroll
    for (int j = 0; j < N; ++j) c[ax][j] = (double)a.c[(int64_t)(ax * N + j) * ld + i];

  // objective: sum_a c^T Q(T) c = T^(1-2p) sum_a c~^T Q(1) c~
  double J = 0.0;
  for (int ax = 0; ax < 3; ++ax) {
    double q = 0.0;
#pragma unroll
    for (int j = P; j < N; ++j)
#pragma unroll
      for (int k = P; k < N; ++k) q += cgram(P, j, k) * c[ax][j] * c[ax][k];
    J += q;
  }
  J *= iTp[2 * P - 1];
  if (a.coeffs != nullptr) {
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int j = 0; j < N; ++j) a.coeffs[(i * 3 + ax) * N + j] = c[ax][j] * iTp[j];
  }
  double rp2 = 0.0, rd2 = 0.0;
  if (a.with_res) {
    // primal: gaps of orders 0..s-1 between this segment's end and the next one's start
    if (!last) {
      const double iTn = 1.0 / a.T[i + 1];
      double iTnp = 1.0;
      for (int o = 0; o < S; ++o) {
        for (int ax = 0; ax < 3; ++ax) {
          double xr = 0.0;
#pragma unroll
          for (int j = 0; j < N; ++j) xr += cfall(o, j) * c[ax][j];
          xr *= iTp[o];
          const double xl = cfact(o) * (double)a.c[(int64_t)(ax * N + o) * ld + i + 1] * iTnp;
          rp2 += (xr - xl) * (xr - xl);
        }
        iTnp *= iTn;
      }
    }
    // dual: rho M(T)^T (z~^{k+1} - z~^k), per axis, monomial basis
    const double rho = a.rho[i];
    for (int ax = 0; ax < 3; ++ax) {
      double dL[S], dR[S];
      for (int o = 0; o < S; ++o) {
        const int64_t f = (int64_t)(ax * S + o) * ld;
        dL[o] = first ? 0.0 : (double)a.state[f + i - 1] - (double)a.zold[f + i - 1];
        dR[o] = last ? 0.0 : (double)a.state[f + i] - (double)a.zold[f + i];
      }
#pragma unroll
      for (int j = 0; j < N; ++j) {
        double v = (j < S) ? cfact(j) * dL[j] : 0.0;
        for (int o = 0; o < S && o <= j; ++o) v += cfall(o, j) * Tp[j - o] * dR[o];
        v *= rho;
        rd2 += v * v;
      }
    }
  }
  if (a.part != nullptr) {
    a.part[i] = J;
    a.part[a.S + i] = rp2;
    a.part[2 * a.S + i] = rd2;
    if (!isfinite(J) || !isfinite(rp2) || !isfinite(rd2)) atomicOr(a.nonfinite, 1);
  }
}

// With residual checks the workgroups walk the list of running trajectories (x, grid-stride; y =
// 256-segment chunk of a trajectory): stopped ones keep their final partials.  Otherwise one lane
// per segment.
template <typename R, int P, int S>
__global__ void __launch_bounds__(256) finalize_kernel(FinalArgs<R> a) {
  if (a.done != nullptr) {
    const int n = *a.live_count;
    for (int q = blockIdx.x; q < n; q += gridDim.x) {
      const int b = a.live[q];
      const int64_t i = a.off[b] + (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
      if (i < a.off[b + 1]) finalize_segment<R, P, S>(a, i);
    }
    return;
  }
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.S) finalize_segment<R, P, S>(a, i);
}

// A workgroup converts 128 consecutive segments into LDS, then writes their 128 * 3n contiguous
// output values with consecutive lanes (one segment's 3n values are 144 or 192 bytes apart from the
// next one's, so per-lane stores straight from registers would not coalesce).
template <typename R, int P>
__global__ void __launch_bounds__(128) coeffs_kernel(const R* c, const double* T, int64_t S, int64_t ld,
                                                     double* out) {
  constexpr int N = 2 * P, K = 3 * N;
  __shared__ double buf[128 * K];
  const int t = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * 128;
  const int64_t i = s0 + t;
  if (i < S) {
    const double iT = 1.0 / T[i];
    double iTp = 1.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) buf[t * K + ax * N + j] = (double)c[(int64_t)(ax * N + j) * ld + i] * iTp;
      iTp *= iT;
    }
  }
  __syncthreads();
  const int64_t nseg = S - s0 < 128 ? S - s0 : 128;
  const int total = (int)nseg * K;
  for (int q = t; q < total; q += 128) out[s0 * K + q] = buf[q];
}

template <typename R>
hipError_t launch_coeffs(int p, const R* c, const double* T, int64_t S, int64_t ld, double* out, hipStream_t st) {
  const dim3 grid((unsigned)((S + 127) / 128)), block(128);
  if (p == 3) hipLaunchKernelGGL((coeffs_kernel<R, 3>), grid, block, 0, st, c, T, S, ld, out);
  else if (p == 4) hipLaunchKernelGGL((coeffs_kernel<R, 4>), grid, block, 0, st, c, T, S, ld, out);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}
template hipError_t launch_coeffs<float>(int, const float*, const double*, int64_t, int64_t, double*, hipStream_t);
template hipError_t launch_coeffs<double>(int, const double*, const double*, int64_t, int64_t, double*, hipStream_t);

template <typename R>
hipError_t launch_finalize(const Variant& v, const FinalArgs<R>& a, hipStream_t st) {
  const int bs = 256;
  const dim3 grid = a.done != nullptr ? dim3((unsigned)std::min(a.B, 1024), (unsigned)((a.max_len + bs - 1) / bs))
                                      : dim3((unsigned)((a.S + bs - 1) / bs));
  const dim3 block(bs);
  if (v.p == 3 && v.s == 3) hipLaunchKernelGGL((finalize_kernel<R, 3, 3>), grid, block, 0, st, a);
  else if (v.p == 3 && v.s == 4) hipLaunchKernelGGL((finalize_kernel<R, 3, 4>), grid, block, 0, st, a);
  else if (v.p == 4 && v.s == 4) hipLaunchKernelGGL((finalize_kernel<R, 4, 4>), grid, block, 0, st, a);
  else if (v.p == 4 && v.s == 5) hipLaunchKernelGGL((finalize_kernel<R, 4, 5>), grid, block, 0, st, a);
  else if (v.p == 3 && v.s == 5) hipLaunchKernelGGL((finalize_kernel<R, 3, 5>), grid, block, 0, st, a);
  else if (v.p == 4 && v.s == 7) hipLaunchKernelGGL((finalize_kernel<R, 4, 7>), grid, block, 0, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template hipError_t launch_finalize<float>(const Variant&, const FinalArgs<float>&, hipStream_t);
template hipError_t launch_finalize<double>(const Variant&, const FinalArgs<double>&, hipStream_t);

// Stage 1: one 256-lane workgroup per chunk.  Lane l sums segments l, l+256, ... of the chunk in
// order, each wave folds its lanes with a fixed shuffle tree, and lane 0 adds the four wave sums in
// order.  The three quantities are summed together so their loads overlap.
__global__ void __launch_bounds__(256) reduce_chunks_kernel(ReduceArgs a) {
  __shared__ double wsum[3][4];
  const int c = blockIdx.x;
  if (c >= a.n_chunks) return;
  const int b = a.chunk_traj[c];
  if (a.done != nullptr && a.done[b] != 0) return;  // stopped: its sums are final
  const int64_t s0 = a.off[b] + (int64_t)(c - a.chunk_off[b]) * kReduceChunk;
  const int64_t s1 = s0 + kReduceChunk < a.off[b + 1] ? s0 + kReduceChunk : a.off[b + 1];
  const int t = threadIdx.x;
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
  for (int64_t i = s0 + t; i < s1; i += 256) {
    acc0 += a.part[i];
    acc1 += a.part[a.S + i];
    acc2 += a.part[2 * a.S + i];
  }
  for (int o = 32; o > 0; o >>= 1) {
    acc0 += __shfl_down(acc0, o);
    acc1 += __shfl_down(acc1, o);
    acc2 += __shfl_down(acc2, o);
  }
  if ((t & 63) == 0) {
    wsum[0][t >> 6] = acc0;
    wsum[1][t >> 6] = acc1;
    wsum[2][t >> 6] = acc2;
  }
  __syncthreads();
  if (t < 3) {
    const double v = ((wsum[t][0] + wsum[t][1]) + wsum[t][2]) + wsum[t][3];
    a.chunk_sum[(int64_t)t * a.n_chunks + c] = v;
  }
}

// Stage 2: one lane per trajectory adds its chunk sums in chunk order.
__global__ void reduce_traj_kernel(ReduceArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.B) return;
  if (a.done != nullptr && a.done[b] != 0) return;
  for (int q = 0; q < 3; ++q) {
    double acc = 0.0;
    for (int c = a.chunk_off[b]; c < a.chunk_off[b + 1]; ++c) acc += a.chunk_sum[(int64_t)q * a.n_chunks + c];
    a.out[(int64_t)q * a.B + b] = (q == 0) ? acc : sqrt(acc);
  }
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st) {
  if (a.n_chunks > 0) hipLaunchKernelGGL(reduce_chunks_kernel, dim3(a.n_chunks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(reduce_traj_kernel, dim3((a.B + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

__global__ void copy_kernel(const double* src, double* dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

hipError_t launch_copy_rows(const double* src, double* dst, int n, hipStream_t st) {
  hipLaunchKernelGGL(copy_kernel, dim3((n + 255) / 256), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

}  // namespace top
