// Deterministic block reductions for 64-wide wavefronts (fixed tree, no atomics).
#pragma once

#include <hip/hip_runtime.h>

namespace igafd {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum over a block of NTH threads; the result is valid in thread 0.
template <int NTH = kBlock>
__device__ inline double block_sum(double v) {
  __shared__ double part[NTH / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) part[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NTH / 64; ++w) s += part[w];
  return s;
}

// Two simultaneous sums (e.g. (r,z) and (r,z_old)) over a block of NT
// threads; the results are valid in thread 0.
template <int NT = kBlock>
__device__ inline void block_sum2(double& a, double& b) {
  __shared__ double part[2][NT / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    part[0][wid] = a;
    part[1][wid] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = b = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
      a += part[0][w];
      b += part[1][w];
    }
  }
}

}  // namespace igafd
