// Block-level and grid-level deterministic reductions (device helpers).
#pragma once
#include <hip/hip_runtime.h>

namespace hdg {

__device__ inline double wave_sum64(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// sum over a block of NT threads (NT a multiple of 64); result in thread 0
template <int NT>
__device__ inline double block_sum_t(double v, double* sh) {
  v = wave_sum64(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NT / 64; ++w) s += sh[w];
  return s;
}

}  // namespace hdg
