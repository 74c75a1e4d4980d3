// Workgroup-wide exclusive scan built from wave shuffles.
#pragma once

#include <hip/hip_runtime.h>

namespace lif {

// Exclusive scan of one value per thread over a workgroup of NT threads
// (NT a multiple of 64, at most 4096): shuffle scans within each wave, one
// wave scans the wave totals, two barriers.  *total receives the
// workgroup's sum.  `sh` is LDS for NT / 64 values; every thread must call.
template <typename T, int NT>
__device__ T block_exclusive_scan(T v, T* sh, T* total) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  if (w == 0) {
    T t = lane < NW ? sh[lane] : T(0);
#pragma unroll
    for (int off = 1; off < NW; off <<= 1) {
      const T y = __shfl_up(t, off, 64);
      if (lane >= off) t += y;
    }
    if (lane < NW) sh[lane] = t;
  }
  __syncthreads();
  *total = sh[NW - 1];
  return (w ? sh[w - 1] : T(0)) + x - v;
}

}  // namespace lif
