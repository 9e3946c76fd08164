// Deterministic FP64 block reductions over 64-wide waves.
#pragma once
#include <hip/hip_runtime.h>

namespace wh {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  return v;
}

// Sum over the NWAVES*64 threads of the block; the result is valid in thread 0.
// Fixed order (shuffle tree per wave, then adjacent pairs of waves, level by level), so results are
// reproducible run to run.  Every thread of the block must call it.
template <int NWAVES>
__device__ __forceinline__ double block_sum(double v, int tid) {
  static_assert(NWAVES == 2 || NWAVES == 4 || NWAVES == 8 || NWAVES == 16, "waves per block");
  __shared__ double sm[NWAVES];
  v = wave_sum(v);
  if ((tid & 63) == 0) sm[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (tid == 0) {
    double t[NWAVES];
#pragma unroll
    for (int i = 0; i < NWAVES; ++i) t[i] = sm[i];
#pragma unroll
    for (int w = NWAVES / 2; w >= 1; w >>= 1)
#pragma unroll
      for (int i = 0; i < w; ++i) t[i] = t[2 * i] + t[2 * i + 1];
    s = t[0];
  }
  __syncthreads();
  return s;
}

__device__ __forceinline__ double block_sum256(double v, int tid) { return block_sum<4>(v, tid); }

__device__ __forceinline__ double block_max256(double v, int tid) {
  __shared__ double sm[4];
  v = wave_max(v);
  if ((tid & 63) == 0) sm[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (tid == 0) s = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
  __syncthreads();
  return s;
}

}  // namespace wh
