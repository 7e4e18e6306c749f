// Deterministic reductions for wave64 / 256-thread workgroups.
#pragma once

#include <hip/hip_runtime.h>

namespace gkb {

// Butterfly sum across the 64 lanes of a wavefront (fixed order).
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Maximum of an int over the 64 lanes of a wavefront, as a wave-uniform
// (scalar) value.  Every lane of the wavefront must take part.
__device__ inline int wave_max(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return __builtin_amdgcn_readfirstlane(v);
}

// Minimum of an int over the 64 lanes of a wavefront, wave-uniform.  Every
// lane of the wavefront must take part.
__device__ inline int wave_min(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return __builtin_amdgcn_readfirstlane(v);
}

// Sum over a workgroup of NT threads; the result is valid in thread 0.
// `lds` holds NT/64 doubles.  Fixed order: lane butterfly, then waves 0..NT/64-1.
template <int NT>
__device__ inline double block_sum(double v, double *lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) r += lds[i];
  }
  return r;
}

// Result broadcast to every thread of the block.
template <int NT>
__device__ inline double block_sum_all(double v, double *lds) {
  double r = block_sum<NT>(v, lds);
  __syncthreads();
  if (threadIdx.x == 0) lds[0] = r;
  __syncthreads();
  r = lds[0];
  __syncthreads();
  return r;
}

// Sum of nb per-workgroup partial results p[i * stride] (i < nb), in a fixed
// order; valid in thread 0.  Used by the finalising kernels that run after the
// kernel that wrote the partials (the kernel boundary orders the two, so no
// workgroup of the producing kernel has to wait for or signal another).
template <int NT>
__device__ inline double partial_total(const double *__restrict__ p, unsigned nb, unsigned stride, double *lds) {
  double a = 0.0;
  for (unsigned i = threadIdx.x; i < nb; i += NT) a += p[(size_t)i * stride];
  return block_sum<NT>(a, lds);
}

}  // namespace gkb
