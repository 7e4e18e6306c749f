// Small device helpers shared by the projector kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace gkb {

// two consecutive elements, 4-byte (float) or 8-byte (double) aligned
template <typename T>
struct Pair;
template <>
struct Pair<float> {
  typedef float v2 __attribute__((ext_vector_type(2), aligned(4)));
};
template <>
struct Pair<double> {
  typedef double v2 __attribute__((ext_vector_type(2), aligned(8)));
};
template <typename T>
__device__ inline typename Pair<T>::v2 load_pair(const T *p) {
  return *reinterpret_cast<const typename Pair<T>::v2 *>(p);
}

// reciprocal: hardware approximation (1 ulp) in float, exact division in double
__device__ inline float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double fast_rcp(double x) { return 1.0 / x; }

// reciprocal square root: hardware approximation (1 ulp) in float, correctly
// rounded square root and division in double
__device__ inline float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double fast_rsq(double x) { return 1.0 / sqrt(x); }

// max(w, 0) for a weight w <= 1 (every hat weight 1 - |x| s with s >= 0):
// written as a clamp to [0, 1], which the compiler folds into the clamp bit
// of the instruction that forms w
template <typename T>
__device__ inline T hat_clamp(T w) {
  return fmin(fmax(w, T(0)), T(1));
}

// min(max(x, lo), hi) for lo <= hi and finite x: one median-of-three in float
__device__ inline float clampv(float x, float lo, float hi) { return __builtin_amdgcn_fmed3f(x, lo, hi); }
__device__ inline double clampv(double x, double lo, double hi) { return fmin(fmax(x, lo), hi); }

// value of v in lane l of the wavefront (l uniform)
__device__ inline float lane_value(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ inline double lane_value(double v, int l) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

}  // namespace gkb
