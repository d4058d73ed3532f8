// pp_device.h -- small device helpers shared by the kernel sources.
#pragma once

#include <hip/hip_runtime.h>

namespace ppk {

// Knuth's two-sum: s + c absorbs t; the rounding error of s + t goes into c.
__device__ __forceinline__ void two_sum(float& s, float& c, float t) {
  const float u = s + t;
  const float bp = u - s;
  const float err = (s - (u - bp)) + (t - bp);
  s = u;
  c += err;
}

__device__ __forceinline__ void two_sum(double& s, double& c, double t) {
  const double u = s + t;
  const double bp = u - s;
  const double err = (s - (u - bp)) + (t - bp);
  s = u;
  c += err;
}

// Adds the compensated pair (t, tc) into (s, c).
__device__ __forceinline__ void two_sum_pair(float& s, float& c, float t, float tc) {
  two_sum(s, c, t);
  c += tc;
}

}  // namespace ppk
