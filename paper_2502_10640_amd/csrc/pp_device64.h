// pp_device64.h -- FP64 device helpers shared by the FP64 pair-sum kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace ppk {

// r2^(-3/2), the factor of the Coulomb term of Eq. (A) with softening folded
// into r2, and optionally r2^(-1/2) (the potential), in FP64.
//
// v_rsq_f64 on gfx950 gives y ~ 1/sqrt(r2) to about 2^-24 relative (measured:
// 4.7e8 units of 2^-53 at worst), so it needs refining.  With
// e = 1 - r2 y^2 (|e| < 2^-23), the binomial series of (1 - e)^(-1/2) and
// (1 - e)^(-3/2) give
//   r2^(-1/2) = y   (1 + e/2  + 3 e^2/8  + O(e^3)),
//   r2^(-3/2) = y^3 (1 + 3e/2 + 15 e^2/8 + O(e^3)),
// whose dropped terms are below 2^-66.  Rounding leaves at most ~2.5 units of
// 2^-53 in r2^(-3/2) (y^2 and y^3 rounded, the error of y^2 entering e with
// weight -3/2), against ~6 for two Newton steps on y followed by y^3.
//
// The r^-3 correction is e (c.c15 + c.c1875 e), with 1.5 held in a VGPR pair
// and 1.875 in an SGPR pair by the caller (SeriesConst): gfx950's FP64 VOP3
// instructions take no literal and read at most one scalar operand, so with
// both as compile-time constants the compiler either rebuilt 1.5 with two
// v_mov per pair or folded 1.875 into the two-operand fmac, which overwrites
// its addend and so costs a v_mov_b64 of 1.5 per pair.  Held in registers the
// step is one v_fma_f64: 6 FP64 operations after the estimate (10 for Newton +
// cube); the potential adds 3.
struct SeriesConst {
  double c15, c1875;
};

__device__ __forceinline__ SeriesConst series_const() {
  // opaque to the optimiser (empty asm statements), so the values stay in
  // registers instead of being rebuilt at each use
  double a = 1.5, b = 1.875;
  asm volatile("" : "+v"(a));
  asm volatile("" : "+s"(b));
  return {a, b};
}

template <bool WANT_INV>
__device__ __forceinline__ double inv_r3_64(double r2, const SeriesConst& c, double& inv) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double y2 = y * y;
  const double e = fma(-r2, y2, 1.0);
  const double y3 = y2 * y;
  if (WANT_INV) inv = fma(y, e * fma(e, 0.375, 0.5), y);
  return fma(y3, e * fma(e, c.c1875, c.c15), y3);
}

}  // namespace ppk
