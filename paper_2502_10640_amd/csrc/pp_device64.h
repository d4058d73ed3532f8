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
// The corrections are formed as c1 e + c2 e^2 so that no instruction needs
// two constants: gfx950's FP64 VOP3 instructions take no literal, and a
// Horner step fma(e, c2, c1) would make the compiler rebuild c1 in VGPRs with
// two v_mov per pair; here each constant is the one scalar operand of its
// instruction.  7 FP64 operations after the estimate (10 for Newton + cube).
template <bool WANT_INV>
__device__ __forceinline__ double inv_r3_64(double r2, double& inv) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double y2 = y * y;
  const double e = fma(-r2, y2, 1.0);
  const double y3 = y2 * y;
  const double ee = e * e;
  if (WANT_INV) inv = fma(y, fma(ee, 0.375, 0.5 * e), y);
  return fma(y3, fma(ee, 1.875, 1.5 * e), y3);
}

}  // namespace ppk
