// slope.hpp -- the Van Leer limited slope of section 4.3.2 without a branch.
// vl_slope (kernels.hpp) skips the quotient when ab <= 0; here it is always
// formed and then selected, so that a wavefront whose lanes disagree on the
// sign does not split, and the compiler can interleave the slopes of a face.
// The same quotient: the hardware reciprocal of a + b refined by two Newton
// steps, then 2ab times it with one correction (within a few ulp of the
// IEEE quotient); 0 when ab <= 0; b when unlimited.
#pragma once
#include <hip/hip_runtime.h>

namespace hofks {

__device__ __forceinline__ double vl_slope_sel(double a, double b, int unlimited = 0) {
  const double ab = a * b;
  const double den = a + b;
  double r = __builtin_amdgcn_rcp(den);
  r = fma(fma(-den, r, 1.0), r, r);
  r = fma(fma(-den, r, 1.0), r, r);
  const double q = 2.0 * ab * r;
  const double v = fma(fma(-den, q, 2.0 * ab), r, q);
  return unlimited ? b : (ab > 0.0 ? v : 0.0);
}

}  // namespace hofks
