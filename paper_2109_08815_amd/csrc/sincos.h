// Single-precision sine, cosine and reciprocal for the dynamics kernels.
//
// x = k pi/2 + r with k = rint(2x/pi) and r reduced by a three-part
// splitting of pi/2 (Cody and Waite), each part subtracted with one fused
// multiply-add; on |r| <= pi/4 the Taylor series of sin (to r^9) and cos
// (to r^10) truncate below 2e-9 relative, so the result is within one unit
// in the last place of the float result.  The quadrant k mod 4 picks and
// signs the two series.  The reduction stays exact while k is an exact
// float integer (|x| below about 2^24); Inf and NaN give NaN.  No branch,
// no table.  No HIP headers: the host tests compile it.
#pragma once

#include <cmath>

#ifndef __HIPCC__
#ifndef __host__
#define __host__
#endif
#ifndef __device__
#define __device__
#endif
#endif

namespace pds {

__host__ __device__ inline void sincos_fast(float x, float* sn, float* cs) {
  constexpr float kTwoOverPi = 0.636619746685028076171875f;
  // pi/2 = kPio2A + kPio2B + kPio2C + O(1e-23)
  constexpr float kPio2A = 1.57079637050628662109375f;
  constexpr float kPio2B = -4.37113882867379300296306610107421875e-08f;
  constexpr float kPio2C = -1.715124510005881870e-15f;
  const float k = std::rint(x * kTwoOverPi);
  float r = std::fma(-k, kPio2A, x);
  r = std::fma(-k, kPio2B, r);
  r = std::fma(-k, kPio2C, r);
  const float r2 = r * r;
  // 1/3!, 1/5!, 1/7!, 1/9! and 1/2!, 1/4!, ..., 1/10!
  const float sp =
      r + r * r2 * (-1.0f / 6.0f + r2 * (1.0f / 120.0f + r2 * (-1.0f / 5040.0f + r2 * (1.0f / 362880.0f))));
  const float cp =
      1.0f + r2 * (-0.5f + r2 * (1.0f / 24.0f + r2 * (-1.0f / 720.0f + r2 * (1.0f / 40320.0f + r2 * (-1.0f / 3628800.0f)))));
  const int q = static_cast<int>(k) & 3;
  float s = (q & 1) ? cp : sp;
  float c = (q & 1) ? sp : cp;
  if (q & 2) s = -s;
  if ((q + 1) & 2) c = -c;
  *sn = s;
  *cs = c;
}

// 1 / x: the hardware reciprocal estimate refined by one Newton step
// r' = r + r (1 - x r) (two fused multiply-adds), within about half a unit
// in the last place for normal x; host builds divide.
__host__ __device__ inline float recip(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const float r = __builtin_amdgcn_rcpf(x);
  return std::fma(std::fma(-x, r, 1.0f), r, r);
#else
  return 1.0f / x;
#endif
}

// FP64 overload for host-side checks of the step functions.  It lives beside
// the float one: declared in a nested namespace it would hide the float
// version from unqualified calls there, and float arguments would be divided
// in full precision instead.
__host__ __device__ inline double recip(double x) { return 1.0 / x; }

}  // namespace pds
