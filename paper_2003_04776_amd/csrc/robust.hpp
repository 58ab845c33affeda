// Device-side robust scalar primitives for the blocked eigenvector kernels.
//
// Overflow protection follows Section 4 of Kjelgaard Mikkelsen & Myllykoski,
// "Parallel Robust Computation of Generalized Eigenvectors of Matrix Pencils":
//   ProtectDivision(b, t) returns xi in (0, 1] with  xi |b| <= |t| Omega,
//   ProtectUpdate(t, x, y) returns xi in (0, 1] with  xi (t x + y) <= Omega,
// and scale factors are integer powers of two (Section 5), so every xi is carried as
// its exponent q (xi = 2^-q) in an int.  Applying a factor is one v_ldexp_f64, which
// is exact unless the result leaves the normal range.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rgev {

// Omega = 2^1020: a factor 16 below the largest double, which leaves room for the
// rounding growth of long sums and for |Re| + |Im| magnitudes.
constexpr int kOmegaExp = 1020;
constexpr double kUnitRoundoff = 1.1102230246251565e-16;   // 2^-53
constexpr double kTiny = 2.2250738585072014e-308;          // smallest normal double
constexpr double kPuMargin = 8.8817841970012523e-16;        // 2^-50

__device__ __forceinline__ double pow2_scale(double x, int e) { return ldexp(x, e); }

// least q >= 0 with 2^-q * b <= t * Omega  (b = |numerator| <= Omega, t = |divisor| > 0)
__device__ __forceinline__ int protect_division(double b, double t) {
  if (!(b > 0.0) || t >= 1.0) return 0;
  const double tw = ldexp(t, kOmegaExp);          // exact: t < 1 cannot overflow
  if (b <= tw) return 0;
  int eb, et;
  const double mb = frexp(b, &eb);
  const double mt = frexp(tw, &et);
  return eb - et + (mb > mt ? 1 : 0);
}

// least q >= 0 with 2^-q * (t x + y) <= Omega (1 - 2^-50), for t, x, y in [0, Omega];
// t x is formed from mantissas and exponents because it may exceed the double range.
__device__ __forceinline__ int protect_update(double t, double x, double y) {
  int et = 0, ex = 0, ey = 0;
  const double mt = t > 0.0 ? frexp(t, &et) : 0.0;
  const double mx = x > 0.0 ? frexp(x, &ex) : 0.0;
  const double my = y > 0.0 ? frexp(y, &ey) : 0.0;
  const double mp = mt * mx;
  const int ep = et + ex;
  if (mp == 0.0 && my == 0.0) return 0;
  const int E = (mp == 0.0) ? ey : (my == 0.0 ? ep : (ep > ey ? ep : ey));
  const double s = (mp == 0.0 ? 0.0 : ldexp(mp, ep - E)) + (my == 0.0 ? 0.0 : ldexp(my, ey - E));
  int es;
  const double ms = frexp(s, &es);
  const int q = es + E - kOmegaExp + (ms > 1.0 - kPuMargin ? 1 : 0);
  return q > 0 ? q : 0;
}

// The same two functions with the common case decided by one comparison, and the exact
// function evaluated only where that fails on an active lane (inactive lanes get 0):
//  - division: b <= t 2^1020 is the first exit of protect_division (for t >= 1 the scaled
//    t is at least 2^1020, or infinite, and protect_division returns 0 as well);
//  - update: fl(t x + y) <= 2^1019 bounds the exact sum by 2^1019 (1 + 2^-52) < Omega
//    (1 - 2^-50), where protect_update returns 0 as well (an overflowing t x gives infinity
//    and takes the exact path).
__device__ __forceinline__ int protect_division_fast(double b, double t, bool active = true) {
  int q = 0;
  if (active && !(b <= ldexp(t, kOmegaExp))) q = protect_division(b, t);
  return q;
}
__device__ __forceinline__ int protect_update_fast(double t, double x, double y, bool active = true) {
  int q = 0;
  if (active && !(fma(t, x, y) <= 0x1p1019)) q = protect_update(t, x, y);
  return q;
}

// 1/x from the hardware reciprocal estimate refined by two Newton-Raphson steps
// (r <- r + r (1 - x r); each step squares the relative error), for normal x whose
// reciprocal is normal: the divisions of the diagonal solves, whose divisors are at least
// smin >= the smallest normal number and whose quotients are bounded by ProtectDivision.
// A shorter dependent chain than the correctly rounded division, within a few ulps of it.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

__device__ __forceinline__ double abs1(double x, double y) { return fabs(x) + fabs(y); }

// info bits (per pencil), shared with the host header
enum : int32_t {
  kInfoNonFinite = 1,
  kInfoBadStructure = 2,
  kInfoRealPair = 4,
  kInfoIndefinite = 8,
  kInfoPerturbed = 16,
  kInfoSelectClosure = 32,
  kInfoRefine = 64,
  kInfoWatchdog = 128,
  kInfoPrescaled = 256,
};

}  // namespace rgev
