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

// Complex quotient (a + ib) / (c + id) by Smith's method, with the refinements of
// Baudin & Smith (2012) for intermediate products that underflow.  Requires |d| <= |c|.
__device__ __forceinline__ void smith_core(double a, double b, double c, double d, double& e, double& f) {
  const double r = d * recip(c);
  const double t = recip(c + d * r);
  if (r != 0.0 || d == 0.0) {
    // (d == 0 lands here too: r = 0 and the products with r vanish)
    const double br = b * r;
    e = (br != 0.0) ? (a + br) * t : a * t + (b * t) * r;
    const double ar = a * r;
    f = (ar != 0.0) ? (b - ar) * t : b * t - (a * t) * r;
  } else {
    // d / c underflowed
    e = (a + d * (b / c)) * t;
    f = (b - d * (a / c)) * t;
  }
}

// The larger of |c|, |d| goes to the divisor's real slot; the swap is done with
// selects so lanes with different orderings share one instruction stream.
__device__ __forceinline__ void complex_div(double a, double b, double c, double d, double& e, double& f) {
  const bool sw = fabs(d) > fabs(c);
  double e1, f1;
  smith_core(sw ? b : a, sw ? a : b, sw ? d : c, sw ? c : d, e1, f1);
  e = e1;
  f = sw ? -f1 : f1;
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
