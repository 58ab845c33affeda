// Split operands for the mixed-precision tile update: a double is carried as a power-of-two
// scale and kSlices signed 7-bit slices, so products of slices are exact in the int8
// matrix instruction's int32 accumulators.
//
// The two halves of a row of [S_kr | T_kr] (S part, T part) and of a column of
// W = [X D ; -X B] are scaled apart by 2^D_r, one offset per source tile row r: the S half of
// row i by 2^a_i, its T half by 2^(a_i + D_r), the X D half of column c by 2^b_c and its
// -X B half by 2^(b_c - D_r), so both halves' products carry the one exponent a_i + b_c and
// are folded together.  D_r is the exponent of |T| minus that of |S| in the columns of tile
// r; with a_i and b_c the least exponents that cover both halves, a pencil whose T is far
// smaller (or larger) than its S loses no bits in either half (with one scale per row and
// column it would lose their ratio in both operands of the same products).
// For a row (or column) scaled by 2^e so that its entries are below one, every
// entry x gives y = x 2^-e in (-1, 1) and
//     y = sum_{p=1..7} a_p 2^(-7p) + rho,   a_p in [-127, 127] integers,  |rho| < 2^-49,
// each a_p the integer part of the running remainder times 2^7 (exact in FP64).  A product
// of two split operands is then 2^(e + f) sum_{p,q} 2^(-7(p+q)) sum_k a_p[i,k] w_q[k,c];
// the pairs with p + q <= 8 are kept (the rest weigh below 2^-63 of the product), and the
// pairs of one level L = p + q are summed exactly in int32 (|sum| <= 7 K 127^2 < 2^31 for
// K <= 256).  The error is at most about 2 K 2^-49 2^(a_i + b_c) per source.
//
// Fragment layout (matches the 16x16x64 int8 matrix instruction): a 16-byte packet per lane
// holds 16 consecutive K values of one row (A) or one column (W); lane l of a 64-lane
// fragment covers row/column 16 b + l % 16 and K values 64 s + 16 (l / 16) + 0..15.
//   A slices of tile pair (k, r): [pair][p][kstep][row block][lane]
//   W slices of tile (r, j):      [slot][p][kstep][col block][lane]
// with K = [S columns | T columns] (A) = [X D rows | -X B rows] (W), each half padded to
// kHalfK(MB) = MB rounded up to 64.
#pragma once
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

namespace rgev {

constexpr int kSlices = 7;
constexpr int kSliceLevels = kSlices;   // levels L = 2 .. kSlices + 1

__host__ __device__ constexpr int slice_half_k(int mb) { return (mb + 63) / 64 * 64; }
__host__ __device__ constexpr int slice_ksteps(int mb) { return 2 * slice_half_k(mb) / 64; }
// int4 packets per slice of one A (or W) tile
__host__ __device__ constexpr int64_t slice_packets(int mb) { return (int64_t)slice_ksteps(mb) * (mb / 16) * 64; }
// triangular index of the tile pair (k, r), k < r
__host__ __device__ inline int64_t pair_index(int k, int r) { return (int64_t)r * (r - 1) / 2 + k; }

// 16 values (already scaled into (-1, 1)) -> kSlices packets of 16 signed bytes.  The
// slices a_p = trunc(128 r_{p-1}) with r_0 = |y|, r_p = 128 r_{p-1} - a_p (each step exact)
// are the base-128 digits of N = floor(|y| 2^49), signed like y.  N is formed exactly in two
// parts, hi = floor(|y| 2^21) (3 digits) and lo = floor((|y| 2^21 - hi) 2^28) (4 digits),
// so the digits come from integer shifts instead of seven dependent FP64 steps.
static_assert(kSlices == 7, "the digit split below is for 7 slices of 7 bits");
__device__ __forceinline__ void slice16(const double (&y)[16], int4 (&out)[kSlices]) {
  int w[kSlices][4] = {};
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    const double ay = fabs(y[b]);
    const double h = trunc(ay * 2097152.0);                     // |y| 2^21, exact
    const int hi = (int)h;
    const int lo = (int)((ay * 2097152.0 - h) * 268435456.0);  // exact fraction times 2^28, truncated
    const bool neg = y[b] < 0.0;
#pragma unroll
    for (int p = 0; p < kSlices; ++p) {
      const int d = p < 3 ? (hi >> (7 * (2 - p))) & 127 : (lo >> (7 * (6 - p))) & 127;
      w[p][b / 4] |= ((neg ? -d : d) & 0xff) << (8 * (b % 4));
    }
  }
#pragma unroll
  for (int p = 0; p < kSlices; ++p) out[p] = make_int4(w[p][0], w[p][1], w[p][2], w[p][3]);
}

// exponent e with |x| < 2^e for the largest magnitude x of a row or column (0 for zero)
__device__ __forceinline__ int slice_exponent(double vmax) {
  int e = 0;
  if (vmax > 0.0) frexp(vmax, &e);
  return e;
}

// The same for an operand of two halves scaled apart by 2^d (the second half's entries are
// taken in units of 2^(e + d)): the least e with |first| < 2^e and |second| < 2^(e + d).
__device__ __forceinline__ int slice_exponent2(double max_first, double max_second, int d) {
  int e1 = INT_MIN / 2, e2 = INT_MIN / 2;
  if (max_first > 0.0) frexp(max_first, &e1);
  if (max_second > 0.0) {
    frexp(max_second, &e2);
    e2 -= d;
  }
  const int e = e1 > e2 ? e1 : e2;
  return e == INT_MIN / 2 ? 0 : e;
}

// D_r from the largest |S| and |T| of the columns of tile r (as bits of non-negative doubles)
__device__ __forceinline__ int half_offset(const unsigned long long* stmax, int mmax, int r) {
  const double s = __longlong_as_double((long long)stmax[r]);
  const double t = __longlong_as_double((long long)stmax[mmax + r]);
  if (!(s > 0.0) || !(t > 0.0)) return 0;
  int es, et;
  frexp(s, &es);
  frexp(t, &et);
  return et - es;
}

}  // namespace rgev
