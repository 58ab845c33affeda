// Complex-arithmetic pencils (the conclusion's extension, Section 7): S and T complex upper
// triangular of order m, no 2x2 blocks.  The eigenvector of eigenvalue k solves
// (beta S - alpha T) z = 0 (Section 2) with complex alpha.
//
// The path runs them through the real blocked solver.  Scaling row i of both matrices by a
// nonzero w_i leaves every right eigenvector unchanged; with w_i = conj(t_ii) 2^-e (a power
// of two keeps it near unit size) the diagonal of T becomes real, exactly: w_i t_ii =
// 2^-e (Re^2 + Im^2).  Each complex entry x + i y then becomes the real 2 x 2 block
// [[x, -y], [y, x]] (the real form of multiplication by x + i y), which gives a real pencil
// of order 2m in generalized real Schur form: its diagonal block i is
// [[a, -b], [b, a]] with T block c I, so a complex eigenvalue (a + i b) / c is a 2x2 block
// carrying the pair (a +- i b) / c, and an exactly real one (b = 0) two 1x1 blocks.  A
// right eigenvector v of the complex pencil for eigenvalue lambda is v (x) (1, -i) in the
// real form (interleaved rows), and conj(v) (x) (1, i) for conj(lambda).  So:
//   - for b > 0 the real solver's pair vector u (the eigenvector of the eigenvalue with
//     positive imaginary part) is a multiple of v (x) (1, -i), and its tip u_2k+1 = 1 makes
//     the multiple i: v_j = -i u_2j;
//   - for b < 0 it belongs to conj(lambda): u = -i conj(v) (x) (1, i), v_j = -i conj(u_2j);
//   - for b = 0 the real vector with its tip at row 2k is Re(v (x) (1, -i)) with v_k = 1:
//     v_j = u_2j + i u_2j+1 (the solver does not need the second 1x1 block's vector, whose
//     eigenvalue repeats, so it is not selected).
// A complex column's 2x2 blocks are solved in its invariant subspace (cform in the solve).
// The real form does twice the arithmetic of complex contractions (each 2x2 block repeats
// its two numbers), in exchange for every kernel of the real path (robust solves, FP64 and
// mixed-precision tile updates, schedules) running unchanged.
#include <hip/hip_runtime.h>

#include "complex.hpp"
#include "layout.hpp"
#include "robust.hpp"

namespace rgev {

// row scale w_i: conj(t_ii) 2^-e, or conj(s_ii) 2^-e when t_ii = 0 (an infinite eigenvalue),
// else 1
__device__ __forceinline__ void row_scale(const ComplexDesc& C, int64_t i, double& wr, double& wi) {
  const double* ts = C.T + 2 * (i + i * C.ldt);
  const double* ss = C.S + 2 * (i + i * C.lds);
  double xr = ts[0], xi = ts[1];
  if (xr == 0.0 && xi == 0.0) {
    xr = ss[0];
    xi = ss[1];
  }
  if (xr == 0.0 && xi == 0.0) {
    wr = 1.0;
    wi = 0.0;
    return;
  }
  int e;
  frexp(fabs(xr) + fabs(xi), &e);
  wr = ldexp(xr, -e);
  wi = -ldexp(xi, -e);
}

// One thread per complex entry (i, j) of column j = blockIdx.y: writes the real 2 x 2 block
// of S2 and T2 (zero below the diagonal; the diagonal block of T2 is c I with c exact) and,
// on the diagonal, the selection of the real form.
__global__ __launch_bounds__(256) void complex_realify_kernel(ComplexDesc C) {
  const int64_t j = blockIdx.y;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t m = C.m;
  if (i >= m || j >= m) return;
  const int64_t ld2 = 2 * m;
  double s00 = 0.0, s10 = 0.0, t00 = 0.0, t10 = 0.0;   // (x, y) of the scaled entries
  if (i <= j) {
    double wr, wi;
    row_scale(C, i, wr, wi);
    const double* sp = C.S + 2 * (i + j * C.lds);
    const double* tp = C.T + 2 * (i + j * C.ldt);
    s00 = wr * sp[0] - wi * sp[1];
    s10 = wr * sp[1] + wi * sp[0];
    t00 = wr * tp[0] - wi * tp[1];
    t10 = wr * tp[1] + wi * tp[0];
    if (i == j) t10 = 0.0;   // exactly zero already when w_i comes from t_ii; (t_ii = 0: both zero)
  }
  double* s2 = C.S2 + (2 * i) + (2 * j) * ld2;
  double* t2 = C.T2 + (2 * i) + (2 * j) * ld2;
  // block [[x, -y], [y, x]]: column 2j holds (x, y), column 2j + 1 holds (-y, x)
  s2[0] = s00;
  s2[1] = s10;
  s2[ld2] = -s10;
  s2[ld2 + 1] = s00;
  t2[0] = t00;
  t2[1] = (i == j) ? 0.0 : t10;
  t2[ld2] = -t10;
  t2[ld2 + 1] = t00;
  if (i == j) {
    const int32_t want = C.select ? (C.select[j] != 0) : 1;
    C.sel2[2 * j] = want;
    C.sel2[2 * j + 1] = s10 != 0.0 ? want : 0;   // the repeated 1x1 eigenvalue is not needed
  }
}

// One workgroup per eigenvalue k: v from the real solver's vector, then normalised (or with
// its exponent), written into column k of Z (rows below k zero).
constexpr int kExtractThreads = 256;
__global__ __launch_bounds__(kExtractThreads) void complex_extract_kernel(ComplexDesc C) {
  __shared__ double red[kExtractThreads / 64];
  const int64_t k = blockIdx.x;
  const int64_t m = C.m;
  if (k >= m) return;
  const int64_t ld2 = 2 * m;
  double* zc = C.Z + 2 * (k * C.ldz);
  const bool want = C.select ? (C.select[k] != 0) : true;
  if (!want) {
    for (int64_t i = threadIdx.x; i < m; i += kExtractThreads) {
      zc[2 * i] = 0.0;
      zc[2 * i + 1] = 0.0;
    }
    if (threadIdx.x == 0 && C.scales) C.scales[k] = 0;
    return;
  }
  const double b = C.S2[(2 * k + 1) + (2 * k) * ld2];   // imaginary part of the scaled s_kk
  const bool pair = b != 0.0;
  const double* x = C.Z2 + (2 * k) * ld2;
  const double* y = x + ld2;
  // The real solver's vector represents 2^scales2 u with its tip fixed: a pair has
  // u_2k+1 = 1 (real), a real eigenvalue u_2k = 1.  With u = c v (x) (1, -i) (b > 0) that gives
  // c = i, so v_j = -i u_2j; with u = c conj(v) (x) (1, i) (b < 0), c = -i and v_j = -i conj(u_2j);
  // a real eigenvalue's u is Re(v (x) (1, -i)) = (Re v_j, Im v_j) interleaved.  No division:
  // the tip entry itself may have underflowed in a normalised vector.
  double nm = 0.0;
  for (int64_t j = threadIdx.x; j <= k; j += kExtractThreads) {
    double vr, vi;
    if (!pair) {
      vr = x[2 * j];
      vi = x[2 * j + 1];
    } else if (b > 0.0) {
      vr = y[2 * j];
      vi = -x[2 * j];
    } else {
      vr = -y[2 * j];
      vi = -x[2 * j];
    }
    zc[2 * j] = vr;
    zc[2 * j + 1] = vi;
    nm = fmax(nm, fabs(vr) + fabs(vi));
  }
  for (int64_t j = k + 1 + threadIdx.x; j < m; j += kExtractThreads) {
    zc[2 * j] = 0.0;
    zc[2 * j + 1] = 0.0;
  }
  if (C.normalize) {
    for (int off = 32; off > 0; off >>= 1) nm = fmax(nm, __shfl_xor(nm, off));
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = nm;
    __syncthreads();
    double mx = 0.0;
    for (int i = 0; i < kExtractThreads / 64; ++i) mx = fmax(mx, red[i]);
    if (mx > 0.0)
      for (int64_t j = threadIdx.x; j <= k; j += kExtractThreads) {
        zc[2 * j] = zc[2 * j] / mx;
        zc[2 * j + 1] = zc[2 * j + 1] / mx;
      }
    if (threadIdx.x == 0 && C.scales) C.scales[k] = 0;
  } else if (threadIdx.x == 0 && C.scales) {
    C.scales[k] = C.scales2[2 * k];
  }
}

void launch_complex_realify(const ComplexDesc& C, hipStream_t s) {
  complex_realify_kernel<<<dim3((unsigned)((C.m + 255) / 256), (unsigned)C.m), 256, 0, s>>>(C);
}

void launch_complex_extract(const ComplexDesc& C, hipStream_t s) {
  complex_extract_kernel<<<(unsigned)C.m, kExtractThreads, 0, s>>>(C);
}

}  // namespace rgev
