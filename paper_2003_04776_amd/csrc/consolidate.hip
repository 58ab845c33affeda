// Post-processing (Section 5, fourth task type): enforce one consistent scaling on
// every eigenvector.  Segment (k, c) represents 2^exps[k][c] * Z[rows of tile k, c];
// the column's common exponent is E_c = max_k exps[k][c], and each segment is
// rescaled by the exact power of two 2^(exps[k][c] - E_c) (flushing to zero when the
// gap exceeds the exponent range).  Optionally each eigenvector is then divided by
// max_i (|x_i| + |y_i|), which comes from the per-segment maxima the solves recorded
// (segn, scaled by the same powers of two), so Z is read and written once.  Rows below
// the eigenvector's tile and unselected columns are zeroed (for one pencil by a second
// launch, one workgroup per column).  One workgroup per eigenvalue (a complex pair is
// handled as one).
#include <hip/hip_runtime.h>

#include "layout.hpp"
#include "robust.hpp"

namespace rgev {

constexpr int kConsThreads = 256;

__device__ __forceinline__ double block_max(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  const int w = threadIdx.x / 64;
  if (threadIdx.x % 64 == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < kConsThreads / 64; ++i) r = fmax(r, red[i]);
  __syncthreads();
  return r;
}

// kZeros: the workgroup also writes the column's zeros (the batched kernel); otherwise
// zero_below_kernel writes them.
template <bool kZeros>
__device__ __forceinline__ void consolidate_body(const PencilDesc& P, int64_t c) {
  __shared__ double red[kConsThreads / 64];
  const int64_t m = P.m;
  if (c >= m) return;
  const int kind = P.blk[c];
  if (kind == 2) return;
  const bool cplx = kind == 1;
  const int jt = P.tileof[c];
  double* zx = P.Z + c * P.ldz;
  double* zy = cplx ? zx + P.ldz : nullptr;
  if (!P.sel[c]) {
    if (kZeros) {
      for (int64_t i = threadIdx.x; i < m; i += kConsThreads) {
        zx[i] = 0.0;
        if (cplx) zy[i] = 0.0;
      }
    }
    if (threadIdx.x == 0 && P.scales) {
      P.scales[c] = 0;
      if (cplx) P.scales[c + 1] = 0;
    }
    return;
  }
  // common exponent
  int E = INT_MIN;
  for (int k = threadIdx.x; k <= jt; k += kConsThreads) E = max(E, P.exps[(int64_t)k * m + c]);
  double Ed = block_max((double)E, red);   // exponents are exact in double
  E = (int)Ed;
  // the normalisation: max_i |x_i| + |y_i| over the rescaled segments
  double nm = 0.0;
  if (P.normalize) {
    for (int k = threadIdx.x; k <= jt; k += kConsThreads)
      nm = fmax(nm, ldexp(P.segn[(int64_t)k * m + c], P.exps[(int64_t)k * m + c] - E));
    nm = block_max(nm, red);
  }
  // rescale every segment to the common exponent (and divide by the norm): a step covers
  // kConsThreads / mb whole segments, thread t row t mod mb of segment t / mb (so its
  // exponent is one load, not one per row), and a thread's kUnroll steps are loaded before
  // any is stored, keeping that many loads of the column in flight
  const bool div = P.normalize && nm > 0.0;
  constexpr int kUnroll = 4;
  const int mb = P.mb;
  const int segs = kConsThreads / mb;   // segments per step (mb divides kConsThreads)
  const int tr = threadIdx.x % mb, ts = threadIdx.x / mb;
  for (int k0 = 0; k0 <= jt; k0 += kUnroll * segs) {
    double x[kUnroll], y[kUnroll];
    int d[kUnroll];
    int64_t row[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int k = k0 + u * segs + ts;
      const int kr = k <= jt ? k : jt;
      const int64_t i = P.edges[kr] + tr;
      row[u] = (k <= jt && i < P.edges[kr + 1]) ? i : -1;   // (-1: no row; a valid one is read)
      const int64_t ir = row[u] >= 0 ? i : P.edges[kr];
      x[u] = zx[ir];
      y[u] = cplx ? zy[ir] : 0.0;
      d[u] = P.exps[(int64_t)kr * m + c] - E;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (row[u] >= 0) {
        const double xs = ldexp(x[u], d[u]);
        zx[row[u]] = div ? xs / nm : xs;
        if (cplx) {
          const double ys = ldexp(y[u], d[u]);
          zy[row[u]] = div ? ys / nm : ys;
        }
      }
    }
  }
  if (kZeros) {
    for (int64_t i = P.edges[jt + 1] + threadIdx.x; i < m; i += kConsThreads) {
      zx[i] = 0.0;
      if (cplx) zy[i] = 0.0;
    }
  }
  if (threadIdx.x == 0 && P.scales) {
    const int sc = P.normalize ? 0 : E;
    P.scales[c] = sc;
    if (cplx) P.scales[c + 1] = sc;
  }
}

// The zeros of column c: rows below the tile of its eigenvalue, or the whole column when the
// eigenvalue is not selected (a complex pair follows its first column).  For one pencil they
// are written by a launch of their own: with the rescaling and the zeros of a column in one
// workgroup, m = 32768 took 3.44 ms where the two launches take 2.13 + 0.81 ms.  A batch of
// short columns (orders up to 2048) keeps them in the rescaling workgroup: there the second
// launch made the consolidation 3.54 ms per call against 3.08 ms.
__device__ __forceinline__ void zero_below_body(const PencilDesc& P) {
  const int64_t c = blockIdx.x;
  const int64_t m = P.m;
  if (c >= m) return;
  const int64_t c1 = P.blk[c] == 2 ? c - 1 : c;
  const int64_t lo = P.sel[c1] ? P.edges[P.tileof[c1] + 1] : 0;
  double* z = P.Z + c * P.ldz;
  for (int64_t i = lo + threadIdx.x; i < m; i += kConsThreads) z[i] = 0.0;
}

// Column of workgroup b: workgroups go to the eight XCDs in turn, and each XCD takes runs of
// 32 adjacent columns (XCD x the runs x, x + 8, ...), so the segment tables' lines (32
// exponents, 16 maxima) are read into one XCD's L2 once rather than into all eight (with
// column = b, 0.7 GB more was read at m = 32768).  The blocks past the last whole group of
// 256 keep their own column.
__device__ __forceinline__ int64_t cons_column(int64_t b, int64_t n) {
  if (b >= n / 256 * 256) return b;
  const int64_t x = b % 8, i = b / 8;
  return 256 * (i / 32) + 32 * x + i % 32;
}

__global__ __launch_bounds__(kConsThreads) void consolidate_kernel(PencilDesc P) {
  consolidate_body<false>(P, cons_column(blockIdx.x, gridDim.x));
}
__global__ __launch_bounds__(kConsThreads) void zero_below_kernel(PencilDesc P) { zero_below_body(P); }

// one pencil per blockIdx.y of a table
__global__ __launch_bounds__(kConsThreads) void consolidate_batched(const PencilDesc* __restrict__ D) {
  const PencilDesc P = D[blockIdx.y];
  consolidate_body<true>(P, blockIdx.x);
}

void launch_consolidate(const PencilDesc& P, hipStream_t s) {
  consolidate_kernel<<<(unsigned)P.m, kConsThreads, 0, s>>>(P);
  zero_below_kernel<<<(unsigned)P.m, kConsThreads, 0, s>>>(P);
}

void launch_consolidate_batched(const PencilDesc* D, int n, int64_t max_m, hipStream_t s) {
  if (n <= 0 || max_m <= 0) return;
  consolidate_batched<<<dim3((unsigned)max_m, (unsigned)n), kConsThreads, 0, s>>>(D);
}

// eigenvalues in the caller's layout: conjugate in the second column of a pair
__global__ void eigvals_out_kernel(PencilDesc P, double* are, double* aim, double* bet) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= P.m) return;
  are[c] = P.ar[c];
  aim[c] = P.blk[c] == 2 ? -P.ai[c] : P.ai[c];
  bet[c] = P.be[c];
}

void launch_eigvals_out(const PencilDesc& P, double* are, double* aim, double* bet, hipStream_t s) {
  eigvals_out_kernel<<<(unsigned)((P.m + 255) / 256), 256, 0, s>>>(P, are, aim, bet);
}

}  // namespace rgev
