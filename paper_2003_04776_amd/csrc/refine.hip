// Refinement of the mixed-precision eigenvectors against an FP64 residual.
//
// For an eigenvector z of eigenvalue (alpha, beta) the residual is r = (beta S - alpha T) z
// (Section 2: the columns of S V D - T V B).  The sweeps run before the consolidation, on the
// augmented form the solve leaves: segment (t, c) of Z is a mantissa with exponent exps[t][c]
// (Section 4), so an eigenvector whose entries span far more than the double range (about a
// bit per row for these pencils: thousands of bits at m = 32768) is still held to full
// precision, tile by tile.  A sweep
//   1. estimates, for every column still under refinement, the componentwise backward
//      error  omega = ||r||_1 / || beta |S| |z| + |alpha| |T| |z| ||_1  with a sketch: the
//      numerator from kSketch Cauchy projections g_t . r (the median of |g_t . r| estimates
//      ||r||_1), the denominator exactly from the column sums of |S| and |T|; all of it in
//      O(m^2) work for the whole pencil;
//   2. flags the columns whose estimate exceeds tau;
//   3. forms r in FP64 for the flagged columns and solves (beta S - alpha T) d = r on the
//      rows above each tip with d = 0 at the tip (the blocked robust solver in correction
//      mode: the same solve and update kernels, Z replaced by r);
//   4. replaces z by z - d, segment by segment (the consolidation follows the sweeps).
// A final estimate sets info bit 64 when a column is still above tau.  Everything is FP64
// except the correction solve's tile updates, which keep the mixed-precision contraction.
#include <hip/hip_runtime.h>
#include <limits.h>

#include "layout.hpp"
#include "robust.hpp"

namespace rgev {

constexpr int kRefThreads = 256;
constexpr int kChunkRows = 1024;               // rows per chunk of the sketch and projection passes
constexpr int kFields = 2 * kSketch + 2;       // partial sums per (chunk, column)

// ---- sketch rows: Cauchy variables from a counter-based generator ----
// SplitMix64 (Steele, Lea and Flood, 2014) of the entry's index gives 53 uniform bits u in
// (0, 1); tan(pi (u - 1/2)) is standard Cauchy.  |g| is clipped at 2^20 (probability about
// 6e-7 per entry), which keeps every sum in range and does not move the median.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ __launch_bounds__(kRefThreads) void refine_g_kernel(PencilDesc P, RefineDesc R) {
  const int64_t n = P.m * kSketch;
  for (int64_t e = blockIdx.x * (int64_t)kRefThreads + threadIdx.x; e < n; e += (int64_t)gridDim.x * kRefThreads) {
    const unsigned long long h = splitmix64((unsigned long long)e);
    const double u = ((double)(h >> 11) + 0.5) * 0x1p-53;
    const double g = tan(3.141592653589793 * (u - 0.5));
    R.G[e] = fmin(fmax(g, -0x1p20), 0x1p20);
  }
}

// Power-of-two scale of the sketch: every column sum of |psc S| is below m 2^Enu, with 2^Enu
// above the largest prescaled tile-pair norm, so with sk = 2^-(Enu + 48) and |g| <= 2^20 no
// sum leaves the range (for m up to 2^20).  Exact, so the estimate's ratio is unchanged.
__device__ __forceinline__ double sketch_scale(const PencilDesc& P) {
  const double numax = __longlong_as_double((long long)P.ctrl->numax_bits);   // units of 2^-32
  int e = 0;
  if (numax > 0.0) frexp(numax, &e);
  int sigma = 0;
  frexp(P.ctrl->psc, &sigma);   // psc = 2^(sigma - 1)
  int E = e + 32 + (sigma - 1);
  if (E < 0) E = 0;
  return ldexp(P.ctrl->psc, -(E + 48));
}

// ---- GS = sk psc (G^T S)^T, GT likewise, column sums of |S| and |T| ----
// One workgroup per (strip of 64 columns, chunk of kChunkRows rows): the chunk's rows are
// walked in 64 x 64 tiles through LDS (coalesced down the columns), each thread accumulating
// 4 sketch rows of one column; partial sums per chunk, summed over the chunks in a fixed
// order by refine_sketch_reduce (reproducible bit for bit; the chunks balance the long strips
// of the triangle's right end against the short ones).
__global__ __launch_bounds__(kRefThreads) void refine_sketch_kernel(PencilDesc P, RefineDesc R) {
  __shared__ double Sl[64][65], Tl[64][65];
  __shared__ double Gl[64][kSketch];
  const int64_t m = P.m;
  const int64_t j0 = (int64_t)blockIdx.x * 64;
  const int64_t r0 = (int64_t)blockIdx.y * kChunkRows;
  const int64_t iend = min(min(j0 + 64 + 1, m), r0 + kChunkRows);  // rows reach the sub-diagonal of the last column
  if (j0 >= m || r0 >= iend) return;
  const int tid = threadIdx.x;
  const int col = tid % 64, tg = tid / 64;   // column of the strip, group of 4 sketch rows
  const int64_t jc = j0 + col;
  double aS[4] = {0.0, 0.0, 0.0, 0.0}, aT[4] = {0.0, 0.0, 0.0, 0.0};
  double absS = 0.0, absT = 0.0;
  for (int64_t i0 = r0; i0 < iend; i0 += 64) {
    __syncthreads();
    for (int q = tid; q < 64 * 64; q += kRefThreads) {
      const int r = q % 64, c = q / 64;
      const int64_t i = i0 + r, j = j0 + c;
      const bool okS = i < iend && j < m && i <= j + 1;
      const bool okT = i < iend && j < m && i <= j;
      Sl[r][c] = okS ? P.S[i + j * P.lds] : 0.0;
      Tl[r][c] = okT ? P.T[i + j * P.ldt] : 0.0;
    }
    for (int q = tid; q < 64 * kSketch; q += kRefThreads) {
      const int r = q / kSketch, t = q % kSketch;
      Gl[r][t] = (i0 + r < iend) ? R.G[(i0 + r) * kSketch + t] : 0.0;
    }
    __syncthreads();
    for (int r = 0; r < 64; ++r) {
      const double sv = Sl[r][col], tv = Tl[r][col];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        aS[q] = fma(Gl[r][4 * tg + q], sv, aS[q]);
        aT[q] = fma(Gl[r][4 * tg + q], tv, aT[q]);
      }
      absS += fabs(sv);
      absT += fabs(tv);
    }
  }
  if (jc < m) {
    double* pp = R.part + ((int64_t)blockIdx.y * m + jc) * kFields;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      pp[4 * tg + q] = aS[q];
      pp[kSketch + 4 * tg + q] = aT[q];
    }
    if (tg == 0) {
      pp[2 * kSketch] = absS;
      pp[2 * kSketch + 1] = absT;
    }
  }
}

// chunks holding rows of column j (rows 0 .. j + 1)
__device__ __forceinline__ int64_t sketch_chunks(int64_t m, int64_t j) {
  return min(j + 2, m) / kChunkRows + (min(j + 2, m) % kChunkRows ? 1 : 0);
}

__global__ __launch_bounds__(kRefThreads) void refine_sketch_reduce(PencilDesc P, RefineDesc R) {
  const int64_t m = P.m;
  const int64_t e = blockIdx.x * (int64_t)kRefThreads + threadIdx.x;
  if (e >= m * kFields) return;
  const int64_t j = e / kFields;
  const int f = (int)(e % kFields);
  const int64_t nch = sketch_chunks(m, j);
  double v = 0.0;
  for (int64_t h = 0; h < nch; ++h) v += R.part[(h * m + j) * kFields + f];
  const double sk = sketch_scale(P);
  if (f < kSketch) R.GS[j * kSketch + f] = sk * v;
  else if (f < 2 * kSketch) R.GT[j * kSketch + f - kSketch] = sk * v;
  else if (f == 2 * kSketch) R.cS[j] = sk * v;
  else R.cT[j] = sk * v;
}

__device__ __forceinline__ double wg_max(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  const int w = threadIdx.x / 64;
  __syncthreads();
  if (threadIdx.x % 64 == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < kRefThreads / 64; ++i) s = fmax(s, red[i]);
  return s;
}

__device__ __forceinline__ double wg_min(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  const int w = threadIdx.x / 64;
  __syncthreads();
  if (threadIdx.x % 64 == 0) red[w] = v;
  __syncthreads();
  double s = red[0];
  for (int i = 1; i < kRefThreads / 64; ++i) s = fmin(s, red[i]);
  return s;
}

// Is column c under refinement in this pass?  Pass 0: every selected column; later passes:
// the columns the previous pass flagged (the others did not change).
__device__ __forceinline__ bool active_column(const PencilDesc& P, const RefineDesc& R, int64_t c, int pass) {
  return pass == 0 ? P.sel[c] != 0 : R.rf[c] != 0;
}

// A column can be refined only while, inside every segment, its entries (down to its
// eigenvalue's block) lie within 2^-kRefineSpan of the segment's largest: the overflow-stress
// eigenvectors grow by hundreds of bits per row, so entries inside one tile underflow to zero,
// and at the first such row the FP64 residual is that row's whole diagonal term (the terms of
// the zeroed entries are missing), from which the correction solve returns d = z above it.
// Such columns are left as they are (and reported through info bit 64 when above tau).
constexpr int kRefineSpan = 900;
static_assert(kSketch == 4 * (kRefThreads / 64), "four sketch rows per group of 64 threads");

// exponent of the largest entry of segment (t, c): exps[t][c] + the exponent of its norm
// (a very negative value for a zero segment)
constexpr int kNoExp = -(1 << 28);
__device__ __forceinline__ int seg_top(const PencilDesc& P, int t, int64_t c) {
  const int64_t e = (int64_t)t * P.m + c;
  const double n = P.norms[e];
  if (!(n > 0.0)) return kNoExp;
  int ex;
  frexp(n, &ex);
  return P.exps[e] + ex;
}

// Per column under refinement: Ec, the largest exponent over its segments (z' = 2^-Ec z,
// segment by segment), and (pass 0) whether every entry down to the eigenvalue's block lies
// within 2^-kRefineSpan of its segment's largest (a pair by |x_i| + |y_i|: the tip's y entry is
// zero by the phase convention).  A workgroup per column, a bounded grid striding over them.
__global__ __launch_bounds__(kRefThreads) void refine_colexp_kernel(PencilDesc P, RefineDesc R, int pass) {
  __shared__ double red[kRefThreads / 64];
  const int64_t m = P.m;
  if (blockIdx.x == 0)
    for (int t = threadIdx.x; t < P.Mmax; t += kRefThreads) R.tflag[t] = 0;
  for (int64_t c = blockIdx.x; c < m; c += gridDim.x) {
    if (!active_column(P, R, c, pass)) continue;
    __syncthreads();   // the previous column is done with red
    const int jt = P.tileof[c];
    double top = (double)kNoExp;
    for (int t = threadIdx.x; t <= jt; t += kRefThreads) top = fmax(top, (double)seg_top(P, t, c));
    top = -wg_min(-top, red);
    bool ok = true;
    if (pass == 0) {
      const int kd = P.blk[c];
      const int64_t blk_end = (kd == 2 ? c - 1 : c) + (kd == 0 ? 1 : 2);
      const int64_t cp = kd == 1 ? c + 1 : (kd == 2 ? c - 1 : c);
      const double* z = P.Z + c * P.ldz;
      const double* zp = P.Z + cp * P.ldz;
      for (int64_t i = threadIdx.x; i < blk_end; i += kRefThreads) {
        const int64_t so = (int64_t)P.tileof[i] * m;
        const double v = fabs(z[i]) + (kd != 0 ? fabs(zp[i]) : 0.0);
        const double nmax = fmax(P.norms[so + c], kd != 0 ? P.norms[so + cp] : 0.0);
        ok = ok && v >= ldexp(nmax, -kRefineSpan);
      }
    }
    const bool fit = wg_min(ok ? 1.0 : 0.0, red) > 0.0;
    if (threadIdx.x == 0) {
      R.zexp[c] = (int)top;
      if (pass == 0) R.fits[c] = fit ? 1 : 0;
    }
  }
}

// Projections G S z'_c, G T z'_c and the denominators' parts cS . |z'_c|, cT . |z'_c|: one
// workgroup per (strip of 64 columns, chunk of kChunkRows rows), the rows walked in 64 x 64
// tiles of z' through LDS (coalesced, each entry brought from its segment's unit to 2^-Ec as
// it is staged); partial sums per chunk, summed in a fixed order by refine_project_reduce.
__global__ __launch_bounds__(kRefThreads) void refine_project_kernel(PencilDesc P, RefineDesc R, int pass) {
  __shared__ double Zl[64][65];
  __shared__ double GSl[64][kSketch], GTl[64][kSketch];
  __shared__ double cSl[64], cTl[64];
  __shared__ int64_t rowsl[64];
  __shared__ int tl[64];
  __shared__ int any;
  const int64_t m = P.m;
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  const int64_t r0 = (int64_t)blockIdx.y * kChunkRows;
  const int tid = threadIdx.x;
  if (tid == 0) any = 0;
  __syncthreads();
  if (tid < 64) {
    const int64_t c = c0 + tid;
    const bool act = c < m && active_column(P, R, c, pass);
    rowsl[tid] = act ? (int64_t)P.edges[P.tileof[c] + 1] : 0;   // zero below the column's tile
    if (act && rowsl[tid] > r0) atomicOr(&any, 1);
  }
  __syncthreads();
  if (!any) return;
  int64_t rmax = 0;
  for (int q = 0; q < 64; ++q) rmax = max(rmax, rowsl[q]);
  const int64_t iend = min(rmax, r0 + kChunkRows);
  const int col = tid % 64, tg = tid / 64;
  double ps[4] = {0.0, 0.0, 0.0, 0.0}, pt[4] = {0.0, 0.0, 0.0, 0.0}, dsum = 0.0;
  for (int64_t i0 = r0; i0 < iend; i0 += 64) {
    __syncthreads();
    if (tid < 64) tl[tid] = (i0 + tid < m) ? P.tileof[i0 + tid] : 0;
    for (int q = tid; q < 64 * kSketch; q += kRefThreads) {
      const int r = q / kSketch, t = q % kSketch;
      const bool ok = i0 + r < iend;
      GSl[r][t] = ok ? R.GS[(i0 + r) * kSketch + t] : 0.0;
      GTl[r][t] = ok ? R.GT[(i0 + r) * kSketch + t] : 0.0;
    }
    if (tid < 64) {
      const bool ok = i0 + tid < iend;
      cSl[tid] = ok ? R.cS[i0 + tid] : 0.0;
      cTl[tid] = ok ? R.cT[i0 + tid] : 0.0;
    }
    __syncthreads();
    for (int q = tid; q < 64 * 64; q += kRefThreads) {
      const int r = q % 64, c = q / 64;
      const int64_t i = i0 + r, cc = c0 + c;
      double z = 0.0;
      if (i < rowsl[c]) z = ldexp(P.Z[i + cc * P.ldz], P.exps[(int64_t)tl[r] * m + cc] - R.zexp[cc]);
      Zl[r][c] = z;
    }
    __syncthreads();
    for (int r = 0; r < 64; ++r) {
      const double z = Zl[r][col];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ps[q] = fma(GSl[r][4 * tg + q], z, ps[q]);
        pt[q] = fma(GTl[r][4 * tg + q], z, pt[q]);
      }
      dsum = fma(tg == 0 ? cSl[r] : cTl[r], fabs(z), dsum);   // (groups 0 and 1 only keep theirs)
    }
  }
  const int64_t c = c0 + col;
  if (c < m && rowsl[col] > r0) {
    double* pp = R.part + ((int64_t)blockIdx.y * m + c) * kFields;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      pp[4 * tg + q] = ps[q];
      pp[kSketch + 4 * tg + q] = pt[q];
    }
    if (tg < 2) pp[2 * kSketch + tg] = dsum;
  }
}

__global__ __launch_bounds__(kRefThreads) void refine_project_reduce(PencilDesc P, RefineDesc R, int pass) {
  const int64_t m = P.m;
  for (int64_t e = blockIdx.x * (int64_t)kRefThreads + threadIdx.x; e < m * kFields;
       e += (int64_t)gridDim.x * kRefThreads) {
    const int64_t c = e / kFields;
    const int f = (int)(e % kFields);
    if (!active_column(P, R, c, pass)) continue;
    const int64_t rows = P.edges[P.tileof[c] + 1];
    const int64_t nch = (rows + kChunkRows - 1) / kChunkRows;
    double v = 0.0;
    for (int64_t h = 0; h < nch; ++h) v += R.part[(h * m + c) * kFields + f];
    if (f < kSketch) R.PS[c * kSketch + f] = v;
    else if (f < 2 * kSketch) R.PT[c * kSketch + f - kSketch] = v;
    else if (f == 2 * kSketch) R.dS[c] = v;
    else R.dT[c] = v;
  }
}

// median of 16 non-negative values: the mean of the 8th and 9th smallest
__device__ __forceinline__ double median16(const double (&v)[kSketch]) {
  double lo = 0.0, hi = 0.0;
#pragma unroll
  for (int i = 0; i < kSketch; ++i) {
    int below = 0, equal_before = 0;
#pragma unroll
    for (int k = 0; k < kSketch; ++k) {
      below += v[k] < v[i] ? 1 : 0;
      equal_before += (v[k] == v[i] && k < i) ? 1 : 0;
    }
    const int rank = below + equal_before;   // distinct ranks 0..15
    if (rank == kSketch / 2 - 1) lo = v[i];
    if (rank == kSketch / 2) hi = v[i];
  }
  return 0.5 * (lo + hi);
}

// ---- decision per eigenvalue: estimate, flag, common exponent of a pair ----
// final_pass: only report (info bit 64) the columns still above tau.  Pass 0 also leaves out
// the columns that cannot be refined (fits = 0; reported through info bit 64 when above tau).
__global__ __launch_bounds__(kRefThreads) void refine_decide_kernel(PencilDesc P, RefineDesc R, int pass,
                                                                    int final_pass) {
  const int64_t c = blockIdx.x * (int64_t)kRefThreads + threadIdx.x;
  if (c >= P.m) return;
  const int kind = P.blk[c];
  if (kind == 2) return;
  const bool act = active_column(P, R, c, pass);
  if (!act) {
    if (pass == 0 && !final_pass) {
      R.rf[c] = 0;
      if (kind == 1) R.rf[c + 1] = 0;
    }
    return;
  }
  const double a = P.ar[c], be = P.be[c];
  double est, den;
  int ze;
  if (kind == 0) {
    double g[kSketch];
#pragma unroll
    for (int t = 0; t < kSketch; ++t) g[t] = fabs(be * R.PS[c * kSketch + t] - a * R.PT[c * kSketch + t]);
    est = median16(g);
    den = be * R.dS[c] + fabs(a) * R.dT[c];
    ze = R.zexp[c];
  } else {
    const double b = P.ai[c];
    const int ex = R.zexp[c], ey = R.zexp[c + 1];
    ze = ex > ey ? ex : ey;
    const int fx = ex - ze, fy = ey - ze;
    double gx[kSketch], gy[kSketch];
#pragma unroll
    for (int t = 0; t < kSketch; ++t) {
      const double sx = ldexp(R.PS[c * kSketch + t], fx), tx = ldexp(R.PT[c * kSketch + t], fx);
      const double sy = ldexp(R.PS[(c + 1) * kSketch + t], fy), ty = ldexp(R.PT[(c + 1) * kSketch + t], fy);
      // r = beta S z - alpha T z with z = x + i y, alpha = a + i b
      gx[t] = fabs(be * sx - a * tx + b * ty);
      gy[t] = fabs(be * sy - b * tx - a * ty);
    }
    est = median16(gx) + median16(gy);
    den = be * (ldexp(R.dS[c], fx) + ldexp(R.dS[c + 1], fy)) +
          (fabs(a) + fabs(b)) * (ldexp(R.dT[c], fx) + ldexp(R.dT[c + 1], fy));
  }
  bool flag = den > 0.0 ? est > R.tau * den : est > 0.0;
  if (final_pass) {
    if (flag) atomicOr(P.info, (int)kInfoRefine);
    return;
  }
  if (flag && pass == 0 && !(R.fits[c] && (kind == 0 || R.fits[c + 1]))) {
    atomicOr(P.info, (int)kInfoRefine);
    flag = false;
  }
  R.rf[c] = flag ? 1 : 0;
  if (kind == 1) R.rf[c + 1] = flag ? 1 : 0;
  R.zexp[c] = ze;
  if (kind == 1) R.zexp[c + 1] = ze;
  if (flag) atomicOr(&R.tflag[P.tileof[c]], 1);
}

// ---- residual of the flagged columns: r = psc (beta S - alpha T) z ----
// One workgroup per tile pair (k, j), k <= j, of a tile column holding a flagged column:
// r on the rows of tile k for every column of tile j (zero for columns not flagged and on
// the rows at and below each eigenvalue's own block), in units of 2^E_kc with E_kc the largest
// segment exponent of column c over tiles k .. j (every z segment is brought to that unit as it
// is staged), written into Zc with the exponents cexps and norms cnorms (the solve's starting
// Y in correction mode).  LDS-staged FP64 VALU
// contraction over the rows l the columns reach: r = sum_l S(i, l) U(l, n) - T(i, l) V(l, n),
// U = beta z', V = z' B (the 2x2 real form of alpha for a pair).
template <int MB>
__device__ __forceinline__ void residual_pair(const PencilDesc& P, const RefineDesc& R, int64_t pid) {
  constexpr int KB = 16;                 // K step
  constexpr int TN = 16;                 // thread grid 16 x 16
  constexpr int UR = (MB + TN - 1) / TN; // outputs per thread and dimension
  constexpr int LDM = MB + 1;
  __shared__ double Sl[KB][LDM], Tl[KB][LDM], Ul[KB][LDM], Vl[KB][LDM];
  __shared__ double cmaxw[TN][MB];
  __shared__ int Ek[MB];
  // (k, j) from the pair index, column-major over the upper triangle: pid = j (j + 1) / 2 + k
  int j = (int)((sqrt(8.0 * (double)pid + 1.0) - 1.0) * 0.5);
  while ((int64_t)j * (j + 1) / 2 > pid) --j;
  while ((int64_t)(j + 1) * (j + 2) / 2 <= pid) ++j;
  const int k = (int)(pid - (int64_t)j * (j + 1) / 2);
  if (!R.tflag[j]) return;
  __syncthreads();   // the previous pair's shared memory is free
  const int64_t m = P.m;
  const int k0 = P.edges[k], hk = P.edges[k + 1] - k0;
  const int c0 = P.edges[j], hj = P.edges[j + 1] - c0;
  const double psc = P.ctrl->psc;
  const int tid = threadIdx.x, ty = tid / TN, tx = tid % TN;
  // E_kc over the segments t = k .. j (common to the two columns of a pair)
  for (int n = tid; n < hj; n += kRefThreads) {
    int e = kNoExp;
    for (int t = k; t <= j; ++t) e = max(e, seg_top(P, t, c0 + n));
    Ek[n] = e;
  }
  __syncthreads();
  for (int n = tid; n < hj; n += kRefThreads)
    if (P.blk[c0 + n] == 1) {
      const int e = max(Ek[n], Ek[n + 1]);
      Ek[n] = e;
      Ek[n + 1] = e;
    }
  __syncthreads();
  double acc[UR][UR];
#pragma unroll
  for (int u = 0; u < UR; ++u)
#pragma unroll
    for (int v = 0; v < UR; ++v) acc[u][v] = 0.0;
  const int l_lo = k0 > 0 ? k0 - 1 : 0, l_hi = c0 + hj;   // rows of z the tile's columns reach
  for (int l0 = l_lo; l0 < l_hi; l0 += KB) {
    __syncthreads();
    for (int q = tid; q < KB * MB; q += kRefThreads) {
      const int i = q % MB, kk = q / MB;
      const int64_t row = k0 + i, l = l0 + kk;
      const bool in = i < hk && l < l_hi;
      Sl[kk][i] = (in && row <= l + 1) ? psc * P.S[row + l * P.lds] : 0.0;
      Tl[kk][i] = (in && row <= l) ? psc * P.T[row + l * P.ldt] : 0.0;
    }
    for (int q = tid; q < KB * MB; q += kRefThreads) {
      const int kk = q % KB, n = q / KB;
      const int64_t l = l0 + kk, c = c0 + n;
      double u = 0.0, v = 0.0;
      if (n < hj && l < l_hi && R.rf[c]) {
        const int kd = P.blk[c];
        const int ze = Ek[n] - P.exps[(int64_t)P.tileof[l] * m + c];   // the segment's unit to 2^E_kc
        const double z = ldexp(P.Z[l + c * P.ldz], -ze);
        const double a = P.ar[c], be = P.be[c];
        u = be * z;
        if (kd == 0) {
          v = a * z;
        } else {
          const double b = P.ai[c];   // positive for both columns of a pair
          const int64_t cp = kd == 1 ? c + 1 : c - 1;
          const double zp = ldexp(P.Z[l + cp * P.ldz], -ze);
          // [x y] [[a, b], [-b, a]] = [a x - b y, b x + a y]
          v = kd == 1 ? (a * z - b * zp) : (b * zp + a * z);
        }
      }
      Ul[kk][n] = u;
      Vl[kk][n] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < KB; ++kk) {
      double sv[UR], tv[UR], uv[UR], vv[UR];
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        const int i = ty + TN * u;
        sv[u] = i < MB ? Sl[kk][i] : 0.0;
        tv[u] = i < MB ? Tl[kk][i] : 0.0;
      }
#pragma unroll
      for (int v = 0; v < UR; ++v) {
        const int n = tx + TN * v;
        uv[v] = n < MB ? Ul[kk][n] : 0.0;
        vv[v] = n < MB ? Vl[kk][n] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UR; ++u)
#pragma unroll
        for (int v = 0; v < UR; ++v) acc[u][v] = fma(sv[u], uv[v], fma(-tv[u], vv[v], acc[u][v]));
    }
  }
  // epilogue: zero on and below each eigenvalue's own block, column maxima of the segment
#pragma unroll
  for (int v = 0; v < UR; ++v) {
    const int n = tx + TN * v;
    double cm = 0.0;
    if (n < hj) {
      const int64_t c = c0 + n;
      const int64_t p0 = P.blk[c] == 2 ? c - 1 : c;   // first row of the eigenvalue's block
      const bool fl = R.rf[c] != 0;
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        const int i = ty + TN * u;
        if (i < hk) {
          const int64_t row = k0 + i;
          const double r = (fl && row < p0) ? acc[u][v] : 0.0;
          R.Zc[row + c * m] = r;
          cm = fmax(cm, fabs(r));
        }
      }
    }
    if (n < MB) cmaxw[ty][n] = cm;
  }
  __syncthreads();
  for (int n = tid; n < hj; n += kRefThreads) {
    double cm = 0.0;
    for (int t = 0; t < TN; ++t) cm = fmax(cm, cmaxw[t][n]);
    const int64_t c = c0 + n;
    R.cexps[(int64_t)k * m + c] = Ek[n] == kNoExp ? 0 : Ek[n];
    R.cnorms[(int64_t)k * m + c] = cm;
  }
}

template <int MB>
__global__ __launch_bounds__(kRefThreads) void refine_residual_kernel(PencilDesc P, RefineDesc R) {
  const int M = P.ctrl->M;
  const int64_t pairs = (int64_t)M * (M + 1) / 2;
  for (int64_t pid = blockIdx.x; pid < pairs; pid += gridDim.x) residual_pair<MB>(P, R, pid);
}

// ---- z <- z - d for the flagged eigenvalues, segment by segment ----
// Segment (t, c) of z is 2^exps[t][c] times its mantissa, that of d 2^cexps[t][c] times its
// mantissa; the segment norms are brought up to date for the next sweep's estimate.
__device__ __forceinline__ void apply_column(const PencilDesc& P, const RefineDesc& R, int64_t c, double* red) {
  const int64_t m = P.m;
  const int kind = P.blk[c];
  if (kind == 2 || !R.rf[c]) return;
  const int jt = P.tileof[c];
  const int64_t blk_end = c + (kind == 0 ? 1 : 2);
  const bool pair = kind == 1;
  // a pair's two columns together (they share every segment exponent), so the segment's
  // max |x_i| + |y_i| is formed as well
  double* zx = P.Z + c * P.ldz;
  double* zy = pair ? zx + P.ldz : zx;
  const double* dx = R.Zc + c * m;
  const double* dy = pair ? dx + m : dx;
  for (int t = 0; t <= jt; ++t) {
    const int r0 = P.edges[t], r1 = P.edges[t + 1];
    const int64_t e = (int64_t)t * m + c;
    const int shx = R.cexps[e] - P.exps[e];
    const int shy = pair ? R.cexps[e + 1] - P.exps[e + 1] : shx;
    double nx = 0.0, ny = 0.0, ns = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kRefThreads) {
      double x = zx[i], y = pair ? zy[i] : 0.0;
      if (i < blk_end) {
        x -= ldexp(dx[i], shx);
        zx[i] = x;
        if (pair) {
          y -= ldexp(dy[i], shy);
          zy[i] = y;
        }
      }
      nx = fmax(nx, fabs(x));
      ny = fmax(ny, fabs(y));
      ns = fmax(ns, fabs(x) + fabs(y));
    }
    nx = wg_max(nx, red);
    ny = wg_max(ny, red);
    ns = wg_max(ns, red);
    if (threadIdx.x == 0) {
      P.norms[e] = nx;
      P.segn[e] = ns;
      if (pair) {
        P.norms[e + 1] = ny;
        P.segn[e + 1] = ns;
      }
    }
  }
}

// one workgroup per eigenvector, a bounded grid striding over the columns
__global__ __launch_bounds__(kRefThreads) void refine_apply_kernel(PencilDesc P, RefineDesc R) {
  __shared__ double red[kRefThreads / 64];
  for (int64_t c = blockIdx.x; c < P.m; c += gridDim.x) apply_column(P, R, c, red);
}

void launch_refine_setup(const PencilDesc& P, const RefineDesc& R, hipStream_t s) {
  const int64_t n = P.m * kSketch;
  refine_g_kernel<<<(unsigned)std::min<int64_t>((n + kRefThreads - 1) / kRefThreads, 4096), kRefThreads, 0, s>>>(P, R);
  const unsigned strips = (unsigned)((P.m + 63) / 64), chunks = (unsigned)((P.m + kChunkRows - 1) / kChunkRows);
  refine_sketch_kernel<<<dim3(strips, chunks), kRefThreads, 0, s>>>(P, R);
  refine_sketch_reduce<<<(unsigned)((P.m * kFields + kRefThreads - 1) / kRefThreads), kRefThreads, 0, s>>>(P, R);
}

void launch_refine_estimate(const PencilDesc& P, const RefineDesc& R, int pass, bool final_pass, hipStream_t s) {
  const unsigned strips = (unsigned)((P.m + 63) / 64), chunks = (unsigned)((P.m + kChunkRows - 1) / kChunkRows);
  refine_colexp_kernel<<<(unsigned)std::min<int64_t>(P.m, pass == 0 ? 8192 : kRhsGrid), kRefThreads, 0, s>>>(P, R, pass);
  refine_project_kernel<<<dim3(strips, chunks), kRefThreads, 0, s>>>(P, R, pass);
  refine_project_reduce<<<(unsigned)std::min<int64_t>((P.m * kFields + kRefThreads - 1) / kRefThreads, 8192),
                          kRefThreads, 0, s>>>(P, R, pass);
  refine_decide_kernel<<<(unsigned)((P.m + kRefThreads - 1) / kRefThreads), kRefThreads, 0, s>>>(P, R, pass,
                                                                                                  final_pass ? 1 : 0);
}

void launch_refine_residual(const PencilDesc& P, const RefineDesc& R, hipStream_t s) {
  const unsigned pairs = (unsigned)std::min<int64_t>((int64_t)P.Mmax * (P.Mmax + 1) / 2, kRhsGrid);
  switch (P.mb) {
    case 32: refine_residual_kernel<32><<<pairs, kRefThreads, 0, s>>>(P, R); break;
    case 64: refine_residual_kernel<64><<<pairs, kRefThreads, 0, s>>>(P, R); break;
    default: refine_residual_kernel<128><<<pairs, kRefThreads, 0, s>>>(P, R); break;
  }
}

void launch_refine_apply(const PencilDesc& P, const RefineDesc& R, hipStream_t s) {
  refine_apply_kernel<<<(unsigned)std::min<int64_t>(P.m, kRhsGrid), kRefThreads, 0, s>>>(P, R);
}

}  // namespace rgev
