// Refinement of the mixed-precision eigenvectors against an FP64 residual.
//
// For an eigenvector z of eigenvalue (alpha, beta) the residual is r = (beta S - alpha T) z
// (Section 2: the columns of S V D - T V B).  A sweep
//   1. estimates, for every column still under refinement, the componentwise backward
//      error  omega = ||r||_1 / || beta |S| |z| + |alpha| |T| |z| ||_1  with a sketch: the
//      numerator from kSketch Cauchy projections g_t . r (the median of |g_t . r| estimates
//      ||r||_1), the denominator exactly from the column sums of |S| and |T|; all of it in
//      O(m^2) work for the whole pencil;
//   2. flags the columns whose estimate exceeds tau;
//   3. forms r in FP64 for the flagged columns and solves (beta S - alpha T) d = r on the
//      rows above each tip with d = 0 at the tip (the blocked robust solver in correction
//      mode: the same solve and update kernels, Z replaced by r);
//   4. replaces z by z - d (and normalises again).
// A final estimate sets info bit 64 when a column is still above tau.  Everything is FP64
// except the correction solve's tile updates, which keep the mixed-precision contraction.
#include <hip/hip_runtime.h>

#include "layout.hpp"
#include "robust.hpp"

namespace rgev {

constexpr int kRefThreads = 256;

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
// One workgroup per strip of 64 columns; the strip's rows are walked in 64 x 64 tiles
// through LDS (coalesced down the columns), each thread accumulating 4 sketch rows of one
// column in a fixed order (the result is reproducible bit for bit).
__global__ __launch_bounds__(kRefThreads) void refine_sketch_kernel(PencilDesc P, RefineDesc R) {
  __shared__ double Sl[64][65], Tl[64][65];
  __shared__ double Gl[64][kSketch];
  const int64_t m = P.m;
  const int64_t j0 = (int64_t)blockIdx.x * 64;
  if (j0 >= m) return;
  const double sk = sketch_scale(P);
  const int tid = threadIdx.x;
  const int col = tid % 64, tg = tid / 64;   // column of the strip, group of 4 sketch rows
  const int64_t jc = j0 + col;
  const int64_t iend = min(j0 + 64 + 1, m);  // rows reach the sub-diagonal of the last column
  double aS[4] = {0.0, 0.0, 0.0, 0.0}, aT[4] = {0.0, 0.0, 0.0, 0.0};
  double absS = 0.0, absT = 0.0;
  for (int64_t i0 = 0; i0 < iend; i0 += 64) {
    __syncthreads();
    for (int q = tid; q < 64 * 64; q += kRefThreads) {
      const int r = q % 64, c = q / 64;
      const int64_t i = i0 + r, j = j0 + c;
      const bool okS = i < m && j < m && i <= j + 1;
      const bool okT = i < m && j < m && i <= j;
      Sl[r][c] = okS ? P.S[i + j * P.lds] : 0.0;
      Tl[r][c] = okT ? P.T[i + j * P.ldt] : 0.0;
    }
    for (int q = tid; q < 64 * kSketch; q += kRefThreads) {
      const int r = q / kSketch, t = q % kSketch;
      Gl[r][t] = (i0 + r < m) ? R.G[(i0 + r) * kSketch + t] : 0.0;
    }
    __syncthreads();
    for (int r = 0; r < 64; ++r) {
      const double s = Sl[r][col], t = Tl[r][col];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        aS[q] = fma(Gl[r][4 * tg + q], s, aS[q]);
        aT[q] = fma(Gl[r][4 * tg + q], t, aT[q]);
      }
      absS += fabs(s);
      absT += fabs(t);
    }
  }
  if (jc < m) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      R.GS[jc * kSketch + 4 * tg + q] = sk * aS[q];
      R.GT[jc * kSketch + 4 * tg + q] = sk * aT[q];
    }
    if (tg == 0) {
      R.cS[jc] = sk * absS;
      R.cT[jc] = sk * absT;
    }
  }
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

// Is column c under refinement in this pass?  Pass 0: every selected column; later passes:
// the columns the previous pass flagged (the others did not change).
__device__ __forceinline__ bool active_column(const PencilDesc& P, const RefineDesc& R, int64_t c, int pass) {
  return pass == 0 ? P.sel[c] != 0 : R.rf[c] != 0;
}

// ---- projections of each column: G S z'_c, G T z'_c and the denominators' parts ----
// One workgroup per kProjCols columns; wave w accumulates sketch rows 4w .. 4w+3 over all
// rows (lanes stride the rows), wave 0 also the denominators; z'_c = 2^-zexp z_c with
// max |z'_c| in [1/2, 1).
constexpr int kProjCols = 2;
static_assert(kSketch == 4 * (kRefThreads / 64), "four sketch rows per wave");

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__global__ __launch_bounds__(kRefThreads) void refine_project_kernel(PencilDesc P, RefineDesc R, int pass) {
  __shared__ double red[kRefThreads / 64];
  const int64_t m = P.m;
  const int64_t cb = (int64_t)blockIdx.x * kProjCols;
  if (blockIdx.x == 0)
    for (int t = threadIdx.x; t < P.Mmax; t += kRefThreads) R.tflag[t] = 0;
  bool act[kProjCols];
  int64_t rows[kProjCols];
  bool any = false;
#pragma unroll
  for (int q = 0; q < kProjCols; ++q) {
    const int64_t c = cb + q;
    act[q] = c < m && active_column(P, R, c, pass);
    rows[q] = act[q] ? (int64_t)P.edges[P.tileof[c] + 1] : 0;   // zero below the column's tile
    any = any || act[q];
  }
  if (!any) return;
  // exponent of each column's largest entry
  int ze[kProjCols];
#pragma unroll
  for (int q = 0; q < kProjCols; ++q) {
    double mx = 0.0;
    if (act[q]) {
      const double* z = P.Z + (cb + q) * P.ldz;
      for (int64_t i = threadIdx.x; i < rows[q]; i += kRefThreads) mx = fmax(mx, fabs(z[i]));
    }
    mx = wg_max(mx, red);
    ze[q] = 0;
    if (mx > 0.0) frexp(mx, &ze[q]);
  }
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int t0 = 4 * wave;
  double ps[kProjCols][4], pt[kProjCols][4], ds[kProjCols], dt[kProjCols];
#pragma unroll
  for (int q = 0; q < kProjCols; ++q) {
    ds[q] = 0.0;
    dt[q] = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) ps[q][t] = pt[q][t] = 0.0;
  }
  int64_t rmax = 0;
#pragma unroll
  for (int q = 0; q < kProjCols; ++q) rmax = rows[q] > rmax ? rows[q] : rmax;
  for (int64_t i = lane; i < rmax; i += 64) {
    double gs[4], gt[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      gs[t] = R.GS[i * kSketch + t0 + t];
      gt[t] = R.GT[i * kSketch + t0 + t];
    }
    const double cs = R.cS[i], ct = R.cT[i];
#pragma unroll
    for (int q = 0; q < kProjCols; ++q) {
      const double z = (i < rows[q]) ? ldexp(P.Z[i + (cb + q) * P.ldz], -ze[q]) : 0.0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        ps[q][t] = fma(gs[t], z, ps[q][t]);
        pt[q][t] = fma(gt[t], z, pt[q][t]);
      }
      ds[q] = fma(cs, fabs(z), ds[q]);
      dt[q] = fma(ct, fabs(z), dt[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < kProjCols; ++q) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      ps[q][t] = wave_sum(ps[q][t]);
      pt[q][t] = wave_sum(pt[q][t]);
    }
    ds[q] = wave_sum(ds[q]);
    dt[q] = wave_sum(dt[q]);
  }
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < kProjCols; ++q) {
      if (!act[q]) continue;
      const int64_t c = cb + q;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        R.PS[c * kSketch + t0 + t] = ps[q][t];
        R.PT[c * kSketch + t0 + t] = pt[q][t];
      }
      if (wave == 0) {
        R.dS[c] = ds[q];
        R.dT[c] = dt[q];
        R.zexp[c] = ze[q];
      }
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
// final_pass: only report (info bit 64) the columns still above tau.
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
  const bool flag = den > 0.0 ? est > R.tau * den : est > 0.0;
  if (final_pass) {
    if (flag) atomicOr(P.info, (int)kInfoRefine);
    return;
  }
  R.rf[c] = flag ? 1 : 0;
  if (kind == 1) R.rf[c + 1] = flag ? 1 : 0;
  R.zexp[c] = ze;
  if (kind == 1) R.zexp[c + 1] = ze;
  if (flag) atomicOr(&R.tflag[P.tileof[c]], 1);
}

// ---- residual of the flagged columns: r = psc (beta S - alpha T) z' ----
// One workgroup per tile pair (k, j), k <= j, of a tile column holding a flagged column:
// r on the rows of tile k for every column of tile j (zero for columns not flagged and on
// the rows at and below each eigenvalue's own block), written into Zc with exponent 0 and the
// segment norms (the solve's starting Y in correction mode).  LDS-staged FP64 VALU
// contraction over the rows l the columns reach: r = sum_l S(i, l) U(l, n) - T(i, l) V(l, n),
// U = beta z', V = z' B (the 2x2 real form of alpha for a pair).
template <int MB>
__global__ __launch_bounds__(kRefThreads) void refine_residual_kernel(PencilDesc P, RefineDesc R) {
  constexpr int KB = 16;                 // K step
  constexpr int TN = 16;                 // thread grid 16 x 16
  constexpr int UR = (MB + TN - 1) / TN; // outputs per thread and dimension
  constexpr int LDM = MB + 1;
  __shared__ double Sl[KB][LDM], Tl[KB][LDM], Ul[KB][LDM], Vl[KB][LDM];
  __shared__ double cmaxw[TN][MB];
  const int M = P.ctrl->M;
  const int64_t pairs = (int64_t)M * (M + 1) / 2;
  const int64_t pid = blockIdx.x;
  if (pid >= pairs) return;
  // (k, j) from the pair index, column-major over the upper triangle: pid = j (j + 1) / 2 + k
  int j = (int)((sqrt(8.0 * (double)pid + 1.0) - 1.0) * 0.5);
  while ((int64_t)j * (j + 1) / 2 > pid) --j;
  while ((int64_t)(j + 1) * (j + 2) / 2 <= pid) ++j;
  const int k = (int)(pid - (int64_t)j * (j + 1) / 2);
  if (!R.tflag[j]) return;
  const int64_t m = P.m;
  const int k0 = P.edges[k], hk = P.edges[k + 1] - k0;
  const int c0 = P.edges[j], hj = P.edges[j + 1] - c0;
  const double psc = P.ctrl->psc;
  const int tid = threadIdx.x, ty = tid / TN, tx = tid % TN;
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
        const int ze = R.zexp[c];
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
    P.exps[(int64_t)k * m + c] = 0;
    P.norms[(int64_t)k * m + c] = cm;
  }
}

// ---- z <- z - 2^zexp d for the flagged eigenvalues, then normalise again ----
__global__ __launch_bounds__(kRefThreads) void refine_apply_kernel(PencilDesc P, RefineDesc R) {
  __shared__ double red[kRefThreads / 64];
  const int64_t c = blockIdx.x;
  const int64_t m = P.m;
  if (c >= m) return;
  const int kind = P.blk[c];
  if (kind == 2 || !R.rf[c]) return;
  const bool cplx = kind == 1;
  const int64_t rend = P.edges[P.tileof[c] + 1];
  const int ze = R.zexp[c];
  double* zx = P.Z + c * P.ldz;
  double* zy = cplx ? zx + P.ldz : nullptr;
  const double* dx = R.Zc + c * m;
  const double* dy = cplx ? dx + m : nullptr;
  double nm = 0.0;
  for (int64_t i = threadIdx.x; i < rend; i += kRefThreads) {
    const int64_t so = (int64_t)P.tileof[i] * m;
    const double x = zx[i] - ldexp(dx[i], P.exps[so + c] + ze);
    zx[i] = x;
    double v = fabs(x);
    if (cplx) {
      const double y = zy[i] - ldexp(dy[i], P.exps[so + c + 1] + ze);
      zy[i] = y;
      v += fabs(y);
    }
    nm = fmax(nm, v);
  }
  nm = wg_max(nm, red);
  if (P.normalize && nm > 0.0)
    for (int64_t i = threadIdx.x; i < rend; i += kRefThreads) {
      zx[i] = zx[i] / nm;
      if (cplx) zy[i] = zy[i] / nm;
    }
}

void launch_refine_setup(const PencilDesc& P, const RefineDesc& R, hipStream_t s) {
  const int64_t n = P.m * kSketch;
  refine_g_kernel<<<(unsigned)std::min<int64_t>((n + kRefThreads - 1) / kRefThreads, 4096), kRefThreads, 0, s>>>(P, R);
  refine_sketch_kernel<<<(unsigned)((P.m + 63) / 64), kRefThreads, 0, s>>>(P, R);
}

void launch_refine_estimate(const PencilDesc& P, const RefineDesc& R, int pass, bool final_pass, hipStream_t s) {
  refine_project_kernel<<<(unsigned)((P.m + kProjCols - 1) / kProjCols), kRefThreads, 0, s>>>(P, R, pass);
  refine_decide_kernel<<<(unsigned)((P.m + kRefThreads - 1) / kRefThreads), kRefThreads, 0, s>>>(P, R, pass,
                                                                                                  final_pass ? 1 : 0);
}

void launch_refine_residual(const PencilDesc& P, const RefineDesc& R, hipStream_t s) {
  const unsigned pairs = (unsigned)((int64_t)P.Mmax * (P.Mmax + 1) / 2);
  switch (P.mb) {
    case 32: refine_residual_kernel<32><<<pairs, kRefThreads, 0, s>>>(P, R); break;
    case 64: refine_residual_kernel<64><<<pairs, kRefThreads, 0, s>>>(P, R); break;
    default: refine_residual_kernel<128><<<pairs, kRefThreads, 0, s>>>(P, R); break;
  }
}

void launch_refine_apply(const PencilDesc& P, const RefineDesc& R, hipStream_t s) {
  refine_apply_kernel<<<(unsigned)P.m, kRefThreads, 0, s>>>(P, R);
}

}  // namespace rgev
