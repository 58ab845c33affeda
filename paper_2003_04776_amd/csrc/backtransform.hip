// Back-transformation: the eigenvectors of the original pencil from those of its Schur
// form.  With the real Schur decomposition S = U^T A V, T = U^T B V of the introduction
// (Section 1; U, V orthogonal), S z = lambda T z gives A (V z) = U S z = lambda U T z =
// lambda B (V z), so the eigenvectors of (A, B) are X = V Z (the introduction writes U z;
// it is V z that satisfies the equation).
//
// Z (the output of the eigenvector solve) is upper quasi-triangular: column c has
// non-zeros in rows 0 .. c, and row c + 1 too when c is the first column of a complex
// pair.  The product is a dense-times-triangular contraction on the FP64 matrix cores:
// output tile (I, J) sums V_{I,K} Z_{K,J} over the rows K that column tile J reaches.
// Every column keeps a power-of-two exponent: 2^xs[c] X_c = V (2^scales[c] Z_c), with
// Z_c scaled down by 2^-q_c (exact) before the product when m max|V| max|Z_c| could
// exceed Omega, so no partial sum overflows.  With normalisation each eigenvector is
// divided by max_i |x_i| (real) or max_i |x_i| + |y_i| (complex pair) and xs = 0.
//
// Kernels, in stream order: a scan (block structure from S's sub-diagonal, column maxima
// of Z, the maximum of |V|), a pack of Z into the matrix-core operand order (scaled, the
// entries below the quasi-diagonal written as zeros), the contraction, and a finishing
// pass (normalisation or exponents).  Z is fully packed before X is written, so X may be
// Z itself.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "back.hpp"
#include "robust.hpp"

namespace rgev {

typedef double bd4 __attribute__((ext_vector_type(4)));

constexpr int kBackScanThreads = 256;

// ---- scan: one workgroup per column ----
__global__ __launch_bounds__(kBackScanThreads) void back_scan_kernel(BackDesc B) {
  const int64_t m = B.m;
  const int64_t c = blockIdx.x;
  const int tid = threadIdx.x;
  __shared__ double red[2][kBackScanThreads / 64];
  const bool first = c + 1 < m && B.S[(c + 1) + c * B.lds] != 0.0;
  if (tid == 0) {
    const bool second = c > 0 && B.S[c + (c - 1) * B.lds] != 0.0;
    B.blk[c] = first ? 1 : (second ? 2 : 0);
  }
  const int64_t zrows = first ? c + 2 : c + 1;   // rows 0 .. c (and c + 1 for a pair's first column)
  double zm = 0.0, vm = 0.0;
  for (int64_t i = tid; i < zrows; i += kBackScanThreads) {
    const double z = fabs(B.Z[i + c * B.ldz]);
    zm = (z != z || zm != zm) ? z + zm : fmax(zm, z);   // a NaN propagates
  }
  for (int64_t i = tid; i < m; i += kBackScanThreads) {
    const double v = fabs(B.V[i + c * B.ldv]);
    vm = (v != v || vm != vm) ? v + vm : fmax(vm, v);   // a NaN propagates
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double y = __shfl_xor(zm, o);
    zm = (y != y || zm != zm) ? y + zm : fmax(zm, y);
    const double w = __shfl_xor(vm, o);
    vm = (w != w || vm != vm) ? w + vm : fmax(vm, w);
  }
  if (tid % 64 == 0) {
    red[0][tid / 64] = zm;
    red[1][tid / 64] = vm;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < kBackScanThreads / 64; ++w) {
      const double y = red[0][w];
      zm = (y != y || zm != zm) ? y + zm : fmax(zm, y);
      const double x = red[1][w];
      vm = (x != x || vm != vm) ? x + vm : fmax(vm, x);
    }
    if (!(vm <= 1.7976931348623157e308) || !(zm <= 1.7976931348623157e308)) {
      atomicOr(B.info, kBackInfoNonFinite);
      vm = fmin(vm, 1.7976931348623157e308);   // (NaN -> the largest double)
      zm = fmin(zm, 1.7976931348623157e308);
    }
    B.zmax[c] = zm;
    // the bits of non-negative doubles order as the values do
    atomicMax(B.vmax, (unsigned long long)__double_as_longlong(vm));
  }
}

// exponent q >= 0 with m max|V| max|Z_c| 2^-q < 2^(Omega exponent - 1): every partial sum of
// V (2^-q Z_c) stays below Omega
__device__ __forceinline__ int back_scale(int64_t m, double vmax, double zmax) {
  if (vmax == 0.0 || zmax == 0.0) return 0;
  int ev, ez;
  frexp(vmax, &ev);   // vmax < 2^ev
  frexp(zmax, &ez);
  int em = 0;
  while (((int64_t)1 << em) < m) ++em;   // m <= 2^em
  const int q = em + ev + ez - kOmegaExp + 1;
  return q > 0 ? q : 0;
}

// the exponent shared by the column(s) of the eigenvector that column c belongs to
__device__ __forceinline__ int back_column_q(const BackDesc& B, int64_t c, double vmax) {
  const int kind = B.blk[c];
  const int64_t p = kind == 2 ? c - 1 : c;
  double zm = B.zmax[p];
  if (B.blk[p] == 1 && p + 1 < B.m) zm = fmax(zm, B.zmax[p + 1]);
  return back_scale(B.m, vmax, zm);
}

// ---- pack: Z tile column J into operand order [step][column block][lane] ----
// element (t, cb, l) = 2^-q_c Z[4 t + l / 16][c], c = mb J + 16 cb + l % 16, zero below the
// quasi-diagonal and past the matrix.  grid (steps / 4 rounded up, tile columns); a
// workgroup of 256 threads writes 4 steps.
__global__ __launch_bounds__(256) void back_pack_kernel(BackDesc B) {
  const int J = blockIdx.y;
  const int mb = B.mb;
  const int64_t m = B.m;
  const int steps = back_steps(m, mb, J);
  const int per_step = 4 * mb;                  // (mb / 16) blocks x 64 lanes
  const double vmax = __longlong_as_double((long long)*B.vmax);
  double* out = B.Zp + back_tile_offset(mb, J);
  for (int e = threadIdx.x; e < 4 * per_step; e += 256) {
    const int t = blockIdx.x * 4 + e / per_step;
    if (t >= steps) break;
    const int r = e % per_step, cb = r / 64, l = r % 64;
    const int64_t row = 4 * (int64_t)t + l / 16;
    const int64_t c = (int64_t)mb * J + 16 * cb + l % 16;
    double v = 0.0;
    if (c < m && row < m) {
      const int64_t last = (B.blk[c] == 1) ? c + 1 : c;   // last row of column c
      if (row <= last) v = ldexp(B.Z[row + c * B.ldz], -back_column_q(B, c, vmax));
    }
    out[(int64_t)t * per_step + r] = v;
  }
}

// ---- contraction: X tile (I, J) = V_{I, 0:K_J} Zp_J ----
// One workgroup (2 x 2 waves) per output tile; each wave streams its matrix-core fragments
// straight from global memory into registers (A from column-major V: four 128-byte lines
// per fragment; B from the packed Z: one 512-byte run), three register slots rotating so
// the loads of step t + 2 are in flight while step t runs.  Every load is unconditional
// (past the last step the loader repeats it; those steps are multiplied by zero), so a
// wave waits only for the slot it is about to use.  Operands are swapped so that a lane's
// four accumulators are one row of four columns of X.  Tiles go to the XCDs in 8 x 8
// blocks (the 64 workgroups an XCD holds at once share 8 row and 8 column panels in its
// L2), blocks dealt round-robin over the XCDs from the longest column tiles down.
template <int MB>
__global__ __launch_bounds__(256, 2) void back_gemm_kernel(BackDesc B) {
  constexpr int WR = MB / 2, WC = MB / 2;
  constexpr int RB = WR / 16, CB = WC / 16;
  constexpr int NS = 3;
  const int64_t m = B.m;
  const int nt = B.nt;
  const int nb = (nt + 7) / 8;
  const int xcd = (int)(blockIdx.x % 8), local = (int)(blockIdx.x / 8);
  const int g = (local / 64) * 8 + xcd, w64 = local % 64;
  if (g >= nb * nb) return;
  const int I = 8 * (g % nb) + w64 % 8;
  const int J = 8 * (nb - 1 - g / nb) + w64 / 8;
  if (I >= nt || J >= nt) return;

  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wr = wave / 2, wc = wave % 2;
  const int li = lane % 16, lk = lane / 16;
  const int64_t r0 = (int64_t)MB * I, c0 = (int64_t)MB * J;
  const int hi = (int)(m - r0 < MB ? m - r0 : MB), hj = (int)(m - c0 < MB ? m - c0 : MB);
  const int nst = back_steps(m, MB, J);
  const double* zp = B.Zp + back_tile_offset(MB, J) + (CB * wc) * 64 + lane;

  int64_t rowA[RB];
#pragma unroll
  for (int a = 0; a < RB; ++a) {
    const int64_t r = r0 + WR * wr + 16 * a + li;
    rowA[a] = r < m ? r : m - 1;
  }
  int ls = 0;   // next step to load
  auto load = [&](double (&af)[RB], double (&bf)[CB]) {
    const int64_t col = 4 * (int64_t)ls + lk < m ? 4 * (int64_t)ls + lk : m - 1;
    const double* colp = B.V + col * B.ldv;
#pragma unroll
    for (int a = 0; a < RB; ++a) af[a] = colp[rowA[a]];
    const double* wp = zp + (int64_t)ls * (4 * MB);
#pragma unroll
    for (int q = 0; q < CB; ++q) bf[q] = wp[q * 64];
    if (ls + 1 < nst) ++ls;
  };
  bd4 acc[RB][CB];
#pragma unroll
  for (int a = 0; a < RB; ++a)
#pragma unroll
    for (int q = 0; q < CB; ++q) acc[a][q] = bd4{0.0, 0.0, 0.0, 0.0};
  auto use = [&](double (&af)[RB], double (&bf)[CB], bool live) {
    if (!live) {
#pragma unroll
      for (int q = 0; q < CB; ++q) bf[q] = 0.0;
    }
#pragma unroll
    for (int a = 0; a < RB; ++a)
#pragma unroll
      for (int q = 0; q < CB; ++q)
        acc[a][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[q], af[a], acc[a][q], 0, 0, 0);
  };
  double af[NS][RB], bf[NS][CB];
  const int nrun = (nst + NS - 1) / NS * NS;
#pragma unroll
  for (int u = 0; u < NS - 1; ++u) load(af[u], bf[u]);
  for (int t0 = 0; t0 < nrun; t0 += NS) {
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      load(af[(u + NS - 1) % NS], bf[(u + NS - 1) % NS]);
      use(af[u], bf[u], t0 + u < nst);
    }
  }
  // lane: row 16 a + li of the wave's rows, columns 16 q + lk + 4 v of its columns
#pragma unroll
  for (int q = 0; q < CB; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int n = WC * wc + 16 * q + lk + 4 * v;
      if (n < hj) {
        double* xc = B.X + (r0 + WR * wr + li) + (c0 + n) * B.ldx;
#pragma unroll
        for (int a = 0; a < RB; ++a)
          if (WR * wr + 16 * a + li < hi) xc[16 * a] = acc[a][q][v];
      }
    }
}

// ---- finish: one workgroup per eigenvector (the second column of a pair exits) ----
__global__ __launch_bounds__(kBackScanThreads) void back_finish_kernel(BackDesc B) {
  const int64_t m = B.m;
  const int64_t c = blockIdx.x;
  const int kind = B.blk[c];
  if (kind == 2) return;
  const bool pair = kind == 1 && c + 1 < m;
  const int tid = threadIdx.x;
  if (!B.normalize) {
    if (tid == 0) {
      const double vmax = __longlong_as_double((long long)*B.vmax);
      const int xs = (B.scales ? B.scales[c] : 0) + back_column_q(B, c, vmax);
      B.xscales[c] = xs;
      if (pair) B.xscales[c + 1] = xs;
    }
    return;
  }
  __shared__ double red[kBackScanThreads / 64];
  double* x = B.X + c * B.ldx;
  double* y = pair ? x + B.ldx : nullptr;
  double t = 0.0;
  for (int64_t i = tid; i < m; i += kBackScanThreads) t = fmax(t, fabs(x[i]) + (pair ? fabs(y[i]) : 0.0));
  for (int o = 32; o > 0; o >>= 1) t = fmax(t, __shfl_xor(t, o));
  if (tid % 64 == 0) red[tid / 64] = t;
  __syncthreads();
  t = red[0];
  for (int w = 1; w < kBackScanThreads / 64; ++w) t = fmax(t, red[w]);
  if (t > 0.0) {
    for (int64_t i = tid; i < m; i += kBackScanThreads) {
      x[i] = x[i] / t;
      if (pair) y[i] = y[i] / t;
    }
  }
  if (tid == 0) {
    B.xscales[c] = 0;
    if (pair) B.xscales[c + 1] = 0;
  }
}

__global__ void back_reset_kernel(BackDesc B) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *B.vmax = 0ull;
    *B.info = 0;
  }
}

void launch_backtransform(const BackDesc& B, hipStream_t s) {
  const int64_t m = B.m;
  back_reset_kernel<<<1, 64, 0, s>>>(B);
  back_scan_kernel<<<(unsigned)m, kBackScanThreads, 0, s>>>(B);
  const int max_steps = back_steps(m, B.mb, B.nt - 1);
  back_pack_kernel<<<dim3((unsigned)((max_steps + 3) / 4), (unsigned)B.nt), 256, 0, s>>>(B);
  const int nb = (B.nt + 7) / 8;
  const unsigned grid = (unsigned)((nb * nb + 7) / 8) * 8 * 64;
  if (B.mb == 64)
    back_gemm_kernel<64><<<grid, 256, 0, s>>>(B);
  else
    back_gemm_kernel<128><<<grid, 256, 0, s>>>(B);
  back_finish_kernel<<<(unsigned)m, kBackScanThreads, 0, s>>>(B);
}

}  // namespace rgev
