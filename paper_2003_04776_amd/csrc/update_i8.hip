// Mixed-precision tile update: the same robust band update as update_tile.hpp (Algorithm 3
// with the scales of Algorithm 2, one ProtectUpdate per column), with the contraction
// [S_kr | T_kr] W_rj emulated on the int8 matrix cores from split operands (slices.hpp):
// for each source of the band and each K step of 64, the slice products with p + q <= 8
// are summed exactly per level L = p + q in int32, and each level is folded into an FP64
// accumulator with the row and column exponents once per source.
//
// A workgroup covers one 32-column group of a target tile (all MB rows): MB/32 waves on
// top of each other, each 32 x 32 (2 x 2 blocks of 16 x 16), two waves per SIMD.  Per K
// step a wave loads the seven A-slice fragments of its rows and, one slice at a time, the
// W-slice fragments of its columns, straight from global memory in the instruction's own
// layout (16 contiguous bytes per lane): the workgroup's waves share the W fragments
// through L1, the column groups of a tile share the A fragments through the XCD's L2
// (they are neighbours in the XCD-blocked order).  Seven int32 level accumulators per
// block take the 28 slice products.
#include <hip/hip_runtime.h>

#include "slices.hpp"
#include "update_tile.hpp"

namespace rgev {

typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4i ld4(const int4* p) {
  const int4 v = *p;
  return v4i{v.x, v.y, v.z, v.w};
}

template <int MB> struct I8Shape {
  static constexpr int WR = MB / 32;             // waves over the rows
  static constexpr int NW = WR;
  static constexpr int COLS = 32;                // columns per workgroup
  static constexpr int NCG = MB / COLS;          // workgroups per tile
};

template <int MB>
__device__ __forceinline__ void update_i8_tile(const PencilDesc& P, const UpdRange& U, int k, int j, int cg) {
  constexpr int WRN = I8Shape<MB>::WR, COLS = I8Shape<MB>::COLS;
  constexpr int KS = slice_ksteps(MB), RBN = MB / 16, CBM = MB / 16;
  constexpr int64_t NPK = slice_packets(MB);
  __shared__ int sfY[COLS], sfA[COLS], seN[COLS];
  __shared__ int sgc[kMaxBand][COLS];
  __shared__ double red[WRN][COLS];

  const int M = P.ctrl->M;
  const int64_t m = P.m;
  const int k0 = P.edges[k], hk = P.edges[k + 1] - k0;
  const int c0 = P.edges[j], hj = P.edges[j + 1] - c0;
  const int g0 = COLS * cg;               // first column of the workgroup inside tile j
  if (g0 >= hj) return;
  const int s_end = min(min(U.s_hi, M - 1), j);
  const int ns = s_end - U.s_lo + 1;
  const bool first = (j <= U.s_hi);
  const int tid = threadIdx.x;
  const int lane = tid % 64, li = lane % 16, lk = lane / 16;
  const int wave = tid / 64;               // row group of this wave
  const int n0 = g0;

  if (tid < COLS) {
    const int n = g0 + tid;
    int fy = 0, fa = 0, en = 0;
    int g[kMaxBand] = {};
    if (n < hj) band_column_scales(P, U, k, c0 + n, first, ns, fy, fa, en, g);
    sfY[tid] = fy;
    sfA[tid] = fa;
    seN[tid] = en;
#pragma unroll
    for (int i = 0; i < kMaxBand; ++i) sgc[i][tid] = g[i];
  }
  __syncthreads();

  // lane's outputs: rows 32 wave + 16 a + li, columns n0 + 16 q + 4 lk + v (a, q, v = 0..1, 0..1, 0..3)
  double acc[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[a][q][v] = 0.0;
  v4i lev[kSliceLevels][2][2];
  auto clear_levels = [&]() {
#pragma unroll
    for (int L = 0; L < kSliceLevels; ++L)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int q = 0; q < 2; ++q) lev[L][a][q] = v4i{0, 0, 0, 0};
  };

  // step t = (source si = t / KS, K step ks = t % KS)
  const int nsteps = ns * KS;
  auto load_a = [&](int t, v4i (&af)[kSlices][2]) {
    const int si = t / KS, ks = t % KS;
    const int s = U.s_lo + si;
    const int4* Ab = P.Aslc + pair_index(k, s) * kSlices * NPK + ((int64_t)ks * RBN + 2 * wave) * 64 + lane;
#pragma unroll
    for (int p = 0; p < kSlices; ++p)
#pragma unroll
      for (int a = 0; a < 2; ++a) af[p][a] = ld4(Ab + (int64_t)p * NPK + a * 64);
  };
  // operands swapped: the product is (A W)^T, so a lane holds one row, four columns
  auto mma = [&](const v4i (&af)[kSlices][2], int t) {
    const int si = t / KS, ks = t % KS;
    const int s = U.s_lo + si;
    const int4* Wb = P.Wslc + ((int64_t)(s % P.wslots) * P.Mmax + j) * kSlices * NPK +
                     ((int64_t)ks * CBM + n0 / 16) * 64 + lane;
#pragma unroll
    for (int qq = 0; qq < kSlices; ++qq) {
      v4i wf[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) wf[q] = ld4(Wb + (int64_t)qq * NPK + q * 64);
#pragma unroll
      for (int pp = 0; pp + qq < kSliceLevels; ++pp)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int q = 0; q < 2; ++q)
            lev[pp + qq][a][q] = __builtin_amdgcn_mfma_i32_16x16x64_i8(wf[q], af[pp][a], lev[pp + qq][a][q], 0, 0, 0);
    }
  };
  // fold: 2^(eA + eW + g) sum_L 2^(-7 (L + 2)) level_L  (each level term is exact in FP64)
  auto fold = [&](int si) {
    const int s = U.s_lo + si;
    const int64_t pair = pair_index(k, s);
    const int slot = s % P.wslots;
    int ea[2], ew[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a) ea[a] = P.Aexp[pair * MB + 32 * wave + 16 * a + li];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int nl = 16 * q + 4 * lk + v;
        ew[q][v] = (n0 + nl < hj) ? P.Wexp[(int64_t)slot * m + c0 + n0 + nl] + sgc[si][nl] : 0;
      }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double t = 0.0;
#pragma unroll
          for (int L = kSliceLevels - 1; L >= 0; --L) t += ldexp((double)lev[L][a][q][v], -7 * (L + 2));
          acc[a][q][v] += ldexp(t, ea[a] + ew[q][v]);
        }
  };

  // A fragments double-buffered in registers (the next step's load is in flight during this
  // step's products); W fragments (shared with the workgroup's other waves, mostly L1 hits)
  // are loaded at the start of their step
  clear_levels();
  for (int t = 0; t < nsteps; ++t) {
    v4i af[kSlices][2];
    load_a(t, af);
    mma(af, t);
    if ((t + 1) % KS == 0) {
      fold(t / KS);
      clear_levels();
    }
  }

  // ---- epilogue: Y <- 2^fY Y - 2^fA acc and the new segment norms ----
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int nl = 16 * q + 4 * lk + v, n = n0 + nl, ng = nl;
      double cmx = 0.0;
      if (n < hj) {
        const int fy = sfY[ng], fa = sfA[ng];
        double* zc = P.Z + (k0 + 32 * wave + li) + (int64_t)(c0 + n) * P.ldz;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const int i = 32 * wave + 16 * a + li;
          if (i < hk) {
            const double yo = first ? 0.0 : zc[16 * a];
            const double yn = ldexp(yo, fy) - ldexp(acc[a][q][v], fa);
            zc[16 * a] = yn;
            cmx = fmax(cmx, fabs(yn));
          }
        }
      }
      cmx = fmax(cmx, __shfl_xor(cmx, 1));
      cmx = fmax(cmx, __shfl_xor(cmx, 2));
      cmx = fmax(cmx, __shfl_xor(cmx, 4));
      cmx = fmax(cmx, __shfl_xor(cmx, 8));
      if (li == 0) red[wave][ng] = cmx;
    }
  __syncthreads();
  if (tid < COLS && g0 + tid < hj) {
    const int64_t c = c0 + g0 + tid;
    double nx = red[0][tid];
#pragma unroll
    for (int w = 1; w < WRN; ++w) nx = fmax(nx, red[w][tid]);
    P.exps[(int64_t)k * m + c] = seN[tid];
    P.norms[(int64_t)k * m + c] = nx;
  }
}

// two waves per SIMD
template <int MB>
__global__ __launch_bounds__(64 * I8Shape<MB>::NW, 2)
void update_i8_kernel(PencilDesc P, UpdRange U) {
  constexpr int NCG = I8Shape<MB>::NCG;   // workgroups per tile
  const int M = P.ctrl->M;
  if (U.j_lo >= M || U.k_hi <= U.k_lo || U.s_lo >= M) return;
  const int nk = U.k_hi - U.k_lo, nj = M - U.j_lo;
  const int nbk = (nk + 7) / 8, nbj = (nj + 7) / 8;
  const int per = (int)(gridDim.x / 8);
  const int idx = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  const int cg = idx % NCG, t = idx / NCG;
  if (t >= nbk * nbj * 64) return;
  const int blk = t / 64, w64 = t % 64;
  const int k = U.k_lo + 8 * (blk % nbk) + (w64 % 8);
  const int j = U.j_lo + 8 * (blk / nbk) + (w64 / 8);
  if (k >= U.k_hi || j >= M) return;
  update_i8_tile<MB>(P, U, k, j, cg);
}

void launch_update_i8(const PencilDesc& P, const UpdRange& U, hipStream_t s) {
  const int64_t nbk = (U.k_hi - U.k_lo + 7) / 8, nbj = (P.Mmax - U.j_lo + 7) / 8;
  switch (P.mb) {
    case 32:
      update_i8_kernel<32><<<(unsigned)(nbk * nbj * 64 * I8Shape<32>::NCG), 64 * I8Shape<32>::NW, 0, s>>>(P, U);
      break;
    case 64:
      update_i8_kernel<64><<<(unsigned)(nbk * nbj * 64 * I8Shape<64>::NCG), 64 * I8Shape<64>::NW, 0, s>>>(P, U);
      break;
    default:
      update_i8_kernel<128><<<(unsigned)(nbk * nbj * 64 * I8Shape<128>::NCG), 64 * I8Shape<128>::NW, 0, s>>>(P, U);
      break;
  }
}

}  // namespace rgev
