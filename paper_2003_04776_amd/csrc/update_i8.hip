// Mixed-precision tile update: the same robust band update as update_tile.hpp (Algorithm 3
// with the scales of Algorithm 2, one ProtectUpdate per column), with the contraction
// [S_kr | T_kr] W_rj emulated on the int8 matrix cores from split operands (slices.hpp):
// for each source of the band and each K step of 64, the slice products with p + q <= 8
// are summed exactly per level L = p + q in int32, and each level is folded into an FP64
// accumulator with the row and column exponents once per source.
//
// A workgroup covers one 32-column group of a target tile (all MB rows): MB/32 waves on
// top of each other, each 32 x 32 (2 x 2 blocks of 16 x 16), two waves per SIMD.  Per K
// step of 64 the 14 W fragments of the group's columns (7 slices x 2 column blocks, 1 KB
// each) go straight from global memory into one of two LDS stages, shared by the waves;
// each wave keeps its 14 A fragments of the step, and those of the next step, in registers
// (loaded in the instruction's own layout, 16 contiguous bytes per lane; the column groups
// of a tile share them through the XCD's L2).  Seven int32 level accumulators per block
// take the 28 slice products; the FP64 accumulators sit in LDS, folded into once per source.
#include <hip/hip_runtime.h>

#include "slices.hpp"
#include "update_tile.hpp"

namespace rgev {

typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4i ld4(const int4* p) {
  const int4 v = *p;
  return v4i{v.x, v.y, v.z, v.w};
}

// 16 bytes a lane straight from global memory into LDS: the wave's 1 KB lands contiguously
// at lds (wave-uniform) + 16 lane
__device__ __forceinline__ void lds_load16(const int4* g, void* lds) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)g,
                                   (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}
// wait until every load of this wave has landed (vmcnt 0; expcnt and lgkmcnt untouched)
__device__ __forceinline__ void wait_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }

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
  static_assert(KS % 2 == 0, "the A fragments alternate between two buffers per K step");
  constexpr int64_t NPK = slice_packets(MB);
  __shared__ int sfY[COLS], sfA[COLS], seN[COLS];
  __shared__ int sgc[kMaxBand][COLS];
  __shared__ double red[WRN][COLS];
  // FP64 accumulators of the waves (kept out of registers, which hold the int32 levels
  // and two K steps of A fragments): [wave][a][q][v][lane]
  __shared__ double accs[WRN][2 * 2 * 4 * 64];
  // W fragments of one K step for the workgroup's 32 columns, shared by its waves, in two
  // stages: [stage][slice][column block][lane]
  __shared__ int4 Wst[2][kSlices][2][64];
  constexpr int NW = I8Shape<MB>::NW;

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
  double* acw = accs[wave];
#pragma unroll
  for (int e = 0; e < 16; ++e) acw[e * 64 + lane] = 0.0;
  __syncthreads();

  v4i lev[kSliceLevels][2][2];
  auto clear_levels = [&]() {
#pragma unroll
    for (int L = 0; L < kSliceLevels; ++L)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int q = 0; q < 2; ++q) lev[L][a][q] = v4i{0, 0, 0, 0};
  };

  // fragment addresses of source si, K step ks (the loads past the band's last step repeat
  // it, so every load is unconditional)
  auto a_ptr = [&](int si, int ks) {
    return P.Aslc + pair_index(k, U.s_lo + si) * kSlices * NPK + ((int64_t)ks * RBN + 2 * wave) * 64 + lane;
  };
  auto w_ptr = [&](int si, int ks) {
    return P.Wslc + ((int64_t)((U.s_lo + si) % P.wslots) * P.Mmax + j) * kSlices * NPK +
           ((int64_t)ks * CBM + n0 / 16) * 64 + lane;
  };
  auto load_a = [&](const int4* Ab, v4i (&af)[kSlices][2]) {
#pragma unroll
    for (int p = 0; p < kSlices; ++p)
#pragma unroll
      for (int a = 0; a < 2; ++a) af[p][a] = ld4(Ab + (int64_t)p * NPK + a * 64);
  };
  // the step's 14 W packets (7 slices x 2 column blocks, 1 KB each) straight into stage st,
  // shared out among the waves
  auto issue_w = [&](const int4* Wb, int st) {
    for (int u = wave; u < 2 * kSlices; u += NW) {
      const int qq = u / 2, q = u % 2;
      lds_load16(Wb + (int64_t)qq * NPK + q * 64, &Wst[st][qq][q][0]);
    }
  };
  // one K step from stage st; operands swapped so a lane holds one row, four columns
  auto step = [&](const v4i (&af)[kSlices][2], int st) {
#pragma unroll
    for (int qq = 0; qq < kSlices; ++qq) {
      v4i wf[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) wf[q] = ld4(&Wst[st][qq][q][lane]);
#pragma unroll
      for (int pp = 0; pp + qq < kSliceLevels; ++pp)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int q = 0; q < 2; ++q)
            lev[pp + qq][a][q] = __builtin_amdgcn_mfma_i32_16x16x64_i8(wf[q], af[pp][a], lev[pp + qq][a][q], 0, 0, 0);
    }
  };
  // fold: acc += 2^(eA + eW + g) sum_L 2^(-7 (L + 2)) level_L  (each level term is exact in FP64)
  auto fold = [&](const int (&ea)[2], const int (&ew)[2][4]) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double t = 0.0;
#pragma unroll
          for (int L = kSliceLevels - 1; L >= 0; --L) t += ldexp((double)lev[L][a][q][v], -7 * (L + 2));
          double& ac = acw[((a * 2 + q) * 4 + v) * 64 + lane];
          ac += ldexp(t, ea[a] + ew[q][v]);
        }
  };
  auto load_exps = [&](int si, int (&ea)[2], int (&ew)[2][4]) {
    const int s = U.s_lo + si;
    const int64_t pair = pair_index(k, s);
    const int slot = s % P.wslots;
#pragma unroll
    for (int a = 0; a < 2; ++a) ea[a] = P.Aexp[pair * MB + 32 * wave + 16 * a + li];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int nl = 16 * q + 4 * lk + v;
        ew[q][v] = P.Wexp[(int64_t)slot * m + c0 + min(n0 + nl, hj - 1)];   // columns past the tile: never stored
      }
  };

  // A fragments double-buffered in registers, W in two LDS stages: the loads of step t + 1
  // (every one unconditional: past the band's last step they repeat it) are in flight while
  // the matrix cores run step t; one barrier per step
  v4i aA[kSlices][2], aB[kSlices][2];
  load_a(a_ptr(0, 0), aA);
  issue_w(w_ptr(0, 0), 0);
  wait_loads();
  __syncthreads();
  for (int si = 0; si < ns; ++si) {
    int ea[2], ew[2][4];
    load_exps(si, ea, ew);
    clear_levels();
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const bool last_ks = ks + 1 == KS;
      const int nsi = last_ks ? (si + 1 < ns ? si + 1 : si) : si;
      const int nks = last_ks ? (si + 1 < ns ? 0 : ks) : ks + 1;
      issue_w(w_ptr(nsi, nks), (ks + 1) % 2);   // stage left by every wave at the last barrier
      if (ks % 2 == 0) {
        load_a(a_ptr(nsi, nks), aB);
        step(aA, 0);
      } else {
        load_a(a_ptr(nsi, nks), aA);
        step(aB, 1);
      }
      wait_loads();
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) ew[q][v] += sgc[si][16 * q + 4 * lk + v];
    fold(ea, ew);
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
            const double yn = ldexp(yo, fy) - ldexp(acw[((a * 2 + q) * 4 + v) * 64 + lane], fa);
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
