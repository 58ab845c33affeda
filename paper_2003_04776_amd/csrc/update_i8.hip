// Mixed-precision tile update: the same robust band update as update_tile.hpp (Algorithm 3
// with the scales of Algorithm 2, one ProtectUpdate per column), with the contraction
// [S_kr | T_kr] W_rj emulated on the int8 matrix cores from split operands (slices.hpp):
// for each source of the band and each K step of 64, the slice products with p + q <= 8
// are summed exactly per level L = p + q in int32, and each level is folded into an FP64
// accumulator with the row and column exponents once per source.
//
// A workgroup covers a 32-column group and a row group of up to 64 rows of a target tile:
// its (up to) four waves each hold 16 rows x 32 columns (2 blocks of 16 x 16), so the seven
// int32 level accumulators take 56 registers, the two K steps of A fragments in flight
// another 56, the FP64 accumulators 16, and three waves fit on a SIMD.  Per K step of 64 the
// 14 W fragments of the group's columns (7 slices x 2 column blocks, 1 KB each) go straight
// from global memory into one of two LDS stages, shared by the waves; each wave loads its 7
// A fragments of the next step into registers (the instruction's own layout, 16 contiguous
// bytes per lane; the column groups of a tile share them through the XCD's L2).  When a
// tile has several row groups (mb = 128), their column norms meet in an atomic maximum and
// are published after the launch (publish_kernel).
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
// 2^(-7 n) as a compile-time constant (n <= 9)
__device__ __forceinline__ constexpr double exp2_neg7(int n) {
  double r = 1.0;
  for (int i = 0; i < n; ++i) r *= 1.0 / 128.0;
  return r;
}

template <int MB> struct I8Shape {
  static constexpr int NW = MB / 16 < 4 ? MB / 16 : 4;   // waves (16 rows each)
  static constexpr int ROWS = 16 * NW;                   // rows per workgroup
  static constexpr int NRG = MB / ROWS;                  // row groups per tile
  static constexpr int COLS = 32;                        // columns per workgroup
  static constexpr int NCG = MB / COLS;                  // column groups per tile
};

template <int MB>
__device__ __forceinline__ void update_i8_tile(const PencilDesc& P, const UpdRange& U, int k, int j, int cg,
                                               int rg) {
  constexpr int NW = I8Shape<MB>::NW, COLS = I8Shape<MB>::COLS;
  constexpr int NRG = I8Shape<MB>::NRG;
  constexpr int KS = slice_ksteps(MB), RBN = MB / 16, CBM = MB / 16;
  static_assert(KS % 2 == 0, "the A fragments alternate between two buffers per K step");
  constexpr int64_t NPK = slice_packets(MB);
  __shared__ int sfY[COLS], sfA[COLS], seN[COLS];
  __shared__ int sgc[kMaxBand][COLS];
  __shared__ double red[NW][COLS];
  // W fragments of one K step for the workgroup's 32 columns, shared by its waves, in two
  // stages: [stage][slice][column block][lane]
  __shared__ int4 Wst[2][kSlices][2][64];

  const int M = P.ctrl->M;
  const int64_t m = P.m;
  const int k0 = P.edges[k], hk = P.edges[k + 1] - k0;
  const int c0 = P.edges[j], hj = P.edges[j + 1] - c0;
  const int g0 = COLS * cg;               // first column of the workgroup inside tile j
  if (g0 >= hj) return;
  const int s_end = min(min(U.s_hi, M - 1), j);
  const int ns = s_end - U.s_lo + 1;
  const bool first = (j <= U.s_hi) && !P.rhs;   // (correction mode: Y starts as the right-hand side)
  const int tid = threadIdx.x;
  const int lane = tid % 64, li = lane % 16, lk = lane / 16;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int rb = rg * NW + wave;           // the wave's row block (16 rows) in the tile
  const int n0 = g0;

  // lane's outputs: row 16 rb + li, columns n0 + 16 q + 4 lk + v (q = 0..1, v = 0..3)
  double acc[2][4];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[q][v] = 0.0;
  v4i lev[kSliceLevels][2];
  auto clear_levels = [&]() {
#pragma unroll
    for (int L = 0; L < kSliceLevels; ++L)
#pragma unroll
      for (int q = 0; q < 2; ++q) lev[L][q] = v4i{0, 0, 0, 0};
  };

  // fragment addresses of source si, K step ks (the loads past the band's last step repeat
  // it, so every load is unconditional); A as a uniform base plus the lane's offset
  auto a_ptr = [&](int si, int ks) {
    return P.Aslc + pair_index(k, U.s_lo + si) * kSlices * NPK + ((int64_t)ks * RBN + rb) * 64;
  };
  auto w_ptr = [&](int si, int ks) {
    return P.Wslc + ((int64_t)((U.s_lo + si) % P.wslots) * P.Mmax + j) * kSlices * NPK +
           ((int64_t)ks * CBM + n0 / 16) * 64 + lane;
  };
  auto load_a = [&](const int4* Ab, v4i (&af)[kSlices]) {
#pragma unroll
    for (int p = 0; p < kSlices; ++p) af[p] = ld4(Ab + ((int64_t)p * NPK + lane));
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
  auto step = [&](const v4i (&af)[kSlices], int st) {
#pragma unroll
    for (int qq = 0; qq < kSlices; ++qq) {
      v4i wf[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) wf[q] = ld4(&Wst[st][qq][q][lane]);
#pragma unroll
      for (int pp = 0; pp + qq < kSliceLevels; ++pp)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          lev[pp + qq][q] = __builtin_amdgcn_mfma_i32_16x16x64_i8(wf[q], af[pp], lev[pp + qq][q], 0, 0, 0);
    }
  };
  // fold: acc += 2^(eA + eW + g) sum_L 2^(-7 (L + 2)) level_L  (each level term is exact in
  // FP64; an fma by an exact power of two rounds as the addition of the exact term)
  auto fold = [&](int ea, const int (&ew)[2][4]) {
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double t = 0.0;
#pragma unroll
        for (int L = kSliceLevels - 1; L >= 0; --L) t = fma((double)lev[L][q][v], exp2_neg7(L + 2), t);
        acc[q][v] += ldexp(t, ea + ew[q][v]);
      }
  };
  auto load_exps = [&](int si, int& ea, int (&ew)[2][4]) {
    const int s = U.s_lo + si;
    const int64_t pair = pair_index(k, s);
    const int slot = s % P.wslots;
    ea = P.Aexp[pair * MB + 16 * rb + li];
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
  // (the first step's loads are issued before the per-column scales are computed, so their
  // latency and that of the scales' loads overlap)
  v4i aA[kSlices], aB[kSlices];
  load_a(a_ptr(0, 0), aA);
  issue_w(w_ptr(0, 0), 0);
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

  wait_loads();
  __syncthreads();   // also publishes the per-column scales
  for (int si = 0; si < ns; ++si) {
    int ea, ew[2][4];
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
  // (the lane's old Y is loaded at once, from addresses clamped into the tile, so the
  // epilogue waits for memory once; only the stores are masked)
  const int i = 16 * rb + li;            // the lane's row in the tile
  double yo[2][4];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int n = min(n0 + 16 * q + 4 * lk + v, hj - 1);
      const double z = P.Z[(k0 + min(i, hk - 1)) + (int64_t)(c0 + n) * P.ldz];   // (unused on a first update)
      yo[q][v] = first ? 0.0 : z;
    }
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int nl = 16 * q + 4 * lk + v, n = n0 + nl;
      double cmx = 0.0;
      if (n < hj && i < hk) {
        const int fy = sfY[nl], fa = sfA[nl];
        double* zc = P.Z + (k0 + i) + (int64_t)(c0 + n) * P.ldz;
        const double yn = ldexp(yo[q][v], fy) - ldexp(acc[q][v], fa);
        *zc = yn;
        cmx = fabs(yn);
      }
      cmx = fmax(cmx, __shfl_xor(cmx, 1));
      cmx = fmax(cmx, __shfl_xor(cmx, 2));
      cmx = fmax(cmx, __shfl_xor(cmx, 4));
      cmx = fmax(cmx, __shfl_xor(cmx, 8));
      if (li == 0) red[wave][nl] = cmx;
    }
  __syncthreads();
  if (tid < COLS && g0 + tid < hj) {
    const int64_t c = c0 + g0 + tid;
    double nx = red[0][tid];
#pragma unroll
    for (int w = 1; w < NW; ++w) nx = fmax(nx, red[w][tid]);
    if (NRG == 1) {
      P.exps[(int64_t)k * m + c] = seN[tid];
      P.norms[(int64_t)k * m + c] = nx;
    } else {
      // other row groups of the tile may still read the old segment: combine, publish later
      P.exps_next[(int64_t)k * m + c] = seN[tid];
      atomicMax(&P.norms_next[(int64_t)k * m + c], (unsigned long long)__double_as_longlong(nx));
    }
  }
}

// up to three waves per SIMD
template <int MB>
__global__ __launch_bounds__(64 * I8Shape<MB>::NW, 3)
void update_i8_kernel(PencilDesc P, UpdRange U) {
  constexpr int NCG = I8Shape<MB>::NCG, NRG = I8Shape<MB>::NRG;   // workgroups per tile
  const int M = P.ctrl->M;
  if (U.j_lo >= M || U.k_hi <= U.k_lo || U.s_lo >= M) return;
  const int nk = U.k_hi - U.k_lo, nj = M - U.j_lo;
  const int nbk = (nk + 7) / 8, nbj = (nj + 7) / 8;
  if (P.rhs) {
    // correction mode: a bounded grid walks the target tiles and skips the tile columns that
    // hold no refined column (so an empty sweep dispatches few workgroups)
    const int total = nbk * nbj * 64 * NCG * NRG;
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
      const int cg = u % NCG, rg = (u / NCG) % NRG, t = u / (NCG * NRG);
      const int blk = t / 64, w64 = t % 64;
      const int k = U.k_lo + 8 * (blk % nbk) + (w64 % 8);
      const int j = U.j_lo + 8 * (blk / nbk) + (w64 / 8);
      if (k >= U.k_hi || j >= M || !P.tflag[j]) continue;
      __syncthreads();   // the previous tile's shared memory is free
      update_i8_tile<MB>(P, U, k, j, cg, rg);
    }
    return;
  }
  const int per = (int)(gridDim.x / 8);
  const int idx = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  const int cg = idx % NCG, rg = (idx / NCG) % NRG, t = idx / (NCG * NRG);
  if (t >= nbk * nbj * 64) return;
  const int blk = t / 64, w64 = t % 64;
  const int k = U.k_lo + 8 * (blk % nbk) + (w64 % 8);
  const int j = U.j_lo + 8 * (blk / nbk) + (w64 / 8);
  if (k >= U.k_hi || j >= M) return;
  update_i8_tile<MB>(P, U, k, j, cg, rg);
}

// After a launch whose tiles had several row groups: the combined segment exponents and
// norms of the launch's tiles become current, and their scratch is cleared for the next.
__global__ void publish_kernel(PencilDesc P, UpdRange U) {
  const int M = P.ctrl->M;
  if (U.j_lo >= M || U.k_hi <= U.k_lo || U.s_lo >= M) return;   // the launch did nothing
  const int k = U.k_lo + (int)blockIdx.y;
  if (k >= U.k_hi || k >= M) return;
  const int64_t m = P.m;
  for (int64_t c = P.edges[U.j_lo] + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < m;
       c += (int64_t)gridDim.x * blockDim.x) {
    if (P.rhs && !P.tflag[P.tileof[c]]) continue;   // (tile column skipped by the launch)
    const int64_t e = (int64_t)k * m + c;
    P.norms[e] = __longlong_as_double((long long)P.norms_next[e]);
    P.exps[e] = P.exps_next[e];
    P.norms_next[e] = 0ull;
  }
}

template <int MB>
static void launch_i8(const PencilDesc& P, const UpdRange& U, hipStream_t s) {
  constexpr int NCG = I8Shape<MB>::NCG, NRG = I8Shape<MB>::NRG;
  const int64_t nbk = (U.k_hi - U.k_lo + 7) / 8, nbj = (P.Mmax - U.j_lo + 7) / 8;
  const int64_t grid = nbk * nbj * 64 * NCG * NRG;
  update_i8_kernel<MB><<<(unsigned)(P.rhs ? std::min<int64_t>(grid, kRhsGrid) : grid), 64 * I8Shape<MB>::NW, 0, s>>>(P, U);
  if (NRG > 1) publish_kernel<<<dim3(16, (unsigned)(U.k_hi - U.k_lo)), 256, 0, s>>>(P, U);
}

void launch_update_i8(const PencilDesc& P, const UpdRange& U, hipStream_t s) {
  switch (P.mb) {
    case 32: launch_i8<32>(P, U, s); break;
    case 64: launch_i8<64>(P, U, s); break;
    default: launch_i8<128>(P, U, s); break;
  }
}

}  // namespace rgev
