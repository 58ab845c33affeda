// Robust tile update of Algorithm 1 (Section 3, kernel 2):
//     Y_kj <- Y_kj - (S_kr X D_jj - T_kr X B_jj),   X = Y_rj already solved,
// done as one dense contraction [S_kr | T_kr] * W on the FP64 matrix cores, with
// W = 2^-g [X D ; -X B] formed once per solved tile by the solve kernel (Algorithm 2
// with a scale that bounds each W segment by one).  The left update is Algorithm 3
// (Section 4): both operands are brought to a common scale, ProtectUpdate bounds the
// result by Omega, and the scale of X is applied to the product instead of to X
// itself (the product is bounded by the tile norm nu because |W| <= 1, so it cannot
// overflow), which leaves X untouched for the other tiles that read it.
//
// One workgroup per target tile (k, j); wave w owns columns [32w, 32w + 32) of the
// tile and all of its rows: 16x16x4 FP64 MFMA blocks, MB/16 row blocks by 2 column
// blocks, accumulators in registers, operands streamed straight from L2/HBM with the
// next K step prefetched.  Each wave owns whole segments, so the new segment norms
// need no cross-wave reduction.
#include <hip/hip_runtime.h>

#include "layout.hpp"
#include "robust.hpp"

namespace rgev {

typedef double d4 __attribute__((ext_vector_type(4)));

template <int MB>
__global__ __launch_bounds__(MB * 2) void update_kernel(PencilDesc P, int r) {
  constexpr int RB = MB / 16;    // row blocks
  constexpr int CBM = MB / 16;   // column blocks of a W tile
  const int M = P.ctrl->M;
  if (r >= M || r == 0) return;
  const int ntiles = r * (M - r);
  // XCD-aware order: workgroup b runs on XCD b % 8; give each XCD a contiguous range
  // of tiles (k fastest) so the W tile of a column and neighbouring S/T tiles stay in
  // that XCD's L2.  The grid is a multiple of 8, so this is a bijection.
  const int per = (int)(gridDim.x / 8);
  const int t = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (t >= ntiles) return;
  const int k = t % r;
  const int j = r + t / r;
  const int64_t m = P.m;
  const int k0 = P.edges[k], hk = P.edges[k + 1] - k0;
  const int r0 = P.edges[r], hr = P.edges[r + 1] - r0;
  const int c0 = P.edges[j], hj = P.edges[j + 1] - c0;
  const bool first = (j == r);   // the first update of (k, j): Y is still zero
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int li = lane % 16, lk = lane / 16;

  // ---- per-column scales (Algorithm 3): common exponent, ProtectUpdate ----
  const double nu = P.nu[(int64_t)k * P.Mmax + r];
  int fY[2], fA[2], eN[2];
  bool colok[2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int n = 32 * wave + 16 * cb + li;
    colok[cb] = n < hj;
    fY[cb] = 0; fA[cb] = 0; eN[cb] = 0;
    if (colok[cb]) {
      const int64_t c = c0 + n;
      const int kind = P.blk[c];
      int eY = 0;
      double nY = 0.0;
      if (!first) {
        eY = P.exps[(int64_t)k * m + c];
        nY = P.norms[(int64_t)k * m + c];
        if (kind == 1) nY += P.norms[(int64_t)k * m + c + 1];
        else if (kind == 2) nY += P.norms[(int64_t)k * m + c - 1];
      }
      const int eW = P.eW[c];
      const double nW = P.nW[c];
      const int ks = eY > eW ? eY : eW;
      const int q = protect_update(nu, ldexp(nW, eW - ks), ldexp(nY, eY - ks));
      eN[cb] = ks + q;
      fY[cb] = eY - eN[cb];
      fA[cb] = eW - eN[cb];
    }
  }
  __syncthreads();   // every segment's old scale is read before any is rewritten
  if (32 * wave >= hj) return;

  // ---- K loop: acc = [S_kr | T_kr] * W ----
  const double psc = P.ctrl->psc;
  const int KP = (hr + 3) & ~3;
  const int KH = KP / 4;          // K steps per half
  const int KS = 2 * KH;
  const double* __restrict__ Wp = P.W + (int64_t)j * w_tile_doubles(MB) + (int64_t)(2 * wave) * 64 + lane;
  const double* __restrict__ pS = P.S + (k0 + li) + (int64_t)(r0 + lk) * P.lds;
  const double* __restrict__ pT = P.T + (k0 + li) + (int64_t)(r0 + lk) * P.ldt;
  bool rowok[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) rowok[rb] = 16 * rb + li < hk;

  d4 acc[RB][2];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = d4{0.0, 0.0, 0.0, 0.0};

  double a_cur[RB], b_cur[2], a_nxt[RB], b_nxt[2];
  auto load = [&](int s, double* av, double* bv) {
    const bool lower = s >= KH;
    const int kk = 4 * (lower ? s - KH : s);
    const bool colok_k = kk + lk < hr;
    const double* base = lower ? pT + (int64_t)kk * P.ldt : pS + (int64_t)kk * P.lds;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) av[rb] = (rowok[rb] && colok_k) ? base[16 * rb] : 0.0;
    bv[0] = Wp[(int64_t)(s * CBM) * 64];
    bv[1] = Wp[(int64_t)(s * CBM + 1) * 64];
  };
  load(0, a_cur, b_cur);
  for (int s = 0; s < KS; ++s) {
    if (s + 1 < KS) load(s + 1, a_nxt, b_nxt);
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const double av = a_cur[rb] * psc;
      acc[rb][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b_cur[0], acc[rb][0], 0, 0, 0);
      acc[rb][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b_cur[1], acc[rb][1], 0, 0, 0);
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) a_cur[rb] = a_nxt[rb];
    b_cur[0] = b_nxt[0];
    b_cur[1] = b_nxt[1];
  }

  // ---- epilogue: Y <- 2^fY Y - 2^fA acc, new segment norms ----
  // accumulator layout of the 16x16x4 FP64 instruction: lane holds column lane % 16,
  // rows lane / 16 + 4 * v for v = 0..3
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int n = 32 * wave + 16 * cb + li;
    double cmx = 0.0;
    if (colok[cb]) {
      double* zc = P.Z + (k0 + lk) + (int64_t)(c0 + n) * P.ldz;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * rb + lk + 4 * v;
          if (i < hk) {
            const double yo = first ? 0.0 : zc[16 * rb + 4 * v];
            const double yn = ldexp(yo, fY[cb]) - ldexp(acc[rb][cb][v], fA[cb]);
            zc[16 * rb + 4 * v] = yn;
            cmx = fmax(cmx, fabs(yn));
          }
        }
    }
    cmx = fmax(cmx, __shfl_xor(cmx, 16));
    cmx = fmax(cmx, __shfl_xor(cmx, 32));
    if (colok[cb] && lk == 0) {
      const int64_t c = c0 + n;
      P.exps[(int64_t)k * m + c] = eN[cb];
      P.norms[(int64_t)k * m + c] = cmx;
    }
  }
}

template <int MB>
static void launch_update_t(const PencilDesc& P, int r, hipStream_t s) {
  const int64_t tiles = (int64_t)r * (P.Mmax - r);
  const int64_t grid = (tiles + 7) / 8 * 8;
  update_kernel<MB><<<(unsigned)grid, MB * 2, 0, s>>>(P, r);
}

void launch_update(const PencilDesc& P, int r, hipStream_t s) {
  if (r <= 0) return;
  switch (P.mb) {
    case 32: launch_update_t<32>(P, r, s); break;
    case 64: launch_update_t<64>(P, r, s); break;
    default: launch_update_t<128>(P, r, s); break;
  }
}

}  // namespace rgev
