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
// A launch applies a band of source rows s in [s_lo, s_hi] (only s <= j for tile column
// j) to the target tiles k in [k_lo, k_hi), j in [j_lo, M): each source's W keeps its
// own exponent, the per-column factors that bring the band to one exponent are exact
// powers of two applied while W is staged, and one ProtectUpdate bounds the sum.
//
// One workgroup per target tile (k, j).  The K dimension (2 h_s per source, each half
// padded to 16) is streamed in chunks of 16 through two LDS stages; the loads of the
// chunk after next are issued before the matrix cores start on the current chunk, so
// every global load has two chunks of compute to arrive (one barrier per chunk).  The
// waves split the tile into a WGR x WGC grid (2 x 4 for MB = 128: 64 x 32 per wave,
// so four waves share each SIMD when two workgroups share a CU).  Tiles are visited in
// 8 x 8 blocks, each XCD taking a contiguous range of blocks, so the S/T and W tiles
// that neighbouring workgroups share stay in that XCD's L2.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>

#include "layout.hpp"
#include "robust.hpp"

namespace rgev {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kChunk = 16;   // K rows per LDS stage

template <int MB> struct UpdShape;   // wave grid per tile size
template <> struct UpdShape<128> { static constexpr int R = 2, C = 4; };
template <> struct UpdShape<64> { static constexpr int R = 2, C = 4; };
template <> struct UpdShape<32> { static constexpr int R = 2, C = 2; };

struct UpdRange {
  int k_lo, k_hi;   // target tile rows [k_lo, k_hi)
  int j_lo;         // target tile columns [j_lo, M)
  int s_lo, s_hi;   // source tile rows (all below every target row)
};

// Per-column scales of a band update of tile (k, j), column c (Algorithm 3 with the band's
// sources brought to one exponent): the common exponent of Y and of the sources' W
// segments, one ProtectUpdate bounding the sum by the tile-pair norms, and the exponent
// g[i] of source i's W relative to the band's.  Returns fy, fa (the factors 2^fy on Y and
// 2^fa on the product) and en, the new exponent of the segment.
__device__ __forceinline__ void band_column_scales(const PencilDesc& P, const UpdRange& U, int k, int64_t c,
                                                   bool first, int ns, int& fy, int& fa, int& en,
                                                   int (&g)[kMaxBand]) {
  const int64_t m = P.m;
  const int WSL = P.wslots;
  const int kind = P.blk[c];
  int eY = 0;
  double nY = 0.0;
  if (!first) {
    eY = P.exps[(int64_t)k * m + c];
    nY = P.norms[(int64_t)k * m + c];
    if (kind == 1) nY += P.norms[(int64_t)k * m + c + 1];
    else if (kind == 2) nY += P.norms[(int64_t)k * m + c - 1];
  }
  int eWs[kMaxBand];
  double nWs[kMaxBand], nus[kMaxBand];
  int ew = INT_MIN;
#pragma unroll
  for (int i = 0; i < kMaxBand; ++i) {
    if (i < ns) {
      const int s = U.s_lo + i;
      const int64_t slot = (int64_t)(s % WSL) * m + c;
      eWs[i] = P.eW[slot];
      nWs[i] = P.nW[slot];
      nus[i] = P.nu[(int64_t)k * P.Mmax + s];
      ew = max(ew, eWs[i]);
    }
  }
  const int ks = eY > ew ? eY : ew;
  // |sum_s [S_ks | T_ks] W_s| <= sum_s nu_ks ||W_s|| (each term <= 2^1000, no overflow)
  double xb = 0.0;
#pragma unroll
  for (int i = 0; i < kMaxBand; ++i) {
    g[i] = 0;
    if (i < ns) {
      xb += nus[i] * ldexp(nWs[i], eWs[i] - ks);
      g[i] = eWs[i] - ew;
    }
  }
  const int q = protect_update(1.0, xb, ldexp(nY, eY - ks));
  en = ks + q;
  fy = eY - en;
  fa = ew - en;
}

// Shared memory of one tile update with a WGR-row wave grid.
template <int MB, int WGR>
struct UpdSmem {
  double As[2][kChunk * MB];   // [k][row]
  double Ws[2][kChunk * MB];   // packed [kstep][col block][lane]
  int sfY[MB], sfA[MB], seN[MB];
  int sg[kMaxBand][MB];        // exponent of each source's W relative to the band's
  int sgany[kMaxBand];
  double red[WGR][MB];
};

// Update of target tile (k, j) of one pencil by the band of sources in U (a workgroup of
// 64 WGR WGC threads, the waves on a WGR x WGC grid over the tile).
template <int MB, int WGR, int WGC>
__device__ __forceinline__ void update_tile(const PencilDesc& P, const UpdRange& U, int k, int j,
                                            UpdSmem<MB, WGR>& sm) {
  constexpr int kUpdThreads = 64 * WGR * WGC;
  constexpr int WR = MB / WGR;          // rows per wave
  constexpr int WC = MB / WGC;          // columns per wave
  constexpr int RB = WR / 16;           // row blocks per wave
  constexpr int CB = WC / 16;           // column blocks per wave
  constexpr int CBM = MB / 16;          // column blocks of a W tile
  constexpr int TPR = kUpdThreads / MB; // threads per A row in the stage load
  constexpr int AK = kChunk / TPR;      // A values per thread per stage
  constexpr int WV = kChunk * MB / kUpdThreads;   // W values per thread per stage
  auto& As = sm.As;
  auto& Ws = sm.Ws;
  auto& sfY = sm.sfY;
  auto& sfA = sm.sfA;
  auto& seN = sm.seN;
  auto& sg = sm.sg;
  auto& sgany = sm.sgany;
  auto& red = sm.red;

  const int M = P.ctrl->M;

  const int64_t m = P.m;
  const int WSL = P.wslots;
  const int k0 = P.edges[k], hk = P.edges[k + 1] - k0;
  const int c0 = P.edges[j], hj = P.edges[j + 1] - c0;
  // sources that reach column tile j: s_lo .. s_end (the source row j itself, when in the
  // band, makes this the first update of (k, j): Y is still zero)
  const int s_end = min(min(U.s_hi, M - 1), j);
  const int ns = s_end - U.s_lo + 1;
  const bool first = (j <= U.s_hi);
  int cs[kMaxBand + 1];     // cumulative K chunks per source
  cs[0] = 0;
#pragma unroll
  for (int i = 0; i < kMaxBand; ++i) {
    const int s = U.s_lo + i;
    const int hs = i < ns ? P.edges[s + 1] - P.edges[s] : 0;
    cs[i + 1] = cs[i] + 2 * ((hs + 15) & ~15) / kChunk;
  }
  const int tid = threadIdx.x;
  if (tid < kMaxBand) sgany[tid] = 0;
  __syncthreads();
  const int wave = tid / 64, lane = tid % 64;
  const int wr = wave / WGC, wc = wave % WGC;
  const int li = lane % 16, lk = lane / 16;

  // ---- per-column scales (Algorithm 3): common exponent, ProtectUpdate ----
  if (tid < MB) {
    const int n = tid;
    int fy = 0, fa = 0, en = 0;
    int g[kMaxBand] = {};
    if (n < hj) band_column_scales(P, U, k, c0 + n, first, ns, fy, fa, en, g);
    sfY[n] = fy;
    sfA[n] = fa;
    seN[n] = en;
#pragma unroll
    for (int i = 0; i < kMaxBand; ++i) {
      sg[i][n] = g[i];
      if (g[i] != 0) atomicOr(&sgany[i], 1);
    }
  }

  // ---- K loop ----
  const double psc = P.ctrl->psc;
  const int nch = cs[ns];
  const int arow = tid % MB;           // stage-load row of this thread
  const int akof = tid / MB;           // first k of this thread (stride TPR)
  const bool arow_ok = arow < hk;
  const double* __restrict__ Srow = P.S + (k0 + arow);
  const double* __restrict__ Trow = P.T + (k0 + arow);

  // chunk c -> source index i, lower (T) half or not, first K row of the chunk
  struct ChunkPos { int i, kb, hs; bool lower; int cc; };
  auto where = [&](int c) {
    ChunkPos p{0, 0, 0, false, 0};
#pragma unroll
    for (int i = 1; i < kMaxBand; ++i)
      if (i < ns && c >= cs[i]) p.i = i;
    const int s = U.s_lo + p.i;
    const int e_s = P.edges[s];
    p.hs = P.edges[s + 1] - e_s;
    p.cc = c - cs[p.i];
    const int half = (cs[p.i + 1] - cs[p.i]) / 2;
    p.lower = p.cc >= half;
    p.kb = e_s + kChunk * (p.lower ? p.cc - half : p.cc);   // absolute column of S or T
    return p;
  };

  // Every load is unconditional (a masked element reads a valid address), and the
  // zero mask is applied only when the chunk is written to LDS, so the loads stay in
  // flight while the matrix cores work.
  const double* safe = P.S;
  auto fetch = [&](int c, double (&ra)[AK], double (&rw)[WV]) {
    const ChunkPos p = where(c);
    const int s = U.s_lo + p.i;
    const int64_t ld = p.lower ? P.ldt : P.lds;
    const double* pa = (p.lower ? Trow : Srow) + (int64_t)(p.kb + akof) * ld;
    const int64_t step = (int64_t)TPR * ld;
    const int krel = p.kb - P.edges[s] + akof;
#pragma unroll
    for (int i = 0; i < AK; ++i) {
      const bool ok = arow_ok && (krel + TPR * i < p.hs);
      ra[i] = *(ok ? pa + i * step : safe);
    }
    const double* wsrc = P.W + ((int64_t)(s % WSL) * P.Mmax + j) * w_tile_doubles(MB) +
                         (int64_t)p.cc * kChunk * MB + tid;
#pragma unroll
    for (int i = 0; i < WV; ++i) rw[i] = wsrc[i * kUpdThreads];
  };
  auto stash = [&](int b, int c, const double (&ra)[AK], const double (&rw)[WV]) {
    const ChunkPos p = where(c);
    const int krel = p.kb - P.edges[U.s_lo + p.i] + akof;
#pragma unroll
    for (int i = 0; i < AK; ++i) {
      const bool ok = arow_ok && (krel + TPR * i < p.hs);
      As[b][(akof + TPR * i) * MB + arow] = ok ? psc * ra[i] : 0.0;
    }
    if (sgany[p.i]) {
#pragma unroll
      for (int i = 0; i < WV; ++i) {
        const int n = 16 * (((i * kUpdThreads + tid) / 64) % CBM) + tid % 16;
        Ws[b][i * kUpdThreads + tid] = ldexp(rw[i], sg[p.i][n]);
      }
    } else {
#pragma unroll
      for (int i = 0; i < WV; ++i) Ws[b][i * kUpdThreads + tid] = rw[i];
    }
  };

  d4 acc[RB][CB];
#pragma unroll
  for (int a = 0; a < RB; ++a)
#pragma unroll
    for (int b = 0; b < CB; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  double ra0[AK], rw0[WV], ra1[AK], rw1[WV], ra2[AK], rw2[WV];
  fetch(0, ra0, rw0);
  if (1 < nch) fetch(1, ra1, rw1);
  __syncthreads();   // per-column scales published; old scales all read before any rewrite
  stash(0, 0, ra0, rw0);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int b = c & 1;
    if (c + 2 < nch) fetch(c + 2, ra2, rw2);
#pragma unroll
    for (int s = 0; s < kChunk / 4; ++s) {
      double af[RB], bf[CB];
#pragma unroll
      for (int a = 0; a < RB; ++a) af[a] = As[b][(4 * s + lk) * MB + WR * wr + 16 * a + li];
#pragma unroll
      for (int q = 0; q < CB; ++q) bf[q] = Ws[b][(s * CBM + CB * wc + q) * 64 + lane];
      // operands swapped: acc holds (A W)^T blocks, so a lane's four accumulator
      // registers are one C row of four columns and a wave's store covers whole lines
#pragma unroll
      for (int a = 0; a < RB; ++a)
#pragma unroll
        for (int q = 0; q < CB; ++q)
          acc[a][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[q], af[a], acc[a][q], 0, 0, 0);
    }
    if (c + 1 < nch) stash(b ^ 1, c + 1, ra1, rw1);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < AK; ++i) ra1[i] = ra2[i];
#pragma unroll
    for (int i = 0; i < WV; ++i) rw1[i] = rw2[i];
  }

  // ---- epilogue: Y <- 2^fY Y - 2^fA acc and the new segment norms ----
  // block (a, q) of the transposed product: lane holds C row 16 a + lane % 16 (within
  // the wave's rows) for columns 16 q + lane / 16 + 4 v, v = 0..3
#pragma unroll
  for (int q = 0; q < CB; ++q) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int n = WC * wc + 16 * q + lk + 4 * v;
      double cmx = 0.0;
      if (n < hj) {
        const int fy = sfY[n], fa = sfA[n];
        double* zc = P.Z + (k0 + WR * wr + li) + (int64_t)(c0 + n) * P.ldz;
#pragma unroll
        for (int a = 0; a < RB; ++a) {
          const int i = WR * wr + 16 * a + li;
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
      if (li == 0) red[wr][n] = cmx;
    }
  }
  __syncthreads();
  if (tid < hj) {
    const int64_t c = c0 + tid;
    double nx = red[0][tid];
#pragma unroll
    for (int w = 1; w < WGR; ++w) nx = fmax(nx, red[w][tid]);
    P.exps[(int64_t)k * m + c] = seN[tid];
    P.norms[(int64_t)k * m + c] = nx;
  }
}

}  // namespace rgev
