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
// powers of two applied to the W fragments as they are loaded, and one ProtectUpdate
// bounds the sum.
//
// One workgroup per target tile (k, j); its waves split the tile into a WGR x WGC grid
// (2 x 2 for MB = 128: 64 x 64 per wave, 16 independent accumulators, two waves per SIMD
// when two workgroups share a CU; batches: one wave for MB = 64, eight workgroups per CU).  Each wave streams its own matrix-core fragments straight from global memory into
// registers, with no LDS staging and no barrier in the K loop: an A fragment (16 rows x 4
// K values of column-major S or T) is four fully used 128-byte lines, a W fragment one
// 512-byte run of the packed W tile, and the waves sharing rows or columns of the tile
// meet in L1.  The loads of step t + 2 are in flight while the matrix cores run step t.
// The padded K rows need no mask: their W rows are zero and the A columns they meet are
// clamped to the source tile's last column (finite values); A rows past the target tile
// are clamped into the matrix and their outputs never stored.  Tiles are visited in 8 x 8
// blocks, each XCD taking a contiguous range of blocks, so the S/T and W tiles that
// neighbouring workgroups share stay in that XCD's L2.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>

#include "layout.hpp"
#include "robust.hpp"

namespace rgev {

typedef double d4 __attribute__((ext_vector_type(4)));


constexpr int kChunk = 16;   // source heights are padded to a multiple of kChunk rows

// wave grid R x C per tile size, S the register slots of the fragment pipeline and W the
// waves per SIMD the kernel is compiled for (W = 2: 256 registers per lane).
//  - UpdShape (one pencil): four waves per tile, so a launch of few tiles (the update of the
//    next band, on the critical path of the band schedule) ends soon;
//  - BatchUpdShape (lock-step batches, launches of thousands of tiles, bound by throughput):
//    a wave holds at most a 64 x 64 block (16 accumulators), so tiles of 64 and 32 are one
//    wave each and a wave's loads per matrix instruction are as for the tile of 128.
template <int MB> struct UpdShape { static constexpr int R = 2, C = 2, S = 3, W = 2; };
template <int MB> struct BatchUpdShape { static constexpr int R = 1, C = 1, S = 3, W = 2; };
template <> struct BatchUpdShape<128> { static constexpr int R = 2, C = 2, S = 3, W = 2; };

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
  // every load is issued at once (the pair partner's norm and the sources past ns from
  // clamped addresses, then discarded), so the prologue waits for memory only once
  const int kind = P.blk[c];
  const int64_t yo = (int64_t)k * m;
  const int eY0 = P.exps[yo + c];
  const double nY0 = P.norms[yo + c];
  const double nYp = P.norms[yo + min(c + 1, m - 1)], nYm = P.norms[yo + max(c - 1, (int64_t)0)];
  int eWs[kMaxBand];
  double nWs[kMaxBand], nus[kMaxBand];
#pragma unroll
  for (int i = 0; i < kMaxBand; ++i) {
    const int s = U.s_lo + min(i, max(ns - 1, 0));
    const int64_t slot = (int64_t)(s % WSL) * m + c;
    eWs[i] = P.eW[slot];
    nWs[i] = P.nW[slot];
    nus[i] = P.nu[(int64_t)k * P.Mmax + s];
  }
  const int eY = first ? 0 : eY0;
  const double nY = first ? 0.0 : (kind == 1 ? nY0 + nYp : (kind == 2 ? nY0 + nYm : nY0));
  int ew = INT_MIN;
#pragma unroll
  for (int i = 0; i < kMaxBand; ++i)
    if (i < ns) ew = max(ew, eWs[i]);
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
  int sfY[MB], sfA[MB], seN[MB];
  int sg[kMaxBand][MB];        // exponent of each source's W relative to the band's
  int sgw[(MB + 63) / 64];     // per wave of column threads: bit i set if some sg[i] != 0
  double red[WGR][MB];
};

// Update of target tile (k, j) of one pencil by the band of sources in U (a workgroup of
// 64 WGR WGC threads, the waves on a WGR x WGC grid over the tile; kOpaque as for solve_tile).
template <int MB, int WGR, int WGC, int NS = 3, bool kOpaque = false>
__device__ __forceinline__ void update_tile(const PencilDesc& P, const UpdRange& U, int k, int j,
                                            UpdSmem<MB, WGR>& sm) {
  constexpr int WR = MB / WGR;          // rows per wave
  constexpr int WC = MB / WGC;          // columns per wave
  constexpr int RB = WR / 16;           // row blocks per wave
  constexpr int CB = WC / 16;           // column blocks per wave
  constexpr int CBM = MB / 16;          // column blocks of a W tile
  auto& sfY = sm.sfY;
  auto& sfA = sm.sfA;
  auto& seN = sm.seN;
  auto& sg = sm.sg;
  auto& sgw = sm.sgw;
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
  // (in correction mode Y starts as the right-hand side, so every update accumulates)
  const bool first = (j <= U.s_hi) && !P.rhs;
  int cs[kMaxBand + 1];     // cumulative K chunks per source
  int es[kMaxBand + 1];     // first row of each source tile (and the end of the last)
  int ev[kMaxBand + 1];     // (edges past the band from clamped addresses, discarded: these
#pragma unroll              // loads need not wait for M)
  for (int i = 0; i <= kMaxBand; ++i) ev[i] = P.edges[min(U.s_lo + i, P.Mmax)];
  cs[0] = 0;
  es[0] = ev[0];
#pragma unroll
  for (int i = 0; i < kMaxBand; ++i) {
    es[i + 1] = i < ns ? ev[i + 1] : es[i];
    cs[i + 1] = cs[i] + 2 * ((es[i + 1] - es[i] + 15) & ~15) / kChunk;
  }
  const int tid = kOpaque ? opaque_tid() : (int)threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  const int wr = wave / WGC, wc = wave % WGC;
  const int li = lane % 16, lk = lane / 16;

  // ---- K loop: fragments straight from global memory into registers ----
  // K step t of a source (4 K values) with q = KP / 4 steps per half: the S columns
  // e_s + 4 t + 0..3 for t < q, else the T columns e_s + 4 (t - q) + 0..3.  A lane's A
  // fragment element is row 16 a + li of its wave's rows and K value lk; its W fragment
  // element is the packed entry (step, column block, lane) of the source's W tile.
  // The first slots are loaded before the per-column scales are computed, so their
  // latency and that of the scales' loads overlap; their W exponent fixups (which need
  // the scales) are read once the scales are published.
  const double psc = P.ctrl->psc;
  const int nst = cs[ns] * (kChunk / 4);   // K steps of the band
  int sgbits = 0;    // sources whose W exponents differ from the band's in some column
  const bool fix_a = psc != 1.0;

  int rowA[RB];      // clamped matrix rows of the lane's A elements
#pragma unroll
  for (int a = 0; a < RB; ++a) rowA[a] = min(k0 + WR * wr + 16 * a + li, (int)m - 1);
  // loader state: the next K step to load
  int ls_i = 0, ls_t = 0, ls_q = 0, ls_es = 0, ls_clast = 0;
  const double* ls_w = nullptr;
  auto enter_source = [&](int i) {
    ls_i = i;
    ls_t = 0;
    ls_es = es[i];
    ls_clast = es[i + 1] - 1;
    ls_q = ((es[i + 1] - es[i] + 15) & ~15) / 4;
    ls_w = P.W + ((int64_t)((U.s_lo + i) % WSL) * P.Mmax + j) * w_tile_doubles(MB) + (CB * wc) * 64 + lane;
  };
  enter_source(0);
  // Loads are unconditional (past the band's last step the loader stays on that step and
  // reloads it), so the compiler's count of loads in flight stays exact and a wave waits
  // only for the slot it is about to use; everything that needs the data (the rare
  // scalings, the zeroing of the steps past the end) happens when the slot is used.
  auto load = [&](double (&af)[RB], double (&bf)[CB], int (&sgl)[CB], int& src) {
    src = ls_i;
    const bool lower = ls_t >= ls_q;
    const double* base = lower ? P.T : P.S;
    const int64_t ld = lower ? P.ldt : P.lds;
    const int col = min(ls_es + 4 * (lower ? ls_t - ls_q : ls_t) + lk, ls_clast);
    const double* colp = base + (int64_t)col * ld;
#pragma unroll
    for (int a = 0; a < RB; ++a) af[a] = colp[rowA[a]];
    const double* wp = ls_w + (int64_t)ls_t * (CBM * 64);
#pragma unroll
    for (int q = 0; q < CB; ++q) bf[q] = wp[q * 64];
    if (sgbits) {
#pragma unroll
      for (int q = 0; q < CB; ++q) sgl[q] = sg[ls_i][16 * (CB * wc + q) + li];
    }
    if (ls_t + 1 < 2 * ls_q) ++ls_t;
    else if (ls_i + 1 < ns) enter_source(ls_i + 1);
  };

  d4 acc[RB][CB];
#pragma unroll
  for (int a = 0; a < RB; ++a)
#pragma unroll
    for (int b = 0; b < CB; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  // operands swapped: acc holds (A W)^T blocks, so a lane's four accumulator registers
  // are one C row of four columns and a wave's store covers whole lines
  auto mma = [&](const double (&af)[RB], const double (&bf)[CB]) {
#pragma unroll
    for (int a = 0; a < RB; ++a)
#pragma unroll
      for (int q = 0; q < CB; ++q)
        acc[a][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[q], af[a], acc[a][q], 0, 0, 0);
  };
  auto use = [&](double (&af)[RB], double (&bf)[CB], const int (&sgl)[CB], bool live) {
    if (!live) {             // a step past the band's end: W = 0
#pragma unroll
      for (int q = 0; q < CB; ++q) bf[q] = 0.0;
    } else {
      // rare: a prescaled pencil, or sources whose W exponents differ from the band's
      if (fix_a) {
#pragma unroll
        for (int a = 0; a < RB; ++a) af[a] *= psc;
      }
      if (sgbits) {
#pragma unroll
        for (int q = 0; q < CB; ++q) bf[q] = ldexp(bf[q], sgl[q]);
      }
    }
    mma(af, bf);
  };

  // NS register slots rotate through an unrolled loop: the loads of step t + NS - 1 are in
  // flight while the matrix cores run step t; the step count is rounded up to NS
  double af[NS][RB], bf[NS][CB];
  int sgl[NS][CB] = {};
  int src[NS];
  const int nrun = (nst + NS - 1) / NS * NS;
#pragma unroll
  for (int u = 0; u < NS - 1; ++u) load(af[u], bf[u], sgl[u], src[u]);

  // ---- per-column scales (Algorithm 3): common exponent, ProtectUpdate ----
  if (tid < MB) {
    const int n = tid;
    int fy = 0, fa = 0, en = 0;
    int g[kMaxBand] = {};
    if (n < hj) band_column_scales(P, U, k, c0 + n, first, ns, fy, fa, en, g);
    sfY[n] = fy;
    sfA[n] = fa;
    seN[n] = en;
    int bits = 0;
#pragma unroll
    for (int i = 0; i < kMaxBand; ++i) {
      sg[i][n] = g[i];
      bits |= (__ballot(g[i] != 0) != 0) << i;
    }
    if (lane == 0) sgw[wave] = bits;
  }
  __syncthreads();   // per-column scales and W exponent flags published
#pragma unroll
  for (int w = 0; w < (MB + 63) / 64; ++w) sgbits |= sgw[w];
  if (sgbits) {
#pragma unroll
    for (int u = 0; u < NS - 1; ++u)
#pragma unroll
      for (int q = 0; q < CB; ++q) sgl[u][q] = sg[src[u]][16 * (CB * wc + q) + li];
  }

  if (!fix_a && !sgbits) {
    // The common case: no scaling of the fragments and no step past the end inside the
    // loop (the last nst mod NS steps, already loaded, run after it), so the loop body is
    // the loader, loads and matrix instructions.
    int t0 = 0;
    for (; t0 + NS <= nst; t0 += NS) {
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        load(af[(u + NS - 1) % NS], bf[(u + NS - 1) % NS], sgl[(u + NS - 1) % NS], src[(u + NS - 1) % NS]);
        mma(af[u], bf[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < NS - 1; ++u)
      if (t0 + u < nst) mma(af[u], bf[u]);
  } else {
    for (int t0 = 0; t0 < nrun; t0 += NS) {
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        load(af[(u + NS - 1) % NS], bf[(u + NS - 1) % NS], sgl[(u + NS - 1) % NS], src[(u + NS - 1) % NS]);
        use(af[u], bf[u], sgl[u], t0 + u < nst);
      }
    }
  }

  // ---- epilogue: Y <- 2^fY Y - 2^fA acc and the new segment norms ----
  // block (a, q) of the transposed product: lane holds C row 16 a + lane % 16 (within
  // the wave's rows) for columns 16 q + lane / 16 + 4 v, v = 0..3.  The old Y of column
  // block q + 1 is loaded before block q is written (from addresses clamped into the
  // tile; only the stores are masked), so the epilogue waits for memory about once.
  auto load_yo = [&](double (&y)[4][RB], int q) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int nc = min(WC * wc + 16 * q + lk + 4 * v, hj - 1);
#pragma unroll
      for (int a = 0; a < RB; ++a) {
        const int ic = min(WR * wr + 16 * a + li, hk - 1);
        const double z = P.Z[(k0 + ic) + (int64_t)(c0 + nc) * P.ldz];   // (unused on a first update)
        y[v][a] = first ? 0.0 : z;
      }
    }
  };
  double yo[2][4][RB];
  load_yo(yo[0], 0);
#pragma unroll
  for (int q = 0; q < CB; ++q) {
    if (q + 1 < CB) load_yo(yo[(q + 1) % 2], q + 1);
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
            const double yn = ldexp(yo[q % 2][v][a], fy) - ldexp(acc[a][q][v], fa);
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
