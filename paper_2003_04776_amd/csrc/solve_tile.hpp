// Diagonal-tile solves of Algorithm 1 (Section 3): kernel 1 computes the tips Y_jj,
// the eigenvectors of the small pencil (S_jj, T_jj); kernel 3 solves
// S_ii Z D_jj - T_ii Z B_jj = Y_ij.  Both are robust back-substitution over the
// 1x1/2x2 blocks of the diagonal tile (Section 4: every division protected by
// ProtectDivision, every column update by ProtectUpdate, scale factors as integer
// exponents).  After the solve, the tile is turned into the right-updated operand of
// Algorithm 2, W = 2^-g [X D ; -X B], packed for the FP64 matrix instruction.
//
// One workgroup per tile (i, j); one thread per eigenvector column of tile j (a complex
// pair belongs to the thread of its first column), plus as many threads again for the
// matrix-core and copy phases.  The tile Y_ij lives in LDS for the whole solve.  Its
// rows are taken in groups of 8 (a 2x2 block is never split): inside a group each
// thread substitutes its own column(s) with the unsolved rows in registers; at the end
// of the group one ProtectUpdate bounds its effect on the rows above, which all waves
// then apply as one rank-16 FP64-MFMA update.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "layout.hpp"
#include "robust.hpp"
#include "slices.hpp"

namespace rgev {

struct Cx {
  double r, i;
};
__device__ __forceinline__ Cx cx(double r, double i) { return Cx{r, i}; }
__device__ __forceinline__ Cx cmul(Cx x, Cx y) { return Cx{x.r * y.r - x.i * y.i, x.r * y.i + x.i * y.r}; }
__device__ __forceinline__ Cx csub(Cx x, Cx y) { return Cx{x.r - y.r, x.i - y.i}; }
__device__ __forceinline__ double cn1(Cx x) { return fabs(x.r) + fabs(x.i); }
// 1/d = 2^-e r for d != 0: with d' = 2^-e d scaled so that max(|Re d'|, |Im d'|) is in
// [1/2, 1), r = conj(d') / |d'|^2, where |d'|^2 is in [1/4, 2) (no overflow or underflow in
// forming it) and |r| = 1/|d'| <= 2.  A quotient x / d is then 2^-e (x r): two rounded
// products more than a correctly rounded quotient, and for |x|_1 <= Omega nothing overflows
// before the final power of two, which the protections bound.
struct CInv {
  Cx r;
  int e;
};
__device__ __forceinline__ CInv cinv(Cx d) {
  int e;
  frexp(fmax(fabs(d.r), fabs(d.i)), &e);
  const double dr = ldexp(d.r, -e), di = ldexp(d.i, -e);
  const double rn = recip(fma(dr, dr, di * di));
  return CInv{Cx{dr * rn, -di * rn}, e};
}
// (ldexp by 0 is the identity, so no select on q is needed)
__device__ __forceinline__ Cx cscl(Cx x, int q) { return Cx{ldexp(x.r, -q), ldexp(x.i, -q)}; }
// x / d as 2^-(q + e) (x r) for the inverse 2^-e r of d: a protection's scale 2^-q of the
// numerator folded into the same power of two
__device__ __forceinline__ Cx cdiv_inv(Cx x, const CInv& v, int q = 0) { return cscl(cmul(x, v.r), q + v.e); }

// When a protection has to scale, the solves scale by 2^128 more than the least
// exponent: any power of two that meets the bound represents the same vector, and the
// head room makes the next scaling (and its pass over the solved rows) rare even when
// the eigenvector keeps growing row after row.
constexpr int kScaleMargin = 128;
__device__ __forceinline__ int with_margin(int q) { return q > 0 ? q + kScaleMargin : 0; }

// pivot threshold: u times the size of the terms of beta S_qq - alpha T_qq
__device__ __forceinline__ double local_smin(double be, double aabs, double smax, double tmax) {
  const double s = kUnitRoundoff * (be * smax + aabs * tmax);
  return s < kTiny ? kTiny : s;
}

// The solves below run on every lane of a wave (their control flow is uniform); act is
// false for a lane whose result is not used, which then neither raises a flag nor runs the
// exact path of a protection.

// (beta s - alpha t) w = y for one row; alpha = a + i b (b = 0 for a real column).
__device__ __forceinline__ Cx solve1(double a, double b, double be, double s, double t, Cx y, int& qs,
                                     int& flags, bool act) {
  Cx d = cx(be * s - a * t, -b * t);
  const double smin = local_smin(be, fabs(a) + fabs(b), fabs(s), fabs(t));
  const bool pert = cn1(d) < smin;
  d = pert ? cx(smin, 0.0) : d;
  flags |= (pert && act) ? kInfoPerturbed : 0;
  // |y/d|_1 <= 2 |y|_1 / |d|_1
  const int q = with_margin(protect_division_fast(cn1(y), 0.5 * cn1(d), act));
  qs += q;
  return cdiv_inv(y, cinv(d), q);
}

// 2x2 block: Gaussian elimination with complete pivoting on |.|_1, every division
// and update protected.  y0, y1 are the block's rows; the solution replaces them.
// (Written with selects only, so nothing is indexed dynamically.)
__device__ __forceinline__ void solve2(double a, double b, double be, double s00, double s01, double s10,
                                       double s11, double t00, double t01, double t11, Cx& y0, Cx& y1,
                                       int& qs, int& flags, bool act) {
  const Cx C00 = cx(be * s00 - a * t00, -b * t00);
  const Cx C01 = cx(be * s01 - a * t01, -b * t01);
  const Cx C10 = cx(be * s10, 0.0);
  const Cx C11 = cx(be * s11 - a * t11, -b * t11);
  const double smax = fmax(fmax(fabs(s00), fabs(s01)), fmax(fabs(s10), fabs(s11)));
  const double tmax = fmax(fmax(fabs(t00), fabs(t01)), fabs(t11));
  const double smin = local_smin(be, fabs(a) + fabs(b), smax, tmax);
  const double v00 = cn1(C00), v01 = cn1(C01), v10 = cn1(C10), v11 = cn1(C11);
  // pivot (ip, jp): the entry of largest |.|_1 (the first of equal ones)
  const bool c01 = v01 > v00;
  const double b0 = c01 ? v01 : v00;
  const bool c10 = v10 > b0;
  const double b1 = c10 ? v10 : b0;
  const bool c11 = v11 > b1;
  const double best = c11 ? v11 : b1;
  const bool pert = best < smin;
  const bool ip = !pert && (c11 || c10);
  const bool jp = !pert && (c11 || (!c10 && c01));
  // rows/columns permuted so the pivot is (0, 0): u11 = C[ip][jp], u12 = C[ip][1-jp],
  // c21 = C[1-ip][jp], c22 = C[1-ip][1-jp]; a block below the threshold is replaced by smin I
  const Cx r0a = ip ? C10 : C00, r0b = ip ? C11 : C01;   // pivot row
  const Cx r1a = ip ? C00 : C10, r1b = ip ? C01 : C11;   // other row
  const Cx u11 = pert ? cx(smin, 0.0) : (jp ? r0b : r0a);
  const Cx u12 = pert ? cx(0.0, 0.0) : (jp ? r0a : r0b);
  const Cx c21 = pert ? cx(0.0, 0.0) : (jp ? r1b : r1a);
  const Cx c22 = pert ? cx(smin, 0.0) : (jp ? r1a : r1b);
  const CInv i11 = cinv(u11);
  const Cx l21 = cdiv_inv(c21, i11);
  Cx u22 = csub(c22, cmul(l21, u12));
  const bool pert2 = cn1(u22) < smin;
  u22 = pert2 ? cx(smin, 0.0) : u22;
  flags |= ((pert || pert2) && act) ? kInfoPerturbed : 0;
  Cx ya = ip ? y1 : y0, yb = ip ? y0 : y1;
  int q = with_margin(protect_update_fast(cn1(l21), cn1(ya), cn1(yb), act));
  ya = cscl(ya, q); yb = cscl(yb, q); qs += q;
  Cx r2 = csub(yb, cmul(l21, ya));
  q = with_margin(protect_division_fast(cn1(r2), 0.5 * cn1(u22), act));
  ya = cscl(ya, q); qs += q;
  Cx w2 = cdiv_inv(r2, cinv(u22), q);
  q = with_margin(protect_update_fast(cn1(u12), cn1(w2), cn1(ya), act));
  w2 = cscl(w2, q); ya = cscl(ya, q); qs += q;
  Cx n1 = csub(ya, cmul(u12, w2));
  q = with_margin(protect_division_fast(cn1(n1), 0.5 * cn1(u11), act));
  w2 = cscl(w2, q); qs += q;
  const Cx w1 = cdiv_inv(n1, i11, q);
  // unknown jp gets w1, the other gets w2
  y0 = jp ? w2 : w1;
  y1 = jp ? w1 : w2;
}

// The real form of a complex pencil (PencilDesc::cform): a complex column's vector is
// v (x) (1, -sg i), so on the 2x2 block [[a_j, -b_j], [b_j, a_j]] (T block c_j I) it is the
// complex 1x1 system (beta (a_j + sg i b_j) - alpha c_j) w = y0 + sg i y1 over 2 (the part of
// (y0, y1) in that subspace), with (y0, y1) = (w, -sg i w); solving it so keeps the other
// subspace, whose pivot beta (a_j - sg i b_j) - alpha c_j may be nearly singular when alpha/beta
// is close to the conjugate of eigenvalue j, at zero.
__device__ __forceinline__ void solve2c(double a, double b, double be, double aj, double bj, double cj, double sg,
                                        Cx& y0, Cx& y1, int& qs, int& flags, bool act) {
  // y0 + sg i y1 = (y0.r - sg y1.i) + i (y0.i + sg y1.r)
  const Cx cv = cx(0.5 * (y0.r - sg * y1.i), 0.5 * (y0.i + sg * y1.r));
  Cx d = cx(be * aj - a * cj, be * sg * bj - b * cj);
  const double smin = local_smin(be, fabs(a) + fabs(b), fmax(fabs(aj), fabs(bj)), fabs(cj));
  const bool pert = cn1(d) < smin;
  d = pert ? cx(smin, 0.0) : d;
  flags |= (pert && act) ? kInfoPerturbed : 0;
  const int q = with_margin(protect_division_fast(cn1(cv), 0.5 * cn1(d), act));
  qs += q;
  const Cx w = cdiv_inv(cv, cinv(d), q);
  y0 = w;
  y1 = cx(sg * w.i, -sg * w.r);   // -sg i w
}

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int solve_threads(int mb) { return mb < 64 ? 64 : mb; }
// the whole workgroup: the column threads plus as many again for the matrix-core and
// copy phases (one wave per SIMD)
constexpr int solve_total(int mb) { return mb < 64 ? 64 : 2 * mb; }
// waves per SIMD the register allocation must allow: two for tiles of 64 and less, whose
// LDS leaves room for several workgroups per CU (a batch's many small tile solves run 12 %
// faster than with the registers of one wave per SIMD), one for 128, whose LDS takes the CU
constexpr int solve_waves_per_simd(int mb) { return mb <= 64 ? 2 : 1; }

// Column slices: columns are independent, so a tile may be solved by CS workgroups, split
// at column SW (moved one right rather than split a complex pair).  With SW = MB / 2 a slice
// needs half the LDS and can share a CU with a tile-update workgroup; measured on the band
// schedule at m = 32768 that is slower (585 ms -> 614 ms: co-resident solves displace update
// workgroups and double the CU time spent in solves), so one workgroup per tile is used.
template <int MB>
struct SolveShape {
  static constexpr int SW = MB;                     // nominal columns per workgroup
  static constexpr int CS = MB / SW;                // workgroups per tile (1 or 2)
  static constexpr int NCY = CS > 1 ? SW + 1 : MB;  // most columns a workgroup holds
  // row stride of the tile in LDS: = 1 mod 32 doubles, so that a thread per row sweeping
  // the columns and a thread per column sweeping the rows are both conflict-free
  static constexpr int LDY = NCY % 32 == 1 ? NCY : NCY + 1;
};

// Shared memory of one tile solve.
template <int MB>
struct SolveSmem {
  static constexpr int LDY = SolveShape<MB>::LDY, BW = SolveShape<MB>::NCY, G = 8;
  double Y[MB * LDY];          // the tile's columns held by this workgroup
  // per column: eigenvalue, block kind, whether it is solved, and the epilogue's values
  double colA[BW], colB[BW], colBe[BW];
  double cmax[BW];
  int ecol[BW];                // exponent of the second column of a pair
  int colG[BW];
  int wexp[BW];                // mixed precision: column exponent of W (X D half)
  int8_t colKind[BW];
  int8_t colOn[BW];            // 1: a selected column of the tile (its B operand is not zero)
  // diagonal block of the group, S (Pn[0]) and T (Pn[1]), by columns: entry (row i,
  // column c) at Pn[.][c][i], so a column's G entries are one aligned vector
  alignas(16) double Pn[2][G][G];
  double tcnS[MB], tcnT[MB];
  int fcol[BW];                // scale exponent still owed by the rows above the group
  int8_t tblk[MB];
};

// Solve of column slice z of tile (r, j) of one pencil (a workgroup of solve_total(MB)
// threads; slices z = 0 .. SolveShape<MB>::CS - 1).  kOpaque: the thread index is read
// through opaque_tid (for a caller that runs several tiles in a loop).
template <int MB, bool kOpaque = false>
__device__ __forceinline__ void solve_tile(const PencilDesc& P, int r, int j, int z, SolveSmem<MB>& sm) {
  constexpr int NTOT = solve_total(MB);
  constexpr int SW = SolveShape<MB>::SW, NCY = SolveShape<MB>::NCY;
  constexpr int LDY = SolveShape<MB>::LDY;
  constexpr int G = 8;          // rows per group (recursive blocking inside the tile)
  auto& Y = sm.Y;
  auto& colOn = sm.colOn;
  auto& Pn = sm.Pn;
  auto& tcnS = sm.tcnS;
  auto& tcnT = sm.tcnT;
  auto& fcol = sm.fcol;
  auto& ecol = sm.ecol;
  auto& tblk = sm.tblk;
  auto& cmax = sm.cmax;
  auto& colA = sm.colA;
  auto& colB = sm.colB;
  auto& colBe = sm.colBe;
  auto& colG = sm.colG;
  auto& colKind = sm.colKind;

  __syncthreads();   // a previous solve in this workgroup is done with the shared memory
  const int M = P.ctrl->M;
  if (r < 0 || r >= M || j >= M) return;
  if (P.rhs && !P.tflag[j]) return;   // correction mode: no column of tile j is refined
  const int64_t m = P.m;
  const int r0 = P.edges[r], hr = P.edges[r + 1] - r0;
  const int c0 = P.edges[j], hj = P.edges[j + 1] - c0;
  // columns [own_lo, own_hi) of tile j: split at SW, moved one right rather than split a pair
  constexpr int CS = SolveShape<MB>::CS;
  int sp = SW;
  if (CS > 1 && sp < hj && P.blk[c0 + sp] == 2) ++sp;
  const int own_lo = z == 0 ? 0 : sp;
  const int own_hi = z == CS - 1 ? hj : min(sp, hj);
  if (own_lo >= own_hi) return;
  const int lo = own_lo, hw = own_hi - own_lo;
  const bool last = own_hi == hj;     // this workgroup also clears W past the tile's columns
  const bool tip = (r == j);
  const double psc = P.ctrl->psc;
  const double* S = P.S;
  const double* T = P.T;
  const int64_t lds = P.lds, ldt = P.ldt, ldz = P.ldz;

  const int lc = kOpaque ? opaque_tid() : (int)threadIdx.x;   // column thread lc holds tile column lo + lc
  const int wave = lc / 64, lane = lc % 64;
  const bool inrange = lc < hw;
  const bool colthr = lc < NCY;
  const int tcol = lo + lc;
  const int64_t c = c0 + tcol;
  const bool own = inrange;
  int kind = 0;
  bool selected = false;
  double a = 0.0, b = 0.0, be = 0.0;
  if (inrange) {
    kind = P.blk[c];
    selected = P.sel[c] != 0;
    a = P.ar[c];
    b = (kind != 0) ? P.ai[c] : 0.0;
    be = P.be[c];
  }
  const int partner = kind == 1 ? lc + 1 : (kind == 2 ? lc - 1 : lc);
  const bool pair = kind == 1;                 // this thread carries the pair (lc, lc + 1)
  const bool owner = selected && kind != 2;
  const int pc = (kind == 2 ? tcol - 1 : tcol) + (c0 - r0);   // local row of own block (tip tile)
  const double aabs = fabs(a) + fabs(b);
  // real form of a complex pencil: the subspace of a complex column, from the sign of the
  // sub-diagonal of its own 2x2 block (its eigenvalue (a + i b) / c has b of that sign)
  const double csg = (P.cform && pair) ? (P.S[(c + 1) + c * P.lds] > 0.0 ? 1.0 : -1.0) : 0.0;
  int e = 0;
  double ybound = 0.0;
  // largest |x_i|, |y_i| and |x_i| + |y_i| of the solved rows, at their current scale (a
  // column's thread; scaling by powers of two keeps them exact): the segment norms
  double tnx = 0.0, tny = 0.0, tns = 0.0;
  int flags = 0;

  // ---- structure and column norms of the diagonal tile, right-hand side Y_rj ----
  if (colthr) {
    colA[lc] = a;
    colB[lc] = b;
    colBe[lc] = be;
    colKind[lc] = (int8_t)kind;
    colOn[lc] = (int8_t)(inrange && selected);
  }
  if (lc < hr) {
    tblk[lc] = P.blk[r0 + lc];
    tcnS[lc] = P.cnS[r0 + lc];
    tcnT[lc] = P.cnT[r0 + lc];
  }
  // (in correction mode the tip tile too starts from the right-hand side held in Z)
  const bool loaded = !tip || P.rhs;
  if (!loaded) {
    // the tip tile starts from zero (the right-hand side of the tip's own system)
    for (int idx = lc; idx < MB * LDY; idx += NTOT) Y[idx] = 0.0;
  } else {
    // thread t reads row t mod MB of one half of the columns (coalesced down the columns),
    // 16 loads in flight; entries of Y past the tile are never used, so nothing is cleared
    static_assert(NTOT >= 2 * MB, "two threads per row");
    const int row = lc % MB, half = (lc / MB) & 1;
    const int hw2 = (hw + 1) / 2, ca = half ? hw2 : 0, cb = half ? hw : hw2;
    if (lc < 2 * MB && row < hr) {
      const double* zrow = P.Z + (r0 + row) + (int64_t)(c0 + lo) * ldz;
      for (int col0 = ca; col0 < cb; col0 += 16) {
        double v[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) v[t] = (col0 + t < cb) ? zrow[(int64_t)(col0 + t) * ldz] : 0.0;
#pragma unroll
        for (int t = 0; t < 16; ++t)
          if (col0 + t < cb) Y[row * LDY + col0 + t] = v[t];
      }
    }
  }
  if (loaded) {
    if (inrange) {
      e = P.exps[(int64_t)r * m + c];
      ybound = P.norms[(int64_t)r * m + c] + (kind != 0 ? P.norms[(int64_t)r * m + c0 + lo + partner] : 0.0);
    }
  }

  // The second rows of the tile's 2x2 blocks as two 64-bit masks, the same in every wave
  // (scalar registers), so the block structure costs no shared-memory read in the loops.
  __syncthreads();   // tblk visible
  const uint64_t two_lo = __ballot(lane < hr && tblk[lane] == 2);
  const uint64_t two_hi = __ballot(64 + lane < hr && tblk[(64 + lane) % MB] == 2);
  auto second = [&](int i) -> bool { return ((i < 64 ? two_lo : two_hi) >> (i & 63)) & 1; };
  // groups of at most G rows from the bottom, never splitting a 2x2 block
  auto group_lo = [&](int g1) {
    int g0 = g1 - G + 1;
    if (g0 < 0) g0 = 0;
    if (g0 > 0 && second(g0)) ++g0;
    return g0;
  };
  // the group's diagonal block of S and T (lanes 0..63 of wave 0 hold one entry each)
  // (loads are unconditional, from a valid address when masked, and the mask is applied
  // at publication, so they stay in flight while the group is solved)
  double pS = 0.0, pT = 0.0;
  bool pOk = false;
  auto panel_fetch = [&](int g0) {
    const int u = lane / G, t = lane % G;
    pOk = wave == 0 && g0 >= 0 && g0 + u < hr && g0 + t < hr;
    const int64_t ro = pOk ? (r0 + g0 + u) : 0, co = pOk ? (r0 + g0 + t) : 0;
    pS = S[ro + co * lds];
    pT = T[ro + co * ldt];
  };
  auto panel_publish = [&]() {
    if (wave == 0) {
      Pn[0][lane % G][lane / G] = pOk ? psc * pS : 0.0;
      Pn[1][lane % G][lane / G] = pOk ? psc * pT : 0.0;
    }
  };
  int g1 = hr - 1;
  int g0 = group_lo(g1);
  panel_fetch(g0);
  panel_publish();
  __syncthreads();

  static_assert(G == 8, "the group's rows are one 8-wide register vector");
  typedef double d8 __attribute__((ext_vector_type(8)));
  // The column waves run the substitution.  A group's rank-2G update of the rows above it is
  // split: the rows of the next group first, by all waves before that group starts, then the
  // rest by the helper waves (the waves past the columns) while the column waves substitute
  // the next group; with no helper wave (tiles of 32) the whole update comes first.
  constexpr int NCW = (NCY + 63) / 64, NHW = NTOT / 64 - NCW;
  // B operand entry (k, n) of the update by the group [bg0, bg1]: row bg0 + (k mod G) of column
  // n, -beta z (k < G) or alpha z (k >= G), own parts (a pair's real part in its first column,
  // imaginary in its second); zero for rows past the group and for columns not solved
  auto bop = [&](int k, int n, int bg0, int bg1) -> double {
    const int i = bg0 + (k & (G - 1));
    const int ir = i <= bg1 ? i : bg1;   // (rows past the group: read in range, dropped)
    const int kd = colKind[n];
    const int np = kd == 1 ? n + 1 : (kd == 2 ? n - 1 : n);
    const double own = Y[ir * LDY + n], oth = Y[ir * LDY + np];
    const double zr = kd == 2 ? oth : own, zi = kd == 0 ? 0.0 : (kd == 1 ? oth : own);
    const double an = colA[n], bn = colB[n];
    const double v = k < G ? -colBe[n] * own : (kd == 2 ? (bn * zr + an * zi) : (an * zr - bn * zi));
    return (i <= bg1 && colOn[n]) ? v : 0.0;
  };
  // Y[rlo:rhi, :] <- 2^-fcol Y[rlo:rhi, :] + [S | T][rlo:rhi, group] * [-beta z ; alpha z] for
  // the group [bg0, bg1] (rhi <= bg0).  A fragments: rows 16 rb + lane % 16 of the group's
  // columns (S then T), masked past the rows above the group and the group's columns.
  auto afrag = [&](int rb, int st, int bg0, int bg1) -> double {
    const int row = 16 * rb + lane % 16;
    const int kk = 4 * st + lane / 16;   // 0..15: S columns 0..7, T columns 8..15
    const int col = bg0 + (kk & (G - 1));
    const bool ok = row < bg0 && col <= bg1;
    const int64_t ro = ok ? r0 + row : 0, co = ok ? r0 + col : 0;
    return kk < G ? S[ro + co * lds] : T[ro + co * ldt];
  };
  // one 16-row block rb of column block cb: acc <- 2^-fs Y + A B, rows in [rlo, rhi) stored
  auto rank_block = [&](const double (&a4)[4], const double (&bf)[4], int rb, int cb, int rlo, int rhi) {
    const int col = 16 * cb + lane % 16;
    const int colr = col < NCY ? col : NCY - 1;   // (columns past those held: dropped)
    const int fs = fcol[colr];
    d4 acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = ldexp(Y[(16 * rb + lane / 16 + 4 * v) * LDY + colr], -fs);
#pragma unroll
    for (int st = 0; st < 4; ++st) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(psc * a4[st], bf[st], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * rb + lane / 16 + 4 * v;
      if (row >= rlo && row < rhi && col < hw) Y[row * LDY + col] = acc[v];
    }
  };
  auto bfrag = [&](double (&bf)[4], int cb, int bg0, int bg1) {
    const int col = 16 * cb + lane % 16;
    const int colr = col < NCY ? col : NCY - 1;
#pragma unroll
    for (int st = 0; st < 4; ++st) bf[st] = bop(4 * st + lane / 16, colr, bg0, bg1);
  };
  // the rows of the next group, [rlo, rhi) within two row blocks from rlo / 16, by every wave
  // (its column blocks strided); the A fragments in au were loaded before
  auto rank_near = [&](const double (&au)[2][4], int rlo, int rhi, int bg0, int bg1) {
    if (rhi <= rlo) return;
    const int rb0 = rlo / 16, nb = (rhi - 1) / 16 - rb0 + 1;   // 1 or 2 row blocks
    const int ncb = (hw + 15) / 16;
    for (int cb = wave; cb < ncb; cb += NTOT / 64) {
      double bf[4];
      bfrag(bf, cb, bg0, bg1);
      rank_block(au[0], bf, rb0, cb, rlo, rhi);
      if (nb > 1) rank_block(au[1], bf, rb0 + 1, cb, rlo, rhi);
    }
  };
  // the rows [0, rhi), by waves wv0 .. wv0 + nwv - 1, each owning whole column blocks: row
  // blocks in chunks of NRC, a chunk's row blocks independent chains issued interleaved.
  // Every operand index is a constant, so the operands stay in registers.
  constexpr int NR0 = MB / 16;
  auto rank_far = [&](auto nrc_c, int rhi, int bg0, int bg1, int wv0, int nwv) {
    constexpr int NRC = decltype(nrc_c)::value;
    if (rhi <= 0 || wave < wv0 || wave >= wv0 + nwv) return;
    const int rb_hi = (rhi + 15) / 16;
    const int ncb = (hw + 15) / 16;
    // every row block's A fragments at once (one memory latency for all of them)
    double af[NR0][4];
#pragma unroll
    for (int rb = 0; rb < NR0; ++rb)
#pragma unroll
      for (int st = 0; st < 4; ++st) af[rb][st] = rb < rb_hi ? afrag(rb, st, bg0, bg1) : 0.0;
    // column blocks (a runtime loop, so its addresses are not hoisted out of the group loop),
    // each with its B fragments formed once and its chunks' row blocks as independent chains
#pragma unroll 1
    for (int cb = wave - wv0; cb < ncb; cb += nwv) {
      const int col = 16 * cb + lane % 16;
      const int colr = col < NCY ? col : NCY - 1;
      const int fs = fcol[colr];
      double bf[4];
      bfrag(bf, cb, bg0, bg1);
#pragma unroll
      for (int ch = 0; ch < NR0 / NRC; ++ch) {
        if (NRC * ch >= rb_hi) continue;
        d4 acc[NRC];
#pragma unroll
        for (int i = 0; i < NRC; ++i)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            acc[i][v] = ldexp(Y[(16 * (NRC * ch + i) + lane / 16 + 4 * v) * LDY + colr], -fs);
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
          for (int i = 0; i < NRC; ++i)
            acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(psc * af[NRC * ch + i][st], bf[st], acc[i], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < NRC; ++i)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = 16 * (NRC * ch + i) + lane / 16 + 4 * v;
            if (row < rhi && col < hw) Y[row * LDY + col] = acc[i][v];
          }
      }
    }
  };
  constexpr int NRC_BIG = NR0 < 4 ? NR0 : 4;
  int dg0 = 0, dg1 = 0, drh = 0;   // deferred: rows [0, drh) take the update of the group [dg0, dg1]
  while (g1 >= 0) {
    const int gn1 = g0 - 1;                       // next group
    const int gn0 = gn1 >= 0 ? group_lo(gn1) : -1;
    panel_fetch(gn0);                             // lands during this group's work
    double yb_above = ybound;   // bound on the rows above the group
    int qsg = 0;                // scaling raised inside the group
    double zng = 0.0;           // largest |z|_1 of the group's solved rows (at their current scale)
    double cng = 0.0;           // sum over the group's rows of beta |S col|_1 + |alpha| |T col|_1

    if (wave < NCW) {
      // ---- blocks of the group, bottom up; updates stay inside the group ----
      // Each column's substitution is private to the thread that owns it (a complex pair
      // belongs to the thread of its first column), so the blocks need no barrier.  The
      // group's rows live in registers, (yr[k], yi[k]) = row g0 + k: a block reads its rows
      // by a uniform index, and its update is applied to all G rows with the block's full
      // panel columns (rows at or below the block are no longer used, so nothing has to
      // move and every other register index is a constant).  Every lane runs the solve;
      // work marks the lanes whose result is used, and the others take z = 0, so their
      // rows are left as they were.
      d8 yr, yi;
      d8 cnv;   // beta |S col|_1 + |alpha| |T col|_1 of the group's rows (zero past the group)
      const int yc0 = lc < NCY ? lc : 0, yc1 = pair ? lc + 1 : yc0;   // (threads past the columns read column 0)
  #pragma unroll
      for (int k = 0; k < G; ++k) {
        const int row = g0 + k <= g1 ? g0 + k : g1;   // (rows past the group: never used)
        yr[k] = Y[row * LDY + yc0];
        yi[k] = pair ? Y[row * LDY + yc1] : 0.0;
        cnv[k] = g0 + k <= g1 ? be * tcnS[row] + aabs * tcnT[row] : 0.0;
      }
      cng = ((cnv[0] + cnv[1]) + (cnv[2] + cnv[3])) + ((cnv[4] + cnv[5]) + (cnv[6] + cnv[7]));
      // a block's solved rows: rescale what is already solved if the block raised the
      // scaling (rare: scaling has head room), store, and extend the group's bound
      auto settle = [&](int q0, int q, int qs, Cx z0, Cx z1, double cn) {
        if (qs > 0) {
          yr = d8{ldexp(yr[0], -qs), ldexp(yr[1], -qs), ldexp(yr[2], -qs), ldexp(yr[3], -qs),
                  ldexp(yr[4], -qs), ldexp(yr[5], -qs), ldexp(yr[6], -qs), ldexp(yr[7], -qs)};
          yi = d8{ldexp(yi[0], -qs), ldexp(yi[1], -qs), ldexp(yi[2], -qs), ldexp(yi[3], -qs),
                  ldexp(yi[4], -qs), ldexp(yi[5], -qs), ldexp(yi[6], -qs), ldexp(yi[7], -qs)};
          for (int i = q + 1; i <= g1; ++i) {
            Y[i * LDY + lc] = ldexp(Y[i * LDY + lc], -qs);
            if (pair) Y[i * LDY + lc + 1] = ldexp(Y[i * LDY + lc + 1], -qs);
          }
          qsg += qs;
          e += qs;
          ybound = ldexp(ybound, -qs);
          yb_above = ldexp(yb_above, -qs);
          zng = ldexp(zng, -qs);
          tnx = ldexp(tnx, -qs);
          tny = ldexp(tny, -qs);
          tns = ldexp(tns, -qs);
        }
        Y[q0 * LDY + lc] = z0.r;
        if (pair) Y[q0 * LDY + lc + 1] = z0.i;
        if (q != q0) {
          Y[q * LDY + lc] = z1.r;
          if (pair) Y[q * LDY + lc + 1] = z1.i;
        }
        const double zn = fmax(cn1(z0), cn1(z1));
        zng = fmax(zng, zn);
        tnx = fmax(tnx, fmax(fabs(z0.r), fabs(z1.r)));
        tny = fmax(tny, fmax(fabs(z0.i), fabs(z1.i)));
        tns = fmax(tns, zn);
        if (q0 > 0) ybound = fma(cn, zn, ybound);
      };
      int q = g1;
      while (q >= g0) {
        // a block: rows q0 .. q (q0 = q for a 1x1 block), local rows lq0 .. lq
        const bool two = second(q);
        const int q0 = two ? q - 1 : q;
        const int lq0 = q0 - g0, lq = q - g0;
        const Cx y0 = cx(yr[lq0], yi[lq0]), y1 = cx(yr[lq], yi[lq]);
        const double cn = two ? cnv[lq0] + cnv[lq] : cnv[lq];
        const bool work = owner && !(tip && q0 > pc);
        const bool at_tip = tip && q0 == pc;   // the column's own block (singular for its eigenvalue)
        const bool act = work && !at_tip;
        int qs = 0;
        Cx z0, z1;
        if (!two) {
          // ---- 1x1 block ----
          z0 = solve1(a, b, be, Pn[0][lq][lq], Pn[1][lq][lq], y1, qs, flags, act);
          z1 = cx(0.0, 0.0);
          if (at_tip) {
            // the tip of a real eigenvalue (zero in correction mode)
            z0 = cx(P.rhs ? 0.0 : 1.0, 0.0);
            qs = 0;
          }
        } else {
          // ---- 2x2 block ----
          const double s00 = Pn[0][lq0][lq0], s10 = Pn[0][lq0][lq], s01 = Pn[0][lq][lq0], s11 = Pn[0][lq][lq];
          const double t00 = Pn[1][lq0][lq0], t01 = Pn[1][lq][lq0], t11 = Pn[1][lq][lq];
          z0 = y0;
          z1 = y1;
          if (P.cform) {
            // real form of a complex pencil: a complex column in its subspace, a real one as usual
            Cx c0 = z0, c1 = z1, g0v = z0, g1v = z1;
            int qc = 0, qg = 0;
            solve2c(a, b, be, s00, s10, t00, csg, c0, c1, qc, flags, act && csg != 0.0);
            solve2(a, b, be, s00, s01, s10, s11, t00, t01, t11, g0v, g1v, qg, flags, act && csg == 0.0);
            z0 = csg != 0.0 ? c0 : g0v;
            z1 = csg != 0.0 ? c1 : g1v;
            qs = csg != 0.0 ? qc : qg;
          } else {
            solve2(a, b, be, s00, s01, s10, s11, t00, t01, t11, z0, z1, qs, flags, act);
          }
          if (tip) {
            // the column's own block: the tip
            Cx tz0 = cx(0.0, 0.0), tz1 = cx(0.0, 0.0);
            int tq = 0;
            if (P.rhs) {
              // correction mode: the correction is zero at the tip (z0 = z1 = 0)
            } else if (csg != 0.0) {
              // real form of a complex pencil: the tip in the column's subspace, (sg i, 1), exactly
              tz0 = cx(0.0, csg);
              tz1 = cx(1.0, 0.0);
            } else {
              // second row of the singular block beta S_b - alpha T_b gives z_p for z_{p+1} = 1
              double m21 = be * s10;
              const Cx nn = cx(-(be * s11 - a * t11), b * t11);
              const double smin = local_smin(be, aabs, fmax(fabs(s10), fabs(s11)), fabs(t11));
              const bool pert = fabs(m21) < smin;
              m21 = pert ? smin : m21;
              flags |= (pert && work && at_tip) ? kInfoPerturbed : 0;
              tq = with_margin(protect_division_fast(cn1(nn), fabs(m21), work && at_tip));
              const Cx ns = cscl(nn, tq);
              const double rm = recip(m21);
              tz0 = cx(ns.r * rm, ns.i * rm);
              tz1 = cx(ldexp(1.0, -tq), 0.0);
            }
            if (at_tip) {
              z0 = tz0;
              z1 = tz1;
              qs = tq;
            }
          }
        }
        if (q0 > 0) {
          // ProtectUpdate for y[0:q0] -= (beta S - alpha T)[0:q0, q0..q] z (inside the group
          // now, above it at the end of the group; the column norms bound both)
          const int qu = with_margin(protect_update_fast(cn, fmax(cn1(z0), cn1(z1)), ldexp(ybound, -qs), work));
          z0 = cscl(z0, qu);
          z1 = cscl(z1, qu);
          qs += qu;
        }
        z0 = work ? z0 : cx(0.0, 0.0);
        z1 = work ? z1 : cx(0.0, 0.0);
        if (work) settle(q0, q, qs, z0, z1, cn);
        // y += S (-beta z) + T (alpha z) with the block's columns
        auto apply = [&](int c, Cx z) {
          const d8 cs = *reinterpret_cast<const d8*>(&Pn[0][c][0]);
          const d8 ct = *reinterpret_cast<const d8*>(&Pn[1][c][0]);
          const double ur = -be * z.r, ui = -be * z.i;
          const double vr = a * z.r - b * z.i, vi = a * z.i + b * z.r;
  #pragma unroll
          for (int k = 0; k < G; ++k) {
            yr[k] = fma(ct[k], vr, fma(cs[k], ur, yr[k]));
            yi[k] = fma(ct[k], vi, fma(cs[k], ui, yi[k]));
          }
        };
        apply(lq0, z0);
        if (two) apply(lq, z1);
        q = q0 - 1;
      }

    } else {
      // the helper waves: the previous group's update of the rows above this group
      rank_far(std::integral_constant<int, NRC_BIG>{}, drh, dg0, dg1, NCW, NHW > 0 ? NHW : 1);
    }
    if (NHW > 0) __syncthreads();   // the rows above are current before the end of the group rescales any
    // A fragments of the next group's rows (they land during the end of the group)
    double au[2][4];
    {
      const int rbn = (gn0 > 0 ? gn0 : 0) / 16;
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int st = 0; st < 4; ++st) au[i][st] = afrag(rbn + i < NR0 ? rbn + i : NR0 - 1, st, g0, g1);
    }

    // ---- end of group: bound the rank-2G update of the rows above, settle scales ----
    if (owner && g0 > 0) {
      const int qg = with_margin(protect_update_fast(cng, zng, yb_above));
      if (qg > 0) {
        for (int i = g0; i <= g1; ++i) {
          Y[i * LDY + lc] = ldexp(Y[i * LDY + lc], -qg);
          if (pair) Y[i * LDY + lc + 1] = ldexp(Y[i * LDY + lc + 1], -qg);
        }
        qsg += qg;
        e += qg;
        yb_above = ldexp(yb_above, -qg);
        zng = ldexp(zng, -qg);
        tnx = ldexp(tnx, -qg);
        tny = ldexp(tny, -qg);
        tns = ldexp(tns, -qg);
      }
      ybound = fma(cng, zng, yb_above);
    }
    if (owner && qsg > 0)   // the solved rows below the group (rare: scaling has head room)
      for (int i = g1 + 1; i < hr; ++i) {
        Y[i * LDY + lc] = ldexp(Y[i * LDY + lc], -qsg);
        if (pair) Y[i * LDY + lc + 1] = ldexp(Y[i * LDY + lc + 1], -qsg);
      }
    if (colthr && kind != 2) {
      fcol[lc] = qsg;
      if (pair) fcol[lc + 1] = qsg;
    }
    __syncthreads();   // the group's solved values and scales are final
    panel_publish();   // the next group's diagonal block (its loads had the whole group)

    // ---- rank-2G update of the rows above the group on the FP64 matrix cores ----
    if (NHW > 0) {
      // the next group's rows now; the rows above it during that group's blocks
      rank_near(au, gn0 > 0 ? gn0 : 0, g0, g0, g1);
      dg0 = g0;
      dg1 = g1;
      drh = gn0 > 0 ? gn0 : 0;
    } else {
      rank_far(std::integral_constant<int, NRC_BIG>{}, g0, g0, g1, 0, 1);
    }
    __syncthreads();
    g1 = gn1;
    g0 = gn0;
  }

  // the second column of a pair takes the exponent its owner carried, and each column its
  // largest |entry|: the maxima its owner kept, or for a column that is not selected, from Y
  // (no wave runs that loop when every column is selected)
  if (colthr && pair) ecol[lc + 1] = e;
  if (colthr) {
    if (selected) {
      if (kind != 2) {
        cmax[lc] = tnx;
        if (pair) cmax[lc + 1] = tny;
      }
    } else {
      double v = 0.0;
      if (inrange)
        for (int i = 0; i < hr; ++i) v = fmax(v, fabs(Y[i * LDY + lc]));
      cmax[lc] = v;
    }
  }
  __syncthreads();
  if (kind == 2) e = ecol[lc];

  // ---- segment norms and exponent ----
  const double nx = colthr ? cmax[lc] : 0.0;   // max |x_i| of this column
  const double ns = owner ? tns : 0.0;         // max |x_i| + |y_i| of a pair (its first column)
  if (own) {
    P.exps[(int64_t)r * m + c] = e;
    P.norms[(int64_t)r * m + c] = nx;
    if (P.segn) {   // (none for a correction solve)
      if (kind == 0) P.segn[(int64_t)r * m + c] = nx;
      if (pair) {
        P.segn[(int64_t)r * m + c] = ns;
        P.segn[(int64_t)r * m + c + 1] = ns;
      }
    }
  }
  if (flags) atomicOr(P.info, flags);
  __syncthreads();
  // Algorithm 2 with a scale that bounds the pair norm of W by one
  {
    const double nxb = colthr ? cmax[lc] + (kind != 0 ? cmax[partner] : 0.0) : 0.0;
    int g = 0;
    if (nxb > 1.0) frexp(nxb, &g);
    if (colthr) colG[lc] = g;
    if (own) {
      const int64_t slot = (int64_t)(r % P.wslots) * m;
      P.eW[slot + c] = e + g;
      P.nW[slot + c] = ldexp(nxb, -g);
    }
  }
  // ---- write the solved tile to Z (thread lc writes row lc: coalesced down each column) ----
  if (lc < hr) {
    double* zrow = P.Z + (r0 + lc) + (int64_t)c0 * ldz;
    for (int col = own_lo; col < own_hi; ++col) zrow[(int64_t)col * ldz] = Y[lc * LDY + (col - lo)];
  }
  __syncthreads();
  // ---- W = 2^-g [X D ; -X B] in operand order: [kstep][col block][lane] ----
  if (P.precision == 1) {
    // split W for the int8 matrix instruction: column exponents, then kSlices slices
    auto& wexp = sm.wexp;
    constexpr int CBM = MB / 16, HK = slice_half_k(MB);
    auto wval = [&](int i, bool lower, int n) -> double {
      const int kd = colKind[n];
      const double x = Y[i * LDY + n];
      if (!lower) return colBe[n] * x;
      const int np = kd == 1 ? n + 1 : (kd == 2 ? n - 1 : n);
      const double xp = Y[i * LDY + np];
      if (kd == 0) return -(colA[n] * x);
      if (kd == 1) return -(colA[n] * x - colB[n] * xp);
      return -(colB[n] * xp + colA[n] * x);
    };
    // the X D half of column c is scaled by 2^b_c, its -X B half by 2^(b_c - D_r)
    const int D = half_offset(P.stmax, P.Mmax, r);
    if (colthr) {
      double mxu = 0.0, mxl = 0.0;
      if (inrange)
        for (int i = 0; i < hr; ++i) {
          mxu = fmax(mxu, fabs(wval(i, false, lc)));
          mxl = fmax(mxl, fabs(wval(i, true, lc)));
        }
      const int f = slice_exponent2(ldexp(mxu, -colG[lc]), ldexp(mxl, -colG[lc]), -D);
      wexp[lc] = f;
      if (own) P.Wexp[(int64_t)(r % P.wslots) * m + c] = f;
    }
    __syncthreads();
    const int64_t npk = slice_packets(MB);
    int4* out = P.Wslc + ((int64_t)(r % P.wslots) * P.Mmax + j) * kSlices * npk;
    // the column blocks this workgroup's columns touch (the last one also clears the blocks
    // past the tile); each packet is one column's, written only by that column's workgroup
    constexpr int KSW = slice_ksteps(MB);
    const int cb_lo = own_lo / 16, cb_hi = last ? CBM : (own_hi + 15) / 16, ob = cb_hi - cb_lo;
    for (int q = lc; q < KSW * ob * 64; q += NTOT) {
      const int l = q % 64, cbo = (q / 64) % ob, ks = q / (64 * ob);
      const int cb = cb_lo + cbo;
      const int64_t pk = ((int64_t)ks * CBM + cb) * 64 + l;
      const int nt = 16 * cb + l % 16;        // tile column
      if (nt < own_lo || (nt >= own_hi && !(last && nt >= hj))) continue;
      const bool nok = nt < own_hi;
      const int n = nok ? nt - lo : 0;        // held column
      const int sh = nok ? colG[n] + wexp[n] - (64 * ks >= HK ? D : 0) : 0;   // (a K step lies in one half)
      double y[16];
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        const int kk = 64 * ks + 16 * (l / 16) + b;
        const bool lower = kk >= HK;
        const int i = lower ? kk - HK : kk;
        y[b] = (nok && i < hr) ? ldexp(wval(i, lower, n), -sh) : 0.0;
      }
      int4 sl[kSlices];
      slice16(y, sl);
#pragma unroll
      for (int p = 0; p < kSlices; ++p) out[p * npk + pk] = sl[p];
    }
  } else {
    constexpr int CBM = MB / 16;
    const int KP = (hr + 15) & ~15;        // rows of each half, padded to the update's K chunk
    const int KS = 2 * KP / 4;
    double* Wj = P.W + ((int64_t)(r % P.wslots) * P.Mmax + j) * w_tile_doubles(MB);
    // a thread keeps one (column block, lane) position of the column blocks this
    // workgroup's columns touch (the last one also clears past the tile) and walks the K
    // steps; an entry is written only by its column's workgroup
    const int cb_lo = own_lo / 16, cb_hi = last ? CBM : (own_hi + 15) / 16;
    for (int q = lc; q < (cb_hi - cb_lo) * 64; q += NTOT) {
      const int cbl = cb_lo * 64 + q;
      const int nt = 16 * (cbl / 64) + cbl % 16;   // tile column
      if (nt < own_lo || (nt >= own_hi && !(last && nt >= hj))) continue;
      const int l16 = (cbl % 64) / 16;
      const bool nok = nt < own_hi;
      const int n = nok ? nt - lo : 0;             // held column
      const int g = nok ? colG[n] : 0;
      const int kd = nok ? colKind[n] : 0;
      const double an = nok ? colA[n] : 0.0, bn = nok ? colB[n] : 0.0, ben = nok ? colBe[n] : 0.0;
      const int np = kd == 1 ? n + 1 : (kd == 2 ? n - 1 : n);
      for (int s = 0; s < KS; ++s) {
        const int kr = 4 * s + l16;
        const bool lower = kr >= KP;
        const int i = lower ? kr - KP : kr;
        double w = 0.0;
        if (nok && i < hr) {
          const double x = Y[i * LDY + n], xp = Y[i * LDY + np];
          if (!lower) w = ben * x;
          else if (kd == 0) w = -(an * x);
          else if (kd == 1) w = -(an * x - bn * xp);
          else w = -(bn * xp + an * x);
          w = ldexp(w, -g);
        }
        Wj[(int64_t)s * (CBM * 64) + cbl] = w;
      }
    }
  }
}

}  // namespace rgev
