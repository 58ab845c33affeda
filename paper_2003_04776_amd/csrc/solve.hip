// Diagonal-tile solves of Algorithm 1 (Section 3): kernel 1 computes the tips Y_jj,
// the eigenvectors of the small pencil (S_jj, T_jj); kernel 3 solves
// S_ii Z D_jj - T_ii Z B_jj = Y_ij.  Both are robust back-substitution over the
// 1x1/2x2 blocks of the diagonal tile (Section 4: every division protected by
// ProtectDivision, every column update by ProtectUpdate, scale factors as integer
// exponents).  After the solve, the tile is turned into the right-updated operand of
// Algorithm 2, W = 2^-g [X D ; -X B], packed for the FP64 matrix instruction.
//
// One workgroup per tile (i, j); one thread per eigenvector column of tile j.  The
// tile Y_ij lives in LDS for the whole solve; the columns of S_ii and T_ii that a step
// needs are staged into LDS one block ahead.  A complex pair occupies two adjacent
// threads that both evaluate the complex pivot arithmetic and keep their own part.
#include <hip/hip_runtime.h>

#include "layout.hpp"
#include "robust.hpp"

namespace rgev {

struct Cx {
  double r, i;
};
__device__ __forceinline__ Cx cx(double r, double i) { return Cx{r, i}; }
__device__ __forceinline__ Cx cmul(Cx x, Cx y) { return Cx{x.r * y.r - x.i * y.i, x.r * y.i + x.i * y.r}; }
__device__ __forceinline__ Cx csub(Cx x, Cx y) { return Cx{x.r - y.r, x.i - y.i}; }
__device__ __forceinline__ double cn1(Cx x) { return fabs(x.r) + fabs(x.i); }
__device__ __forceinline__ Cx cdivx(Cx x, Cx y) {
  Cx z;
  complex_div(x.r, x.i, y.r, y.i, z.r, z.i);
  return z;
}
__device__ __forceinline__ Cx cscl(Cx x, int q) { return q ? Cx{ldexp(x.r, -q), ldexp(x.i, -q)} : x; }

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

// (beta s - alpha t) w = y for one row; alpha = a + i b (b = 0 for a real column).
__device__ __forceinline__ Cx solve1(double a, double b, double be, double s, double t, Cx y, int& qs,
                                     int& flags) {
  Cx d = cx(be * s - a * t, -b * t);
  const double smin = local_smin(be, fabs(a) + fabs(b), fabs(s), fabs(t));
  if (cn1(d) < smin) {
    d = cx(smin, 0.0);
    flags |= kInfoPerturbed;
  }
  // |y/d|_1 <= 2 |y|_1 / |d|_1
  const int q = with_margin(protect_division(cn1(y), 0.5 * cn1(d)));
  qs += q;
  return cdivx(cscl(y, q), d);
}

// 2x2 block: Gaussian elimination with complete pivoting on |.|_1, every division
// and update protected.  y0, y1 are the block's rows; the solution replaces them.
// (Written with selects only, so nothing is indexed dynamically.)
__device__ __forceinline__ void solve2(double a, double b, double be, double s00, double s01, double s10,
                                       double s11, double t00, double t01, double t11, Cx& y0, Cx& y1,
                                       int& qs, int& flags) {
  const Cx C00 = cx(be * s00 - a * t00, -b * t00);
  const Cx C01 = cx(be * s01 - a * t01, -b * t01);
  const Cx C10 = cx(be * s10, 0.0);
  const Cx C11 = cx(be * s11 - a * t11, -b * t11);
  const double smax = fmax(fmax(fabs(s00), fabs(s01)), fmax(fabs(s10), fabs(s11)));
  const double tmax = fmax(fmax(fabs(t00), fabs(t01)), fabs(t11));
  const double smin = local_smin(be, fabs(a) + fabs(b), smax, tmax);
  const double v00 = cn1(C00), v01 = cn1(C01), v10 = cn1(C10), v11 = cn1(C11);
  // pivot (ip, jp): the entry of largest |.|_1
  int ip = 0, jp = 0;
  double best = v00;
  if (v01 > best) { best = v01; ip = 0; jp = 1; }
  if (v10 > best) { best = v10; ip = 1; jp = 0; }
  if (v11 > best) { best = v11; ip = 1; jp = 1; }
  Cx u11, u12, c21, c22;
  if (best < smin) {
    u11 = cx(smin, 0.0); u12 = cx(0.0, 0.0); c21 = cx(0.0, 0.0); c22 = cx(smin, 0.0);
    ip = 0; jp = 0;
    flags |= kInfoPerturbed;
  } else {
    // rows/columns permuted so the pivot is (0, 0): u11 = C[ip][jp], u12 = C[ip][1-jp],
    // c21 = C[1-ip][jp], c22 = C[1-ip][1-jp]
    const Cx r0a = ip ? C10 : C00, r0b = ip ? C11 : C01;   // pivot row
    const Cx r1a = ip ? C00 : C10, r1b = ip ? C01 : C11;   // other row
    u11 = jp ? r0b : r0a;
    u12 = jp ? r0a : r0b;
    c21 = jp ? r1b : r1a;
    c22 = jp ? r1a : r1b;
  }
  const Cx l21 = cdivx(c21, u11);
  Cx u22 = csub(c22, cmul(l21, u12));
  if (cn1(u22) < smin) {
    u22 = cx(smin, 0.0);
    flags |= kInfoPerturbed;
  }
  Cx ya = ip ? y1 : y0, yb = ip ? y0 : y1;
  int q = with_margin(protect_update(cn1(l21), cn1(ya), cn1(yb)));
  ya = cscl(ya, q); yb = cscl(yb, q); qs += q;
  Cx r2 = csub(yb, cmul(l21, ya));
  q = with_margin(protect_division(cn1(r2), 0.5 * cn1(u22)));
  r2 = cscl(r2, q); ya = cscl(ya, q); qs += q;
  Cx w2 = cdivx(r2, u22);
  q = with_margin(protect_update(cn1(u12), cn1(w2), cn1(ya)));
  w2 = cscl(w2, q); ya = cscl(ya, q); qs += q;
  Cx n1 = csub(ya, cmul(u12, w2));
  q = with_margin(protect_division(cn1(n1), 0.5 * cn1(u11)));
  n1 = cscl(n1, q); w2 = cscl(w2, q); qs += q;
  const Cx w1 = cdivx(n1, u11);
  // unknown jp gets w1, the other gets w2
  y0 = jp ? w2 : w1;
  y1 = jp ? w1 : w2;
}

template <int MB>
__global__ __launch_bounds__(MB) void solve_kernel(PencilDesc P, int r) {
  constexpr int LDY = MB + 1;   // odd stride: row and column sweeps are both conflict-free
  constexpr int PW = 4;         // columns per staged panel of S_rr and T_rr
  __shared__ double Y[MB * LDY];
  __shared__ double stS[2][PW][MB];   // [panel slot][column in panel][row]
  __shared__ double stT[2][PW][MB];
  __shared__ double tcnS[MB], tcnT[MB];
  __shared__ int8_t tblk[MB];
  __shared__ double cmax[MB];
  __shared__ double colA[MB], colB[MB], colBe[MB];
  __shared__ int colG[MB];
  __shared__ int8_t colKind[MB];

  const int M = P.ctrl->M;
  const int j = r + (int)blockIdx.x;
  if (r >= M || j >= M) return;
  const int64_t m = P.m;
  const int r0 = P.edges[r], hr = P.edges[r + 1] - r0;
  const int c0 = P.edges[j], hj = P.edges[j + 1] - c0;
  const bool tip = (r == j);
  const double psc = P.ctrl->psc;
  const double* S = P.S;
  const double* T = P.T;
  const int64_t lds = P.lds, ldt = P.ldt, ldz = P.ldz;

  const int lc = threadIdx.x;
  const bool inrange = lc < hj;
  const int64_t c = c0 + lc;
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
  const int pc = (kind == 2 ? lc - 1 : lc) + (c0 - r0);   // local row of own block (tip tile)
  const double aabs = fabs(a) + fabs(b);
  int e = 0;
  double ybound = 0.0;
  int flags = 0;

  // ---- structure and column norms of the diagonal tile, right-hand side Y_rj ----
  if (lc < hr) {
    tblk[lc] = P.blk[r0 + lc];
    tcnS[lc] = P.cnS[r0 + lc];
    tcnT[lc] = P.cnT[r0 + lc];
  }
  for (int idx = lc; idx < MB * LDY; idx += MB) Y[idx] = 0.0;
  __syncthreads();
  if (!tip) {
    // thread lc reads row lc of every column (coalesced down the columns), 16 loads in flight
    if (lc < hr) {
      const double* zrow = P.Z + (r0 + lc) + (int64_t)c0 * ldz;
      for (int col0 = 0; col0 < hj; col0 += 16) {
        double v[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) v[t] = (col0 + t < hj) ? zrow[(int64_t)(col0 + t) * ldz] : 0.0;
#pragma unroll
        for (int t = 0; t < 16; ++t)
          if (col0 + t < hj) Y[lc * LDY + col0 + t] = v[t];
      }
    }
    if (inrange) {
      e = P.exps[(int64_t)r * m + c];
      ybound = P.norms[(int64_t)r * m + c] + (kind != 0 ? P.norms[(int64_t)r * m + c0 + partner] : 0.0);
    }
  }

  // ---- panels of S_rr, T_rr: panel p = columns [PW p, PW p + PW), slot p % 2 ----
  double pfS[PW], pfT[PW];
  auto panel_fetch = [&](int p) {
#pragma unroll
    for (int t = 0; t < PW; ++t) {
      const int col = PW * p + t;
      const bool ok = p >= 0 && col < hr && lc < hr;
      pfS[t] = ok ? S[(r0 + lc) + (r0 + col) * lds] : 0.0;
      pfT[t] = ok ? T[(r0 + lc) + (r0 + col) * ldt] : 0.0;
    }
  };
  auto panel_publish = [&](int p) {
#pragma unroll
    for (int t = 0; t < PW; ++t) {
      stS[p & 1][t][lc] = psc * pfS[t];
      stT[p & 1][t][lc] = psc * pfT[t];
    }
  };
  auto SC = [&](int col) -> const double* { return stS[(col / PW) & 1][col % PW]; };
  auto TC = [&](int col) -> const double* { return stT[(col / PW) & 1][col % PW]; };

  int plow = (hr - 1) / PW;   // lowest-numbered panel resident in LDS
  panel_fetch(plow);
  panel_publish(plow);
  panel_fetch(plow - 1);
  if ((tblk[hr - 1] == 2 ? hr - 2 : hr - 1) < PW * plow) {   // the first block reaches below
    --plow;
    panel_publish(plow);
    panel_fetch(plow - 1);
  }
  __syncthreads();

  int q = hr - 1;
  while (q >= 0) {
    const int q0 = (tblk[q] == 2) ? q - 1 : q;
    const int nb = q - q0 + 1;
    // ---- phase A: small solve of the block (rows q0..q) ----
    const bool work = selected && !(tip && q0 > pc);
    Cx z0 = cx(0.0, 0.0), z1 = cx(0.0, 0.0);
    int qs = 0;
    double cn = 0.0;
    if (work) {
      auto yv = [&](int row) -> Cx {
        if (kind == 0) return cx(Y[row * LDY + lc], 0.0);
        const double own = Y[row * LDY + lc], oth = Y[row * LDY + partner];
        return kind == 1 ? cx(own, oth) : cx(oth, own);
      };
      if (tip && q0 == pc) {
        if (nb == 1) {
          z0 = cx(1.0, 0.0);
        } else {
          // second row of the singular block beta S_b - alpha T_b gives z_p for z_{p+1} = 1
          const double s21 = SC(q0)[q], s22 = SC(q)[q], t22 = TC(q)[q];
          double m21 = be * s21;
          const Cx nn = cx(-(be * s22 - a * t22), b * t22);
          const double smin = local_smin(be, aabs, fmax(fabs(s21), fabs(s22)), fabs(t22));
          if (fabs(m21) < smin) { m21 = smin; flags |= kInfoPerturbed; }
          const int qd = with_margin(protect_division(cn1(nn), fabs(m21)));
          const Cx ns = cscl(nn, qd);
          z0 = cx(ns.r / m21, ns.i / m21);
          z1 = cx(ldexp(1.0, -qd), 0.0);
          qs += qd;
        }
      } else if (nb == 1) {
        z0 = solve1(a, b, be, SC(q)[q], TC(q)[q], yv(q), qs, flags);
      } else {
        z0 = yv(q0);
        z1 = yv(q);
        solve2(a, b, be, SC(q0)[q0], SC(q)[q0], SC(q0)[q], SC(q)[q], TC(q0)[q0], TC(q)[q0], TC(q)[q],
               z0, z1, qs, flags);
      }
      if (q0 > 0) {
        // ProtectUpdate for y[0:q0] -= (beta S - alpha T)[0:q0, q0..q] z
        cn = be * tcnS[q0] + aabs * tcnT[q0];
        if (nb == 2) cn += be * tcnS[q] + aabs * tcnT[q];
        const double zn = fmax(cn1(z0), cn1(z1));
        const int qu = with_margin(protect_update(cn, zn, ldexp(ybound, -qs)));
        z0 = cscl(z0, qu);
        z1 = cscl(z1, qu);
        qs += qu;
      }
    }
    __syncthreads();   // every thread has read rows q0..q before any is overwritten
    if (work) {
      // the scale applies to the whole segment: the solved rows below now, the rows
      // above inside the update loop (f is an exact power of two)
      double f = 1.0;
      if (qs > 0) {
        for (int i = q + 1; i < hr; ++i) Y[i * LDY + lc] = ldexp(Y[i * LDY + lc], -qs);
        if (qs <= 1000) {
          f = ldexp(1.0, -qs);
        } else {
          for (int i = 0; i < q0; ++i) Y[i * LDY + lc] = ldexp(Y[i * LDY + lc], -qs);
        }
        e += qs;
        ybound = ldexp(ybound, -qs);
      }
      const bool im = (kind == 2);
      Y[q0 * LDY + lc] = im ? z0.i : z0.r;
      if (nb == 2) Y[q * LDY + lc] = im ? z1.i : z1.r;
      if (q0 > 0) {
        // u = beta z, v = alpha z (own real or imaginary part)
        const double u0 = be * (im ? z0.i : z0.r);
        const double v0 = im ? (b * z0.r + a * z0.i) : (a * z0.r - b * z0.i);
        const double* sc0 = SC(q0);
        const double* tc0 = TC(q0);
        if (nb == 1) {
#pragma unroll 4
          for (int i = 0; i < q0; ++i) {
            const double y = Y[i * LDY + lc];
            Y[i * LDY + lc] = y * f - (sc0[i] * u0 - tc0[i] * v0);
          }
        } else {
          const double u1 = be * (im ? z1.i : z1.r);
          const double v1 = im ? (b * z1.r + a * z1.i) : (a * z1.r - b * z1.i);
          const double* sc1 = SC(q);
          const double* tc1 = TC(q);
#pragma unroll 4
          for (int i = 0; i < q0; ++i) {
            const double y = Y[i * LDY + lc];
            Y[i * LDY + lc] = y * f - ((sc0[i] * u0 - tc0[i] * v0) + (sc1[i] * u1 - tc1[i] * v1));
          }
        }
        ybound += cn * fmax(cn1(z0), cn1(z1));
      }
    }
    // the next block ends at q0 - 1; publish the panel below when it reaches into it
    const int qn = q0 - 1;
    if (qn >= 0) {
      const int qn0 = (tblk[qn] == 2) ? qn - 1 : qn;
      if (qn0 < PW * plow) {
        --plow;
        panel_publish(plow);
        panel_fetch(plow - 1);
      }
    }
    __syncthreads();
    q = q0 - 1;
  }

  // ---- segment norm and exponent ----
  double nx = 0.0;
  for (int i = 0; i < hr; ++i) nx = fmax(nx, fabs(Y[i * LDY + lc]));
  cmax[lc] = nx;
  colA[lc] = a;
  colB[lc] = b;
  colBe[lc] = be;
  colKind[lc] = (int8_t)kind;
  if (inrange) {
    P.exps[(int64_t)r * m + c] = e;
    P.norms[(int64_t)r * m + c] = nx;
  }
  if (flags) atomicOr(P.info, flags);
  __syncthreads();
  // Algorithm 2 with a scale that bounds the pair norm of W by one
  {
    const double nxb = cmax[lc] + (kind != 0 ? cmax[partner] : 0.0);
    int g = 0;
    if (nxb > 1.0) frexp(nxb, &g);
    colG[lc] = g;
    if (inrange) {
      const int64_t slot = (int64_t)(r % P.wslots) * m;
      P.eW[slot + c] = e + g;
      P.nW[slot + c] = ldexp(nxb, -g);
    }
  }
  // ---- write the solved tile to Z (thread lc writes row lc: coalesced down each column) ----
  if (lc < hr) {
    double* zrow = P.Z + (r0 + lc) + (int64_t)c0 * ldz;
    for (int col = 0; col < hj; ++col) zrow[(int64_t)col * ldz] = Y[lc * LDY + col];
  }
  __syncthreads();
  // ---- W = 2^-g [X D ; -X B] in operand order: [kstep][col block][lane] ----
  {
    constexpr int CBM = MB / 16;
    const int KP = (hr + 15) & ~15;        // rows of each half, padded to the update's K chunk
    const int KS = 2 * KP / 4;
    const int total = KS * CBM * 64;
    double* Wj = P.W + ((int64_t)(r % P.wslots) * P.Mmax + j) * w_tile_doubles(MB);
    for (int idx = lc; idx < total; idx += MB) {
      const int s = idx / (CBM * 64);
      const int rem = idx % (CBM * 64);
      const int cb = rem / 64, l = rem % 64;
      const int kr = 4 * s + l / 16;
      const int n = 16 * cb + l % 16;
      double w = 0.0;
      if (n < hj) {
        const bool lower = kr >= KP;
        const int i = lower ? kr - KP : kr;
        if (i < hr) {
          const int g = colG[n];
          const int kd = colKind[n];
          const double x = Y[i * LDY + n];
          if (!lower) {
            w = colBe[n] * x;
          } else {
            const double an = colA[n], bn = colB[n];
            if (kd == 0) w = an * x;
            else if (kd == 1) w = an * x - bn * Y[i * LDY + n + 1];
            else w = bn * Y[i * LDY + n - 1] + an * x;
            w = -w;
          }
          w = ldexp(w, -g);
        }
      }
      Wj[idx] = w;
    }
  }
}

template <int MB>
static void launch_solve_t(const PencilDesc& P, int r, hipStream_t s) {
  solve_kernel<MB><<<P.Mmax - r, MB, 0, s>>>(P, r);
}

void launch_solve(const PencilDesc& P, int r, hipStream_t s) {
  switch (P.mb) {
    case 32: launch_solve_t<32>(P, r, s); break;
    case 64: launch_solve_t<64>(P, r, s); break;
    default: launch_solve_t<128>(P, r, s); break;
  }
}

}  // namespace rgev
