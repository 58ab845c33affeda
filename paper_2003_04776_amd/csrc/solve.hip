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
  const int q = protect_division(cn1(y), 0.5 * cn1(d));
  qs += q;
  return cdivx(cscl(y, q), d);
}

// 2x2 block: Gaussian elimination with complete pivoting on |.|_1, every division
// and update protected.  y[0], y[1] are the block's rows; the solution replaces them.
__device__ __forceinline__ void solve2(double a, double b, double be, const double s[2][2],
                                       const double t[2][2], Cx y[2], int& qs, int& flags) {
  Cx C[2][2];
  double smax = 0.0, tmax = 0.0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const double tv = (i > j) ? 0.0 : t[i][j];
      C[i][j] = cx(be * s[i][j] - a * tv, -b * tv);
      smax = fmax(smax, fabs(s[i][j]));
      tmax = fmax(tmax, fabs(tv));
    }
  const double smin = local_smin(be, fabs(a) + fabs(b), smax, tmax);
  int ip = 0, jp = 0;
  double best = -1.0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const double v = cn1(C[i][j]);
      if (v > best) { best = v; ip = i; jp = j; }
    }
  if (best < smin) {
    C[0][0] = cx(smin, 0.0); C[0][1] = cx(0.0, 0.0);
    C[1][0] = cx(0.0, 0.0); C[1][1] = cx(smin, 0.0);
    ip = 0; jp = 0;
    flags |= kInfoPerturbed;
  }
  const int io = 1 - ip, jo = 1 - jp;
  const Cx u11 = C[ip][jp], u12 = C[ip][jo];
  const Cx l21 = cdivx(C[io][jp], u11);
  Cx u22 = csub(C[io][jo], cmul(l21, u12));
  if (cn1(u22) < smin) {
    u22 = cx(smin, 0.0);
    flags |= kInfoPerturbed;
  }
  Cx y1 = y[ip], y2 = y[io];
  int q = protect_update(cn1(l21), cn1(y1), cn1(y2));
  y1 = cscl(y1, q); y2 = cscl(y2, q); qs += q;
  Cx r2 = csub(y2, cmul(l21, y1));
  q = protect_division(cn1(r2), 0.5 * cn1(u22));
  r2 = cscl(r2, q); y1 = cscl(y1, q); qs += q;
  Cx w2 = cdivx(r2, u22);
  q = protect_update(cn1(u12), cn1(w2), cn1(y1));
  w2 = cscl(w2, q); y1 = cscl(y1, q); qs += q;
  Cx n1 = csub(y1, cmul(u12, w2));
  q = protect_division(cn1(n1), 0.5 * cn1(u11));
  n1 = cscl(n1, q); w2 = cscl(w2, q); qs += q;
  const Cx w1 = cdivx(n1, u11);
  y[jp] = w1;
  y[jo] = w2;
}

template <int MB>
__global__ __launch_bounds__(MB) void solve_kernel(PencilDesc P, int r) {
  constexpr int LDY = MB + 1;   // odd stride: row and column sweeps are both conflict-free
  __shared__ double Y[MB * LDY];
  __shared__ double stS[2][2][MB];   // [buffer][slot: 0 = column q, 1 = column q-1][row]
  __shared__ double stT[2][2][MB];
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

  // ---- right-hand side Y_rj (zero for the tip tile) ----
  for (int idx = lc; idx < MB * LDY; idx += MB) Y[idx] = 0.0;
  __syncthreads();
  if (!tip) {
    for (int idx = lc; idx < hr * hj; idx += MB) {
      const int i = idx % hr, col = idx / hr;
      Y[i * LDY + col] = P.Z[(r0 + i) + (c0 + col) * ldz];
    }
    if (inrange) {
      e = P.exps[(int64_t)r * m + c];
      ybound = P.norms[(int64_t)r * m + c] + (kind != 0 ? P.norms[(int64_t)r * m + c0 + partner] : 0.0);
    }
  }
  // ---- stage the first block's two columns ----
  {
    const int qa = hr - 1, qb = hr - 2;
    if (lc < hr) {
      stS[0][0][lc] = psc * S[(r0 + lc) + (r0 + qa) * lds];
      stT[0][0][lc] = psc * T[(r0 + lc) + (r0 + qa) * ldt];
      stS[0][1][lc] = qb >= 0 ? psc * S[(r0 + lc) + (r0 + qb) * lds] : 0.0;
      stT[0][1][lc] = qb >= 0 ? psc * T[(r0 + lc) + (r0 + qb) * ldt] : 0.0;
    }
  }
  __syncthreads();

  int buf = 0;
  int q = hr - 1;
  while (q >= 0) {
    const int q0 = (P.blk[r0 + q] == 2) ? q - 1 : q;
    const int nb = q - q0 + 1;
    const int s0 = nb - 1;   // stage slot of column q0
    // prefetch the next block's two columns
    const int qn = q0 - 1;
    double pS0 = 0.0, pT0 = 0.0, pS1 = 0.0, pT1 = 0.0;
    if (qn >= 0 && lc < hr) {
      pS0 = S[(r0 + lc) + (r0 + qn) * lds];
      pT0 = T[(r0 + lc) + (r0 + qn) * ldt];
      if (qn >= 1) {
        pS1 = S[(r0 + lc) + (r0 + qn - 1) * lds];
        pT1 = T[(r0 + lc) + (r0 + qn - 1) * ldt];
      }
    }
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
          const double s21 = stS[buf][1][q], s22 = stS[buf][0][q], t22 = stT[buf][0][q];
          double m21 = be * s21;
          const Cx nn = cx(-(be * s22 - a * t22), b * t22);
          const double smin = local_smin(be, aabs, fmax(fabs(s21), fabs(s22)), fabs(t22));
          if (fabs(m21) < smin) { m21 = smin; flags |= kInfoPerturbed; }
          const int qd = protect_division(cn1(nn), fabs(m21));
          const Cx ns = cscl(nn, qd);
          z0 = cx(ns.r / m21, ns.i / m21);
          z1 = cx(ldexp(1.0, -qd), 0.0);
          qs += qd;
        }
      } else if (nb == 1) {
        z0 = solve1(a, b, be, stS[buf][0][q], stT[buf][0][q], yv(q), qs, flags);
      } else {
        const double s2[2][2] = {{stS[buf][1][q0], stS[buf][0][q0]}, {stS[buf][1][q], stS[buf][0][q]}};
        const double t2[2][2] = {{stT[buf][1][q0], stT[buf][0][q0]}, {0.0, stT[buf][0][q]}};
        Cx yy[2] = {yv(q0), yv(q)};
        solve2(a, b, be, s2, t2, yy, qs, flags);
        z0 = yy[0];
        z1 = yy[1];
      }
      if (q0 > 0) {
        // ProtectUpdate for y[0:q0] -= (beta S - alpha T)[0:q0, q0..q] z
        cn = be * P.cnS[r0 + q0] + aabs * P.cnT[r0 + q0];
        if (nb == 2) cn += be * P.cnS[r0 + q] + aabs * P.cnT[r0 + q];
        const double zn = fmax(cn1(z0), cn1(z1));
        const int qu = protect_update(cn, zn, ldexp(ybound, -qs));
        z0 = cscl(z0, qu);
        z1 = cscl(z1, qu);
        qs += qu;
      }
    }
    __syncthreads();   // every thread has read rows q0..q before any is overwritten
    if (work) {
      if (qs > 0) {
        for (int i = 0; i < hr; ++i) Y[i * LDY + lc] = ldexp(Y[i * LDY + lc], -qs);
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
        const double* sc0 = stS[buf][s0];
        const double* tc0 = stT[buf][s0];
        if (nb == 1) {
#pragma unroll 4
          for (int i = 0; i < q0; ++i) {
            double y = Y[i * LDY + lc];
            y -= sc0[i] * u0 - tc0[i] * v0;
            Y[i * LDY + lc] = y;
          }
        } else {
          const double u1 = be * (im ? z1.i : z1.r);
          const double v1 = im ? (b * z1.r + a * z1.i) : (a * z1.r - b * z1.i);
          const double* sc1 = stS[buf][0];
          const double* tc1 = stT[buf][0];
#pragma unroll 4
          for (int i = 0; i < q0; ++i) {
            double y = Y[i * LDY + lc];
            y -= (sc0[i] * u0 - tc0[i] * v0) + (sc1[i] * u1 - tc1[i] * v1);
            Y[i * LDY + lc] = y;
          }
        }
        ybound += cn * fmax(cn1(z0), cn1(z1));
      }
    }
    // publish the prefetched columns for the next block
    if (qn >= 0 && lc < hr) {
      stS[buf ^ 1][0][lc] = psc * pS0;
      stT[buf ^ 1][0][lc] = psc * pT0;
      stS[buf ^ 1][1][lc] = psc * pS1;
      stT[buf ^ 1][1][lc] = psc * pT1;
    }
    __syncthreads();
    buf ^= 1;
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
      const int64_t slot = (int64_t)(r % P.band) * m;
      P.eW[slot + c] = e + g;
      P.nW[slot + c] = ldexp(nxb, -g);
    }
  }
  // ---- write the solved tile to Z (coalesced down each column) ----
  for (int idx = lc; idx < hr * hj; idx += MB) {
    const int i = idx % hr, col = idx / hr;
    P.Z[(r0 + i) + (c0 + col) * ldz] = Y[i * LDY + col];
  }
  __syncthreads();
  // ---- W = 2^-g [X D ; -X B] in operand order: [kstep][col block][lane] ----
  {
    constexpr int CBM = MB / 16;
    const int KP = (hr + 15) & ~15;        // rows of each half, padded to the update's K chunk
    const int KS = 2 * KP / 4;
    const int total = KS * CBM * 64;
    double* Wj = P.W + ((int64_t)(r % P.band) * P.Mmax + j) * w_tile_doubles(MB);
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
