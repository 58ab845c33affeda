// Pre-processing (Section 5, first task type): block structure, tile partition,
// normalised eigenvalues (alpha, beta) and every norm the robust updates and solves
// need (Section 4: norms of all super-diagonal tiles of S and T, and of the columns
// the diagonal solves update), plus a common power-of-two prescale of S and T when
// a tile norm would exceed the bound.
#include <hip/hip_runtime.h>

#include "layout.hpp"
#include "robust.hpp"
#include "slices.hpp"

namespace rgev {

// Block structure from S's sub-diagonal (Section 2: blocks of order 1 or 2), the
// selection closed under conjugation (Section 5), and the info word reset.
__device__ __forceinline__ void pre_reset_body(const PencilDesc& P) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *P.info = 0;
    P.ctrl->numax_bits = 0;
    P.ctrl->psc = 1.0;
  }
  if (P.precision == 1 && blockIdx.x == 0)
    for (int i = threadIdx.x; i < 2 * P.Mmax; i += blockDim.x) P.stmax[i] = 0ull;
}

__device__ __forceinline__ void pre_structure_body(const PencilDesc& P) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t m = P.m;
  if (k >= m) return;
  const double sub_k = (k + 1 < m) ? P.S[(k + 1) + k * P.lds] : 0.0;
  const double sub_km1 = (k > 0) ? P.S[k + (k - 1) * P.lds] : 0.0;
  const double sub_km2 = (k > 1) ? P.S[(k - 1) + (k - 2) * P.lds] : 0.0;
  int8_t kind = 0;
  // a first row needs S[k+1,k] != 0 with row k not already the second row of a pair
  if (sub_k != 0.0 && sub_km1 == 0.0) kind = 1;
  else if (sub_km1 != 0.0 && sub_km2 == 0.0) kind = 2;
  if (sub_k != 0.0 && sub_km1 != 0.0) atomicOr(P.info, (int)kInfoBadStructure);
  P.blk[k] = kind;
  int8_t s = 1;
  if (P.select) {
    const int64_t partner = kind == 1 ? k + 1 : (kind == 2 ? k - 1 : k);
    const int a = P.select[k] != 0, b = P.select[partner] != 0;
    s = (int8_t)(a | b);
    if (a != b) atomicOr(P.info, (int)kInfoSelectClosure);
  }
  P.sel[k] = s;
}

// Greedy tile partition: boundaries every MB rows, moved up one row when a boundary
// would split a 2x2 block (Section 3: any partition that does not split a 2x2 block;
// Section 5.1: the default adjusted minimally).  One thread; O(M).
__device__ __forceinline__ void pre_partition_body(const PencilDesc& P) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t m = P.m;
  int M = 0;
  int64_t e = 0;
  P.edges[0] = 0;
  while (e < m && M < P.Mmax) {
    int64_t nx = e + P.mb;
    if (nx >= m) nx = m;
    else if (P.blk[nx] == 2) nx -= 1;
    P.edges[++M] = (int32_t)nx;
    e = nx;
  }
  P.ctrl->M = M;
  P.ctrl->psc = 1.0;
}

__device__ __forceinline__ void pre_tileof_body(const PencilDesc& P) {
  const int t = blockIdx.x;
  if (t >= P.ctrl->M) return;
  const int e0 = P.edges[t], e1 = P.edges[t + 1];
  for (int i = e0 + threadIdx.x; i < e1; i += blockDim.x) P.tileof[i] = t;
}

// Eigenvalue (alpha, beta) of the diagonal block of column c, normalised so that
// max(beta, |Re alpha| + |Im alpha|) lies in (1/2, 1] (the real encoding of
// equations DB1/DB2 then has ||D_jj||, ||B_jj|| <= 1).
__device__ __forceinline__ void pre_eig_body(const PencilDesc& P) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= P.m) return;
  const int8_t kind = P.blk[c];
  const int64_t p = kind == 2 ? c - 1 : c;
  const double* S = P.S;
  const double* T = P.T;
  const int64_t lds = P.lds, ldt = P.ldt;
  double a, b, bt;
  int info = 0;
  if (kind == 0) {
    a = S[p + p * lds];
    bt = T[p + p * ldt];
    if (bt < 0.0 || (bt == 0.0 && signbit(bt))) { a = -a; bt = -bt; }
    b = 0.0;
    if (a == 0.0 && bt == 0.0) info |= kInfoIndefinite;
  } else {
    double s11 = S[p + p * lds], s12 = S[p + (p + 1) * lds];
    double s21 = S[(p + 1) + p * lds], s22 = S[(p + 1) + (p + 1) * lds];
    double t11 = T[p + p * ldt], t12 = T[p + (p + 1) * ldt], t22 = T[(p + 1) + (p + 1) * ldt];
    const double ms = fmax(fmax(fabs(s11), fabs(s12)), fmax(fabs(s21), fabs(s22)));
    const double mt = fmax(fmax(fabs(t11), fabs(t12)), fabs(t22));
    int es = 0, et = 0;
    if (ms > 0.0) frexp(ms, &es);
    if (mt > 0.0) frexp(mt, &et);
    s11 = ldexp(s11, -es); s12 = ldexp(s12, -es); s21 = ldexp(s21, -es); s22 = ldexp(s22, -es);
    t11 = ldexp(t11, -et); t12 = ldexp(t12, -et); t22 = ldexp(t22, -et);
    // det(S_b - lambda T_b) = q2 lambda^2 - q1 lambda + q0
    double q2 = t11 * t22;
    double q1 = s11 * t22 + s22 * t11 - s21 * t12;
    double q0 = s11 * s22 - s12 * s21;
    if (q2 < 0.0) { q2 = -q2; q1 = -q1; q0 = -q0; }
    double disc = q1 * q1 - 4.0 * q2 * q0;
    if (disc >= 0.0) { info |= kInfoRealPair; disc = 0.0; }
    a = 0.5 * q1;
    b = 0.5 * sqrt(-disc);
    bt = q2;
    if (a == 0.0 && b == 0.0 && bt == 0.0) info |= kInfoIndefinite;
    const int d = es - et;   // alpha carries 2^es, beta 2^et
    if (d >= 0) bt = ldexp(bt, -d);
    else { a = ldexp(a, d); b = ldexp(b, d); }
  }
  const double n = fmax(bt, fabs(a) + fabs(b));
  if (n > 0.0) {
    int e;
    frexp(n, &e);
    a = ldexp(a, -e); b = ldexp(b, -e); bt = ldexp(bt, -e);
  }
  P.ar[c] = a;
  P.ai[c] = b;
  P.be[c] = bt;
  if (info) atomicOr(P.info, info);
}

// Tile norms, computed in units of 2^-32 so that no finite input can overflow the
// sums; pre_fixup_kernel converts them after choosing the prescale.
//   k < r : nu[k][r] = max over rows i of tile k of sum_{l in tile r} |S_il| + |T_il|
//   k = r : cnS[c], cnT[c] = max over rows of the tile above c's diagonal block
// One workgroup per tile pair; threads run down rows so every load is coalesced.
constexpr int kNormThreads = 256;

__device__ __forceinline__ void pre_norms_body(const PencilDesc& P) {
  const int M = P.ctrl->M;
  // decode the upper-triangular pair index: bid -> (k, r), k <= r
  const int64_t bid = blockIdx.x;
  const int64_t npairs = (int64_t)M * (M + 1) / 2;
  if (bid >= npairs) return;
  int r = (int)((sqrt(8.0 * (double)bid + 1.0) - 1.0) * 0.5);
  while ((int64_t)(r + 1) * (r + 2) / 2 <= bid) ++r;
  while ((int64_t)r * (r + 1) / 2 > bid) --r;
  const int k = (int)(bid - (int64_t)r * (r + 1) / 2);
  const int k0 = P.edges[k], hk = P.edges[k + 1] - k0;
  const int c0 = P.edges[r], hc = P.edges[r + 1] - c0;
  const double sc = 2.3283064365386963e-10;  // 2^-32
  const double* S = P.S;
  const double* T = P.T;
  const int64_t lds = P.lds, ldt = P.ldt;
  __shared__ double part[kNormThreads];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  if (k < r) {
    // rows spread over threads; the remaining threads take column halves
    const int nrg = (hk + 63) / 64 * 64;   // rows padded to whole waves
    const int groups = kNormThreads / 64;
    double best = 0.0;
    double smx = 0.0, tmx = 0.0;   // largest |S| and |T| of the pair (mixed precision: D_r)
    int nonfinite = 0;
    // each thread owns rows i = tid % 64 + 64 * u and columns l = group, group + groups, ...
    const int lane = threadIdx.x % 64, grp = threadIdx.x / 64;
    for (int i0 = 0; i0 < nrg; i0 += 64) {
      const int i = i0 + lane;
      double s = 0.0;
      if (i < hk) {
        for (int l = grp; l < hc; l += groups) {
          const double sv = S[(k0 + i) + (int64_t)(c0 + l) * lds];
          const double tv = T[(k0 + i) + (int64_t)(c0 + l) * ldt];
          s += fabs(sv) * sc + fabs(tv) * sc;
          smx = fmax(smx, fabs(sv) * sc);
          tmx = fmax(tmx, fabs(tv) * sc);
          nonfinite |= !(isfinite(sv) && isfinite(tv));
        }
      }
      part[threadIdx.x] = s;
      __syncthreads();
      if (grp == 0 && i < hk) {
        double tot = part[lane];
        for (int g = 1; g < groups; ++g) tot += part[lane + 64 * g];
        best = fmax(best, tot);
      }
      __syncthreads();
    }
    if (nonfinite) atomicOr(&bad, 1);
    if (P.precision == 1) {
      for (int off = 32; off > 0; off >>= 1) {
        smx = fmax(smx, __shfl_xor(smx, off));
        tmx = fmax(tmx, __shfl_xor(tmx, off));
      }
      if (lane == 0) {
        if (isfinite(smx)) atomicMax(&P.stmax[r], (unsigned long long)__double_as_longlong(smx));
        if (isfinite(tmx)) atomicMax(&P.stmax[P.Mmax + r], (unsigned long long)__double_as_longlong(tmx));
      }
    }
    // reduce best over the first wave
    if (grp == 0) {
      for (int off = 32; off > 0; off >>= 1) best = fmax(best, __shfl_xor(best, off));
      if (lane == 0) {
        // margin for the rounding of the sums (<= 256 terms) and for underflowed terms
        const double v = best * (1.0 + 9.094947017729282e-13) + 1e-300;
        P.nu[(int64_t)k * P.Mmax + r] = v;
        atomicMax(&P.ctrl->numax_bits, (unsigned long long)__double_as_longlong(v));
      }
    }
  } else {
    // diagonal tile: column norms above each column's diagonal block, and the
    // largest diagonal-block row sum (folded into numax so the prescale covers it)
    for (int l = threadIdx.x; l < hc; l += blockDim.x) {
      const int64_t c = c0 + l;
      const int top = (P.blk[c] == 2) ? l - 1 : l;   // first row of c's diagonal block
      double ms = 0.0, mt = 0.0;
      int nonfinite = 0;
      for (int i = 0; i < top; ++i) {
        const double sv = S[(c0 + i) + c * lds];
        const double tv = T[(c0 + i) + c * ldt];
        ms = fmax(ms, fabs(sv) * sc);
        mt = fmax(mt, fabs(tv) * sc);
        nonfinite |= !(isfinite(sv) && isfinite(tv));
      }
      for (int i = top; i <= l + (P.blk[c] == 1 ? 1 : 0) && i < hc; ++i) {
        const double sv = S[(c0 + i) + c * lds];
        const double tv = (i <= l) ? T[(c0 + i) + c * ldt] : 0.0;
        nonfinite |= !(isfinite(sv) && isfinite(tv));
      }
      P.cnS[c] = ms;
      P.cnT[c] = mt;
      if (nonfinite) atomicOr(&bad, 1);
    }
    // a bound on the row sums of the diagonal tile keeps its entries inside the range too
    double best = 0.0;
    for (int i = threadIdx.x; i < hc; i += blockDim.x) {
      double s = 0.0;
      for (int l = (i > 0 ? i - 1 : 0); l < hc; ++l)
        s += fabs(S[(c0 + i) + (int64_t)(c0 + l) * lds]) * sc + (l >= i ? fabs(T[(c0 + i) + (int64_t)(c0 + l) * ldt]) * sc : 0.0);
      best = fmax(best, s);
    }
    part[threadIdx.x] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
      double v = 0.0;
      for (int t = 0; t < kNormThreads; ++t) v = fmax(v, part[t]);
      if (isfinite(v)) atomicMax(&P.ctrl->numax_bits, (unsigned long long)__double_as_longlong(v));
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && bad) atomicOr(P.info, (int)kInfoNonFinite);
}

// Choose the prescale 2^-sigma so that every tile norm is at most 2^1000 (well below
// Omega), then convert the norms from units of 2^-32.
__device__ __forceinline__ void pre_fixup_body(const PencilDesc& P) {
  const int M = P.ctrl->M;
  const double numax_s = __longlong_as_double((long long)P.ctrl->numax_bits);
  int sigma = 0;
  if (numax_s > 0.0) {
    int e;
    frexp(numax_s, &e);             // numax_s < 2^e
    const int etrue = e + 32;       // true norm < 2^etrue
    if (etrue > 1000) sigma = etrue - 1000;
  }
  const int shift = 32 - sigma;
  const int64_t n_nu = (int64_t)P.Mmax * P.Mmax;
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (tid == 0) {
    P.ctrl->psc = ldexp(1.0, -sigma);
    if (sigma > 0) atomicOr(P.info, (int)kInfoPrescaled);
  }
  for (int64_t i = tid; i < n_nu; i += stride) {
    const int k = (int)(i / P.Mmax), r = (int)(i % P.Mmax);
    if (k < r && r < M) P.nu[i] = ldexp(P.nu[i], shift);
  }
  for (int64_t c = tid; c < P.m; c += stride) {
    P.cnS[c] = ldexp(P.cnS[c], shift) * (1.0 + 2.220446049250313e-16);
    P.cnT[c] = ldexp(P.cnT[c], shift) * (1.0 + 2.220446049250313e-16);
  }
  if (P.precision == 1)   // the mixed-precision updates combine their norms here
    for (int64_t i = tid; i < (int64_t)P.Mmax * P.m; i += stride) P.norms_next[i] = 0ull;
}

// Mixed precision: split every super-diagonal tile pair A = [S_kr | T_kr] (prescaled)
// into row exponents and kSlices int8 slices in the matrix-instruction layout (see
// slices.hpp).  One workgroup per pair (k, r), k < r; runs after pre_fixup (psc known).
constexpr int kSliceThreads = 256;

template <int MB>
__device__ __forceinline__ void pre_slices_tile(const PencilDesc& P, int k, int r) {
  constexpr int HK = slice_half_k(MB), KS = slice_ksteps(MB), RBN = MB / 16;
  __shared__ int rowexp[MB];
  __shared__ double rowmax[2][kSliceThreads / MB > 0 ? kSliceThreads / MB : 1][MB];
  const int k0 = P.edges[k], hk = P.edges[k + 1] - k0;
  const int c0 = P.edges[r], hc = P.edges[r + 1] - c0;
  const double psc = P.ctrl->psc;
  const int64_t lds = P.lds, ldt = P.ldt;
  const int64_t pair = pair_index(k, r);
  // row maxima: thread (g, i) scans columns g, g + G, ... of row i (coalesced down columns)
  constexpr int G = kSliceThreads / MB > 0 ? kSliceThreads / MB : 1;
  const int tid = threadIdx.x;
  if (tid < G * MB) {
    const int i = tid % MB, g = tid / MB;
    double mxs = 0.0, mxt = 0.0;
    if (i < hk)
      for (int l = g; l < hc; l += G) {
        mxs = fmax(mxs, fabs(P.S[(k0 + i) + (int64_t)(c0 + l) * lds]));
        mxt = fmax(mxt, fabs(P.T[(k0 + i) + (int64_t)(c0 + l) * ldt]));
      }
    rowmax[0][g][i] = psc * mxs;
    rowmax[1][g][i] = psc * mxt;
  }
  __syncthreads();
  // the S half of row i is scaled by 2^a_i, its T half by 2^(a_i + D_r)
  const int D = half_offset(P.stmax, P.Mmax, r);
  if (tid < MB) {
    double ms = rowmax[0][0][tid], mt = rowmax[1][0][tid];
    for (int g = 1; g < G; ++g) {
      ms = fmax(ms, rowmax[0][g][tid]);
      mt = fmax(mt, rowmax[1][g][tid]);
    }
    const int e = slice_exponent2(ms, mt, D);
    rowexp[tid] = e;
    P.Aexp[pair * MB + tid] = e;
  }
  __syncthreads();
  // packets: (kstep, row block, lane) -> 16 K values of one row, kSlices slices each
  const int64_t npk = slice_packets(MB);
  int4* out = P.Aslc + pair * kSlices * npk;
  for (int64_t pk = tid; pk < npk; pk += kSliceThreads) {
    const int l = (int)(pk % 64), rb = (int)((pk / 64) % RBN), ks = (int)(pk / (64 * RBN));
    const int i = 16 * rb + l % 16;
    // a K step of 64 lies in one half (HK is a multiple of 64)
    const int e = rowexp[i] + (64 * ks >= HK ? D : 0);
    double y[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) {
      const int kk = 64 * ks + 16 * (l / 16) + b;
      const bool lower = kk >= HK;
      const int cc = lower ? kk - HK : kk;
      double x = 0.0;
      if (i < hk && cc < hc)
        x = lower ? P.T[(k0 + i) + (int64_t)(c0 + cc) * ldt] : P.S[(k0 + i) + (int64_t)(c0 + cc) * lds];
      y[b] = ldexp(psc * x, -e);
    }
    int4 sl[kSlices];
    slice16(y, sl);
#pragma unroll
    for (int p = 0; p < kSlices; ++p) out[p * npk + pk] = sl[p];
  }
  (void)KS;
}

__device__ __forceinline__ void pre_slices_body(const PencilDesc& P) {
  const int M = P.ctrl->M;
  const int64_t bid = blockIdx.x;
  if (bid >= (int64_t)M * (M - 1) / 2) return;
  int r = (int)((1.0 + sqrt(1.0 + 8.0 * (double)bid)) * 0.5);
  while ((int64_t)r * (r - 1) / 2 > bid) --r;
  while ((int64_t)(r + 1) * r / 2 <= bid) ++r;
  const int k = (int)(bid - (int64_t)r * (r - 1) / 2);
  switch (P.mb) {
    case 32: pre_slices_tile<32>(P, k, r); break;
    case 64: pre_slices_tile<64>(P, k, r); break;
    default: pre_slices_tile<128>(P, k, r); break;
  }
}

// Kernels: one pencil (descriptor by value), or one pencil per blockIdx.y of a table.
#define RGEV_PRE_KERNELS(name, bounds)                                                      \
  __global__ bounds void name##_kernel(PencilDesc P) { name##_body(P); }                  \
  __global__ bounds void name##_batched(const PencilDesc* __restrict__ D) {              \
    const PencilDesc P = D[blockIdx.y];                                                   \
    name##_body(P);                                                                       \
  }
RGEV_PRE_KERNELS(pre_reset, )
RGEV_PRE_KERNELS(pre_structure, )
RGEV_PRE_KERNELS(pre_partition, )
RGEV_PRE_KERNELS(pre_tileof, )
RGEV_PRE_KERNELS(pre_eig, )
RGEV_PRE_KERNELS(pre_norms, __launch_bounds__(kNormThreads))
RGEV_PRE_KERNELS(pre_fixup, )
RGEV_PRE_KERNELS(pre_slices, __launch_bounds__(kSliceThreads))
#undef RGEV_PRE_KERNELS

void launch_preprocess(const PencilDesc& P, hipStream_t s) {
  const int64_t m = P.m;
  const int nb = (int)((m + 255) / 256);
  pre_reset_kernel<<<1, 64, 0, s>>>(P);
  pre_structure_kernel<<<nb, 256, 0, s>>>(P);
  pre_partition_kernel<<<1, 64, 0, s>>>(P);
  pre_tileof_kernel<<<P.Mmax, 128, 0, s>>>(P);
  pre_eig_kernel<<<nb, 256, 0, s>>>(P);
  const int64_t npairs = (int64_t)P.Mmax * (P.Mmax + 1) / 2;
  pre_norms_kernel<<<(unsigned)npairs, kNormThreads, 0, s>>>(P);
  pre_fixup_kernel<<<64, 256, 0, s>>>(P);
  if (P.precision == 1 && P.Mmax > 1)
    pre_slices_kernel<<<(unsigned)((int64_t)P.Mmax * (P.Mmax - 1) / 2), kSliceThreads, 0, s>>>(P);
}

// The same sequence for n pencils of one table (orders <= max_m, tile counts <= max_tiles).
void launch_preprocess_batched(const PencilDesc* D, int n, int64_t max_m, int max_tiles, hipStream_t s) {
  if (n <= 0) return;
  const unsigned nb = (unsigned)((max_m + 255) / 256);
  const unsigned npairs = (unsigned)((int64_t)max_tiles * (max_tiles + 1) / 2);
  const unsigned un = (unsigned)n;
  pre_reset_batched<<<dim3(1, un), 64, 0, s>>>(D);
  pre_structure_batched<<<dim3(nb, un), 256, 0, s>>>(D);
  pre_partition_batched<<<dim3(1, un), 64, 0, s>>>(D);
  pre_tileof_batched<<<dim3((unsigned)max_tiles, un), 128, 0, s>>>(D);
  pre_eig_batched<<<dim3(nb, un), 256, 0, s>>>(D);
  pre_norms_batched<<<dim3(npairs, un), kNormThreads, 0, s>>>(D);
  pre_fixup_batched<<<dim3(8, un), 256, 0, s>>>(D);
}

}  // namespace rgev
