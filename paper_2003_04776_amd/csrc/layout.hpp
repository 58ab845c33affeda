// Per-pencil descriptor shared by the host driver and every kernel, and the
// carve-up of the caller's workspace.
//
// Data layout in HBM (m = order, MB = nominal tile size, Mmax = bound on the tile
// count M, which is only known on the device after the structure scan):
//   S, T, Z            caller's column-major matrices (ld >= m)
//   blk[m]   int8      0 = 1x1 block, 1 = first row of a 2x2 block, 2 = second row
//   sel[m]   int8      selection after closure under conjugation
//   tileof[m] int32    tile index of each row/column
//   edges[Mmax+1]      tile boundaries (greedy: MB rows, or MB-1 if MB would split a pair)
//   ar, ai, be [m]     normalised eigenvalue of each column (ai > 0 for both columns of a pair)
//   cnS, cnT [m]       per column: largest |S|, |T| above the column's diagonal block
//                      inside its own diagonal tile (norms for the diagonal solves)
//   nu[Mmax*Mmax]      nu[k*Mmax + r] >= max_i sum_l |S_il| + |T_il| over tile pair (k, r)
//   exps[Mmax*m]       exponent of segment (tile row k, column c): value = 2^e * mantissa
//   norms[Mmax*m]      infinity norm (upper bound) of that segment's mantissa
//   W[2R * Mmax * WS]  right-updated tiles of the last 2R solved source rows (Algorithm 2),
//                      slot (r % 2R) * Mmax + j (two bands, so a band's solves never
//                      overwrite what the previous band's update still reads), packed in
//                      the operand order of the FP64 matrix instruction
//   eW, nW [2R * m]    exponent and norm bound of W per source-row slot and column
//   (the persistent walker keeps W, eW, nW of every source row: Mmax slots, and its
//   work list and counters, see WalkDesc)
//   Aslc, Aexp         mixed precision: split slices and row exponents of every tile pair
//                      (k, r), k < r (triangular index), written by pre-processing
//   Wslc, Wexp         mixed precision: split slices and column exponents of W per slot
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rgev {

struct Ctrl {
  int32_t M;          // number of tiles
  int32_t pad0;
  double psc;         // common power-of-two prescale of S and T (1 = none)
  unsigned long long numax_bits;  // largest scaled tile-pair norm (as bits, >= 0)
  int32_t info_local; // info target when the caller passed NULL
  int32_t pad1[9];
};

struct PencilDesc {
  int64_t m, lds, ldt, ldz;
  const double* S;
  const double* T;
  double* Z;
  int32_t* scales;
  const int32_t* select;
  int32_t* info;
  int8_t* blk;
  int8_t* sel;
  int32_t* tileof;
  int32_t* edges;
  double* ar;
  double* ai;
  double* be;
  double* cnS;
  double* cnT;
  double* nu;
  int32_t* exps;
  double* norms;
  // segn[t][c]: max over the rows of segment (t, c) of |x_i| + |y_i| for a complex pair (x
  // its first column, y its second; stored at both), |x_i| for a real column, in the units
  // of the segment's exponent: the final segments' norms for the normalisation (NULL in
  // the descriptor of a refinement's correction solve, which leaves them alone)
  double* segn;
  double* W;
  int32_t* eW;
  double* nW;
  Ctrl* ctrl;
  // mixed precision (split operands for the int8 matrix instruction, see slices.hpp)
  int4* Aslc;         // slices of every super-diagonal tile pair [S_kr | T_kr]
  int32_t* Aexp;      // [pair][MB] row exponents of those tiles (S half; T half + D_r)
  int4* Wslc;         // slices of W per source-row slot and tile column
  int32_t* Wexp;      // [slot][m] column exponents of W (X D half; -X B half - D_r)
  unsigned long long* stmax;   // [2][Mmax] largest |S| and |T| (bits, >= 0) in the columns of
                               // tile r above its diagonal tile: D_r from their exponents
  // the new segment exponents and norms of a mixed-precision update launch whose tiles are
  // split over several workgroups (row groups): norms combined by an atomic maximum on the
  // bits of the non-negative doubles, published into exps/norms (and cleared) once the
  // launch is done, so that no workgroup reads a segment another one has already rewritten
  int32_t* exps_next;            // [Mmax * m]
  unsigned long long* norms_next; // [Mmax * m], zero between launches
  // refinement of the mixed-precision result: in correction mode (rhs = 1) the tile rows of
  // Z hold a right-hand side (the residual) instead of starting at zero, the tip block's
  // correction is zero, and only tile columns j with tflag[j] != 0 are solved and updated
  int32_t* tflag;     // [Mmax], read in correction mode only
  int32_t rhs;
  // the real form of a complex pencil (complex.hip): every 2x2 diagonal block is
  // [[a, -b], [b, a]] with T block c I, and a complex column's vector lies in one of the two
  // invariant subspaces of the form, so its 2x2 blocks are solved as complex 1x1 systems
  int32_t cform;
  int32_t mb;
  int32_t Mmax;
  int32_t normalize;
  int32_t band;       // R: tile rows per update band
  int32_t split;      // tiles per launch of a band's update of the rows above it (0: one launch)
  int32_t wslots;     // 2R source-row slots of W, eW, nW
  int32_t precision;  // 0: FP64 contraction; 1: split operands on the int8 matrix cores
};

constexpr int kMaxBand = 8;

// Refinement of the mixed-precision result against an FP64 residual.  A sketch with
// kSketch Cauchy rows G estimates the 1-norm of each column's residual r = (beta S - alpha T) z
// (the median of |g_t . r| over the rows is a consistent estimate of ||r||_1 for Cauchy g);
// the column is flagged when that estimate exceeds tau times the exact
// || beta |S| |z| + |alpha| |T| |z| ||_1 (a componentwise backward error, at the level of u for an
// FP64 substitution); flagged columns get r in FP64 and a correction solve.
constexpr int kSketch = 16;
// workgroups of a correction-mode launch (they stride over the tiles of the launch)
constexpr int kRhsGrid = 1536;

struct RefineDesc {
  double* G;          // [m][kSketch] sketch rows, row-major by matrix row
  double* GS;         // [m][kSketch] sk * psc * (G S)^T: entry (j, t) = sum_i G(i, t) S(i, j)
  double* GT;         // [m][kSketch] the same for T
  double* cS;         // [m] sk * psc * column sums of |S| (and |T|)
  double* cT;
  double* PS;         // [m][kSketch] projections G S z'_c, G T z'_c of each column of Z
  double* PT;
  double* dS;         // [m] cS . |z'_c| and cT . |z'_c|
  double* dT;
  int32_t* zexp;      // [m] z'_c = 2^-zexp[c] z_c (common to the two columns of a pair)
  int8_t* rf;         // [m] flagged by the latest pass
  int8_t* fits;       // [m] every entry within the range a refinement can handle (pass 0)
  int32_t* tflag;     // [Mmax] tile column holds a flagged column
  double* part;       // [ceil(m / 1024) * m * (2 kSketch + 2)] partial sums per row chunk
  double* Zc;         // [m * m] residual in, correction out (leading dimension m)
  int32_t* cexps;     // [Mmax * m] segment exponents and norms of Zc (the correction solve's)
  double* cnorms;
  double tau;         // flag threshold on the backward-error estimate
};

// Work list and dependency counters of the persistent walker (schedule 2).
struct WalkDesc {
  int32_t* cnt;       // [Mmax * Mmax] updates applied to tile (k, j)
  int32_t* solved;    // [Mmax * Mmax] tile (r, j) solved
  int4* tickets;      // tasks in priority order: (type 0 solve / 1 update, k, r, j)
  int64_t* levels;    // [2 Mmax + 1] first ticket of each level; the last entry is the count
  int32_t* next;      // ticket dispenser
  int32_t spin_limit; // bound on every dependency wait
  int32_t grid;       // workgroups to launch (0: as many as are resident at once; capped there)
};

// number of walker tasks for M tiles: per distance d = j - r, M - d solves and
// (M - 1 - d)(M - d)/2 updates
__host__ __device__ inline int64_t walk_tasks(int64_t M) {
  int64_t n = 0;
  for (int64_t d = 0; d < M; ++d) n += (M - d) + (M - 1 - d) * (M - d) / 2;
  return n;
}

// W tile of one (source row, tile column) pair: 2*MB K-rows x MB columns.
__host__ __device__ constexpr int64_t w_tile_doubles(int mb) { return 2LL * mb * mb; }

// The thread's index in the workgroup through a move the compiler cannot see through: each
// call is a new value, so a kernel that runs several tiles in a loop keeps nothing derived from
// the index live from one tile to the next (it recomputes it).
__device__ __forceinline__ int opaque_tid() {
  int t;
  asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
  return t;
}

__host__ __device__ constexpr int tile_bound(int64_t m, int mb) {
  return m <= 0 ? 0 : (int)((m + (mb - 2)) / (mb - 1)) + 1;
}

}  // namespace rgev
