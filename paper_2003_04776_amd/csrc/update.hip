// Kernels of the tile updates (the tile body is in update_tile.hpp): a band of source
// rows applied to a range of target tiles of one pencil, or one lock-step of a batch.
#include <hip/hip_runtime.h>

#include "update_tile.hpp"

namespace rgev {

// UpdShape<MB>::W waves per SIMD
template <int MB>
__global__ __launch_bounds__(64 * UpdShape<MB>::R * UpdShape<MB>::C, UpdShape<MB>::W)
void update_kernel(PencilDesc P, UpdRange U) {
  const int M = P.ctrl->M;
  if (U.j_lo >= M || U.k_hi <= U.k_lo || U.s_lo >= M) return;
  // ---- tile of this workgroup: 8 x 8 blocks of (k, j), each XCD a contiguous range ----
  const int nk = U.k_hi - U.k_lo, nj = M - U.j_lo;
  const int nbk = (nk + 7) / 8, nbj = (nj + 7) / 8;
  const int per = (int)(gridDim.x / 8);
  const int idx = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (idx >= nbk * nbj * 64) return;
  const int blk = idx / 64, w64 = idx % 64;
  const int k = U.k_lo + 8 * (blk % nbk) + (w64 % 8);
  const int j = U.j_lo + 8 * (blk / nbk) + (w64 / 8);
  if (k >= U.k_hi || j >= M) return;
  if (P.rhs && !P.tflag[j]) return;   // correction mode: no column of tile j is refined
  __shared__ UpdSmem<MB, UpdShape<MB>::R> sm;
  update_tile<MB, UpdShape<MB>::R, UpdShape<MB>::C, UpdShape<MB>::S>(P, U, k, j, sm);
}

// one update of a batch's lock-step t for pencil p = blockIdx.y, in its band B_p - 1 - t
// (tile rows [r_lo, r_hi]); the ranges are those of the single-pencil band schedule:
//   part 0: the in-band update after the solve of row r = r_hi - a: targets k in [r_lo, r),
//           j >= r, source r;
//   part 1: the band applied to the next band's rows, targets [r_lo - R, r_lo), j >= r_lo;
//   part 2: the band applied to rows [max(0, hi - c), hi) above those, hi = r_lo - R - a.
// blockIdx.x enumerates (k - k_lo, j - j_lo) with J columns.
template <int MB>
__global__ __launch_bounds__(64 * BatchUpdShape<MB>::R * BatchUpdShape<MB>::C, BatchUpdShape<MB>::W)
void update_batched_kernel(const PencilDesc* __restrict__ D, int R, int t, int part, int a, int c, int J) {
  const PencilDesc P = D[blockIdx.y];
  const int M = P.ctrl->M;
  const int b = (M + R - 1) / R - 1 - t;
  if (b < 0) return;
  const int r_lo = R * b, r_hi = min(r_lo + R - 1, M - 1);
  UpdRange U;
  if (part == 0) {
    const int r = r_hi - a;
    if (r <= r_lo) return;
    U = UpdRange{r_lo, r, r, r, r};
  } else if (part == 1) {
    if (r_lo == 0) return;
    U = UpdRange{max(r_lo - R, 0), r_lo, r_lo, r_lo, r_hi};
  } else {
    const int hi = r_lo - R - a;
    if (hi <= 0) return;
    U = UpdRange{max(hi - c, 0), hi, r_lo, r_lo, r_hi};
  }
  const int kk = (int)blockIdx.x / J, jj = (int)blockIdx.x % J;
  const int k = U.k_lo + kk, j = U.j_lo + jj;
  if (k >= U.k_hi || j >= M) return;
  __shared__ UpdSmem<MB, BatchUpdShape<MB>::R> sm;
  update_tile<MB, BatchUpdShape<MB>::R, BatchUpdShape<MB>::C, BatchUpdShape<MB>::S>(P, U, k, j, sm);
}

// The same update with BatchUpdShape's tiles (one wave per tile of 64): for launches of at
// least kFarTiles tiles (the updates of the rows above a band in larger pencils), which are
// bound by throughput.
constexpr int64_t kFarTiles = 4096;
template <int MB>
__global__ __launch_bounds__(64 * BatchUpdShape<MB>::R * BatchUpdShape<MB>::C, BatchUpdShape<MB>::W)
void update_far_kernel(PencilDesc P, UpdRange U) {
  const int M = P.ctrl->M;
  if (U.j_lo >= M || U.k_hi <= U.k_lo || U.s_lo >= M) return;
  const int nk = U.k_hi - U.k_lo, nj = M - U.j_lo;
  const int nbk = (nk + 7) / 8, nbj = (nj + 7) / 8;
  const int per = (int)(gridDim.x / 8);
  const int idx = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (idx >= nbk * nbj * 64) return;
  const int blk = idx / 64, w64 = idx % 64;
  const int k = U.k_lo + 8 * (blk % nbk) + (w64 % 8);
  const int j = U.j_lo + 8 * (blk / nbk) + (w64 / 8);
  if (k >= U.k_hi || j >= M) return;
  if (P.rhs && !P.tflag[j]) return;
  __shared__ UpdSmem<MB, BatchUpdShape<MB>::R> sm;
  update_tile<MB, BatchUpdShape<MB>::R, BatchUpdShape<MB>::C, BatchUpdShape<MB>::S>(P, U, k, j, sm);
}

template <int MB>
static void launch_update_t(const PencilDesc& P, const UpdRange& U, hipStream_t s) {
  // upper bound on the 8 x 8 blocked tile range (the true tile count is on the device)
  const int64_t nbk = (U.k_hi - U.k_lo + 7) / 8, nbj = (P.Mmax - U.j_lo + 7) / 8;
  const int64_t grid = nbk * nbj * 64;
  if constexpr (MB == 64) {
    // (a launch of fewer tiles ends sooner with four waves per tile)
    if ((int64_t)(U.k_hi - U.k_lo) * (P.Mmax - U.j_lo) >= kFarTiles) {
      update_far_kernel<MB><<<(unsigned)grid, 64 * BatchUpdShape<MB>::R * BatchUpdShape<MB>::C, 0, s>>>(P, U);
      return;
    }
  }
  update_kernel<MB><<<(unsigned)grid, 64 * UpdShape<MB>::R * UpdShape<MB>::C, 0, s>>>(P, U);
}

// Apply source rows [s_lo, s_hi] to target rows [k_lo, k_hi) of every tile column
// j >= j_lo.  Returns false when there is nothing to launch.
void launch_update_i8(const PencilDesc& P, const UpdRange& U, hipStream_t s);

bool launch_update(const PencilDesc& P, int k_lo, int k_hi, int j_lo, int s_lo, int s_hi, hipStream_t s) {
  if (k_hi <= k_lo || j_lo >= P.Mmax) return false;
  const UpdRange U{k_lo, k_hi, j_lo, s_lo, s_hi};
  if (P.precision == 1) {
    launch_update_i8(P, U, s);
    return true;
  }
  switch (P.mb) {
    case 32: launch_update_t<32>(P, U, s); break;
    case 64: launch_update_t<64>(P, U, s); break;
    default: launch_update_t<128>(P, U, s); break;
  }
  return true;
}

// Batch lock-step t, band R (see update_batched_kernel): kmax bounds the target rows of the
// part over the group's pencils (R - 1 in a band, R for the next band, c for a part of the
// rows above), and the columns j - j_lo < R (t + 1).
void launch_update_batched(const PencilDesc* D, int n, int mb, int max_tiles, int R, int t, int part, int a, int c,
                           int kmax, hipStream_t s) {
  const int64_t J = (R * (t + 1) < max_tiles) ? R * (t + 1) : max_tiles;
  if (kmax <= 0 || J <= 0 || n <= 0) return;
  const dim3 grid((unsigned)(kmax * J), (unsigned)n);
  const int Ji = (int)J;
  switch (mb) {
    case 32: update_batched_kernel<32><<<grid, 64 * BatchUpdShape<32>::R * BatchUpdShape<32>::C, 0, s>>>(D, R, t, part, a, c, Ji); break;
    case 64: update_batched_kernel<64><<<grid, 64 * BatchUpdShape<64>::R * BatchUpdShape<64>::C, 0, s>>>(D, R, t, part, a, c, Ji); break;
    default: update_batched_kernel<128><<<grid, 64 * BatchUpdShape<128>::R * BatchUpdShape<128>::C, 0, s>>>(D, R, t, part, a, c, Ji); break;
  }
}

}  // namespace rgev
