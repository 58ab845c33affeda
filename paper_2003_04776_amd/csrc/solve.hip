// Kernels of the diagonal solves (the tile body is in solve_tile.hpp): one tile row of
// one pencil per launch, or one lock-step of a batch.
#include <hip/hip_runtime.h>

#include "solve_tile.hpp"
#include "update_tile.hpp"
#include "chain.hpp"

namespace rgev {

// Registers are capped at 256 a lane (the rank-2G update's accumulators in ordinary vector
// registers, which the build asks for): a tile-update workgroup holds 256 a lane, so a solve
// fits beside one of them.  A solve that needed the whole register file of its CU would wait,
// while a large update launch runs, until none of that launch's workgroups were left to
// start, delaying the chain of solves that every band of the schedule waits for.
// tile row r of one pencil: tiles (r, j), j = r .. M-1
template <int MB>
__global__ __launch_bounds__(solve_total(MB), solve_waves_per_simd(MB)) __attribute__((amdgpu_num_vgpr(256))) void solve_kernel(PencilDesc P, int r) {
  constexpr int CS = SolveShape<MB>::CS;
  __shared__ SolveSmem<MB> sm;
  solve_tile<MB>(P, r, r + (int)blockIdx.x / CS, (int)blockIdx.x % CS, sm);
}

// The chain of one band, C(b) of the band schedule, in one launch: the band's rows r_hi ..
// r_lo, each solve followed by the update of the band's rows above it by that row.  For a
// tile column j these steps read and write only column j's tiles (and the band's tiles of S
// and T), so one workgroup per tile column j = r_lo + blockIdx.x runs them in order, and the
// launch has to be placed on the GPU once rather than once per step.  Every tile gets the
// same operations in the same order as with one launch per step, so the results are the same
// bit for bit.  The update runs on the workgroup's own waves (a 2 x 2 wave grid for tiles
// of 128, 1 x 2 for 64, one wave for 32) with its shared memory in the solve's.  Tiles of
// 128 run band_chain_kernel_128 (chain128.hip), held to 256 registers a lane.
template <int MB>
__global__ __launch_bounds__(solve_total(MB), solve_waves_per_simd(MB)) __attribute__((amdgpu_num_vgpr(256))) void band_chain_kernel(PencilDesc P, int r_lo, int r_hi) {
  constexpr int WGR = ChainUpdShape<MB>::R, WGC = ChainUpdShape<MB>::C;
  static_assert(64 * WGR * WGC == solve_total(MB), "chain workgroup size");
  static_assert(SolveShape<MB>::CS == 1, "one workgroup per tile");
  __shared__ ChainSmem<MB> sm;
  const int M = P.ctrl->M;
  const int j = r_lo + (int)blockIdx.x;
  if (j >= M) return;
  // (correction mode: tile columns with no refined column take no update, as in the
  // update kernels; their solves still run)
  const bool upd = !(P.rhs && !P.tflag[j]);
  const int top = min(r_hi, j);
  for (int r = top; r >= r_lo; --r) {
    solve_tile<MB>(P, r, j, 0, sm.s);
    if (r > r_lo && upd) {
      const UpdRange U{r_lo, r, r, r, r};
      for (int k = r_lo; k < r; ++k) {
        __syncthreads();   // the solve's (or the previous update's) shared memory is free
        update_tile<MB, WGR, WGC>(P, U, k, j, sm.u);
      }
    }
    __syncthreads();   // every store of the step is visible to the workgroup's next step
  }
}

hipError_t launch_band_chain(const PencilDesc& P, int r_lo, int r_hi, hipStream_t s) {
  const int grid = P.Mmax - r_lo;
  if (grid <= 0) return hipSuccess;
  switch (P.mb) {
    case 32: band_chain_kernel<32><<<grid, solve_total(32), 0, s>>>(P, r_lo, r_hi); return hipSuccess;
    case 64: band_chain_kernel<64><<<grid, solve_total(64), 0, s>>>(P, r_lo, r_hi); return hipSuccess;
    default: return launch_band_chain_128(P, r_lo, r_hi, grid, s);
  }
}

// one solve of a batch's lock-step t: in band B_p - 1 - t of every pencil p = blockIdx.y
// (bands of R tile rows from the top, B_p of them), the row io places above the band's
// last row; tiles (r, j), j >= r
template <int MB>
__global__ __launch_bounds__(solve_total(MB), solve_waves_per_simd(MB)) __attribute__((amdgpu_num_vgpr(256))) void solve_batched_kernel(const PencilDesc* __restrict__ D, int R, int t, int io) {
  constexpr int CS = SolveShape<MB>::CS;
  __shared__ SolveSmem<MB> sm;
  const PencilDesc P = D[blockIdx.y];
  const int M = P.ctrl->M;
  const int b = (M + R - 1) / R - 1 - t;
  const int r_hi = min(R * b + R - 1, M - 1);
  const int r = b >= 0 && r_hi - io >= R * b ? r_hi - io : -1;   // -1: no row (solve_tile returns)
  solve_tile<MB>(P, r, r + (int)blockIdx.x / CS, (int)blockIdx.x % CS, sm);
}

template <int MB>
static void launch_solve_t(const PencilDesc& P, int r, hipStream_t s) {
  solve_kernel<MB><<<(P.Mmax - r) * SolveShape<MB>::CS, solve_total(MB), 0, s>>>(P, r);
}

void launch_solve(const PencilDesc& P, int r, hipStream_t s) {
  switch (P.mb) {
    case 32: launch_solve_t<32>(P, r, s); break;
    case 64: launch_solve_t<64>(P, r, s); break;
    default: launch_solve_t<128>(P, r, s); break;
  }
}

// Batch step t for the n pencils of table D (all with tile size mb and at most
// max_tiles tiles): grid (t + 1) x n; pencils with fewer than t + 1 tiles exit at once.
void launch_solve_batched(const PencilDesc* D, int n, int mb, int max_tiles, int R, int t, int io, hipStream_t s) {
  // a band-R lock-step t reaches at most R (t + 1) tile columns: M - R b <= R (t + 1)
  const int gx = (R * (t + 1) < max_tiles) ? R * (t + 1) : max_tiles;
  if (gx <= 0 || n <= 0) return;
  switch (mb) {
    case 32:
      solve_batched_kernel<32><<<dim3(gx * SolveShape<32>::CS, n), solve_total(32), 0, s>>>(D, R, t, io);
      break;
    case 64:
      solve_batched_kernel<64><<<dim3(gx * SolveShape<64>::CS, n), solve_total(64), 0, s>>>(D, R, t, io);
      break;
    default:
      solve_batched_kernel<128><<<dim3(gx * SolveShape<128>::CS, n), solve_total(128), 0, s>>>(D, R, t, io);
      break;
  }
}

}  // namespace rgev
