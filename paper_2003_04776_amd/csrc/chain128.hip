// The chain of one band for tiles of 128 (band_chain_kernel in solve.hip holds the tiles of
// 32 and 64; the steps are the same).  It is a translation unit of its own: its shared memory
// is dynamic, and a kernel with dynamic shared memory in the same module changes how the
// others are compiled.
#include <hip/hip_runtime.h>

#include "chain.hpp"

namespace rgev {

// Tiles of 128: held to 256 registers a lane (two waves per SIMD), so that one update
// workgroup fits beside the chain on a CU.  Two things make that possible: each step reads the
// thread index through an opaque move, so the compiler cannot keep values derived from it live
// from one step to the next (with threadIdx.x itself it kept 110 registers more), and the
// shared memory (142 KB) is dynamic, so the compiler's occupancy bound comes from the registers
// alone (with static shared memory it takes one workgroup per CU as given and ignores the
// two-wave bound).  Four values spill to scratch.
__global__ __launch_bounds__(solve_total(128)) __attribute__((amdgpu_waves_per_eu(2, 2))) void band_chain_kernel_128(PencilDesc P, int r_lo, int r_hi) {
  constexpr int MB = 128, WGR = ChainUpdShape<MB>::R, WGC = ChainUpdShape<MB>::C;
  static_assert(64 * WGR * WGC == solve_total(MB), "chain workgroup size");
  static_assert(SolveShape<MB>::CS == 1, "one workgroup per tile");
  extern __shared__ __align__(16) unsigned char chain_smem[];   // sizeof(ChainSmem<128>) bytes
  ChainSmem<MB>& sm = *reinterpret_cast<ChainSmem<MB>*>(chain_smem);
  const int M = P.ctrl->M;
  const int j = r_lo + (int)blockIdx.x;
  if (j >= M) return;
  const bool upd = !(P.rhs && !P.tflag[j]);
  const int top = min(r_hi, j);
  for (int r = top; r >= r_lo; --r) {
    solve_tile<MB, true>(P, r, j, 0, sm.s);
    if (r > r_lo && upd) {
      const UpdRange U{r_lo, r, r, r, r};
      for (int k = r_lo; k < r; ++k) {
        __syncthreads();   // the solve's (or the previous update's) shared memory is free
        update_tile<MB, WGR, WGC, 3, true>(P, U, k, j, sm.u);
      }
    }
    __syncthreads();   // every store of the step is visible to the workgroup's next step
  }
}

// the dynamic shared memory exceeds the default limit: raised once per device before the
// first launch
static hipError_t chain_smem_limit() {
  static thread_local int done_dev = -1;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev == done_dev) return e;
  e = hipFuncSetAttribute((const void*)band_chain_kernel_128, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)sizeof(ChainSmem<128>));
  if (e == hipSuccess) done_dev = dev;
  return e;
}

hipError_t launch_band_chain_128(const PencilDesc& P, int r_lo, int r_hi, int grid, hipStream_t s) {
  const hipError_t e = chain_smem_limit();
  if (e != hipSuccess) return e;
  band_chain_kernel_128<<<grid, solve_total(128), sizeof(ChainSmem<128>), s>>>(P, r_lo, r_hi);
  return hipSuccess;
}

}  // namespace rgev
