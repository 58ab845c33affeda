// Persistent walker of the task graph of Algorithm 1 (Section 3), the schedule the
// paper leaves to a task runtime (Section 5.3): one launch of resident workgroups that
// take tasks from a ticket list in a fixed priority order and wait on device-side
// dependency counters.
//
// Tasks (tile granularity, one source row per update):
//   Solve(r, j), r <= j        tip (r = j) or diagonal solve of tile (r, j);
//                              ready when cnt(r, j) = j - r
//   Update(k, j; r), k < r <= j  Y_kj -= [S_kr | T_kr] W_rj (Algorithms 2 and 3);
//                              ready when solved(r, j) and cnt(k, j) = j - r
// cnt(k, j) counts the updates applied to tile (k, j).  The second condition makes the
// updates of a tile run in the fixed order r = j, j-1, ..., so results do not depend on
// the schedule (they equal those of the band schedule with one row per band).
//
// Ticket order: level by level, where the level of Solve(r, j) is 2(j - r) and that of
// Update(k, j; r) is 2(j - r) + 1 (every dependency sits on a lower level, so the order
// is topological).  Inside a level, solves go by descending j; updates by distance
// e = r - 1 - k to the diagonal (e = 0 feeds the next solve: critical path first), then
// descending j.  A workgroup takes ticket t only after every workgroup took the tickets
// before it, and those depend only on lower tickets, so the earliest unfinished ticket
// can always run: no deadlock, whatever the number of resident workgroups.
//
// Every wait is bounded (a spin limit): a wait that gives up sets the watchdog bit of
// info and the task runs anyway, so the launch always drains (the results are then not
// to be trusted).
#include <hip/hip_runtime.h>

#include "solve_tile.hpp"
#include "update_tile.hpp"

namespace rgev {

template <int MB> struct WalkShape;   // update wave grid of a walker workgroup
template <> struct WalkShape<32> { static constexpr int R = 1, C = 1; };
template <> struct WalkShape<64> { static constexpr int R = 1, C = 2; };
template <> struct WalkShape<128> { static constexpr int R = 2, C = 2; };

// level offsets: lvl[2d] = first ticket of the solves with j - r = d, lvl[2d+1] of the
// updates with j - r = d; lvl[2M] = total.  One thread.
__global__ void walk_levels_kernel(PencilDesc P, WalkDesc W) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t M = P.ctrl->M;
  int64_t off = 0;
  for (int64_t d = 0; d < M; ++d) {
    W.levels[2 * d] = off;
    off += M - d;
    W.levels[2 * d + 1] = off;
    off += (M - 1 - d) * (M - d) / 2;
  }
  W.levels[2 * M] = off;
  *W.next = 0;
}

// One thread per tile (r, j), r <= j: writes its solve ticket and its updates' tickets;
// also clears the tile's counters.
__global__ void walk_tickets_kernel(PencilDesc P, WalkDesc W) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int Mmax = P.Mmax;
  if (idx >= (int64_t)Mmax * Mmax) return;
  const int r = (int)(idx / Mmax), j = (int)(idx % Mmax);
  W.cnt[idx] = 0;
  W.solved[idx] = 0;
  const int M = P.ctrl->M;
  if (j >= M || r > j) return;
  const int d = j - r;
  W.tickets[W.levels[2 * d] + (M - 1 - j)] = make_int4(0, 0, r, j);
  const int64_t base = W.levels[2 * d + 1];
  for (int k = 0; k < r; ++k) {
    const int64_t e = r - 1 - k;
    const int64_t pos = base + e * (M - 1 - d) - e * (e - 1) / 2 + (M - 1 - j);
    W.tickets[pos] = make_int4(1, k, r, j);
  }
}

__device__ __forceinline__ int load_acquire(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

template <int MB>
__global__ __launch_bounds__(solve_total(MB)) void walker_kernel(PencilDesc P, WalkDesc W) {
  constexpr int WGR = WalkShape<MB>::R, WGC = WalkShape<MB>::C;
  static_assert(64 * WGR * WGC == solve_total(MB), "walker workgroup size");
  union Smem {
    SolveSmem<MB> s;
    UpdSmem<MB, WGR> u;
  };
  __shared__ Smem sm;
  __shared__ int4 task;
  const int Mmax = P.Mmax;
  const int64_t ntasks = W.levels[2 * (int64_t)P.ctrl->M];
  const int limit = W.spin_limit;
  for (;;) {
    __syncthreads();   // the previous task is finished with the shared memory and 'task'
    if (threadIdx.x == 0) {
      const int t = atomicAdd(W.next, 1);
      int4 tk = make_int4(-1, 0, 0, 0);
      if (t < ntasks) {
        tk = W.tickets[t];
        const int k = tk.x == 0 ? tk.z : tk.y, r = tk.z, j = tk.w;
        const int need = j - r;
        const int32_t* c = W.cnt + (int64_t)k * Mmax + j;
        const int32_t* sv = W.solved + (int64_t)r * Mmax + j;
        int spins = 0;
        while ((tk.x == 1 && load_acquire(sv) == 0) || load_acquire(c) < need) {
          __builtin_amdgcn_s_sleep(2);
          if (++spins > limit) {
            atomicOr(P.info, (int)kInfoWatchdog);
            break;
          }
        }
      }
      task = tk;
    }
    __syncthreads();
    const int4 tk = task;
    if (tk.x < 0) break;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // see the producers' results
    if (tk.x == 0) {
      for (int z = 0; z < SolveShape<MB>::CS; ++z) solve_tile<MB>(P, tk.z, tk.w, z, sm.s);
    } else {
      const UpdRange U{tk.y, tk.y + 1, tk.w, tk.z, tk.z};
      update_tile<MB, WGR, WGC>(P, U, tk.y, tk.w, sm.u);
    }
    __syncthreads();   // every store of the task is issued and complete in this workgroup
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      if (tk.x == 0)
        __hip_atomic_store(W.solved + (int64_t)tk.z * Mmax + tk.w, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      else
        __hip_atomic_fetch_add(W.cnt + (int64_t)tk.y * Mmax + tk.w, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <int MB>
static hipError_t launch_walker_t(const PencilDesc& P, const WalkDesc& W, hipStream_t s) {
  // resident workgroups: as many as fit at once (more would only wait for the end), or the
  // caller's smaller count
  static int grid_cache[64] = {0};
  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return err;
  int& grid = grid_cache[dev & 63];
  if (grid == 0) {
    int per_cu = 0, cus = 0;
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, walker_kernel<MB>, solve_total(MB), 0);
    if (err == hipSuccess) err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (err != hipSuccess) return err;
    grid = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
  }
  // a requested count below that: the tasks are taken from the ticket dispenser only by
  // running workgroups, so any count makes progress and computes the same results
  const int g = (W.grid > 0 && W.grid < grid) ? W.grid : grid;
  walker_kernel<MB><<<g, solve_total(MB), 0, s>>>(P, W);
  return hipGetLastError();
}

hipError_t launch_walk(const PencilDesc& P, const WalkDesc& W, hipStream_t s) {
  walk_levels_kernel<<<1, 64, 0, s>>>(P, W);
  const int64_t pairs = (int64_t)P.Mmax * P.Mmax;
  walk_tickets_kernel<<<(unsigned)((pairs + 255) / 256), 256, 0, s>>>(P, W);
  switch (P.mb) {
    case 32: return launch_walker_t<32>(P, W, s);
    case 64: return launch_walker_t<64>(P, W, s);
    default: return launch_walker_t<128>(P, W, s);
  }
}

}  // namespace rgev
