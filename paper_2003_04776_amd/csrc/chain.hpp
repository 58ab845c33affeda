// Shapes shared by the band-chain kernels (solve.hip for tiles of 32 and 64, chain128.hip for
// tiles of 128): the update's wave grid inside a chain workgroup, and the chain's shared
// memory, which the solve and the update use in turn.
#pragma once
#include <hip/hip_runtime.h>

#include "solve_tile.hpp"
#include "update_tile.hpp"

namespace rgev {

template <int MB> struct ChainUpdShape;
template <> struct ChainUpdShape<32> { static constexpr int R = 1, C = 1; };
template <> struct ChainUpdShape<64> { static constexpr int R = 1, C = 2; };
template <> struct ChainUpdShape<128> { static constexpr int R = 2, C = 2; };

template <int MB>
union ChainSmem {
  SolveSmem<MB> s;
  UpdSmem<MB, ChainUpdShape<MB>::R> u;
};

// the chain of tile rows [r_lo, r_hi] for tiles of 128 on grid tile columns (chain128.hip)
hipError_t launch_band_chain_128(const PencilDesc& P, int r_lo, int r_hi, int grid, hipStream_t s);

}  // namespace rgev
