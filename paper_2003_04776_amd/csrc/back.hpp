// Descriptor and packed-operand layout of the back-transformation X = V Z.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace rgev {

constexpr int kBackInfoNonFinite = 1;   // NaN or Inf in V or Z

struct BackDesc {
  int64_t m;
  const double* S;   // sub-diagonal only: the 2 x 2 block structure
  int64_t lds;
  const double* V;
  int64_t ldv;
  const double* Z;
  int64_t ldz;
  const int32_t* scales;   // nullable: all zero
  double* X;
  int64_t ldx;
  int32_t* xscales;
  int32_t* info;
  int mb;          // tile size (64 or 128)
  int nt;          // tiles per dimension, ceil(m / mb)
  int normalize;
  // workspace
  int8_t* blk;               // [m] 0 real, 1 first / 2 second column of a complex pair
  double* zmax;              // [m] max_i |Z_ic| over the quasi-triangle
  unsigned long long* vmax;  // bits of max |V_ik|
  int32_t* info_local;       // info when the caller passes none
  double* Zp;                // packed Z, tile column J at back_tile_offset(mb, J)
};

// K steps (4 rows each) that tile column J reaches: rows 0 .. mb J + h_J (one row past the
// tile for a pair that ends it), at most m
__host__ __device__ inline int back_steps(int64_t m, int mb, int J) {
  int64_t rows = (int64_t)mb * (J + 1) + 1;
  if (rows > m) rows = m;
  return (int)((rows + 3) / 4);
}

// doubles before tile column J in the packed Z: sum over J' < J of (mb (J' + 1) / 4 + 1)
// steps of 4 mb doubles (the bound of back_steps without the cap at m)
__host__ __device__ inline int64_t back_tile_offset(int mb, int J) {
  const int64_t steps = (int64_t)mb * J * (J + 1) / 8 + J;
  return steps * 4 * mb;
}

}  // namespace rgev
