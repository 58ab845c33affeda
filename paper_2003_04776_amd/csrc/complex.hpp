// Descriptor of a complex-pencil call (complex.hip): the caller's complex matrices and the
// real form of order 2m that the real path solves, in the caller's workspace.
#pragma once
#include <stdint.h>

namespace rgev {

struct ComplexDesc {
  int64_t m, lds, ldt, ldz;
  const double* S;     // complex, interleaved (re, im), leading dimension in complex entries
  const double* T;
  double* Z;
  int32_t* scales;
  const int32_t* select;
  double* S2;          // real form, order 2m, leading dimension 2m
  double* T2;
  double* Z2;
  int32_t* sel2;
  int32_t* scales2;
  int32_t normalize;
};

}  // namespace rgev
