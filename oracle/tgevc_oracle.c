/*
 * CPU oracle for the robust generalized eigenvector computation.  TEST
 * INFRASTRUCTURE ONLY: it is built beside the product library so that tests, the
 * smoke check and the CPU baseline of the benchmark can call it; the product path
 * never links, loads or calls it.
 *
 * The arithmetic lives in oracle_impl.h, compiled here twice: in double precision
 * (the precision of the method) and in x86 extended precision (long double, 64-bit
 * significand, 15-bit exponent) as an independent cross-check of conditioning.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

/* ---- double ---- */
#define R double
#define FN(x) x##_d
#define FREXP frexp
#define LDEXP ldexp
#define FABS fabs
#define SQRT sqrt
#define SIGNBIT signbit
#define OMEGA_EXP (DBL_MAX_EXP - 4)        /* Omega = 2^1020 */
#define U_ROUND (DBL_EPSILON / 2)          /* 2^-53 */
#define TINY DBL_MIN
#define MARGIN ((R)0x1p-50)
#include "oracle_impl.h"
#undef R
#undef FN
#undef FREXP
#undef LDEXP
#undef FABS
#undef SQRT
#undef SIGNBIT
#undef OMEGA_EXP
#undef U_ROUND
#undef TINY
#undef MARGIN

/* ---- long double ---- */
#define R long double
#define FN(x) x##_ld
#define FREXP frexpl
#define LDEXP ldexpl
#define FABS fabsl
#define SQRT sqrtl
#define SIGNBIT signbit
#define OMEGA_EXP (LDBL_MAX_EXP - 4)       /* Omega = 2^16380 */
#define U_ROUND (LDBL_EPSILON / 2)         /* 2^-64 */
#define TINY LDBL_MIN
#define MARGIN ((R)0x1p-50)
#include "oracle_impl.h"

/* helpers with double arguments for the tests of the long double scalars */
int oracle_pd_ld_dbl(double b, double t) { return oracle_pd_ld(b, t); }
int oracle_pu_ld_dbl(double t, double x, double y) { return oracle_pu_ld(t, x, y); }
int oracle_omega_exp_d(void) { return DBL_MAX_EXP - 4; }
