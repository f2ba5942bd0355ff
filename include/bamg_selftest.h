/*
 * bamg_selftest.h -- test-only entry points of the bamg library (not part of
 * the solver's interface in bamg.h; exported for the library's own tests).
 */
#ifndef BAMG_SELFTEST_H
#define BAMG_SELFTEST_H

#include "bamg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Self-test of the FP64 matrix-core tile products the coarse factorization is
 * built from: C += X Y^T (mode 0), C += X^T Y (mode 1), C += X Y (mode 2), with
 * X, Y, C 16 x 16 row-major device arrays. Lets a test confirm the operand
 * layout of the MFMA 16x16x4 FP64 instruction on the running GPU. */
ba_status ba_selftest_tile_mma(const double* X, const double* Y, double* C, int32_t mode, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* BAMG_SELFTEST_H */
