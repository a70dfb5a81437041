// Host launchers of the Cholesky factorisation and block triangular solve (chol.hip), complex
// FP64, used to orthonormalise tall blocks by (shifted) Cholesky QR.
#pragma once

#include "common.h"
#include "gemm.h"

namespace mpdo {

// Device doubles of the work array of cholesky_lower / trsm_right_lower_adj for order m: the
// shift and the inverses of the 64 x 64 diagonal blocks of L.
size_t chol_work_doubles(int m);

// L L^H = A + s I for the Hermitian m x m matrix A (only its lower triangle is read; the trailing
// part is overwritten by the updates), s = shift_coef * trace(A) (0: no shift).  L (ld ldl, not
// aliasing A) receives the lower factor, work the diagonal-block inverses.  A pivot that is not
// positive and finite sets flag[0] = 1 (the caller zeroes it first and discards the result).
// The products run on cgemm_ex with opt (its k-split workspace).  No host synchronisation.
hipError_t cholesky_lower(hipStream_t s, double* A, long lda, int m, double shift_coef, double* L, long ldl,
                          double* work, int* flag, const GemmOpts& opt, ProfSink* prof);

// Q = Y L^{-H} for the n x m block Y (ld ldy; overwritten) and the factor of cholesky_lower with its
// work array; Q (ld ldq) must not alias Y or L.
hipError_t trsm_right_lower_adj(hipStream_t s, double* Y, long ldy, int n, int m, const double* L, long ldl,
                                const double* work, double* Q, long ldq, const GemmOpts& opt, ProfSink* prof);

}  // namespace mpdo
