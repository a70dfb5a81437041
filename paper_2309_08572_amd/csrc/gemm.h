// Host launchers of the complex matrix-core GEMM (gemm.hip).
#pragma once

#include "common.h"

namespace mpdo {

// C = alpha * A * B + beta * C over `batch` problems; A is M x K, B is K x N, C is M x N as
// strided views (see CView); batch strides sA, sB, sC are in complex elements.  C must not
// alias A or B.  prof (may be null) brackets the matrix-core kernel as PF_GEMM with its
// algorithmic flop and bytes, and the output pre-scaling of split-k products as PF_OTHER.
// Returns the launch status.
template <typename T>
hipError_t cgemm(hipStream_t s, int M, int N, int K, cd alpha, CView<T> A, CView<T> B, cd beta,
                 CView<T> C, int batch = 1, long sA = 0, long sB = 0, long sC = 0, ProfSink* prof = nullptr);

// C = alpha * A * (b_scale * B + b_diag * I) (B square in its leading K x N block): the shifted
// operand is formed as B's tiles are loaded, so an iteration such as Newton-Schulz,
// X (3/2 I - 1/2 X^H X), needs no separate kernel for it.  C must not alias A or B.
template <typename T>
hipError_t cgemm_shift_b(hipStream_t s, int M, int N, int K, cd alpha, CView<T> A, CView<T> B, double b_scale,
                         double b_diag, CView<T> C, ProfSink* prof = nullptr);

// Number of shape buckets the launch-plan autotuner has settled (MPDO_GEMM_AUTOTUNE=1).
int gemm_tuned_buckets();
}  // namespace mpdo
