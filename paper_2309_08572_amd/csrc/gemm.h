// Host launchers of the complex matrix-core GEMM (gemm.hip).
#pragma once

#include "common.h"

namespace mpdo {

// C = alpha * A * B + beta * C over `batch` problems; A is M x K, B is K x N, C is M x N as
// strided views (see CView); batch strides sA, sB, sC are in complex elements.  C must not
// alias A or B.  prof (may be null) brackets the matrix-core kernel as PF_GEMM with its
// algorithmic flop and bytes.  No workspace: k is never split (see GemmOpts).
// Returns the launch status.
template <typename T>
hipError_t cgemm(hipStream_t s, int M, int N, int K, cd alpha, CView<T> A, CView<T> B, cd beta,
                 CView<T> C, int batch = 1, long sA = 0, long sB = 0, long sC = 0, ProfSink* prof = nullptr);

// Operand transforms applied as B's tiles are loaded, so that no separate kernel forms them:
// op(B) -> (b_scale op(B) + b_diag I) diag(b_col)  (b_diag needs B square in its leading
// K x N block; b_col, if non-null, is a device array of N real factors).  Newton-Schulz,
// X (3/2 I - 1/2 X^H X), and products followed by a column scaling, R (V diag(s)), use them.
struct GemmOpts {
    double b_scale = 1.0;
    double b_diag = 0.0;
    const double* b_col = nullptr;
    // Device workspace for k-split products (the partial tiles of every k-chunk, added in
    // chunk order by a second launch).  Without one, or when it is too small for the plan's
    // split, the product runs with k unsplit.  Either way the result does not depend on the
    // order in which workgroups run.
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // FP32 products only: each operand split into two BF16 terms and the product formed from
    // three BF16 matrix-core products with FP32 accumulation (relative error of an elementary
    // product below 2^-15 instead of 2^-24; the FP32 accumulation is unchanged).  Ignored for
    // FP64 and with operand transforms.
    bool split_bf16 = false;
};

// cgemm with operand transforms.  C must not alias A or B.
template <typename T>
hipError_t cgemm_ex(hipStream_t s, int M, int N, int K, cd alpha, CView<T> A, CView<T> B, cd beta, CView<T> C,
                    const GemmOpts& opt, ProfSink* prof = nullptr, int batch = 1, long sA = 0, long sB = 0,
                    long sC = 0);

// Number of shape buckets the launch-plan autotuner has settled (MPDO_GEMM_AUTOTUNE=1).
int gemm_tuned_buckets();
}  // namespace mpdo
