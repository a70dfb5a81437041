// Host entry of the FP64 Hermitian block-Jacobi eigensolver (eig.hip).
#pragma once

#include "common.h"

namespace mpdo {

// Device scratch bytes eigh() needs for order n.
size_t eigh_work_bytes(int n);

// Device int where eigh() leaves the number of sweeps of an order <= 64 solve (read it after
// the stream reaches that point; eigh() itself only waits for it when sweeps_used is given).
int* eigh_sweep_counter(void* work, int n);

// Eigen-decomposition of the Hermitian n x n complex matrix H (row-major, leading
// dimension ldh, overwritten).  evals[0..n) receives the eigenvalues in descending order,
// V (row-major, leading dimension ldv) the matching unit eigenvectors as columns.  Blocks
// the host once per sweep (reads a convergence counter through host_pinned, a pinned int).
// prof (may be null) receives marks around every kernel launch.  input_eps: the rounding unit
// the entries of H were formed in (a Gram matrix built by FP32 products carries noise of
// ~eps32 ||H||_F); orders <= 64 leave off-diagonal entries below input_eps ||H||_F unrotated,
// since they hold no information beyond that noise.
hipError_t eigh(hipStream_t s, int n, double* H, int ldh, double* V, int ldv, double* evals, void* work,
                int max_sweeps, int* sweeps_used, int* host_pinned, ProfSink* prof = nullptr,
                double input_eps = 2.220446049250313e-16);

}  // namespace mpdo
