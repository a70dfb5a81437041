// Host entry of the tridiagonal Hermitian eigensolver (tri.hip).
#pragma once

#include "common.h"

namespace mpdo {

// Largest order the tridiagonal solver takes (one workgroup holds its vectors in LDS).
constexpr int TRI_MAX = 1024;

// Device scratch bytes eigh_top() needs for order n (n <= TRI_MAX).
size_t tri_work_bytes(int n);

// Eigenpairs of the Hermitian n x n complex matrix H (row-major, leading dimension ldh,
// overwritten) that one deflation level accepts: with lambda_max the largest eigenvalue and
// st0 = lambda_max when level == 0 (st[0] otherwise), the accepted eigenvalues are the
// largest ones above t = max(floor2 * st0, noise * lambda_max, tau * lambda_max), at most
// cap of them.  Writes, on the device and with no host synchronisation: cnt[0] = m (the
// accepted count), evals[0..m) descending, sig[j] = sqrt(lambda_j) and inv[j] = 1/sig[j]
// (either may be null), the unit eigenvectors as columns 0..m) of V (row-major, leading
// dimension ldv), st[1 + level] = t, and at level 0 st[0] = lambda_max and st[4] = trace(H).
// Requires 1 <= n <= TRI_MAX; returns hipErrorInvalidValue otherwise.
hipError_t eigh_top(hipStream_t s, int n, double* H, int ldh, int level, double floor2, double noise, double tau,
                    int cap, double* st, int* cnt, double* evals, double* sig, double* inv, double* V, int ldv,
                    void* work, ProfSink* prof = nullptr);

}  // namespace mpdo
