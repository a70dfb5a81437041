// Host launcher of the pivoted-Cholesky range basis (pchol.hip), complex FP64 Gram matrices.
#pragma once

#include "common.h"

namespace mpdo {

// Largest Gram order (and column count) the one-workgroup kernel takes.
constexpr int PCHOL_MAX = 256;

// Device doubles of the work array for Gram order n (n <= PCHOL_MAX): the Cholesky columns
// (n x n complex) and the inverse of the pivot block (n x n complex).
size_t pchol_work_doubles(int n);

// Algorithmic work of a call that took t pivots at order n: per pivot j a column of L
// (n - j rows, j complex multiply-adds each) and a row of L11^{-1} (j(j+1)/2); bytes: G read
// once, W written.  pchol_basis records its launch with t = cap; the caller amends it.
inline double pchol_flop(int n, int t) {
    return 8.0 * ((double)t * t * (3.0 * n - 2.0 * t) / 6.0 + (double)t * t * t / 6.0);
}
inline double pchol_bytes(int n, int t) { return 16.0 * n * (double)n + 16.0 * n * (double)t; }

// Columns of a range basis of R from its Gram G = R^H R (n x n, Hermitian, complex FP64, row
// major with leading dimension ldg; only read).  A pivoted Cholesky factorisation
// G[P, P] = L11 L11^H takes pivots while the largest remaining Schur-complement diagonal exceeds
//     thr = max(rel * trace(G), floor2 * st[0])
// and at most cap of them.  It writes cnt[0] = t (the pivots taken) and W (n x t, T complex,
// row major, leading dimension ldw) = P L11^{-H}, so that Q = R W has Q^H Q = I up to rounding
// (eps times the squared condition number of the t chosen columns of R) and
// ||R - Q Q^H R||_F^2 = trace of the remaining Schur complement <= (n - t) thr.
// st (device): st[8 + level] = thr; at level 0 also st[0] = st[4] = trace(G), the reference
// the later levels' floor2 is relative to.  work: pchol_work_doubles(n) doubles.
// Requires 0 <= n <= PCHOL_MAX, 0 <= cap <= n, 0 <= level <= 3; hipErrorInvalidValue
// otherwise.  No host synchronisation.
template <typename T>
hipError_t pchol_basis(hipStream_t s, const double* G, long ldg, int n, int level, double floor2, double rel,
                       int cap, double* st, int* cnt, double* work, T* W, long ldw, ProfSink* prof);

}  // namespace mpdo
