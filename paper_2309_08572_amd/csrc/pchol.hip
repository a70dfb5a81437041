// Range bases by pivoted Cholesky of a Gram matrix (gfx950, complex FP64).
//
// For an n x c block R with Gram G = R^H R, a partial Cholesky factorisation with diagonal
// pivoting (the largest remaining Schur-complement diagonal first) stops after t pivots once
// every remaining diagonal is below a threshold thr.  The remaining Schur complement S is
// positive semidefinite and equals (R - Q Q^H R)^H (R - Q Q^H R) for Q = R P L11^{-H}, so the
// part of R outside range(Q) has squared Frobenius norm trace(S) <= (c - t) thr: the chosen
// columns span range(R) down to the threshold.  Q = R W with W = P L11^{-H} is Cholesky QR of
// the chosen columns R P (Q^H Q = L11^{-1} (R P)^H (R P) L11^{-H} = I in exact arithmetic); in
// floating point Q^H Q - I is about eps cond(R P)^2, and a threshold of rel * trace(G) keeps
// cond(R P)^2 near 1/rel, so a few Newton-Schulz steps finish the basis.
//
// This replaces, for the range bases of the split, a Gram eigendecomposition whose accepted
// eigenvectors were only used to form the same kind of basis: the tridiagonal reduction walks
// all c columns, bisection and inverse iteration follow, while the factorisation stops after
// the t accepted pivots.
//
//   pchol_kernel  one workgroup of 512 threads.  Per pivot: an argmax over the remaining
//                 diagonal (wave shuffles, one barrier), the pivot's row of L into LDS, then
//                 column j of L for every remaining row (left-looking: G's pivot row minus the
//                 row's earlier columns times the pivot row's, 2..8 lanes per row) and row j of
//                 L11^{-1} (bordered forward substitution, one thread per column).  L and
//                 L11^{-1} live in the work array (L2-resident); each column of L11^{-1} is
//                 written and read by one thread only.
#include <math.h>

#include "pchol.h"

namespace mpdo {

namespace {

constexpr int PT = 512;
constexpr int PW = PT / 64;

__device__ inline void argmax_wave(double& v, int& k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(v, o);
        const int ok = __shfl_xor(k, o);
        if (ov > v || (ov == v && ok < k)) {
            v = ov;
            k = ok;
        }
    }
}

__device__ inline double sum_wave(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// G: n x n (ld ldg, complex interleaved).  L: n x cap column-major (column j at L + 2 j n).
// X = L11^{-1}: cap x cap row-major (ld cap), lower triangular.  W: n x t (ld ldw).
template <typename T>
__global__ __launch_bounds__(PT) void pchol_kernel(const double* __restrict__ G, long ldg, int n, int level,
                                                   double floor2, double rel, int cap, double* __restrict__ st,
                                                   int* __restrict__ cnt, double* __restrict__ L,
                                                   double* __restrict__ X, T* __restrict__ W, long ldw) {
    __shared__ double d[PCHOL_MAX];       // remaining Schur-complement diagonal
    __shared__ int pos[PCHOL_MAX];        // pivot index of a row, -1 while it remains
    __shared__ double lp[2 * PCHOL_MAX];  // the pivot's row of L (columns < j)
    __shared__ double wv[PW];
    __shared__ int wk[PW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    double tr = 0.0;
    for (int r = tid; r < n; r += PT) {
        const double g = G[2 * ((long)r * ldg + r)];
        d[r] = g;
        pos[r] = -1;
        tr += g > 0.0 ? g : 0.0;
    }
    tr = sum_wave(tr);
    if (lane == 0) wv[wave] = tr;
    __syncthreads();
    tr = 0.0;
#pragma unroll
    for (int w = 0; w < PW; ++w) tr += wv[w];
    const double ref = level == 0 ? tr : st[0];
    double thr = rel * tr;
    if (floor2 * ref > thr) thr = floor2 * ref;
    __syncthreads();   // wv is reused below

    // lanes per row: 8 for n <= 64, 4 for n <= 128, 2 for n <= 256
    const int tpr = n <= 64 ? 8 : (n <= 128 ? 4 : 2);
    const int row = tid / tpr, sub = tid - row * tpr;

    int j = 0;
    for (; j < cap; ++j) {
        double v = -1.0;
        int k = n;
        for (int r = tid; r < n; r += PT)
            if (pos[r] < 0 && d[r] > v) {   // a NaN diagonal is never taken
                v = d[r];
                k = r;
            }
        argmax_wave(v, k);
        if (lane == 0) {
            wv[wave] = v;
            wk[wave] = k;
        }
        __syncthreads();
        v = wv[0];
        k = wk[0];
#pragma unroll
        for (int w = 1; w < PW; ++w)
            if (wv[w] > v || (wv[w] == v && wk[w] < k)) {
                v = wv[w];
                k = wk[w];
            }
        if (!(v > thr) || k >= n) break;   // the same decision in every thread
        const int p = k;
        const double lpp = sqrt(v), ilpp = 1.0 / lpp;
        for (int i = tid; i < j; i += PT) {
            lp[2 * i] = L[2 * ((long)i * n + p)];
            lp[2 * i + 1] = L[2 * ((long)i * n + p) + 1];
        }
        __syncthreads();

        // column j of L: L[r][j] = (G[r][p] - sum_{i<j} L[r][i] conj(L[p][i])) / L[p][j]
        const bool live = row < n && row != p && pos[row] < 0;
        double ar = 0.0, ai = 0.0;
        if (live) {
            for (int i = sub; i < j; i += tpr) {
                const double xr = L[2 * ((long)i * n + row)], xi = L[2 * ((long)i * n + row) + 1];
                const double yr = lp[2 * i], yi = lp[2 * i + 1];
                ar += xr * yr + xi * yi;
                ai += xi * yr - xr * yi;
            }
        }
        for (int o = tpr >> 1; o > 0; o >>= 1) {
            ar += __shfl_xor(ar, o);
            ai += __shfl_xor(ai, o);
        }
        if (sub == 0 && row < n) {
            if (row == p) {
                L[2 * ((long)j * n + p)] = lpp;
                L[2 * ((long)j * n + p) + 1] = 0.0;
                pos[p] = j;
            } else if (live) {
                // G[r][p] = conj(G[p][r]): the pivot's row is read contiguously
                const double gr = G[2 * ((long)p * ldg + row)], gi = -G[2 * ((long)p * ldg + row) + 1];
                const double lr = (gr - ar) * ilpp, li = (gi - ai) * ilpp;
                L[2 * ((long)j * n + row)] = lr;
                L[2 * ((long)j * n + row) + 1] = li;
                d[row] -= lr * lr + li * li;
            }
        }
        // row j of X = L11^{-1}: X[j][c] = -(sum_{c<=m<j} L11[j][m] X[m][c]) / L11[j][j]
        if (tid < j) {
            double sr = 0.0, si = 0.0;
            for (int m = tid; m < j; ++m) {
                const double xr = X[2 * ((long)m * cap + tid)], xi = X[2 * ((long)m * cap + tid) + 1];
                const double yr = lp[2 * m], yi = lp[2 * m + 1];
                sr += yr * xr - yi * xi;
                si += yr * xi + yi * xr;
            }
            X[2 * ((long)j * cap + tid)] = -sr * ilpp;
            X[2 * ((long)j * cap + tid) + 1] = -si * ilpp;
        } else if (tid == j) {
            X[2 * ((long)j * cap + j)] = ilpp;
            X[2 * ((long)j * cap + j) + 1] = 0.0;
        }
        __syncthreads();
    }
    const int t = j;
    if (tid == 0) {
        cnt[0] = t;
        st[8 + level] = thr;
        if (level == 0) {
            st[0] = tr;
            st[4] = tr;
        }
    }
    // W = P L11^{-H}: row r = P e_i (pivot i) holds conj(X[c][i]) for c >= i, other rows 0
    for (long e = tid; e < (long)n * t; e += PT) {
        const int r = (int)(e / t), c = (int)(e - (long)r * t);
        const int i = pos[r];
        double wr = 0.0, wi = 0.0;
        if (i >= 0 && c >= i) {
            wr = X[2 * ((long)c * cap + i)];
            wi = -X[2 * ((long)c * cap + i) + 1];
        }
        W[2 * ((long)r * ldw + c)] = (T)wr;
        W[2 * ((long)r * ldw + c) + 1] = (T)wi;
    }
}

}  // namespace

size_t pchol_work_doubles(int n) {
    const size_t m = (size_t)(n < PCHOL_MAX ? n : PCHOL_MAX);
    return 4 * m * m + 64;
}

template <typename T>
hipError_t pchol_basis(hipStream_t s, const double* G, long ldg, int n, int level, double floor2, double rel,
                       int cap, double* st, int* cnt, double* work, T* W, long ldw, ProfSink* prof) {
    if (n < 0 || n > PCHOL_MAX || cap < 0 || cap > n || level < 0 || level > 3) return hipErrorInvalidValue;
    double* L = work;
    double* X = work + 2 * (size_t)n * (cap > 0 ? cap : 1);
    if (prof) prof->begin(s, PF_PCHOL);
    hipLaunchKernelGGL(pchol_kernel<T>, dim3(1), dim3(PT), 0, s, G, ldg, n, level, floor2, rel, cap, st, cnt, L, X, W,
                       ldw);
    if (prof) prof->end(s, PF_PCHOL, pchol_flop(n, cap), pchol_bytes(n, cap));
    return hipGetLastError();
}

template hipError_t pchol_basis<double>(hipStream_t, const double*, long, int, int, double, double, int, double*,
                                        int*, double*, double*, long, ProfSink*);
template hipError_t pchol_basis<float>(hipStream_t, const double*, long, int, int, double, double, int, double*,
                                       int*, double*, float*, long, ProfSink*);

}  // namespace mpdo
