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
//   pchol_kernel  one workgroup of 512 threads, two barriers per pivot.  Every wave takes the
//                 argmax of the remaining diagonal itself (DPP moves inside rows of 16 lanes,
//                 two shuffles across them), so all waves agree on the pivot without an
//                 exchange; the pivot's row of L goes to LDS (barrier); then column j of L for
//                 every remaining row (left-looking: G's pivot row minus the row's earlier
//                 columns times the pivot row's; TPR lanes per row, summed by DPP) and row j
//                 of L11^{-1} (bordered forward substitution, 2..8 lanes per column) (barrier).
//                 Orders <= 64 keep each row's entries of L in its lanes' registers and
//                 L11^{-1} in LDS; larger orders keep both in the work array (L2-resident).
#include <math.h>

#include "pchol.h"

namespace mpdo {

namespace {

constexpr int PT = 512;
constexpr int PW = PT / 64;

// x from another lane of the same row of 16 (DPP); all lanes must be active
template <int CTRL>
__device__ __forceinline__ double dmov(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ int imov(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}

// sum over aligned groups of G lanes (2, 4 or 8), returned to every lane of the group:
// quad swaps (xor 1, xor 2), then the half-row mirror (lane i with 7 - i)
template <int G>
__device__ __forceinline__ double group_sum(double x) {
    if (G >= 2) x += dmov<0xB1>(x);
    if (G >= 4) x += dmov<0x4E>(x);
    if (G >= 8) x += dmov<0x141>(x);
    return x;
}
__device__ __forceinline__ double group_sum_rt(double x, int g) {
    if (g == 8) return group_sum<8>(x);
    if (g == 4) return group_sum<4>(x);
    return group_sum<2>(x);
}

__device__ __forceinline__ void take(double& v, int& k, double ov, int ok) {
    if (ov > v || (ov == v && ok < k)) {
        v = ov;
        k = ok;
    }
}
// argmax (largest value, then smallest index) over the 64 lanes, returned to every lane
__device__ __forceinline__ void wave_argmax(double& v, int& k) {
    take(v, k, dmov<0xB1>(v), imov<0xB1>(k));     // quad_perm [1,0,3,2]
    take(v, k, dmov<0x4E>(v), imov<0x4E>(k));     // quad_perm [2,3,0,1]
    take(v, k, dmov<0x141>(v), imov<0x141>(k));   // row_half_mirror
    take(v, k, dmov<0x140>(v), imov<0x140>(k));   // row_mirror
    take(v, k, __shfl_xor(v, 16), __shfl_xor(k, 16));
    take(v, k, __shfl_xor(v, 32), __shfl_xor(k, 32));
}
__device__ __forceinline__ double wave_sum(double x) {
    x += dmov<0xB1>(x);
    x += dmov<0x4E>(x);
    x += dmov<0x141>(x);
    x += dmov<0x140>(x);
    x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 32);
    return x;
}

// G: n x n (ld ldg, complex interleaved).  TPR lanes per row of L.  NREG > 0: row r's entry
// L[r][i] in register slot i / TPR of lane i % TPR of the row's group (orders n <= PT / TPR,
// NREG * TPR >= n); NREG == 0: L in Lg, n x cap column-major (column j at Lg + 2 j n).
// XCAP > 0: X = L11^{-1} in LDS (ld XCAP, cap <= XCAP); else in Xg (ld cap).  W: n x t (ld ldw).
template <typename T, int TPR, int NREG, int XCAP>
__global__ __launch_bounds__(PT) void pchol_kernel(const double* __restrict__ G, long ldg, int n, int level,
                                                   double floor2, double rel, int cap, double* __restrict__ st,
                                                   int* __restrict__ cnt, double* __restrict__ Lg,
                                                   double* __restrict__ Xg, T* __restrict__ W, long ldw) {
    constexpr int ROWS = PT / TPR;
    __shared__ double d[ROWS];        // remaining Schur-complement diagonal
    __shared__ int pos[ROWS];         // pivot index of a row, -1 while it remains
    __shared__ double lp[2 * ROWS];   // the pivot's row of L (columns < j)
    __shared__ double wv[PW];
    __shared__ double Xs[XCAP > 0 ? 2 * XCAP * XCAP : 2];
    double* X = XCAP > 0 ? Xs : Xg;
    const long ldx = XCAP > 0 ? XCAP : cap;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int row = tid / TPR, sub = tid - row * TPR;

    double tr = 0.0;
    for (int r = tid; r < n; r += PT) {
        const double g = G[2 * ((long)r * ldg + r)];
        d[r] = g;
        pos[r] = -1;
        tr += g > 0.0 ? g : 0.0;
    }
    tr = wave_sum(tr);
    if (lane == 0) wv[wave] = tr;
    __syncthreads();
    tr = 0.0;
#pragma unroll
    for (int w = 0; w < PW; ++w) tr += wv[w];
    const double ref = level == 0 ? tr : st[0];
    double thr = rel * tr;
    if (floor2 * ref > thr) thr = floor2 * ref;

    double lr_[NREG > 0 ? NREG : 1], li_[NREG > 0 ? NREG : 1];
#pragma unroll
    for (int q = 0; q < (NREG > 0 ? NREG : 1); ++q) {
        lr_[q] = 0.0;
        li_[q] = 0.0;
    }

    int j = 0;
    for (; j < cap; ++j) {
        // every wave finds the pivot from the diagonal in LDS (a NaN is never taken)
        double v = -1.0;
        int k = n;
        for (int r = lane; r < n; r += 64)
            if (pos[r] < 0 && d[r] > v) {
                v = d[r];
                k = r;
            }
        wave_argmax(v, k);
        if (!(v > thr) || k >= n) break;   // the same decision in every thread
        const int p = k;
        const double lpp = sqrt(v), ilpp = 1.0 / lpp;
        const bool live = row < n && row != p && pos[row] < 0;
        // G[r][p] = conj(G[p][r]): the pivot's row, read contiguously, in flight over the barrier
        double gr = 0.0, gi = 0.0;
        if (live) {
            gr = G[2 * ((long)p * ldg + row)];
            gi = -G[2 * ((long)p * ldg + row) + 1];
        }
        if (NREG > 0) {
            if (row == p) {
#pragma unroll
                for (int q = 0; q < (NREG > 0 ? NREG : 1); ++q) {
                    const int i = q * TPR + sub;
                    if (i < j) {
                        lp[2 * i] = lr_[q];
                        lp[2 * i + 1] = li_[q];
                    }
                }
            }
        } else {
            for (int i = tid; i < j; i += PT) {
                lp[2 * i] = Lg[2 * ((long)i * n + p)];
                lp[2 * i + 1] = Lg[2 * ((long)i * n + p) + 1];
            }
        }
        __syncthreads();

        // column j of L: L[r][j] = (G[r][p] - sum_{i<j} L[r][i] conj(L[p][i])) / L[p][j]
        double ar = 0.0, ai = 0.0;
        if (live) {
            if (NREG > 0) {
#pragma unroll
                for (int q = 0; q < (NREG > 0 ? NREG : 1); ++q) {
                    const int i = q * TPR + sub;
                    if (i < j) {
                        const double yr = lp[2 * i], yi = lp[2 * i + 1];
                        ar += lr_[q] * yr + li_[q] * yi;
                        ai += li_[q] * yr - lr_[q] * yi;
                    }
                }
            } else {
#pragma unroll 4
                for (int i = sub; i < j; i += TPR) {
                    const double xr = Lg[2 * ((long)i * n + row)], xi = Lg[2 * ((long)i * n + row) + 1];
                    const double yr = lp[2 * i], yi = lp[2 * i + 1];
                    ar += xr * yr + xi * yi;
                    ai += xi * yr - xr * yi;
                }
            }
        }
        ar = group_sum<TPR>(ar);
        ai = group_sum<TPR>(ai);
        if (live) {
            const double lr = (gr - ar) * ilpp, li = (gi - ai) * ilpp;
            if (NREG > 0) {
#pragma unroll
                for (int q = 0; q < (NREG > 0 ? NREG : 1); ++q)
                    if (q * TPR + sub == j) {
                        lr_[q] = lr;
                        li_[q] = li;
                    }
            } else if (sub == 0) {
                Lg[2 * ((long)j * n + row)] = lr;
                Lg[2 * ((long)j * n + row) + 1] = li;
            }
            if (sub == 0) d[row] -= lr * lr + li * li;
        } else if (row == p && sub == 0) {
            pos[p] = j;
        }
        // row j of X = L11^{-1}: X[j][c] = -(sum_{c<=m<j} L11[j][m] X[m][c]) / L11[j][j],
        // xpr lanes per column c (8 for j <= 64, 4 for j <= 128, 2 beyond)
        {
            const int xpr = j <= 64 ? 8 : (j <= 128 ? 4 : 2);
            const int xc = tid / xpr, xs = tid - xc * xpr;
            double sr = 0.0, si = 0.0;
            if (xc < j) {
#pragma unroll 4
                for (int m = xc + xs; m < j; m += xpr) {
                    const double xr = X[2 * (m * ldx + xc)], xi = X[2 * (m * ldx + xc) + 1];
                    const double yr = lp[2 * m], yi = lp[2 * m + 1];
                    sr += yr * xr - yi * xi;
                    si += yr * xi + yi * xr;
                }
            }
            sr = group_sum_rt(sr, xpr);
            si = group_sum_rt(si, xpr);
            if (xs == 0 && xc < j) {
                X[2 * (j * ldx + xc)] = -sr * ilpp;
                X[2 * (j * ldx + xc) + 1] = -si * ilpp;
            }
            if (tid == 0) {
                X[2 * (j * ldx + j)] = ilpp;
                X[2 * (j * ldx + j) + 1] = 0.0;
            }
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
            wr = X[2 * (c * ldx + i)];
            wi = -X[2 * (c * ldx + i) + 1];
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
    // measured per pivot (one MI355X, random Gram matrices): orders <= 64 about 2.1 us with L in
    // registers and L11^{-1} in LDS; orders 65..128 2.7-3.5 us with both in the work array and
    // four lanes per row (3.8-4.0 us in registers: the 32 predicated slots cost more than the L2
    // reads they save); larger orders two lanes per row, 3.5-4.9 us
    if (n <= 64)
        hipLaunchKernelGGL((pchol_kernel<T, 8, 8, 64>), dim3(1), dim3(PT), 0, s, G, ldg, n, level, floor2, rel, cap, st,
                           cnt, L, X, W, ldw);
    else if (n <= 128)
        hipLaunchKernelGGL((pchol_kernel<T, 4, 0, 0>), dim3(1), dim3(PT), 0, s, G, ldg, n, level, floor2, rel, cap, st,
                           cnt, L, X, W, ldw);
    else
        hipLaunchKernelGGL((pchol_kernel<T, 2, 0, 0>), dim3(1), dim3(PT), 0, s, G, ldg, n, level, floor2, rel, cap, st,
                           cnt, L, X, W, ldw);
    if (prof) prof->end(s, PF_PCHOL, pchol_flop(n, cap), pchol_bytes(n, cap));
    return hipGetLastError();
}

template hipError_t pchol_basis<double>(hipStream_t, const double*, long, int, int, double, double, int, double*,
                                        int*, double*, double*, long, ProfSink*);
template hipError_t pchol_basis<float>(hipStream_t, const double*, long, int, int, double, double, int, double*,
                                       int*, double*, float*, long, ProfSink*);

}  // namespace mpdo
