// Cholesky factorisation and triangular solve for the orthonormalisation of tall blocks
// (gfx950, complex FP64): Q = Y L^{-H} with Y^H Y + s I = L L^H.
//
// Shifted Cholesky QR (Fukaya, Kannan, Nakatsukasa, Zhang, Yamamoto, "Shifted Cholesky QR for
// computing the QR factorization of ill-conditioned matrices", SIAM J. Sci. Comput. 42 (2020)):
// one pass with the shift s = 11 (n m + m (m + 1)) u ||Y||^2 (||Y||_F^2 >= ||Y||_2^2 here, a
// larger and still admissible shift) brings the condition number of Y down to about
// sqrt(||Y||^2 / s) whatever it was below 1/u; two unshifted passes then make the columns
// orthonormal to working precision.  The block subspace iteration of the saturated split uses
// it instead of Gram eigen-decompositions: its blocks (theta Z, 8192 x 768 at chi = 512) have
// condition numbers near 1e10, and the Cholesky passes need matrix products and 64-wide
// diagonal blocks, not a sequential tridiagonal reduction of order 768.
//
//   chol_shift_kernel  s from the trace of G (one workgroup; no host synchronisation)
//   chol_diag_kernel   one workgroup of 1024 threads: the 64 x 64 diagonal block factored in
//                      LDS (right-looking, one barrier per column) and its lower-triangular inverse
//   panel and trailing updates, and the block triangular solve, run on the matrix-core GEMM.
#include <math.h>

#include "chol.h"
#include "gemm.h"

namespace mpdo {

namespace {

constexpr int CB = 64;   // block size of the factorisation and of the solve

__global__ __launch_bounds__(256) void chol_shift_kernel(const double* __restrict__ G, long ldg, int m, double coef,
                                                         double* __restrict__ shift) {
    __shared__ double red[256];
    double t = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) t += G[2 * ((long)i * ldg + i)];
    red[threadIdx.x] = t;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) shift[0] = coef * red[0];
}

// Diagonal block [k0, k0 + kb) of the lower Cholesky factor: A (ld lda) holds the trailing matrix
// already updated by the earlier panels; the block plus shift[0] on its diagonal is factored, L
// (ld ldl) receives the factor (zeros above the diagonal) and Li (kb x kb, ld CB) its inverse.
// A pivot that is not positive and finite sets flag[0] = 1 and is replaced by 1 (the result is
// then discarded by the caller).
//
// The block lives in LDS; thread (c, h) = (t mod 64, t / 64) works on column c, rows
// c + h + 16 k (16 row slices, so a step's longest row list is 4).  Step j of the right-looking
// factorisation reads column j, final since step j - 1, and applies a_rc -= a_rj conj(a_cj) /
// a_jj to the rows r >= c of the columns c > j, so that one barrier per step suffices; the
// columns are scaled by 1 / sqrt(a_jj) at the end.  The block is stored by columns (64 doubles
// apart): the 64 lanes of a wave then read column j at consecutive addresses and update
// a_{c+h+16k, c} on distinct banks.  The inverse X = L^{-1} follows the same pattern: y_c =
// e_c, step q subtracts L_rq y_qc / L_qq from the rows r > q (row slice h of every column;
// the lanes of a wave read the same L_rq and update a row of Y stored by rows), and X_rc =
// y_rc / L_rr at the end.
constexpr int DT = 1024;            // threads of chol_diag_kernel
constexpr int DS = DT / CB;         // row slices
__global__ __launch_bounds__(DT) void chol_diag_kernel(const double* __restrict__ A, long lda, int k0, int kb,
                                                       const double* __restrict__ shift, double* __restrict__ L,
                                                       long ldl, double* __restrict__ Li, int* __restrict__ flag) {
    __shared__ double Ar[CB][CB], Am[CB][CB];           // [column][row]: the block, then its factor
    __shared__ double Yr[CB][CB + 1], Ym[CB][CB + 1];   // [row][column]: the inverse
    __shared__ double dg[CB];                           // sqrt of the pivots
    const int t = threadIdx.x, c = t & (CB - 1), h = t / CB;
    const double s = shift ? shift[0] : 0.0;
    for (int r = h; r < CB; r += DS) {
        double vr = 0.0, vi = 0.0;
        if (r < kb && c < kb && r >= c) {
            const double* a = A + 2 * ((long)(k0 + r) * lda + (k0 + c));
            vr = a[0];
            vi = r == c ? 0.0 : a[1];
        }
        Ar[c][r] = r == c && c < kb ? vr + s : vr;
        Am[c][r] = vi;
    }
    __syncthreads();
    for (int j = 0; j < kb; ++j) {
        double p = Ar[j][j];
        if (!(p > 0.0) || !isfinite(p)) p = 1.0;
        if (c > j && c < kb) {
            const double rp = 1.0 / p;
            const double yr = Ar[j][c] * rp, yi = -Am[j][c] * rp;   // conj(a_cj) / a_jj
            for (int r = c + h; r < kb; r += DS) {
                const double xr = Ar[j][r], xi = Am[j][r];
                Ar[c][r] -= xr * yr - xi * yi;
                Am[c][r] -= xr * yi + xi * yr;
            }
        }
        __syncthreads();
    }
    // scale the columns; the factor to global memory (zero above the diagonal) and to LDS
    if (t < CB) {
        double p = t < kb ? Ar[t][t] : 1.0;
        if (!(p > 0.0) || !isfinite(p)) {
            if (t < kb) flag[0] = 1;
            p = 1.0;
        }
        dg[t] = sqrt(p);
    }
    __syncthreads();
    const double rdc = 1.0 / dg[c];
    for (int r = h; r < CB; r += DS) {
        const bool low = r > c && r < kb && c < kb;
        const double lr = r == c ? dg[c] : (low ? Ar[c][r] * rdc : 0.0);
        const double li = low ? Am[c][r] * rdc : 0.0;
        Ar[c][r] = lr;
        Am[c][r] = li;
        Yr[r][c] = r == c ? 1.0 : 0.0;
        Ym[r][c] = 0.0;
        if (r < kb && c < kb) {
            double* l = L + 2 * ((long)(k0 + r) * ldl + (k0 + c));
            l[0] = lr;
            l[1] = li;
        }
    }
    __syncthreads();
    for (int q = 0; q < kb; ++q) {
        if (c <= q) {
            const double rq = 1.0 / Ar[q][q];
            const double yr = Yr[q][c] * rq, yi = Ym[q][c] * rq;
            for (int r = q + 1 + ((h - (q + 1)) & (DS - 1)); r < kb; r += DS) {   // rows > q of slice h
                const double lr = Ar[q][r], li = Am[q][r];
                Yr[r][c] -= lr * yr - li * yi;
                Ym[r][c] -= lr * yi + li * yr;
            }
        }
        __syncthreads();
    }
    for (int r = h; r < kb; r += DS) {
        const double rr = 1.0 / Ar[r][r];
        Li[2 * ((long)r * CB + c)] = c < kb ? Yr[r][c] * rr : 0.0;
        Li[2 * ((long)r * CB + c) + 1] = c < kb ? Ym[r][c] * rr : 0.0;
    }
}

}  // namespace

size_t chol_work_doubles(int m) {
    const int nb = (m + CB - 1) / CB;
    return (size_t)nb * CB * CB * 2 + 64;
}

hipError_t cholesky_lower(hipStream_t s, double* A, long lda, int m, double shift_coef, double* L, long ldl,
                          double* work, int* flag, const GemmOpts& opt, ProfSink* prof) {
    if (m <= 0) return hipSuccess;
    double* sh = work;
    double* Li = work + 64;
    if (shift_coef > 0.0) hipLaunchKernelGGL(chol_shift_kernel, dim3(1), dim3(256), 0, s, A, lda, m, shift_coef, sh);
    for (int k0 = 0; k0 < m; k0 += CB) {
        const int kb = m - k0 < CB ? m - k0 : CB;
        double* Lik = Li + (size_t)(k0 / CB) * CB * CB * 2;
        hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(DT), 0, s, A, lda, k0, kb, shift_coef > 0.0 ? sh : nullptr,
                           L, ldl, Lik, flag);
        const int rest = m - k0 - kb;
        if (rest <= 0) break;
        // panel: L[k0+kb:, k0:k0+kb] = A[k0+kb:, k0:k0+kb] Li^H
        hipError_t e = cgemm_ex<double>(s, rest, kb, kb, cd{1.0, 0.0}, view<double>(A + 2 * ((long)(k0 + kb) * lda + k0), lda, 1),
                                        adj(view<double>(Lik, CB, 1)), cd{0.0, 0.0},
                                        view<double>(L + 2 * ((long)(k0 + kb) * ldl + k0), ldl, 1), opt, prof);
        if (e != hipSuccess) return e;
        // trailing: A[k0+kb:, k0+kb:] -= L_panel L_panel^H (the whole square; only the lower part is read)
        const CView<double> P = view<double>(L + 2 * ((long)(k0 + kb) * ldl + k0), ldl, 1);
        e = cgemm_ex<double>(s, rest, rest, kb, cd{-1.0, 0.0}, P, adj(P), cd{1.0, 0.0},
                             view<double>(A + 2 * ((long)(k0 + kb) * lda + (k0 + kb)), lda, 1), opt, prof);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t trsm_right_lower_adj(hipStream_t s, double* Y, long ldy, int n, int m, const double* L, long ldl,
                                const double* work, double* Q, long ldq, const GemmOpts& opt, ProfSink* prof) {
    const double* Li = work + 64;
    for (int j0 = 0; j0 < m; j0 += CB) {
        const int jb = m - j0 < CB ? m - j0 : CB;
        if (j0 > 0) {
            // Y_j -= Q_{<j} L[j0:j0+jb, 0:j0]^H
            hipError_t e = cgemm_ex<double>(s, n, jb, j0, cd{-1.0, 0.0}, view<double>(Q, ldq, 1),
                                            adj(view<double>((double*)L + 2 * ((long)j0 * ldl), ldl, 1)), cd{1.0, 0.0},
                                            view<double>(Y + 2 * j0, ldy, 1), opt, prof);
            if (e != hipSuccess) return e;
        }
        // Q_j = Y_j Li_jj^H
        hipError_t e = cgemm_ex<double>(s, n, jb, jb, cd{1.0, 0.0}, view<double>(Y + 2 * j0, ldy, 1),
                                        adj(view<double>((double*)Li + (size_t)(j0 / CB) * CB * CB * 2, CB, 1)),
                                        cd{0.0, 0.0}, view<double>(Q + 2 * j0, ldq, 1), opt, prof);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace mpdo
