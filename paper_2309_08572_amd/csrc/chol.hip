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
//   chol_diag_kernel   one wave: the 64 x 64 diagonal block factored in LDS (right-looking,
//                      column by column) and its lower-triangular inverse by forward
//                      substitution, one column per lane
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
__global__ __launch_bounds__(64) void chol_diag_kernel(const double* __restrict__ A, long lda, int k0, int kb,
                                                       const double* __restrict__ shift, double* __restrict__ L,
                                                       long ldl, double* __restrict__ Li, int* __restrict__ flag) {
    __shared__ double ar[CB][CB + 1], ai[CB][CB + 1];
    __shared__ double xr_s[CB][CB + 1], xi_s[CB][CB + 1];
    const int lane = threadIdx.x;
    const double s = shift ? shift[0] : 0.0;
    for (int idx = lane; idx < kb * kb; idx += 64) {
        const int r = idx / kb, c = idx - (idx / kb) * kb;
        double xr = 0.0, xi = 0.0;
        if (r >= c) {
            const double* a = A + 2 * ((long)(k0 + r) * lda + (k0 + c));
            xr = a[0];
            xi = r == c ? 0.0 : a[1];
            if (r == c) xr += s;
        }
        ar[r][c] = xr;
        ai[r][c] = xi;
    }
    __syncthreads();
    for (int j = 0; j < kb; ++j) {
        double p = ar[j][j];
        if (!(p > 0.0) || !isfinite(p)) {
            if (lane == 0) flag[0] = 1;
            p = 1.0;
        }
        const double dj = sqrt(p), rdj = 1.0 / dj;
        __syncthreads();
        if (lane == 0) ar[j][j] = dj;
        for (int r = j + 1 + lane; r < kb; r += 64) {
            ar[r][j] *= rdj;
            ai[r][j] *= rdj;
        }
        __syncthreads();
        // trailing lower part: a_rc -= l_rj conj(l_cj), j < c <= r
        const int w = kb - j - 1;
        for (int idx = lane; idx < w * w; idx += 64) {
            const int r = j + 1 + idx / w, c = j + 1 + (idx - (idx / w) * w);
            if (c > r) continue;
            const double xr = ar[r][j], xi = ai[r][j], yr = ar[c][j], yi = ai[c][j];
            ar[r][c] -= xr * yr + xi * yi;
            ai[r][c] -= xi * yr - xr * yi;
        }
        __syncthreads();
    }
    // the factor, zero above the diagonal
    for (int idx = lane; idx < kb * kb; idx += 64) {
        const int r = idx / kb, c = idx - (idx / kb) * kb;
        double* l = L + 2 * ((long)(k0 + r) * ldl + (k0 + c));
        l[0] = r >= c ? ar[r][c] : 0.0;
        l[1] = r > c ? ai[r][c] : 0.0;
    }
    // inverse, column c per lane (in LDS): X[r][c] = (delta_rc - sum_{c <= q < r} L[r][q] X[q][c]) / L[r][r]
    if (lane < kb) {
        const int c = lane;
        for (int r = 0; r < kb; ++r) {
            double sr = r == c ? 1.0 : 0.0, si = 0.0;
            for (int q = c; q < r; ++q) {
                const double lr = ar[r][q], li = ai[r][q], yr = xr_s[q][c], yi = xi_s[q][c];
                sr -= lr * yr - li * yi;
                si -= lr * yi + li * yr;
            }
            const double rd = 1.0 / ar[r][r];
            xr_s[r][c] = r < c ? 0.0 : sr * rd;
            xi_s[r][c] = r < c ? 0.0 : si * rd;
        }
        for (int r = 0; r < kb; ++r) {
            Li[2 * ((long)r * CB + c)] = xr_s[r][c];
            Li[2 * ((long)r * CB + c) + 1] = xi_s[r][c];
        }
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
        hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(64), 0, s, A, lda, k0, kb, shift_coef > 0.0 ? sh : nullptr,
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
