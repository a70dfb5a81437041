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
//                      LDS by 16-column panels (a panel in one wave's registers, then a rank-16
//                      update) and its lower-triangular inverse by 16 x 16 blocks
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
// The block lives in LDS, stored by columns; it is factored in panels of PW = 16 columns.
// Panel p (columns j0 = 16 p ..): one wave holds rows 0..63 of the panel in registers (lane r,
// row r) and factors it right-looking, column by column, with the pivot and the multipliers
// taken from other lanes by shuffles, so the 16 steps need no barrier; then every thread applies
// the panel's rank-16 update to the trailing columns (rows r >= c), one barrier.  Columns past
// kb are the identity.  The inverse X = L^{-1} is formed by 16 x 16 blocks: four waves invert
// the diagonal blocks by forward substitution in registers (lane c, column c of the block), then
// block rows I = 1, 2, 3 in turn: T_IJ = sum_{J <= K < I} L_IK X_KJ and X_IJ = -X_II T_IJ for
// all J < I at once.  A pivot that is not positive and finite sets flag[0] = 1 and is replaced
// by 1.
constexpr int DT = 1024;             // threads of chol_diag_kernel
constexpr int DS = DT / CB;         // row slices of the trailing update
constexpr int PW = 8;               // panel width
// x of lane `lane` (the same lane in every active lane of the wave), by two scalar reads
__device__ __forceinline__ double lane_val(double x, int lane) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__global__ __launch_bounds__(DT) void chol_diag_kernel(const double* __restrict__ A, long lda, int k0, int kb,
                                                       const double* __restrict__ shift, double* __restrict__ L,
                                                       long ldl, double* __restrict__ Li, int* __restrict__ flag) {
    __shared__ double Ar[CB][CB], Am[CB][CB];           // [column][row]: the block, then its factor
    __shared__ double Yr[CB][CB + 1], Ym[CB][CB + 1];   // [row][column]: the inverse
    __shared__ double Tr[CB / PW - 1][PW][PW + 1], Tm[CB / PW - 1][PW][PW + 1];
    const int t = threadIdx.x, c = t & (CB - 1), h = t / CB, lane = t & 63, wv = t >> 6;
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
        Yr[r][c] = 0.0;
        Ym[r][c] = 0.0;
    }
    __syncthreads();
    for (int j0 = 0; j0 < CB; j0 += PW) {
        if (wv == 0) {
            const int r = lane;
            double ar[PW], ai[PW];
#pragma unroll
            for (int k = 0; k < PW; ++k) {
                ar[k] = Ar[j0 + k][r];
                ai[k] = Am[j0 + k][r];
            }
#pragma unroll
            for (int jj = 0; jj < PW; ++jj) {
                const int j = j0 + jj;
                double lr, li;
                if (j < kb) {
                    double p = lane_val(ar[jj], j);   // a_jj
                    if (!(p > 0.0) || !isfinite(p)) {
                        if (r == 0) flag[0] = 1;
                        p = 1.0;
                    }
                    const double d = sqrt(p), rd = 1.0 / d;
                    lr = r > j ? ar[jj] * rd : (r == j ? d : 0.0);
                    li = r > j ? ai[jj] * rd : 0.0;
                } else {
                    lr = r == j ? 1.0 : 0.0;
                    li = 0.0;
                }
                ar[jj] = lr;
                ai[jj] = li;
#pragma unroll
                for (int kk = jj + 1; kk < PW; ++kk) {
                    const double cr = lane_val(lr, j0 + kk), ci = lane_val(li, j0 + kk);   // l_{j0+kk, j}
                    ar[kk] -= lr * cr + li * ci;   // a_{r, j0+kk} -= l_rj conj(l_{j0+kk, j})
                    ai[kk] -= li * cr - lr * ci;
                }
            }
#pragma unroll
            for (int k = 0; k < PW; ++k) {
                const bool low = r >= j0 + k;
                Ar[j0 + k][r] = low ? ar[k] : 0.0;
                Am[j0 + k][r] = low ? ai[k] : 0.0;
            }
        }
        __syncthreads();
        // rank-PW update of the trailing columns c >= j0 + PW, rows r >= c
        if (c >= j0 + PW && c < kb) {
            double lcr[PW], lci[PW];
#pragma unroll
            for (int k = 0; k < PW; ++k) {
                lcr[k] = Ar[j0 + k][c];
                lci[k] = -Am[j0 + k][c];   // conj(l_{c, j0+k})
            }
            for (int r = c + h; r < kb; r += DS) {
                double sr = 0.0, si = 0.0;
#pragma unroll
                for (int k = 0; k < PW; ++k) {
                    const double xr = Ar[j0 + k][r], xi = Am[j0 + k][r];
                    sr += xr * lcr[k] - xi * lci[k];
                    si += xr * lci[k] + xi * lcr[k];
                }
                Ar[c][r] -= sr;
                Am[c][r] -= si;
            }
        }
        __syncthreads();
    }
    // the factor to global memory (zeros above the diagonal)
    for (int r = h; r < kb; r += DS)
        if (c < kb) {
            double* l = L + 2 * ((long)(k0 + r) * ldl + (k0 + c));
            l[0] = Ar[c][r];
            l[1] = Am[c][r];
        }
    // inverse: diagonal blocks, one wave each (lanes 0..15: the block's columns)
    // (each lane reads back only the entries of its own column it has written)
    if (wv < CB / PW && lane < PW) {
        const int b0 = PW * wv, cc = lane;
        for (int rr = 0; rr < PW; ++rr) {
            const int row = b0 + rr;
            double sr = rr == cc ? 1.0 : 0.0, si = 0.0;
            for (int k = cc; k < rr; ++k) {
                const double lr = Ar[b0 + k][row], li = Am[b0 + k][row];   // l_{row, b0+k}
                const double yr = Yr[b0 + k][b0 + cc], yi = Ym[b0 + k][b0 + cc];
                sr -= lr * yr - li * yi;
                si -= lr * yi + li * yr;
            }
            const double rd = 1.0 / Ar[row][row];
            Yr[row][b0 + cc] = rr < cc ? 0.0 : sr * rd;
            Ym[row][b0 + cc] = rr < cc ? 0.0 : si * rd;
        }
    }
    __syncthreads();
    // block rows I = 1..3: T_IJ = sum_K L_IK X_KJ, then X_IJ = -X_II T_IJ (J < I)
    for (int I = 1; I < CB / PW; ++I) {
        if (t < I * PW * PW) {
            const int J = t / (PW * PW), rr = (t / PW) % PW, cc = t % PW;
            const int row = PW * I + rr, col = PW * J + cc;
            double sr = 0.0, si = 0.0;
            for (int k = PW * J; k < PW * I; ++k) {
                const double lr = Ar[k][row], li = Am[k][row];   // l_{row, k}
                const double yr = Yr[k][col], yi = Ym[k][col];
                sr += lr * yr - li * yi;
                si += lr * yi + li * yr;
            }
            Tr[J][rr][cc] = sr;
            Tm[J][rr][cc] = si;
        }
        __syncthreads();
        if (t < I * PW * PW) {
            const int J = t / (PW * PW), rr = (t / PW) % PW, cc = t % PW;
            const int row = PW * I + rr;
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int k = 0; k < PW; ++k) {
                const double xr = Yr[row][PW * I + k], xi = Ym[row][PW * I + k];
                const double tr = Tr[J][k][cc], ti = Tm[J][k][cc];
                sr += xr * tr - xi * ti;
                si += xr * ti + xi * tr;
            }
            Yr[row][PW * J + cc] = -sr;
            Ym[row][PW * J + cc] = -si;
        }
        __syncthreads();
    }
    for (int r = h; r < kb; r += DS) {
        Li[2 * ((long)r * CB + c)] = c < kb ? Yr[r][c] : 0.0;
        Li[2 * ((long)r * CB + c) + 1] = c < kb ? Ym[r][c] : 0.0;
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
