// Host launchers of the small kernels (kernels.hip).
#pragma once

#include "common.h"

namespace mpdo {

// Y = alpha op(X) + beta Y elementwise over M x N views (X.p == nullptr reads zeros).
template <typename TX, typename TY>
hipError_t geam(hipStream_t s, int M, int N, cd alpha, CView<TX> X, cd beta, CView<TY> Y);

// Left factor of the gate applied to a site: out (cl*D2) x (r*cm), row (l, s'),
// column (k, m): sum_s X_k[s'][s] A[l][s][m].  X: r x D2 x D2 complex FP64 (device).
template <typename T>
hipError_t phys_left(hipStream_t s, const T* A, int cl, int D2, int cm, const double* X, int r, T* out);

// Right factor: out (r*cm) x (D2*cr), row (k, m), column (s', c): sum_s Y_k[s'][s] B[m][s][c].
template <typename T>
hipError_t phys_right(hipStream_t s, const T* B, int cm, int D2, int cr, const double* Y, int r, T* out);

// y[r] = sum_{l,s} x[l] o[s] A[l][s][r]; x, o, y complex FP64 (device).
template <typename T>
hipError_t transfer_left(hipStream_t s, const T* A, int cl, int D2, int cr, const double* x, const double* o,
                         double* y);

// y[l] = sum_{s,r} A[l][s][r] o[s] x[r].
template <typename T>
hipError_t transfer_right(hipStream_t s, const T* A, int cl, int D2, int cr, const double* x, const double* o,
                          double* y);

// v = x (x) z  (complex FP64 vectors of lengths na, nb).
hipError_t kron_vec(hipStream_t s, const double* x, int na, const double* z, int nb, double* v);

// out2[0] = ||X||_F^2, out2[1] = number of blocks with non-finite entries (FP64), in one
// launch of at most SUMSQ_MAX_BLOCKS blocks.  part: device scratch of 2 SUMSQ_MAX_BLOCKS
// doubles; cnt: a device counter that is 0 before the call (zero it once when it is
// allocated; every call leaves it 0 again).  Calls that share part and cnt must be ordered
// on one stream.
constexpr int SUMSQ_MAX_BLOCKS = 1024;
template <typename T>
hipError_t sumsq(hipStream_t s, CView<T> X, int M, int N, double* out2, double* part, unsigned* cnt);

// L[a][b] = x[a] x[b] for the complex FP64 vector x of length n (n x n, row-major, in T).
template <typename T>
hipError_t outer(hipStream_t s, const double* x, int n, T* L);

// out[0..1] = sum_{a,b} y[a] L[a][b] y[b] (complex, FP64 accumulation).
template <typename T>
hipError_t bilinear(hipStream_t s, const T* L, int n, const double* y, double* out);

// Accept the eigenvalues of one level of the split (see spectrum_cut_kernel).
hipError_t spectrum_cut(hipStream_t s, const double* lam, int n, int level, double floor2, double noise,
                        double tau, int cap, double* st, int* cnt, double* sig, double* inv);

// X[:, j] *= f[j]
template <typename T>
hipError_t scale_cols(hipStream_t s, CView<T> X, int M, int N, const double* f);

// X (M x N view) <- seeded uniform [-1, 1) entries (re and im), reproducible for a seed.
template <typename T>
hipError_t fill_random(hipStream_t s, CView<T> X, int M, int N, uint64_t seed);

// Class of each vectorised physical index eta (D2 <= 16 entries), passed by value.
struct EtaClass {
    static constexpr int MAXD2 = 16;
    int c[MAXD2];
};

// Bond enlargement of a cl x D2 x cr site tensor X by the class of its physical index (the
// crosstalk gate's control bonds), into Y (device, (ncls cl or cl) x D2 x (cr or ncls cr)):
// mode 0 / 3 split the right / left bond into ncls blocks, each keeping the entries of its
// class; mode 1 / 2 replicate the left / right bond ncls times.  Y must not alias X.
template <typename T>
hipError_t class_expand(hipStream_t s, const T* X, int cl, int D2, int cr, int mode, int ncls, const EtaClass& cls,
                        T* Y);

// Purity-Preserving Truncation on the kept spectrum (fac[j] = Lambda~_j / Lambda'_j).
// out: [0] tr before, [1] xi before, [2] theta, [3] feasible, [4] degenerate sigma, [5] x,
//      [6] max |Im T'L'|, [7] |Lambda'|^2, [8] T'.Lambda', [9] sum Im, [10] tr after,
//      [11] xi after, [12] |Lambda~|^2.
hipError_t ppt(hipStream_t s, const double* sig, const double* tl, const double* tr, const double* sc, int k,
               int use_ppt, int renorm, double* fac, double* out);

// B[j, :] *= f[j] for a k x ncol row-major block with leading dimension ld.
template <typename T>
hipError_t scale_rows(hipStream_t s, T* B, int k, int ncol, long ld, const double* f);

hipError_t zero_doubles(hipStream_t s, double* p, int n);

// y[j] = sum_a x[a] M[a, j] for the a x n view M (unconjugated), FP64 accumulation.
template <typename T>
hipError_t gemv_left(hipStream_t s, CView<T> M, int a, int n, const double* x, double* y);

// out[j] = ||X[j, :]|| (FP64) for the k x ncol view X.
template <typename T>
hipError_t row_norms(hipStream_t s, CView<T> X, int k, int ncol, double* out);

// out[0] + i out[1] = sum_a x[a] y[a] (FP64 complex).
hipError_t dot(hipStream_t s, const double* x, const double* y, int n, double* out);

}  // namespace mpdo
