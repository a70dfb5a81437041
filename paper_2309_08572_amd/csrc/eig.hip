// Hermitian eigensolver in FP64 for the Gram matrices of the split (gfx950).
//
// Two-sided cyclic block Jacobi.  The matrix is cut into 32-row blocks; in each round the
// blocks are paired by the circle (round-robin) schedule, every 64 x 64 pair matrix is
// diagonalised completely in LDS by scalar complex Jacobi rotations (one workgroup per
// pair), and the pair rotations are applied to the block rows and block columns of the
// matrix and to the accumulated eigenvectors as 64 x 64 x 64 complex products on the FP64
// matrix cores.  A sweep visits every block pair once; the solver stops after the first
// sweep in which no pair had an off-diagonal entry above
//     tol_rel * sqrt(|h_pp h_qq|) + tol_abs,
// tol_abs = eps * ||H||_F.  The blocked solver applies every block rotation by matrix-core
// products whose rounding leaves noise of order sqrt(K) eps |h_pp| in the rotated rows; where
// a dominant row keeps entries above eps ||H||_F alive (large orders), the floor is raised
// 4-fold per sweep after sweep JAC_RELAX_AFTER, up to 64 n eps ||H||_F, so the solve stops at
// the accuracy the products allow instead of running out of sweeps.
// Matrices of order <= 64 are solved by one workgroup in one launch.
// Output: eigenvalues in descending order and the matching eigenvectors as columns.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>

#include "common.h"
#include "eig.h"
#include "tri.h"

namespace mpdo {

namespace {

constexpr int NB = 16;       // block rows of the blocked solver
constexpr int NP = 2 * NB;   // pair matrix order
constexpr int NS = 64;       // largest order solved by one workgroup in one launch
constexpr int JAC_RELAX_AFTER = 12;   // sweeps at the full floor before it is raised

typedef double v4d __attribute__((ext_vector_type(4)));

template <int N>
struct PairLds {
    static constexpr int LD = N + 1;   // LDS row stride (doubles)
    double Hr[N][LD];
    double Hi[N][LD];
    double Vr[N][LD];
    double Vi[N][LD];
    double c[N / 2], s[N / 2], er[N / 2], ei[N / 2];
    int p[N / 2], q[N / 2];
    int flag;
};

// 1/sqrt(x) and 1/x (1e-290 <= |x| <= 1e290) from the hardware estimates and two Newton
// steps each, to a few ulp: a rotation needs c^2 + s^2 = 1 to rounding, not IEEE rounding of
// every intermediate, and the estimate-and-refine chain is about half as long as sqrt + div.
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double r = fma(-(x * y), y, 1.0);
        y = fma(0.5 * y, r, y);
    }
    return y;
}
__device__ __forceinline__ double rcp_nr2(double x) {
    double y = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double e = fma(-x, y, 1.0);
        y = fma(y, e, y);
    }
    return y;
}

__device__ __forceinline__ void circle_pair(int players, int round, int j, int& a, int& b) {
    // players is even; player players-1 stays fixed
    const int m = players - 1;
    if (j == 0) {
        a = round;
        b = m;
    } else {
        a = (round + j) % m;
        b = (round - j + m) % m;
    }
}

constexpr int JAC_ITEMS = 3;   // updates per thread per round in every launch of this solver

// One update of a round: the 2 x 2 block (rows of pair a) x (columns of pair b) of H.
template <int N>
__device__ __forceinline__ void jac_h_item(PairLds<N>& L, int a, int b) {
    // H block: rows {p_a, q_a} x columns {p_b, q_b}
    const double sa = L.s[a], sb = L.s[b];
    if (sa == 0.0 && sb == 0.0) return;
    const int pa = L.p[a], qa = L.q[a], pb = L.p[b], qb = L.q[b];
    double h11r = L.Hr[pa][pb], h11i = L.Hi[pa][pb];
    double h12r = L.Hr[pa][qb], h12i = L.Hi[pa][qb];
    double h21r = L.Hr[qa][pb], h21i = L.Hi[qa][pb];
    double h22r = L.Hr[qa][qb], h22i = L.Hi[qa][qb];
    if (sa != 0.0) {
        // rows: new_p = c h_p - s e h_q ; new_q = s h_p + c e h_q
        const double c = L.c[a], er = L.er[a], ei = L.ei[a];
        const double e1r = er * h21r - ei * h21i, e1i = er * h21i + ei * h21r;
        const double e2r = er * h22r - ei * h22i, e2i = er * h22i + ei * h22r;
        const double n11r = c * h11r - sa * e1r, n11i = c * h11i - sa * e1i;
        const double n12r = c * h12r - sa * e2r, n12i = c * h12i - sa * e2i;
        h21r = sa * h11r + c * e1r;
        h21i = sa * h11i + c * e1i;
        h22r = sa * h12r + c * e2r;
        h22i = sa * h12i + c * e2i;
        h11r = n11r;
        h11i = n11i;
        h12r = n12r;
        h12i = n12i;
    }
    if (sb != 0.0) {
        // columns: new_p = c x_p - s conj(e) x_q ; new_q = s x_p + c conj(e) x_q
        const double c = L.c[b], er = L.er[b], ei = -L.ei[b];
        const double e1r = er * h12r - ei * h12i, e1i = er * h12i + ei * h12r;
        const double e2r = er * h22r - ei * h22i, e2i = er * h22i + ei * h22r;
        const double n11r = c * h11r - sb * e1r, n11i = c * h11i - sb * e1i;
        const double n21r = c * h21r - sb * e2r, n21i = c * h21i - sb * e2i;
        h12r = sb * h11r + c * e1r;
        h12i = sb * h11i + c * e1i;
        h22r = sb * h21r + c * e2r;
        h22i = sb * h21i + c * e2i;
        h11r = n11r;
        h11i = n11i;
        h21r = n21r;
        h21i = n21i;
    }
    L.Hr[pa][pb] = h11r;
    L.Hi[pa][pb] = h11i;
    L.Hr[pa][qb] = h12r;
    L.Hi[pa][qb] = h12i;
    L.Hr[qa][pb] = h21r;
    L.Hi[qa][pb] = h21i;
    L.Hr[qa][qb] = h22r;
    L.Hi[qa][qb] = h22i;
}

// One update of a round: row k of V on the columns of pair b.
template <int N>
__device__ __forceinline__ void jac_v_item(PairLds<N>& L, int b, int k) {
    // V <- V J on the columns of pair b, row k
    const double sb = L.s[b];
    if (sb == 0.0) return;
    const double c = L.c[b], er = L.er[b], ei = -L.ei[b];
    const int pb = L.p[b], qb = L.q[b];
    const double xpr = L.Vr[k][pb], xpi = L.Vi[k][pb];
    const double xqr = L.Vr[k][qb], xqi = L.Vi[k][qb];
    const double eqr = er * xqr - ei * xqi, eqi = er * xqi + ei * xqr;
    L.Vr[k][pb] = c * xpr - sb * eqr;
    L.Vi[k][pb] = c * xpi - sb * eqi;
    L.Vr[k][qb] = sb * xpr + c * eqr;
    L.Vi[k][qb] = sb * xpi + c * eqi;
}

// Diagonalise the Hermitian n x n matrix in L (n even, <= 64); L.V accumulates the
// rotations (starts as identity).  Each round computes the rotations of the n/2 disjoint
// pairs, then applies H <- J^+ H J and V <- V J in one pass: a thread owns the 2 x 2 block
// (rows of pair a) x (columns of pair b) and applies both rotations to it.
// Returns the number of sweeps that rotated.
template <int N>
__device__ int lds_jacobi(PairLds<N>& L, int n, double tol_rel, double tol_abs, int max_sweeps) {
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const int half = n / 2;
    // A round has half^2 H-block and half * n V-row updates.  Every launch of this solver gives
    // a thread at most JAC_ITEMS of them, the same ones in every round: their indices are
    // computed once here instead of by two integer divisions per update per round.
    const int total = half * half + half * n;
    const bool fixed = total <= JAC_ITEMS * nt;
    int kind[JAC_ITEMS], ia[JAC_ITEMS], ib[JAC_ITEMS];
#pragma unroll
    for (int q = 0; q < JAC_ITEMS; ++q) {
        const int idx = tid + q * nt;
        kind[q] = -1;
        ia[q] = ib[q] = 0;
        if (idx < half * half) {
            kind[q] = 0;
            ia[q] = idx / half;
            ib[q] = idx - ia[q] * half;
        } else if (idx < total) {
            kind[q] = 1;
            ia[q] = (idx - half * half) / n;
            ib[q] = (idx - half * half) - ia[q] * n;
        }
    }
    int sweeps = 0;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        if (tid == 0) L.flag = 0;
        __syncthreads();
        for (int r = 0; r < n - 1; ++r) {
            if (tid < half) {
                int p, q;
                circle_pair(n, r, tid, p, q);
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                const double a = L.Hr[p][p], d = L.Hr[q][q];
                const double br = L.Hr[p][q], bi = L.Hi[p][q];
                const double ab2 = br * br + bi * bi;
                double c = 1.0, s = 0.0, er = 1.0, ei = 0.0;
                // |b| > tol, i.e. |b|^2 > tol^2 (tol >= 0)
                const double tol = tol_rel * sqrt(fabs(a * d)) + tol_abs;
                if (ab2 > tol * tol && ab2 > 0.0) {
                    // 1 / |b|; |b|^2 below 1e-290 (not seen at Gram scales) takes the IEEE route,
                    // where the hardware estimate could overflow
                    const double rab = ab2 >= 1e-290 ? rsqrt_nr(ab2) : 1.0 / sqrt(ab2);
                    const double zeta = 0.5 * (d - a) * rab;
                    const double az = fabs(zeta);
                    // t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), the smaller root; for huge
                    // |zeta| (no overflow of zeta^2) t = 1 / (2 zeta)
                    double t;
                    if (az < 1e100) {
                        const double u = fma(zeta, zeta, 1.0);
                        t = rcp_nr2(az + u * rsqrt_nr(u));
                    } else {
                        t = 0.5 / az;
                    }
                    if (zeta < 0.0) t = -t;
                    c = rsqrt_nr(fma(t, t, 1.0));
                    s = t * c;
                    er = br * rab;
                    ei = bi * rab;
                    L.flag = 1;
                }
                L.c[tid] = c;
                L.s[tid] = s;
                L.er[tid] = er;
                L.ei[tid] = ei;
                L.p[tid] = p;
                L.q[tid] = q;
            }
            __syncthreads();
            const int nh = half * half;
            if (fixed) {
#pragma unroll
                for (int q = 0; q < JAC_ITEMS; ++q) {
                    if (kind[q] == 0)
                        jac_h_item(L, ia[q], ib[q]);
                    else if (kind[q] == 1)
                        jac_v_item(L, ia[q], ib[q]);
                }
            } else {
                for (int idx = tid; idx < nh + half * n; idx += nt) {
                    if (idx < nh)
                        jac_h_item(L, idx / half, idx - (idx / half) * half);
                    else
                        jac_v_item(L, (idx - nh) / n, (idx - nh) - ((idx - nh) / n) * n);
                }
            }
            __syncthreads();
        }
        const int f = L.flag;
        __syncthreads();
        if (!f) break;
        ++sweeps;
    }
    return sweeps;
}

__device__ __forceinline__ void pair_rows(int nblk, int round, int pair, int& P, int& Q) {
    circle_pair(nblk, round, pair, P, Q);
}

__device__ __forceinline__ int pair_index(int P, int Q, int x) {
    return (x < NB ? P : Q) * NB + (x & (NB - 1));
}

// ---------------------------------------------------------------- small matrices
// One workgroup of jac_small_threads(n) threads; ||H||_F (the absolute tolerance's scale) is
// summed while the matrix is loaded.  Only the leading np x np corner of the LDS arrays is
// used (np = n rounded up to even; the padding row and column are zero, with 1 on V's
// diagonal).
__global__ __launch_bounds__(1024) void jac_small_kernel(const double* __restrict__ H, int ld, int n,
                                                        double tol_rel, double abs_eps, int max_sweeps,
                                                        double* __restrict__ evals, double* __restrict__ V, int ldv,
                                                        int* __restrict__ sweeps_out) {
    __shared__ PairLds<NS> L;
    __shared__ int rank[NS];
    __shared__ double red[1024 / 64];
    const int tid = threadIdx.x;
    const int np = (n + 1) & ~1;
    double f2 = 0.0;
    for (int idx = tid; idx < np * np; idx += blockDim.x) {
        const int x = idx / np, y = idx - (idx / np) * np;
        double hr = 0.0, hi = 0.0;
        if (x < n && y < n) {
            hr = H[2 * ((long)x * ld + y)];
            hi = H[2 * ((long)x * ld + y) + 1];
            f2 += hr * hr + hi * hi;
        }
        L.Hr[x][y] = hr;
        L.Hi[x][y] = hi;
        L.Vr[x][y] = (x == y) ? 1.0 : 0.0;
        L.Vi[x][y] = 0.0;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) f2 += __shfl_xor(f2, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = f2;
    __syncthreads();
    double fro2 = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) fro2 += red[w];
    // Hermitian part: average the two triangles, real diagonal
    for (int idx = tid; idx < np * np; idx += blockDim.x) {
        const int x = idx / np, y = idx - (idx / np) * np;
        if (x < y) {
            const double r = 0.5 * (L.Hr[x][y] + L.Hr[y][x]);
            const double i = 0.5 * (L.Hi[x][y] - L.Hi[y][x]);
            L.Hr[x][y] = r;
            L.Hi[x][y] = i;
            L.Hr[y][x] = r;
            L.Hi[y][x] = -i;
        } else if (x == y) {
            L.Hi[x][x] = 0.0;
        }
    }
    __syncthreads();
    const int sw = lds_jacobi<NS>(L, np, tol_rel, abs_eps * sqrt(fro2), max_sweeps);
    if (tid < n) {
        const double lam = L.Hr[tid][tid];
        int rk = 0;
        for (int j = 0; j < n; ++j) {
            const double lj = L.Hr[j][j];
            rk += (lj > lam) || (lj == lam && j < tid);
        }
        rank[tid] = rk;
        evals[rk] = lam;
    }
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += blockDim.x) {
        const int x = idx / n, j = idx % n;
        const int rk = rank[j];
        V[2 * ((long)x * ldv + rk)] = L.Vr[x][j];
        V[2 * ((long)x * ldv + rk) + 1] = L.Vi[x][j];
    }
    if (tid == 0 && sweeps_out) *sweeps_out = sw;
}

// ---------------------------------------------------------------- blocked matrices
__global__ __launch_bounds__(256) void jac_pair_kernel(const double* __restrict__ H, int ld, int n, int nblk,
                                                       int round, double* __restrict__ Vp,
                                                       int* __restrict__ skip, int* __restrict__ nrot,
                                                       const double* __restrict__ fro, double tol_rel,
                                                       double abs_factor, int max_inner) {
    __shared__ PairLds<NP> L;
    __shared__ int any;
    const int tid = threadIdx.x;
    const int pair = blockIdx.x;
    int P, Q;
    pair_rows(nblk, round, pair, P, Q);
    const double tol_abs = abs_factor * fro[0];
    if (tid == 0) any = 0;
    for (int idx = tid; idx < NP * NP; idx += blockDim.x) {
        const int x = idx / NP, y = idx % NP;
        const int gx = pair_index(P, Q, x), gy = pair_index(P, Q, y);
        double hr = 0.0, hi = 0.0;
        if (gx < n && gy < n) {
            hr = H[2 * ((long)gx * ld + gy)];
            hi = H[2 * ((long)gx * ld + gy) + 1];
        }
        L.Hr[x][y] = hr;
        L.Hi[x][y] = hi;
        L.Vr[x][y] = (x == y) ? 1.0 : 0.0;
        L.Vi[x][y] = 0.0;
    }
    __syncthreads();
    for (int idx = tid; idx < NP * NP; idx += blockDim.x) {
        const int x = idx / NP, y = idx % NP;
        if (x < y) {
            const double r = 0.5 * (L.Hr[x][y] + L.Hr[y][x]);
            const double i = 0.5 * (L.Hi[x][y] - L.Hi[y][x]);
            L.Hr[x][y] = r;
            L.Hi[x][y] = i;
            L.Hr[y][x] = r;
            L.Hi[y][x] = -i;
            const double ab = sqrt(r * r + i * i);
            if (ab > tol_rel * sqrt(fabs(L.Hr[x][x] * L.Hr[y][y])) + tol_abs) any = 1;
        } else if (x == y) {
            L.Hi[x][x] = 0.0;
        }
    }
    __syncthreads();
    if (!any) {
        if (tid == 0) skip[pair] = 1;
        return;
    }
    lds_jacobi<NP>(L, NP, tol_rel, tol_abs, max_inner);
    double* out = Vp + (long)pair * NP * NP * 2;
    for (int idx = tid; idx < NP * NP; idx += blockDim.x) {
        const int x = idx / NP, y = idx % NP;
        out[2 * idx] = L.Vr[x][y];
        out[2 * idx + 1] = L.Vi[x][y];
    }
    if (tid == 0) {
        skip[pair] = 0;
        atomicAdd(nrot, 1);
    }
}

// 64 x 64 complex product in LDS on the FP64 matrix cores:
//   Y = op(U) X   (mode 0, op(U) = U^+)   or   Y = X U   (mode 1)
// with U, X staged in (Ur, Ui), (Xr, Xi).  Each wave owns a 32 x 32 quadrant.
struct RotLds {
    static constexpr int LD = NP + 1;
    double Xr[NP][LD];
    double Xi[NP][LD];
    double Ur[NP][LD];
    double Ui[NP][LD];
};

__device__ __forceinline__ v4d mfma64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ void rot_product(const RotLds& L, int mode, v4d cr[2][2], v4d ci[2][2]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            cr[i][j] = (v4d){0, 0, 0, 0};
            ci[i][j] = (v4d){0, 0, 0, 0};
        }
    for (int kk = 0; kk < NP; kk += 4) {
        double ar[2], ai[2], nai[2], br[2], bi[2];
        const int k = kk + lk;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int row = wr * 32 + i * 16 + li;
            if (mode == 0) {  // A = U^+ : A[row][k] = conj(U[k][row])
                ar[i] = L.Ur[k][row];
                ai[i] = -L.Ui[k][row];
            } else {  // A = X
                ar[i] = L.Xr[row][k];
                ai[i] = L.Xi[row][k];
            }
            nai[i] = -ai[i];
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = wc * 32 + j * 16 + li;
            if (mode == 0) {  // B = X
                br[j] = L.Xr[k][col];
                bi[j] = L.Xi[k][col];
            } else {  // B = U
                br[j] = L.Ur[k][col];
                bi[j] = L.Ui[k][col];
            }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                cr[i][j] = mfma64(ar[i], br[j], cr[i][j]);
                cr[i][j] = mfma64(nai[i], bi[j], cr[i][j]);
                ci[i][j] = mfma64(ar[i], bi[j], ci[i][j]);
                ci[i][j] = mfma64(ai[i], br[j], ci[i][j]);
            }
    }
}

__device__ void store_acc(RotLds& L, const v4d cr[2][2], const v4d ci[2][2]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int x = wr * 32 + i * 16 + lk + 4 * r;
                const int y = wc * 32 + j * 16 + li;
                L.Xr[x][y] = cr[i][j][r];
                L.Xi[x][y] = ci[i][j][r];
            }
}

__device__ void load_rot(RotLds& L, const double* Vp, int pair, int skipped) {
    const double* U = Vp + (long)pair * NP * NP * 2;
    for (int idx = threadIdx.x; idx < NP * NP; idx += blockDim.x) {
        const int x = idx / NP, y = idx % NP;
        L.Ur[x][y] = skipped ? (x == y ? 1.0 : 0.0) : U[2 * idx];
        L.Ui[x][y] = skipped ? 0.0 : U[2 * idx + 1];
    }
}

// One launch per round: blocks [0, m^2) apply H_ab <- V_a^+ H_ab V_b to the 64 x 64 block
// (rows of pair a) x (columns of pair b); blocks [m^2, m^2 + m * tiles) apply Z <- Z V_b to a
// 64-row tile of the eigenvector accumulator.  Every block owns the entries it rewrites.
__global__ __launch_bounds__(64) void jac_rot2_kernel(double* __restrict__ H, int ld, double* __restrict__ Z,
                                                       int ldz, int n, int nblk, int round,
                                                       const double* __restrict__ Vp,
                                                       const int* __restrict__ skip) {
    __shared__ RotLds L;
    const int m = nblk / 2;
    const int bid = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
    v4d cr[2][2], ci[2][2];
    if (bid < m * m) {
        const int a = bid / m, b = bid % m;
        const int sa = skip[a], sb = skip[b];
        if (sa && sb) return;
        int Pa, Qa, Pb, Qb;
        pair_rows(nblk, round, a, Pa, Qa);
        pair_rows(nblk, round, b, Pb, Qb);
        for (int idx = threadIdx.x; idx < NP * NP; idx += blockDim.x) {
            const int x = idx / NP, y = idx % NP;
            const int gx = pair_index(Pa, Qa, x), gy = pair_index(Pb, Qb, y);
            double xr = 0.0, xi = 0.0;
            if (gx < n && gy < n) {
                xr = H[2 * ((long)gx * ld + gy)];
                xi = H[2 * ((long)gx * ld + gy) + 1];
            }
            L.Xr[x][y] = xr;
            L.Xi[x][y] = xi;
        }
        load_rot(L, Vp, b, sb);
        __syncthreads();
        rot_product(L, 1, cr, ci);   // X V_b
        __syncthreads();
        store_acc(L, cr, ci);
        load_rot(L, Vp, a, sa);
        __syncthreads();
        rot_product(L, 0, cr, ci);   // V_a^+ (X V_b)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int x = wr * 32 + i * 16 + lk + 4 * r;   // FP64 MFMA row interleave
                    const int y = wc * 32 + j * 16 + li;
                    const int gx = pair_index(Pa, Qa, x), gy = pair_index(Pb, Qb, y);
                    if (gx < n && gy < n) {
                        H[2 * ((long)gx * ld + gy)] = cr[i][j][r];
                        H[2 * ((long)gx * ld + gy) + 1] = ci[i][j][r];
                    }
                }
        return;
    }
    const int idx0 = bid - m * m;
    const int b = idx0 % m, rt = idx0 / m;
    if (skip[b]) return;
    int Pb, Qb;
    pair_rows(nblk, round, b, Pb, Qb);
    const int r0 = rt * NP;
    for (int idx = threadIdx.x; idx < NP * NP; idx += blockDim.x) {
        const int x = idx / NP, y = idx % NP;
        const int gx = r0 + x, gy = pair_index(Pb, Qb, y);
        double xr = 0.0, xi = 0.0;
        if (gx < n && gy < n) {
            xr = Z[2 * ((long)gx * ldz + gy)];
            xi = Z[2 * ((long)gx * ldz + gy) + 1];
        }
        L.Xr[x][y] = xr;
        L.Xi[x][y] = xi;
    }
    load_rot(L, Vp, b, 0);
    __syncthreads();
    rot_product(L, 1, cr, ci);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int x = wr * 32 + i * 16 + lk + 4 * r;
                const int y = wc * 32 + j * 16 + li;
                const int gx = r0 + x, gy = pair_index(Pb, Qb, y);
                if (gx < n && gy < n) {
                    Z[2 * ((long)gx * ldz + gy)] = cr[i][j][r];
                    Z[2 * ((long)gx * ldz + gy) + 1] = ci[i][j][r];
                }
            }
}

__global__ void eye_kernel(double* Z, int ld, int n) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * n) return;
    const int x = (int)(idx / n), y = (int)(idx % n);
    Z[2 * ((long)x * ld + y)] = (x == y) ? 1.0 : 0.0;
    Z[2 * ((long)x * ld + y) + 1] = 0.0;
}

__global__ void zero_ints_kernel(int* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void fro_kernel(const double* __restrict__ H, int ld, int n, double* __restrict__ out) {
    __shared__ double part[256];
    double acc = 0.0;
    for (long idx = threadIdx.x; idx < (long)n * n; idx += blockDim.x) {
        const int x = (int)(idx / n), y = (int)(idx % n);
        const double r = H[2 * ((long)x * ld + y)], i = H[2 * ((long)x * ld + y) + 1];
        acc += r * r + i * i;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sqrt(part[0]);
}

// diag(H) -> descending eigenvalues and the permutation that sorts them
__global__ void jac_sort_kernel(const double* __restrict__ H, int ld, int n, double* __restrict__ evals,
                                int* __restrict__ perm) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double lam = H[2 * ((long)i * ld + i)];
        int rk = 0;
        for (int j = 0; j < n; ++j) {
            const double lj = H[2 * ((long)j * ld + j)];
            rk += (lj > lam) || (lj == lam && j < i);
        }
        evals[rk] = lam;
        perm[rk] = i;
    }
}

__global__ void gather_cols_kernel(const double* __restrict__ Z, int ldz, int n, const int* __restrict__ perm,
                                   double* __restrict__ V, int ldv) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * n) return;
    const int x = (int)(idx / n), r = (int)(idx % n);
    const int src = perm[r];
    V[2 * ((long)x * ldv + r)] = Z[2 * ((long)x * ldz + src)];
    V[2 * ((long)x * ldv + r) + 1] = Z[2 * ((long)x * ldz + src) + 1];
}

}  // namespace

size_t eigh_work_bytes(int n) {
    const int nblk = ((n + NB - 1) / NB + 1) & ~1;
    size_t b = 0;
    b += (size_t)(nblk / 2) * NP * NP * 2 * sizeof(double);  // pair rotations
    b += (size_t)n * n * 2 * sizeof(double);                  // accumulated eigenvectors
    b += 64 * sizeof(double);                                  // norms
    b += (size_t)(nblk / 2 + n + 64) * sizeof(int);            // skip flags, perm, counters
    // the tridiagonal solver (orders up to TRI_MAX) uses the same scratch at other times
    const size_t bt = tri_work_bytes(n < TRI_MAX ? n : TRI_MAX);
    return (b > bt ? b : bt) + 1024;
}

int* eigh_sweep_counter(void* work, int n) {
    const int nblk = ((n + NB - 1) / NB + 1) & ~1;
    char* w = (char*)work;
    w += (size_t)(nblk / 2) * NP * NP * 2 * sizeof(double);
    w += (size_t)n * n * 2 * sizeof(double);
    w += 64 * sizeof(double);
    int* skip = (int*)w;
    return skip + nblk / 2 + n;
}

hipError_t eigh(hipStream_t s, int n, double* H, int ldh, double* V, int ldv, double* evals, void* work,
                int max_sweeps, int* sweeps_used, int* host_pinned, ProfSink* prof, double input_eps) {
    if (n <= 0) return hipSuccess;
    const double tol_rel = 1e-15;
    char* w = (char*)work;
    const int nblk = ((n + NB - 1) / NB + 1) & ~1;
    double* Vp = (double*)w;
    w += (size_t)(nblk / 2) * NP * NP * 2 * sizeof(double);
    double* Z = (double*)w;
    w += (size_t)n * n * 2 * sizeof(double);
    double* fro = (double*)w;
    w += 64 * sizeof(double);
    int* skip = (int*)w;
    int* perm = skip + nblk / 2;
    int* nrot = perm + n;

    if (n <= NS) {
        // a round of the small solver has (n/2)^2 + (n/2) n independent updates: one wave up
        // to order 16, four up to 32; fewer waves make each round's two barriers cheaper
        const int threads = n <= 16 ? 64 : (n <= 32 ? 256 : 1024);
        if (prof) prof->begin(s, PF_EIG_SMALL);
        hipLaunchKernelGGL(jac_small_kernel, dim3(1), dim3(threads), 0, s, H, ldh, n, tol_rel, input_eps,
                           max_sweeps, evals, V, ldv, nrot);
        if (prof) prof->end(s, PF_EIG_SMALL, 0.0, 32.0 * n * n);
        if (sweeps_used) {
            hipError_t e = hipMemcpyAsync(host_pinned, nrot, sizeof(int), hipMemcpyDeviceToHost, s);
            if (e != hipSuccess) return e;
            e = hipStreamSynchronize(s);
            if (e != hipSuccess) return e;
            *sweeps_used = host_pinned[0];
        }
        return hipGetLastError();
    }
    hipLaunchKernelGGL(fro_kernel, dim3(1), dim3(256), 0, s, H, ldh, n, fro);
    // read per call (no shared state between the batch workers' threads)
    int inner_sweeps = 1;
    if (const char* e = getenv("MPDO_JACOBI_INNER_SWEEPS")) {
        inner_sweeps = atoi(e);
        if (inner_sweeps < 1) inner_sweeps = 1;
    }
    const long nn = (long)n * n;
    const double eps = 2.220446049250313e-16;
    double abs_factor = eps;
    hipLaunchKernelGGL(eye_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, Z, n, n);
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, s, nrot, 1);
        for (int r = 0; r < nblk - 1; ++r) {
            const double pairs = nblk / 2;
            if (prof) prof->begin(s, PF_EIG_PAIR);
            hipLaunchKernelGGL(jac_pair_kernel, dim3(nblk / 2), dim3(256), 0, s, H, ldh, n, nblk, r, Vp, skip,
                               nrot, fro, tol_rel, abs_factor, inner_sweeps);
            // one inner sweep: NP-1 rounds; per round NP/2 rotations (~40 flop each), the 2 x 2
            // block updates of H ((NP/2)^2 blocks, 56 flop) and of V (NP * NP/2 pairs, 14 flop)
            const double pair_flop = (double)inner_sweeps * (NP - 1) *
                                     (40.0 * (NP / 2) + 56.0 * (NP / 2) * (NP / 2) + 14.0 * NP * (NP / 2));
            if (prof) prof->end(s, PF_EIG_PAIR, pairs * pair_flop, pairs * NP * NP * 16.0 * 2.0);
            const int tiles = (n + NP - 1) / NP;
            const int m = nblk / 2;
            // per block pair two 64^3 complex products; per Z tile one
            const double rotflop = 8.0 * NP * NP * (double)NP * (2.0 * m * m + (double)m * tiles);
            const double rotbytes = 16.0 * NP * (double)NP * (2.0 * m * m + 2.0 * m * tiles);
            if (prof) prof->begin(s, PF_EIG_ROT);
            hipLaunchKernelGGL(jac_rot2_kernel, dim3(m * m + m * tiles), dim3(64), 0, s, H, ldh, Z, n, n, nblk,
                               r, Vp, skip);
            if (prof) prof->end(s, PF_EIG_ROT, rotflop, rotbytes);
        }
        hipError_t e = hipMemcpyAsync(host_pinned, nrot, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (host_pinned[0] == 0) break;
        if (sweep + 1 >= JAC_RELAX_AFTER) abs_factor = std::min(4.0 * abs_factor, 64.0 * n * eps);
    }
    if (sweeps_used) *sweeps_used = sweep;
    if (getenv("MPDO_DEBUG_CHECKS"))
        fprintf(stderr, "[mpdo check] block Jacobi order %d sweeps %d floor %.1f eps ||H||_F\n", n, sweep,
                abs_factor / eps);
    hipLaunchKernelGGL(jac_sort_kernel, dim3(1), dim3(256), 0, s, H, ldh, n, evals, perm);
    hipLaunchKernelGGL(gather_cols_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, Z, n, n, perm, V,
                       ldv);
    return hipGetLastError();
}

}  // namespace mpdo
