// Hermitian eigensolver in FP64 for the Gram matrices of the split (gfx950).
//
// Two-sided cyclic block Jacobi.  The matrix is cut into 32-row blocks; in each round the
// blocks are paired by the circle (round-robin) schedule, every 64 x 64 pair matrix is
// diagonalised completely in LDS by scalar complex Jacobi rotations (one workgroup per
// pair), and the pair rotations are applied to the block rows and block columns of the
// matrix and to the accumulated eigenvectors as 64 x 64 x 64 complex products on the FP64
// matrix cores.  A sweep visits every block pair once; the solver stops after the first
// sweep in which no pair had an off-diagonal entry above
//     tol_rel * sqrt(|h_pp h_qq|) + tol_abs,   tol_abs = eps * ||H||_F
// (entries below the rounding level of the matrix itself are not rotated away).
// Matrices of order <= 64 are solved by one workgroup in one launch.
// Output: eigenvalues in descending order and the matching eigenvectors as columns.
#include "common.h"
#include "eig.h"

namespace mpdo {

namespace {

constexpr int NB = 32;       // block rows
constexpr int NP = 64;       // pair matrix order
constexpr int LD = NP + 1;   // LDS row stride (doubles)

typedef double v4d __attribute__((ext_vector_type(4)));

struct PairLds {
    double Hr[NP][LD];
    double Hi[NP][LD];
    double Vr[NP][LD];
    double Vi[NP][LD];
    double c[NP / 2], s[NP / 2], er[NP / 2], ei[NP / 2];
    int p[NP / 2], q[NP / 2];
    int flag;
};

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

// Diagonalise the Hermitian n x n matrix in L (n even, <= 64); L.V accumulates the
// rotations (starts as identity).  Returns the number of sweeps that rotated.
__device__ int lds_jacobi(PairLds& L, int n, double tol_rel, double tol_abs, int max_sweeps) {
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const int half = n / 2;
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
                const double ab = sqrt(br * br + bi * bi);
                double c = 1.0, s = 0.0, er = 1.0, ei = 0.0;
                if (ab > tol_rel * sqrt(fabs(a * d)) + tol_abs) {
                    const double zeta = (d - a) / (2.0 * ab);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                    er = br / ab;
                    ei = bi / ab;
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
            // rows: H <- J^+ H ; new_p = c h_p - s e h_q ; new_q = s h_p + c e h_q
            for (int idx = tid; idx < half * n; idx += nt) {
                const int j = idx / n, k = idx - (idx / n) * n;
                const double s = L.s[j];
                if (s == 0.0) continue;
                const double c = L.c[j], er = L.er[j], ei = L.ei[j];
                const int p = L.p[j], q = L.q[j];
                const double hpr = L.Hr[p][k], hpi = L.Hi[p][k];
                const double hqr = L.Hr[q][k], hqi = L.Hi[q][k];
                const double eqr = er * hqr - ei * hqi, eqi = er * hqi + ei * hqr;  // e * h_q
                L.Hr[p][k] = c * hpr - s * eqr;
                L.Hi[p][k] = c * hpi - s * eqi;
                L.Hr[q][k] = s * hpr + c * eqr;
                L.Hi[q][k] = s * hpi + c * eqi;
            }
            __syncthreads();
            // columns: X <- X J for X in {H, V}; new_p = c x_p - s conj(e) x_q ;
            // new_q = s x_p + c conj(e) x_q
            for (int idx = tid; idx < 2 * half * n; idx += nt) {
                const int which = idx / (half * n);
                const int rem = idx - which * half * n;
                const int j = rem / n, k = rem - (rem / n) * n;
                const double s = L.s[j];
                if (s == 0.0) continue;
                const double c = L.c[j], er = L.er[j], ei = -L.ei[j];
                const int p = L.p[j], q = L.q[j];
                double (*Xr)[LD] = which ? L.Vr : L.Hr;
                double (*Xi)[LD] = which ? L.Vi : L.Hi;
                const double xpr = Xr[k][p], xpi = Xi[k][p];
                const double xqr = Xr[k][q], xqi = Xi[k][q];
                const double eqr = er * xqr - ei * xqi, eqi = er * xqi + ei * xqr;
                Xr[k][p] = c * xpr - s * eqr;
                Xi[k][p] = c * xpi - s * eqi;
                Xr[k][q] = s * xpr + c * eqr;
                Xi[k][q] = s * xpi + c * eqi;
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
__global__ __launch_bounds__(256) void jac_small_kernel(const double* __restrict__ H, int ld, int n,
                                                        const double* __restrict__ fro, double tol_rel,
                                                        int max_sweeps, double* __restrict__ evals,
                                                        double* __restrict__ V, int ldv,
                                                        int* __restrict__ sweeps_out) {
    __shared__ PairLds L;
    __shared__ int rank[NP];
    const int tid = threadIdx.x;
    const int np = (n + 1) & ~1;
    for (int idx = tid; idx < NP * NP; idx += blockDim.x) {
        const int x = idx / NP, y = idx % NP;
        double hr = 0.0, hi = 0.0;
        if (x < n && y < n) {
            hr = H[2 * ((long)x * ld + y)];
            hi = H[2 * ((long)x * ld + y) + 1];
        }
        L.Hr[x][y] = hr;
        L.Hi[x][y] = hi;
        L.Vr[x][y] = (x == y) ? 1.0 : 0.0;
        L.Vi[x][y] = 0.0;
    }
    __syncthreads();
    // Hermitian part: average the two triangles, real diagonal
    for (int idx = tid; idx < NP * NP; idx += blockDim.x) {
        const int x = idx / NP, y = idx % NP;
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
    const int sw = lds_jacobi(L, np, tol_rel, 2.220446049250313e-16 * fro[0], max_sweeps);
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
                                                       int max_inner) {
    __shared__ PairLds L;
    __shared__ int any;
    const int tid = threadIdx.x;
    const int pair = blockIdx.x;
    int P, Q;
    pair_rows(nblk, round, pair, P, Q);
    const double tol_abs = 2.220446049250313e-16 * fro[0];
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
    lds_jacobi(L, NP, tol_rel, tol_abs, max_inner);
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

// rows of pair p, columns [64 ct, 64 ct + 64):  X <- Vp^+ X
__global__ __launch_bounds__(256) void jac_rot_rows_kernel(double* __restrict__ H, int ld, int n, int nblk,
                                                           int round, const double* __restrict__ Vp,
                                                           const int* __restrict__ skip) {
    __shared__ RotLds L;
    const int pair = blockIdx.y;
    if (skip[pair]) return;
    int P, Q;
    pair_rows(nblk, round, pair, P, Q);
    const int c0 = blockIdx.x * NP;
    const int tid = threadIdx.x;
    const double* U = Vp + (long)pair * NP * NP * 2;
    for (int idx = tid; idx < NP * NP; idx += blockDim.x) {
        const int x = idx / NP, y = idx % NP;
        const int gx = pair_index(P, Q, x), gy = c0 + y;
        double xr = 0.0, xi = 0.0;
        if (gx < n && gy < n) {
            xr = H[2 * ((long)gx * ld + gy)];
            xi = H[2 * ((long)gx * ld + gy) + 1];
        }
        L.Xr[x][y] = xr;
        L.Xi[x][y] = xi;
        L.Ur[x][y] = U[2 * idx];
        L.Ui[x][y] = U[2 * idx + 1];
    }
    __syncthreads();
    v4d cr[2][2], ci[2][2];
    rot_product(L, 0, cr, ci);
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int x = wr * 32 + i * 16 + lk + 4 * r;   // FP64 MFMA row interleave
                const int y = wc * 32 + j * 16 + li;
                const int gx = pair_index(P, Q, x), gy = c0 + y;
                if (gx < n && gy < n) {
                    H[2 * ((long)gx * ld + gy)] = cr[i][j][r];
                    H[2 * ((long)gx * ld + gy) + 1] = ci[i][j][r];
                }
            }
}

// columns of pair p, rows [64 rt, 64 rt + 64) of H (z = 0) or of Z (z = 1):  X <- X Vp
__global__ __launch_bounds__(256) void jac_rot_cols_kernel(double* __restrict__ H, int ld, double* __restrict__ Z,
                                                           int ldz, int n, int nblk, int round,
                                                           const double* __restrict__ Vp,
                                                           const int* __restrict__ skip) {
    __shared__ RotLds L;
    const int pair = blockIdx.y;
    if (skip[pair]) return;
    int P, Q;
    pair_rows(nblk, round, pair, P, Q);
    double* M = blockIdx.z ? Z : H;
    const int ldm = blockIdx.z ? ldz : ld;
    const int r0 = blockIdx.x * NP;
    const int tid = threadIdx.x;
    const double* U = Vp + (long)pair * NP * NP * 2;
    for (int idx = tid; idx < NP * NP; idx += blockDim.x) {
        const int x = idx / NP, y = idx % NP;
        const int gx = r0 + x, gy = pair_index(P, Q, y);
        double xr = 0.0, xi = 0.0;
        if (gx < n && gy < n) {
            xr = M[2 * ((long)gx * ldm + gy)];
            xi = M[2 * ((long)gx * ldm + gy) + 1];
        }
        L.Xr[x][y] = xr;
        L.Xi[x][y] = xi;
        L.Ur[x][y] = U[2 * idx];
        L.Ui[x][y] = U[2 * idx + 1];
    }
    __syncthreads();
    v4d cr[2][2], ci[2][2];
    rot_product(L, 1, cr, ci);
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int x = wr * 32 + i * 16 + lk + 4 * r;   // FP64 MFMA row interleave
                const int y = wc * 32 + j * 16 + li;
                const int gx = r0 + x, gy = pair_index(P, Q, y);
                if (gx < n && gy < n) {
                    M[2 * ((long)gx * ldm + gy)] = cr[i][j][r];
                    M[2 * ((long)gx * ldm + gy) + 1] = ci[i][j][r];
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
    return b + 1024;
}

hipError_t eigh(hipStream_t s, int n, double* H, int ldh, double* V, int ldv, double* evals, void* work,
                int max_sweeps, int* sweeps_used, int* host_pinned) {
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

    hipLaunchKernelGGL(fro_kernel, dim3(1), dim3(256), 0, s, H, ldh, n, fro);
    if (n <= NP) {
        hipLaunchKernelGGL(jac_small_kernel, dim3(1), dim3(256), 0, s, H, ldh, n, fro, tol_rel, max_sweeps,
                           evals, V, ldv, nrot);
        if (sweeps_used) {
            hipMemcpyAsync(host_pinned, nrot, sizeof(int), hipMemcpyDeviceToHost, s);
            hipError_t e = hipStreamSynchronize(s);
            if (e != hipSuccess) return e;
            *sweeps_used = host_pinned[0];
        }
        return hipGetLastError();
    }
    const long nn = (long)n * n;
    hipLaunchKernelGGL(eye_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, Z, n, n);
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, s, nrot, 1);
        for (int r = 0; r < nblk - 1; ++r) {
            hipLaunchKernelGGL(jac_pair_kernel, dim3(nblk / 2), dim3(256), 0, s, H, ldh, n, nblk, r, Vp, skip,
                               nrot, fro, tol_rel, 30);
            const int tiles = (n + NP - 1) / NP;
            hipLaunchKernelGGL(jac_rot_rows_kernel, dim3(tiles, nblk / 2), dim3(256), 0, s, H, ldh, n, nblk, r,
                               Vp, skip);
            hipLaunchKernelGGL(jac_rot_cols_kernel, dim3(tiles, nblk / 2, 2), dim3(256), 0, s, H, ldh, Z, n, n,
                               nblk, r, Vp, skip);
        }
        hipMemcpyAsync(host_pinned, nrot, sizeof(int), hipMemcpyDeviceToHost, s);
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (host_pinned[0] == 0) break;
    }
    if (sweeps_used) *sweeps_used = sweep;
    hipLaunchKernelGGL(jac_sort_kernel, dim3(1), dim3(256), 0, s, H, ldh, n, evals, perm);
    hipLaunchKernelGGL(gather_cols_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, Z, n, n, perm, V,
                       ldv);
    return hipGetLastError();
}

}  // namespace mpdo
