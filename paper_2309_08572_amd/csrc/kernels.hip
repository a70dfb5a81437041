// Memory-bound and small kernels of the two-site update (gfx950).
//
//  geam            Y = alpha op(X) + beta Y on strided complex views (copies, adjoints,
//                  precision changes, residuals)
//  phys_left/right apply the operator-Schmidt factors of a two-site superoperator to the
//                  physical index of a site tensor (the factored form of the theta
//                  contraction, Sec. III.A)
//  transfer_*      one transfer-matrix step of a trace or expectation contraction
//                  (Sec. III.D trace environment, Sec. III.E linear observables)
//  sumsq           ||X||_F^2 in FP64 with a non-finite flag
//  spectrum_cut    per-level acceptance of Gram eigenvalues (the cut of Sec. III.A)
//  ppt             Purity-Preserving Truncation on the kept spectrum (Sec. III.D,
//                  Eqs. (xiformula), (ppt)) in FP64
#include <math.h>

#include "common.h"
#include "kernels.h"

namespace mpdo {

namespace {

template <typename TX, typename TY>
__global__ void geam_kernel(int M, int N, double ar, double ai, CView<TX> X, double br, double bi, CView<TY> Y) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)M * N) return;
    const int m = (int)(idx / N), n = (int)(idx - (idx / N) * N);
    double xr = 0.0, xi = 0.0;
    if (X.p) {
        const long ox = 2 * ((long)m * X.rs + (long)n * X.cs);
        xr = (double)X.p[ox];
        xi = (double)X.p[ox + 1];
        if (X.conj) xi = -xi;
    }
    const long oy = 2 * ((long)m * Y.rs + (long)n * Y.cs);
    double vr = ar * xr - ai * xi, vi = ar * xi + ai * xr;
    if (br != 0.0 || bi != 0.0) {
        const double yr = (double)Y.p[oy];
        const double yi = Y.conj ? -(double)Y.p[oy + 1] : (double)Y.p[oy + 1];
        vr += br * yr - bi * yi;
        vi += br * yi + bi * yr;
    }
    Y.p[oy] = (TY)vr;
    Y.p[oy + 1] = (TY)(Y.conj ? -vi : vi);
}

// out[l][s'][k][m] = sum_s X[k][s'][s] A[l][s][m]      (out row (l,s'), column (k,m))
template <typename T>
__global__ void phys_left_kernel(const T* __restrict__ A, int cl, int D2, int cm, const double* __restrict__ X,
                                 int r, T* __restrict__ out) {
    extern __shared__ double xs[];  // r * D2 * D2 complex
    const int nx = r * D2 * D2;
    for (int i = threadIdx.x; i < 2 * nx; i += blockDim.x) xs[i] = X[i];
    __syncthreads();
    const long total = (long)cl * D2 * r * cm;
    const long ld = (long)r * cm;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int m = (int)(idx % cm);
        long t = idx / cm;
        const int k = (int)(t % r);
        t /= r;
        const int sp = (int)(t % D2);
        const int l = (int)(t / D2);
        double accr = 0.0, acci = 0.0;
        const double* xk = xs + 2 * ((long)k * D2 * D2 + (long)sp * D2);
        const T* a = A + 2 * ((long)l * D2 * cm + m);
        for (int s = 0; s < D2; ++s) {
            const double xr = xk[2 * s], xi = xk[2 * s + 1];
            if (xr == 0.0 && xi == 0.0) continue;
            const double ar = (double)a[2 * (long)s * cm], ai = (double)a[2 * (long)s * cm + 1];
            accr += xr * ar - xi * ai;
            acci += xr * ai + xi * ar;
        }
        out[2 * ((long)(l * D2 + sp) * ld + (long)k * cm + m)] = (T)accr;
        out[2 * ((long)(l * D2 + sp) * ld + (long)k * cm + m) + 1] = (T)acci;
    }
}

// out[k][m][s'][r] = sum_s Y[k][s'][s] B[m][s][r]      (out row (k,m), column (s',r))
template <typename T>
__global__ void phys_right_kernel(const T* __restrict__ B, int cm, int D2, int cr, const double* __restrict__ Y,
                                  int r, T* __restrict__ out) {
    extern __shared__ double ys[];
    const int ny = r * D2 * D2;
    for (int i = threadIdx.x; i < 2 * ny; i += blockDim.x) ys[i] = Y[i];
    __syncthreads();
    const long total = (long)r * cm * D2 * cr;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int c = (int)(idx % cr);
        long t = idx / cr;
        const int sp = (int)(t % D2);
        t /= D2;
        const int m = (int)(t % cm);
        const int k = (int)(t / cm);
        double accr = 0.0, acci = 0.0;
        const double* yk = ys + 2 * ((long)k * D2 * D2 + (long)sp * D2);
        const T* b = B + 2 * ((long)m * D2 * cr + c);
        for (int s = 0; s < D2; ++s) {
            const double yr = yk[2 * s], yi = yk[2 * s + 1];
            if (yr == 0.0 && yi == 0.0) continue;
            const double br = (double)b[2 * (long)s * cr], bi = (double)b[2 * (long)s * cr + 1];
            accr += yr * br - yi * bi;
            acci += yr * bi + yi * br;
        }
        out[2 * idx] = (T)accr;
        out[2 * idx + 1] = (T)acci;
    }
}

// y[r] = sum_{l, s} x[l] o[s] A[l][s][r]   (A is cl x D2 x cr).  Block: 64 outputs.
template <typename T>
__global__ __launch_bounds__(256) void transfer_left_kernel(const T* __restrict__ A, int cl, int D2, int cr,
                                                            const double* __restrict__ x,
                                                            const double* __restrict__ o,
                                                            double* __restrict__ y) {
    __shared__ double pr[4][64], pi[4][64];
    __shared__ double os[2 * 16];
    __shared__ int nzs[16];
    __shared__ int nnz;
    if (threadIdx.x == 0) {
        int c = 0;
        for (int s = 0; s < D2; ++s) {
            os[2 * s] = o[2 * s];
            os[2 * s + 1] = o[2 * s + 1];
            if (o[2 * s] != 0.0 || o[2 * s + 1] != 0.0) nzs[c++] = s;
        }
        nnz = c;
    }
    __syncthreads();
    const int rloc = threadIdx.x & 63, lg = threadIdx.x >> 6;
    const int rr = blockIdx.x * 64 + rloc;
    double accr = 0.0, acci = 0.0;
    if (rr < cr) {
        for (int l = lg; l < cl; l += 4) {
            const double xr = x[2 * l], xi = x[2 * l + 1];
            double sr = 0.0, si = 0.0;
            for (int t = 0; t < nnz; ++t) {
                const int s = nzs[t];
                const long off = 2 * (((long)l * D2 + s) * cr + rr);
                const double ar = (double)A[off], ai = (double)A[off + 1];
                sr += os[2 * s] * ar - os[2 * s + 1] * ai;
                si += os[2 * s] * ai + os[2 * s + 1] * ar;
            }
            accr += xr * sr - xi * si;
            acci += xr * si + xi * sr;
        }
    }
    pr[lg][rloc] = accr;
    pi[lg][rloc] = acci;
    __syncthreads();
    if (lg == 0 && rr < cr) {
        y[2 * rr] = pr[0][rloc] + pr[1][rloc] + pr[2][rloc] + pr[3][rloc];
        y[2 * rr + 1] = pi[0][rloc] + pi[1][rloc] + pi[2][rloc] + pi[3][rloc];
    }
}

// y[l] = sum_{s, r} A[l][s][r] o[s] x[r].  One wave per output row l.
template <typename T>
__global__ __launch_bounds__(256) void transfer_right_kernel(const T* __restrict__ A, int cl, int D2, int cr,
                                                             const double* __restrict__ x,
                                                             const double* __restrict__ o,
                                                             double* __restrict__ y) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int l = blockIdx.x * 4 + wave;
    if (l >= cl) return;
    double accr = 0.0, acci = 0.0;
    for (int s = 0; s < D2; ++s) {
        const double orr = o[2 * s], oi = o[2 * s + 1];
        if (orr == 0.0 && oi == 0.0) continue;
        double sr = 0.0, si = 0.0;
        for (int r = lane; r < cr; r += 64) {
            const long off = 2 * (((long)l * D2 + s) * cr + r);
            const double ar = (double)A[off], ai = (double)A[off + 1];
            const double xr = x[2 * r], xi = x[2 * r + 1];
            sr += ar * xr - ai * xi;
            si += ar * xi + ai * xr;
        }
        accr += orr * sr - oi * si;
        acci += orr * si + oi * sr;
    }
    for (int off = 32; off > 0; off >>= 1) {
        accr += __shfl_down(accr, off);
        acci += __shfl_down(acci, off);
    }
    if (lane == 0) {
        y[2 * l] = accr;
        y[2 * l + 1] = acci;
    }
}

// v[(a, b)] = x[a] * z[b]  (a < na, b < nb): the trace vector of a block of sites times
// the vectorised operator of one more site
__global__ void kron_kernel(const double* __restrict__ x, int na, const double* __restrict__ z, int nb,
                            double* __restrict__ v) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= na * nb) return;
    const int a = idx / nb, b = idx % nb;
    const double xr = x[2 * a], xi = x[2 * a + 1], zr = z[2 * b], zi = z[2 * b + 1];
    v[2 * idx] = xr * zr - xi * zi;
    v[2 * idx + 1] = xr * zi + xi * zr;
}

// ||X||_F^2 and the count of non-finite entries in one launch: each block stores its partial
// sums in part[2 b], part[2 b + 1] and counts itself in *cnt; the last block to arrive adds the
// partials in block order (the result does not depend on which block finishes when), writes
// out[0..1] and resets *cnt to 0 for the next call.
template <typename T>
__global__ void sumsq_kernel(CView<T> X, int M, int N, double* __restrict__ out, double* __restrict__ part_g,
                             unsigned* __restrict__ cnt) {
    __shared__ double part[256];
    __shared__ double pbad[256];
    __shared__ bool last;
    double acc = 0.0, bad = 0.0;
    const long tot = (long)M * N;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < tot; idx += (long)gridDim.x * blockDim.x) {
        const int m = (int)(idx / N), n = (int)(idx - (idx / N) * N);
        const long off = 2 * ((long)m * X.rs + (long)n * X.cs);
        const double r = (double)X.p[off], i = (double)X.p[off + 1];
        if (!isfinite(r) || !isfinite(i)) bad = 1.0;
        acc += r * r + i * i;
    }
    part[threadIdx.x] = acc;
    pbad[threadIdx.x] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            part[threadIdx.x] += part[threadIdx.x + s];
            pbad[threadIdx.x] += pbad[threadIdx.x + s];
        }
        __syncthreads();
    }
    // The blocks of a launch run on different XCDs, whose L2 caches are not coherent with each
    // other: the partials, the arrival count and its reset all go through device-scope atomic
    // accesses, and the arrival orders them (release by every block, acquire by the last).
    if (threadIdx.x == 0) {
        __hip_atomic_store(&part_g[2 * blockIdx.x], part[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&part_g[2 * blockIdx.x + 1], pbad[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        last = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x) {
        a += __hip_atomic_load(&part_g[2 * i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        b += __hip_atomic_load(&part_g[2 * i + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    part[threadIdx.x] = a;
    pbad[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            part[threadIdx.x] += part[threadIdx.x + s];
            pbad[threadIdx.x] += pbad[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = part[0];
        out[1] = pbad[0];
        __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Accept the eigenvalues of one level of the split.  lam: descending eigenvalues of the
// level's Gram matrix.  st (device, FP64):
//   st[0] = largest eigenvalue of the first level (set when level == 0)
//   st[1 + level] = the level's acceptance threshold
//   st[4] = sum of the first level's non-negative eigenvalues (set when level == 0)
// Accepted: lam_j > max(floor2 * st[0], noise * lam_0, tau * lam_0) and j < cap.
// Writes cnt[0] = accepted count, sig[j] = sqrt(lam_j) for accepted j, and
// inv[j] = 1/sqrt(lam_j) (used to normalise orthonormal-basis columns).
__global__ void spectrum_cut_kernel(const double* __restrict__ lam, int n, int level, double floor2,
                                    double noise, double tau, int cap, double* __restrict__ st,
                                    int* __restrict__ cnt, double* __restrict__ sig, double* __restrict__ inv) {
    __shared__ int c;
    if (threadIdx.x == 0) {
        const double l0 = n > 0 ? lam[0] : 0.0;
        if (level == 0) {
            // st[4]: sum of the non-negative eigenvalues = squared Frobenius norm of the factor
            double tot = 0.0;
            for (int j = 0; j < n; ++j) tot += lam[j] > 0.0 ? lam[j] : 0.0;
            st[0] = l0;
            st[4] = tot;
        }
        double t = floor2 * st[0];
        if (noise * l0 > t) t = noise * l0;
        if (tau * l0 > t) t = tau * l0;
        int k = 0;
        while (k < n && k < cap && lam[k] > t && lam[k] > 0.0) ++k;
        if (!(l0 > 0.0)) k = 0;
        c = k;
        cnt[0] = k;
        st[1 + level] = t;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < c; j += blockDim.x) {
        const double s = sqrt(lam[j]);
        if (sig) sig[j] = s;
        if (inv) inv[j] = 1.0 / s;
    }
}

// Seeded random start block: entry (r, c) of X gets re, im uniform in [-1, 1) from the
// SplitMix64 sequence at counter (seed, r * cols + c) (Steele, Lea, Flood 2014).
__device__ inline uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Bond enlargement for the crosstalk gate.  X: cl x D2 x cr site tensor; the vectorised physical
// index eta has class cls.c[eta] in [0, ncls).  Y (complex, T):
//   mode 0: cl x D2 x (ncls cr), Y[l][eta][a cr + r] = X[l][eta][r] if a == class(eta), else 0
//   mode 1: (ncls cl) x D2 x cr, Y[a cl + l][eta][r] = X[l][eta][r]
//   mode 2: cl x D2 x (ncls cr), Y[l][eta][a cr + r] = X[l][eta][r]
//   mode 3: (ncls cl) x D2 x cr, Y[a cl + l][eta][r] = X[l][eta][r] if a == class(eta), else 0
template <typename T>
__global__ void class_expand_kernel(const T* __restrict__ X, int cl, int D2, int cr, int mode, int ncls, EtaClass cls,
                                    T* __restrict__ Y) {
    const long tot = (long)ncls * cl * D2 * cr;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= tot) return;
    int l, eta, r, a;
    if (mode == 0 || mode == 2) {
        const long wide = (long)ncls * cr;
        const long q = idx / wide;
        const int rr = (int)(idx - q * wide);
        l = (int)(q / D2);
        eta = (int)(q - (long)l * D2);
        a = rr / cr;
        r = rr - a * cr;
    } else {
        const long per = (long)D2 * cr;
        const long ll = idx / per;
        const int rem = (int)(idx - ll * per);
        a = (int)(ll / cl);
        l = (int)(ll - (long)a * cl);
        eta = rem / cr;
        r = rem - eta * cr;
    }
    const bool keep = (mode == 1 || mode == 2) || cls.c[eta] == a;
    const long src = 2 * (((long)l * D2 + eta) * cr + r);
    Y[2 * idx] = keep ? X[src] : (T)0;
    Y[2 * idx + 1] = keep ? X[src + 1] : (T)0;
}

template <typename T>
__global__ void fill_random_kernel(CView<T> X, int M, int N, uint64_t seed) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)M * N) return;
    const long r = idx / N, c = idx - (idx / N) * N;
    const uint64_t h = splitmix64(seed ^ splitmix64((uint64_t)idx));
    const double u0 = (double)(h >> 40) * (1.0 / 16777216.0), u1 = (double)((h >> 16) & 0xFFFFFF) * (1.0 / 16777216.0);
    T* p = X.p + 2 * (r * X.rs + c * X.cs);
    p[0] = (T)(2.0 * u0 - 1.0);
    p[1] = (T)(2.0 * u1 - 1.0);
}

template <typename T>
__global__ void scale_cols_kernel(CView<T> X, int M, int N, const double* __restrict__ f) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)M * N) return;
    const int m = (int)(idx / N), n = (int)(idx - (idx / N) * N);
    const long off = 2 * ((long)m * X.rs + (long)n * X.cs);
    X.p[off] = (T)((double)X.p[off] * f[n]);
    X.p[off + 1] = (T)((double)X.p[off + 1] * f[n]);
}

// PPT on the kept spectrum.  Inputs (device, FP64):
//   sig[k]   kept Schmidt values Lambda'
//   tl[k]    left trace factors  (l . U_j), complex
//   tr[k]    right trace factors (B_j . r), complex; T'_j Lambda'_j = tl_j tr_j
//   sc[0..1] = re, im tr(rho); sc[4] = ||theta||_F^2 (sc[5]: its non-finite count)
// Output: fac[j] = Lambda~_j / Lambda'_j and out[0..15] (see PptOut in kernels.h).
__global__ void ppt_kernel(const double* __restrict__ sig, const double* __restrict__ tl,
                           const double* __restrict__ tr, const double* __restrict__ sc, int k, int use_ppt,
                           int renorm, double* __restrict__ fac, double* __restrict__ out) {
    __shared__ double red[6][256];
    const int tid = threadIdx.x;
    double s_tt = 0, s_tl = 0, s_ll = 0, s_t = 0, s_im = 0, s_imx = 0;
    for (int j = tid; j < k; j += blockDim.x) {
        const double ar = tl[2 * j], ai = tl[2 * j + 1], br = tr[2 * j], bi = tr[2 * j + 1];
        const double pr = ar * br - ai * bi, pim = ar * bi + ai * br;  // T'_j Lambda'_j
        const double l = sig[j];
        const double Tj = l > 0.0 ? pr / l : 0.0;
        s_tt += Tj * Tj;
        s_tl += Tj * l;
        s_ll += l * l;
        s_t += pr;
        s_im += pim;
        s_imx = fmax(s_imx, fabs(pim));
    }
    red[0][tid] = s_tt;
    red[1][tid] = s_tl;
    red[2][tid] = s_ll;
    red[3][tid] = s_t;
    red[4][tid] = s_im;
    red[5][tid] = s_imx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            for (int q = 0; q < 5; ++q) red[q][tid] += red[q][tid + s];
            red[5][tid] = fmax(red[5][tid], red[5][tid + s]);
        }
        __syncthreads();
    }
    __shared__ double xs, cterm, scale_all;
    if (tid == 0) {
        const double tt = red[0][0], tl_ = red[1][0], ll = red[2][0];
        const double trr = sc[0], n2 = sc[4];
        const double nT = sqrt(tt), nL = sqrt(ll);
        double x = 0.0, cth = 1.0, theta = 0.0, sigma = 0.0;
        int feas = 1, dg = 0;
        if (!use_ppt || nT == 0.0 || nL == 0.0 || n2 <= 0.0) {
            dg = use_ppt ? 1 : 0;
        } else {
            // Eq. (xiformula): cos(theta) = |T| cos(phi) / |T'| = tr(rho) / (|Lambda| |T'|)
            cth = trr / (sqrt(n2) * nT);
            if (cth > 1.0) {
                feas = 0;
                theta = 0.0;
            } else {
                theta = acos(fmax(-1.0, cth));
            }
            double cs = tl_ / (nT * nL);
            cs = fmin(1.0, fmax(-1.0, cs));
            sigma = acos(cs);
            if (sin(sigma) < 1e-14) {
                dg = 1;
            } else {
                x = tan(theta) / tan(sigma) - 1.0;   // App. B
            }
        }
        // Eq. (ppt): Lambda~ = Lambda' + x (Lambda' - |Lambda'| cos(sigma) T'/|T'|)
        //          = (1 + x) Lambda' - x (T'.Lambda' / |T'|^2) T'
        xs = dg ? 0.0 : x;
        cterm = (nT > 0.0) ? tl_ / tt : 0.0;
        out[0] = trr;                         // tr rho before
        out[1] = n2 > 0.0 ? n2 / (trr * trr) : 0.0;  // xi before
        out[2] = theta;
        out[3] = feas;
        out[4] = dg;
        out[5] = xs;
        out[6] = red[5][0];                   // max |Im T'_j Lambda'_j|
        out[7] = ll;                          // |Lambda'|^2
        out[8] = red[3][0];                   // T'.Lambda' (tr after plain cut)
        out[9] = red[4][0];
        scale_all = 1.0;
    }
    __syncthreads();
    // renormalisation of the trace (optional): multiply by tr_before / (T'.Lambda~)
    if (renorm) {
        // T'.Lambda~ = T'.Lambda' (Eq. (ppt) keeps the T' component)
        if (tid == 0) {
            const double tpl = red[3][0];
            scale_all = (tpl != 0.0) ? sc[0] / tpl : 1.0;
        }
        __syncthreads();
    }
    double s_lt = 0.0, s_tlt = 0.0;
    for (int j = tid; j < k; j += blockDim.x) {
        const double ar = tl[2 * j], ai = tl[2 * j + 1], br = tr[2 * j], bi = tr[2 * j + 1];
        const double pr = ar * br - ai * bi;
        const double l = sig[j];
        const double Tj = l > 0.0 ? pr / l : 0.0;
        const double lt = ((1.0 + xs) * l - xs * cterm * Tj) * scale_all;
        fac[j] = l > 0.0 ? lt / l : 1.0;
        s_lt += lt * lt;
        s_tlt += Tj * lt;
    }
    red[0][tid] = s_lt;
    red[1][tid] = s_tlt;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            red[0][tid] += red[0][tid + s];
            red[1][tid] += red[1][tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        out[10] = red[1][0];                                       // tr after
        out[11] = red[1][0] != 0.0 ? red[0][0] / (red[1][0] * red[1][0]) : 0.0;  // xi after
        out[12] = red[0][0];                                       // |Lambda~|^2
    }
}

template <typename T>
__global__ void scale_rows_kernel(T* __restrict__ B, int k, int ncol, long ld, const double* __restrict__ f) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)k * ncol) return;
    const int j = (int)(idx / ncol), c = (int)(idx - (idx / ncol) * ncol);
    const long off = 2 * ((long)j * ld + c);
    B[off] = (T)((double)B[off] * f[j]);
    B[off + 1] = (T)((double)B[off + 1] * f[j]);
}

__global__ void zero_doubles_kernel(double* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// y[j] = sum_a x[a] M[a, j] (unconjugated), FP64 accumulation; one block per output j.
template <typename T>
__global__ __launch_bounds__(256) void gemv_left_kernel(CView<T> M, int a, int n, const double* __restrict__ x,
                                                        double* __restrict__ y) {
    __shared__ double pr[256], pi[256];
    const int j = blockIdx.x;
    double sr = 0.0, si = 0.0;
    for (int i = threadIdx.x; i < a; i += blockDim.x) {
        const long off = 2 * ((long)i * M.rs + (long)j * M.cs);
        const double mr = (double)M.p[off];
        const double mi = M.conj ? -(double)M.p[off + 1] : (double)M.p[off + 1];
        const double xr = x[2 * i], xi = x[2 * i + 1];
        sr += xr * mr - xi * mi;
        si += xr * mi + xi * mr;
    }
    pr[threadIdx.x] = sr;
    pi[threadIdx.x] = si;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            pr[threadIdx.x] += pr[threadIdx.x + s];
            pi[threadIdx.x] += pi[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        y[2 * j] = pr[0];
        y[2 * j + 1] = pi[0];
    }
}

// out[j] = ||X[j, :]||_2 for the k x ncol view X, FP64 accumulation; one block per row.
template <typename T>
__global__ __launch_bounds__(256) void row_norms_kernel(CView<T> X, int ncol, double* __restrict__ out) {
    __shared__ double part[256];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
        const long off = 2 * ((long)j * X.rs + (long)c * X.cs);
        const double r = (double)X.p[off], i = (double)X.p[off + 1];
        acc += r * r + i * i;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = sqrt(part[0]);
}

// out[0..1] = sum_a x[a] y[a] (unconjugated complex dot), FP64
__global__ void dot_kernel(const double* __restrict__ x, const double* __restrict__ y, int n,
                           double* __restrict__ out) {
    __shared__ double pr[256], pi[256];
    double sr = 0.0, si = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double xr = x[2 * i], xi = x[2 * i + 1], yr = y[2 * i], yi = y[2 * i + 1];
        sr += xr * yr - xi * yi;
        si += xr * yi + xi * yr;
    }
    pr[threadIdx.x] = sr;
    pi[threadIdx.x] = si;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            pr[threadIdx.x] += pr[threadIdx.x + s];
            pi[threadIdx.x] += pi[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = pr[0];
        out[1] = pi[0];
    }
}

// L[a][b] = x[a] x[b] (complex, no conjugation: both factors are the same vec(rho)), n x n
template <typename T>
__global__ void outer_kernel(const double* __restrict__ x, int n, T* __restrict__ L) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * n) return;
    const int a = (int)(idx / n), b = (int)(idx - (idx / n) * n);
    const double ar = x[2 * a], ai = x[2 * a + 1], br = x[2 * b], bi = x[2 * b + 1];
    L[2 * idx] = (T)(ar * br - ai * bi);
    L[2 * idx + 1] = (T)(ar * bi + ai * br);
}

// out = sum_{a,b} y[a] L[a][b] y[b] (complex, FP64 accumulation), one block
template <typename T>
__global__ void bilinear_kernel(const T* __restrict__ L, int n, const double* __restrict__ y,
                                double* __restrict__ out) {
    __shared__ double pr[256], pi[256];
    double sr = 0.0, si = 0.0;
    for (long idx = threadIdx.x; idx < (long)n * n; idx += blockDim.x) {
        const int a = (int)(idx / n), b = (int)(idx - (idx / n) * n);
        const double lr = (double)L[2 * idx], li = (double)L[2 * idx + 1];
        const double yr = y[2 * a] * y[2 * b] - y[2 * a + 1] * y[2 * b + 1];
        const double yi = y[2 * a] * y[2 * b + 1] + y[2 * a + 1] * y[2 * b];
        sr += lr * yr - li * yi;
        si += lr * yi + li * yr;
    }
    pr[threadIdx.x] = sr;
    pi[threadIdx.x] = si;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            pr[threadIdx.x] += pr[threadIdx.x + s];
            pi[threadIdx.x] += pi[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = pr[0];
        out[1] = pi[0];
    }
}

inline unsigned blocks_for(long n, int bs = 256) {
    long b = (n + bs - 1) / bs;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

template <typename TX, typename TY>
hipError_t geam(hipStream_t s, int M, int N, cd alpha, CView<TX> X, cd beta, CView<TY> Y) {
    if (M <= 0 || N <= 0) return hipSuccess;
    hipLaunchKernelGGL((geam_kernel<TX, TY>), dim3(blocks_for((long)M * N)), dim3(256), 0, s, M, N, alpha.re,
                       alpha.im, X, beta.re, beta.im, Y);
    return hipGetLastError();
}

template <typename T>
hipError_t phys_left(hipStream_t s, const T* A, int cl, int D2, int cm, const double* X, int r, T* out) {
    const long total = (long)cl * D2 * r * cm;
    if (total <= 0) return hipSuccess;
    unsigned nb = blocks_for(total);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(phys_left_kernel<T>, dim3(nb), dim3(256), (size_t)r * D2 * D2 * 2 * sizeof(double), s, A,
                       cl, D2, cm, X, r, out);
    return hipGetLastError();
}

template <typename T>
hipError_t phys_right(hipStream_t s, const T* B, int cm, int D2, int cr, const double* Y, int r, T* out) {
    const long total = (long)r * cm * D2 * cr;
    if (total <= 0) return hipSuccess;
    unsigned nb = blocks_for(total);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(phys_right_kernel<T>, dim3(nb), dim3(256), (size_t)r * D2 * D2 * 2 * sizeof(double), s, B,
                       cm, D2, cr, Y, r, out);
    return hipGetLastError();
}

template <typename T>
hipError_t transfer_left(hipStream_t s, const T* A, int cl, int D2, int cr, const double* x, const double* o,
                         double* y) {
    hipLaunchKernelGGL(transfer_left_kernel<T>, dim3((cr + 63) / 64), dim3(256), 0, s, A, cl, D2, cr, x, o, y);
    return hipGetLastError();
}

template <typename T>
hipError_t transfer_right(hipStream_t s, const T* A, int cl, int D2, int cr, const double* x, const double* o,
                          double* y) {
    hipLaunchKernelGGL(transfer_right_kernel<T>, dim3((cl + 3) / 4), dim3(256), 0, s, A, cl, D2, cr, x, o, y);
    return hipGetLastError();
}

hipError_t kron_vec(hipStream_t s, const double* x, int na, const double* z, int nb, double* v) {
    hipLaunchKernelGGL(kron_kernel, dim3(blocks_for((long)na * nb)), dim3(256), 0, s, x, na, z, nb, v);
    return hipGetLastError();
}

template <typename T>
hipError_t sumsq(hipStream_t s, CView<T> X, int M, int N, double* out2, double* part, unsigned* cnt) {
    unsigned nb = blocks_for((long)M * N);
    if (nb > SUMSQ_MAX_BLOCKS) nb = SUMSQ_MAX_BLOCKS;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(sumsq_kernel<T>, dim3(nb), dim3(256), 0, s, X, M, N, out2, part, cnt);
    return hipGetLastError();
}

hipError_t spectrum_cut(hipStream_t s, const double* lam, int n, int level, double floor2, double noise, double tau,
                        int cap, double* st, int* cnt, double* sig, double* inv) {
    hipLaunchKernelGGL(spectrum_cut_kernel, dim3(1), dim3(256), 0, s, lam, n, level, floor2, noise, tau, cap, st,
                       cnt, sig, inv);
    return hipGetLastError();
}

template <typename T>
hipError_t class_expand(hipStream_t s, const T* X, int cl, int D2, int cr, int mode, int ncls, const EtaClass& cls,
                        T* Y) {
    if (D2 > EtaClass::MAXD2 || mode < 0 || mode > 3 || ncls < 1) return hipErrorInvalidValue;
    const long tot = (long)ncls * cl * D2 * cr;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(class_expand_kernel<T>, dim3(blocks_for(tot)), dim3(256), 0, s, X, cl, D2, cr, mode, ncls, cls, Y);
    return hipGetLastError();
}

template <typename T>
hipError_t fill_random(hipStream_t s, CView<T> X, int M, int N, uint64_t seed) {
    if (M <= 0 || N <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_random_kernel<T>, dim3(blocks_for((long)M * N)), dim3(256), 0, s, X, M, N, seed);
    return hipGetLastError();
}

template <typename T>
hipError_t scale_cols(hipStream_t s, CView<T> X, int M, int N, const double* f) {
    if (M <= 0 || N <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_cols_kernel<T>, dim3(blocks_for((long)M * N)), dim3(256), 0, s, X, M, N, f);
    return hipGetLastError();
}

hipError_t ppt(hipStream_t s, const double* sig, const double* tl, const double* tr, const double* sc, int k,
               int use_ppt, int renorm, double* fac, double* out) {
    hipLaunchKernelGGL(ppt_kernel, dim3(1), dim3(256), 0, s, sig, tl, tr, sc, k, use_ppt, renorm, fac, out);
    return hipGetLastError();
}

template <typename T>
hipError_t scale_rows(hipStream_t s, T* B, int k, int ncol, long ld, const double* f) {
    if (k <= 0 || ncol <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_rows_kernel<T>, dim3(blocks_for((long)k * ncol)), dim3(256), 0, s, B, k, ncol, ld, f);
    return hipGetLastError();
}

hipError_t zero_doubles(hipStream_t s, double* p, int n) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_doubles_kernel, dim3(blocks_for(n)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

template <typename T>
hipError_t gemv_left(hipStream_t s, CView<T> M, int a, int n, const double* x, double* y) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gemv_left_kernel<T>, dim3(n), dim3(256), 0, s, M, a, n, x, y);
    return hipGetLastError();
}

template <typename T>
hipError_t row_norms(hipStream_t s, CView<T> X, int k, int ncol, double* out) {
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(row_norms_kernel<T>, dim3(k), dim3(256), 0, s, X, ncol, out);
    return hipGetLastError();
}

hipError_t dot(hipStream_t s, const double* x, const double* y, int n, double* out) {
    hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(256), 0, s, x, y, n, out);
    return hipGetLastError();
}

template <typename T>
hipError_t outer(hipStream_t s, const double* x, int n, T* L) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(outer_kernel<T>, dim3(blocks_for((long)n * n)), dim3(256), 0, s, x, n, L);
    return hipGetLastError();
}

template <typename T>
hipError_t bilinear(hipStream_t s, const T* L, int n, const double* y, double* out) {
    hipLaunchKernelGGL(bilinear_kernel<T>, dim3(1), dim3(256), 0, s, L, n, y, out);
    return hipGetLastError();
}

#define MPDO_INST_T(T)                                                                                          \
    template hipError_t phys_left<T>(hipStream_t, const T*, int, int, int, const double*, int, T*);             \
    template hipError_t phys_right<T>(hipStream_t, const T*, int, int, int, const double*, int, T*);            \
    template hipError_t transfer_left<T>(hipStream_t, const T*, int, int, int, const double*, const double*,    \
                                         double*);                                                              \
    template hipError_t transfer_right<T>(hipStream_t, const T*, int, int, int, const double*, const double*,   \
                                          double*);                                                             \
    template hipError_t sumsq<T>(hipStream_t, CView<T>, int, int, double*, double*, unsigned*);                \
    template hipError_t outer<T>(hipStream_t, const double*, int, T*);                                          \
    template hipError_t bilinear<T>(hipStream_t, const T*, int, const double*, double*);                         \
    template hipError_t scale_cols<T>(hipStream_t, CView<T>, int, int, const double*);                          \
    template hipError_t fill_random<T>(hipStream_t, CView<T>, int, int, uint64_t);                               \
    template hipError_t class_expand<T>(hipStream_t, const T*, int, int, int, int, int, const EtaClass&, T*);     \
    template hipError_t scale_rows<T>(hipStream_t, T*, int, int, long, const double*);                          \
    template hipError_t gemv_left<T>(hipStream_t, CView<T>, int, int, const double*, double*);                  \
    template hipError_t row_norms<T>(hipStream_t, CView<T>, int, int, double*);

MPDO_INST_T(double)
MPDO_INST_T(float)

template hipError_t geam<double, double>(hipStream_t, int, int, cd, CView<double>, cd, CView<double>);
template hipError_t geam<float, float>(hipStream_t, int, int, cd, CView<float>, cd, CView<float>);
template hipError_t geam<float, double>(hipStream_t, int, int, cd, CView<float>, cd, CView<double>);
template hipError_t geam<double, float>(hipStream_t, int, int, cd, CView<double>, cd, CView<float>);

}  // namespace mpdo
