// Complex GEMM on CDNA4 matrix cores (gfx950), FP64, FP32 and FP32 data by split-BF16 products.
//
//   C = alpha * op(A) * op(B) + beta * C
//
// op(A), op(B) and C are strided complex views (CView): transposes and conjugates are
// expressed in the view, so theta, Gram products, projections and rebuilds all run through
// this one kernel without materialising permuted copies.
//
// Complex products use four real MFMA products per k-step (re*re - im*im, re*im + im*re);
// counted as 8 real flop per complex multiply-add, the same as the algorithm.
// Block tile 64 x 64 or 32 x 32, k-step 32, 256 threads = 4 waves of 64 lanes; each wave owns
// a quadrant of 2 x 2 or 1 x 1 MFMA 16x16 tiles.  Tiles of A and B are staged through LDS as
// separate real and imaginary planes; the global loader walks the contiguous dimension of
// each view so loads coalesce whichever way the view is laid out.  Large-k products with a
// small output (Gram matrices of tall factors) split k over blockIdx.z when the caller lends
// a workspace: every k-chunk writes its partial tile there and a second launch adds the
// partials in chunk order, so a product gives the same bits on every run (no atomics).
//
// One FP64 16x16x4 MFMA occupies a SIMD for 64 cycles (78.6 TFLOP/s over 1024 SIMDs), so a
// workgroup needs 64 WM^2 cycles per unit of k on its compute unit: the small products of an
// update (outputs of a few 64 x 64 tiles) are bound by how many compute units they reach.
// The launcher picks the tile size and the k split from that cost (plan_of).
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <unordered_map>

#include "common.h"
#include "gemm.h"

namespace mpdo {

namespace {

constexpr int BK = 32;

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct Acc;
template <>
struct Acc<double> {
    typedef v4d v;
};
template <>
struct Acc<float> {
    typedef v4f v;
};

// Output row of accumulator register r in lane group lk (= lane / 16) of a 16x16 tile:
// the FP64 instruction interleaves rows (lk + 4 r), the FP32 one blocks them (4 lk + r).
__device__ __forceinline__ int acc_row(double, int lk, int r) { return lk + 4 * r; }
__device__ __forceinline__ int acc_row(float, int lk, int r) { return 4 * lk + r; }

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T>
struct GemmArgs {
    int M, N, K;
    int ksplit;        // number of k-chunks over blockIdx.z (>= 1)
    int kchunk;        // k extent of one chunk (multiple of BK)
    int batch;
    CView<T> A, B, C;
    long sA, sB, sC;   // batch strides in complex elements
    double ar, ai, br, bi;
    T* part;           // non-null: write alpha*AB of k-chunk kc and batch b to part (dense
                       // M x N per (kc, b), beta ignored); the reduce launch forms C
    int bshift;        // 1: op(B) is replaced by bsc op(B) + bdg I as it is loaded
    double bsc, bdg;
    const double* bcol;   // non-null: column n of op(B) is scaled by bcol[n] as it is loaded
};

template <typename T>
__device__ __forceinline__ void load_cplx(const T* p, long off, int conj, T& re, T& im) {
    re = p[2 * off];
    im = p[2 * off + 1];
    if (conj) im = -im;
}

// WM: MFMA tiles per wave along each output dimension; block tile (32 WM) x (32 WM).
// TF: 1 if B's operand transforms (bshift, bcol) may be set; the plain kernel keeps the
// registers they need free (the FP64 64 x 64 kernel stays within two waves per SIMD).
// LDS row padding.  A 16x16x4 MFMA step reads A[16 rows][4 k] and B[4 k][16 columns]; the
// first 32 lanes cover 16 rows (columns) at 2 k.  FP64 elements take two 4-byte banks and the
// +1 padding already spreads them; for FP32 a row stride of 2 (mod 32) words puts the A reads
// on 32 distinct banks and a stride of 16 (mod 32) does the same for B (measured: about two
// conflict cycles per LDS instruction with +1 padding in FP32, none in FP64).
template <typename T>
constexpr int PAD_A = std::is_same<T, float>::value ? 2 : 1;

template <typename T, int BN>
constexpr int PAD_B = std::is_same<T, float>::value ? 16 : 1;

template <typename T, int WM, int TF>
__global__ __launch_bounds__(256) void cgemm_kernel(GemmArgs<T> g) {
    constexpr int BM = 32 * WM, BN = 32 * WM, WQ = 16 * WM;
    __shared__ T sAr[BM][BK + PAD_A<T>];
    __shared__ T sAi[BM][BK + PAD_A<T>];
    __shared__ T sBr[BK][BN + PAD_B<T, BN>];
    __shared__ T sBi[BK][BN + PAD_B<T, BN>];
    __shared__ double sbf[BN];   // column factors of B (b_col)

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1;
    const int wc = wave & 1;
    // Logical tile of this workgroup.  Workgroups are handed to the eight XCDs in turn
    // (linear id w to XCD w mod 8), each XCD with its own L2; mapping the w of one XCD onto a
    // contiguous run of tiles (x fastest, then y, then batch) lets the workgroups that share
    // A row panels and B column panels meet in the same L2.
    const unsigned nx = gridDim.x, ny = gridDim.y;
    const unsigned nw = nx * ny * gridDim.z;
    const unsigned w = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
    const unsigned per = nw / 8, rem = nw % 8, xcd = w % 8;
    const unsigned t = xcd * per + (xcd < rem ? xcd : rem) + w / 8;
    const int m0 = (int)((t / nx) % ny) * BM;
    const int n0 = (int)(t % nx) * BN;
    const int bz = (int)(t / (nx * ny));
    const int b = bz / g.ksplit;
    const int kc = bz - b * g.ksplit;
    const int kbeg = kc * g.kchunk;
    const int kend = min(g.K, kbeg + g.kchunk);

    const T* Ap = g.A.p + 2 * (long)b * g.sA;
    const T* Bp = g.B.p + 2 * (long)b * g.sB;
    T* Cp = g.C.p + 2 * (long)b * g.sC;

    typename Acc<T>::v cr[WM][WM], ci[WM][WM];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WM; ++j) {
            cr[i][j] = (typename Acc<T>::v){0, 0, 0, 0};
            ci[i][j] = (typename Acc<T>::v){0, 0, 0, 0};
        }

    const bool a_kfast = (g.A.cs == 1);
    const bool b_nfast = (g.B.cs == 1);
    const int li = lane & 15;
    const int lk = lane >> 4;

    // The next k-tile is loaded into registers while the current one is multiplied from LDS.
    constexpr int PA = (BM * BK) / 256, PB = (BN * BK) / 256;
    T par[PA], pai[PA], pbr[PB], pbi[PB];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int j = 0; j < PA; ++j) {
            const int e = tid + 256 * j;
            const int m = a_kfast ? e / BK : e % BM, k = a_kfast ? e % BK : e / BM;
            const int gm = m0 + m, gk = k0 + k;
            par[j] = 0;
            pai[j] = 0;
            if (gm < g.M && gk < kend) load_cplx(Ap, (long)gm * g.A.rs + (long)gk * g.A.cs, g.A.conj, par[j], pai[j]);
        }
#pragma unroll
        for (int j = 0; j < PB; ++j) {
            const int e = tid + 256 * j;
            const int n = b_nfast ? e % BN : e / BK, k = b_nfast ? e / BN : e % BK;
            const int gn = n0 + n, gk = k0 + k;
            pbr[j] = 0;
            pbi[j] = 0;
            if (gn < g.N && gk < kend) load_cplx(Bp, (long)gk * g.B.rs + (long)gn * g.B.cs, g.B.conj, pbr[j], pbi[j]);
        }
    };
    // operand transforms of B are applied when a tile is staged (the loaded values are waited
    // for there anyway); the column factors do not depend on k and are read once into LDS
    const bool btf = TF && (g.bshift || g.bcol);
    if (TF && g.bcol) {
        for (int i = tid; i < BN; i += 256) sbf[i] = n0 + i < g.N ? g.bcol[n0 + i] : 1.0;
        __syncthreads();
    }
    if (kbeg < kend) fetch(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        // ---- stage the fetched A tile (BM x BK) and B tile (BK x BN) in LDS
#pragma unroll
        for (int j = 0; j < PA; ++j) {
            const int e = tid + 256 * j;
            const int m = a_kfast ? e / BK : e % BM, k = a_kfast ? e % BK : e / BM;
            sAr[m][k] = par[j];
            sAi[m][k] = pai[j];
        }
#pragma unroll
        for (int j = 0; j < PB; ++j) {
            const int e = tid + 256 * j;
            const int n = b_nfast ? e % BN : e / BK, k = b_nfast ? e / BN : e % BK;
            T br = pbr[j], bi = pbi[j];
            if (btf) {
                // (bsc B + bdg I) diag(bcol); entries outside the product stay zero
                const int gn = n0 + n, gk = k0 + k;
                const double dg = (g.bshift && gk == gn && gn < g.N && gk < kend) ? g.bdg : 0.0;
                const double f = g.bcol ? sbf[n] : 1.0;
                br = (T)((dg + g.bsc * (double)br) * f);
                bi = (T)(g.bsc * (double)bi * f);
            }
            sBr[k][n] = br;
            sBi[k][n] = bi;
        }
        __syncthreads();
        if (k0 + BK < kend) fetch(k0 + BK);
        // unrolled by two: a full unroll hoists all eight k-steps' operands into registers and
        // leaves one wave per SIMD (308 registers); by two the FP64 kernel fits two waves
#pragma unroll 2
        for (int kk = 0; kk < BK; kk += 4) {
            T ar[WM], ai[WM], nai[WM], br[WM], bi[WM];
#pragma unroll
            for (int i = 0; i < WM; ++i) {
                ar[i] = sAr[wr * WQ + i * 16 + li][kk + lk];
                ai[i] = sAi[wr * WQ + i * 16 + li][kk + lk];
                nai[i] = -ai[i];
            }
#pragma unroll
            for (int j = 0; j < WM; ++j) {
                br[j] = sBr[kk + lk][wc * WQ + j * 16 + li];
                bi[j] = sBi[kk + lk][wc * WQ + j * 16 + li];
            }
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WM; ++j) {
                    cr[i][j] = mfma16(ar[i], br[j], cr[i][j]);
                    cr[i][j] = mfma16(nai[i], bi[j], cr[i][j]);
                    ci[i][j] = mfma16(ar[i], bi[j], ci[i][j]);
                    ci[i][j] = mfma16(ai[i], br[j], ci[i][j]);
                }
        }
        __syncthreads();
    }

    // ---- epilogue: lane holds column lane%16 and rows acc_row(lane/16, r) of each tile
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WM; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wr * WQ + i * 16 + acc_row(T(0), lk, r);
                const int gn = n0 + wc * WQ + j * 16 + li;
                if (gm >= g.M || gn >= g.N) continue;
                const double xr = (double)cr[i][j][r], xi = (double)ci[i][j][r];
                const double vr = g.ar * xr - g.ai * xi;
                const double vi = g.ar * xi + g.ai * xr;
                if (g.part) {
                    T* pp = g.part + 2 * (((long)kc * g.batch + b) * g.M * (long)g.N + (long)gm * g.N + gn);
                    pp[0] = (T)vr;
                    pp[1] = (T)vi;
                } else {
                    const long off = 2 * ((long)gm * g.C.rs + (long)gn * g.C.cs);
                    double or_ = 0.0, oi = 0.0;
                    if (g.br != 0.0 || g.bi != 0.0) {
                        const double cr0 = (double)Cp[off];
                        const double ci0 = g.C.conj ? -(double)Cp[off + 1] : (double)Cp[off + 1];
                        or_ = g.br * cr0 - g.bi * ci0;
                        oi = g.br * ci0 + g.bi * cr0;
                    }
                    const double wr_ = vr + or_;
                    const double wi_ = vi + oi;
                    Cp[off] = (T)wr_;
                    Cp[off + 1] = (T)(g.C.conj ? -wi_ : wi_);
                }
            }
}

// ------------------------------------------------------------ split-BF16 products of FP32 data
// Each FP32 operand x is written as hi + lo with hi = bf16(x) and lo = bf16(x - hi) (x - hi is
// exact in FP32; both roundings to nearest even, by the packed hardware conversion), so
// x - hi - lo is below 2^-18 |x|.  A real product a b is then a_hi b_hi + a_hi b_lo + a_lo b_hi
// (the dropped a_lo b_lo is below 2^-18 |a b|), three BF16 matrix-core products with FP32
// accumulation: 16x16x32 MFMAs, one k-step of 32 per tile.  The complex product takes the
// four real products of the FP32 kernel, twelve MFMAs per 16x16 output tile and k-step (the
// negated imaginary part of A by a sign-bit flip, which is exact).
//
// A k-step costs a wave 12 x 16 cycles of matrix core per 16x16 tile, a sixth of the FP32
// kernel's, so the operand traffic and the conversion must be spread over more output: the
// workgroup tile is 128 x 128 (each wave 64 x 64, 4 x 4 MFMA tiles, accumulators in AGPRs),
// i.e. 3072 matrix-core cycles per SIMD and k-step against 32 KB of operands per workgroup.
// Every thread loads 16 complex values of A and 16 of B per k-step at offsets fixed for the
// whole product (one 64-bit base per operand and a constant stride between its 16 values), so
// the next k-step's loads cost one add.  LDS holds hi and lo planes of the real and imaginary
// parts, k contiguous (rows of 40 BF16, 16-byte aligned), so a lane reads the eight k values
// of its row (column) with one 16-byte load; the 16 lanes of a row group then touch 64
// distinct banks.  The same lane-to-k assignment is used for A and B, so the sum over k pairs
// matching terms whatever order the instruction adds them.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef unsigned short v8us __attribute__((ext_vector_type(8)));
constexpr int XK = 32;    // k-step of the split-BF16 kernel
constexpr int XPAD = 8;   // LDS row padding in BF16 elements (rows stay 16-byte aligned)
constexpr int XT = 128;   // workgroup tile (rows of A, columns of B)
constexpr int XL = (XT * XK) / 256;   // complex values of each operand per thread and k-step

// (hi, lo) of x packed as two BF16 (hi in the low half)
__device__ __forceinline__ unsigned split_bf16(float x) {
    const __bf16 h = (__bf16)x;
    const v2bf p = {h, (__bf16)(x - (float)h)};
    return __builtin_bit_cast(unsigned, p);
}

__device__ __forceinline__ v4f mfma_bf16(v8us a, v8us b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0,
                                                   0);
}

// Per-thread load pattern of one operand tile (TILE rows (A) or columns (B) by XK k): value j
// (0 <= j < TILE XK / 256) sits at row r0 + j dr and k k0 + j dk of the tile; `kfast` says
// whether k is the contiguous dimension of the view (then 32 consecutive threads read 32
// consecutive k of a row), else rows are (then TILE consecutive threads read TILE consecutive
// rows).
struct XPat {
    int r0, dr, k0, dk;
};
template <int TILE = XT>
__device__ __forceinline__ XPat xpat(int tid, bool kfast) {
    return kfast ? XPat{tid / XK, 256 / XK, tid % XK, 0} : XPat{tid % TILE, 0, tid / TILE, 256 / TILE};
}

__global__ __launch_bounds__(256) void cgemm_x3_kernel(GemmArgs<float> g) {
    constexpr int WM = 4, WQ = 16 * WM;
    // planes: 0 re hi, 1 re lo, 2 im hi, 3 im lo; [row of A or column of B][k]
    __shared__ __attribute__((aligned(16))) unsigned short sA[4][XT][XK + XPAD];
    __shared__ __attribute__((aligned(16))) unsigned short sB[4][XT][XK + XPAD];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1;
    const int wc = wave & 1;
    // the XCD-aware tile order of cgemm_kernel
    const unsigned nx = gridDim.x, ny = gridDim.y;
    const unsigned nw = nx * ny * gridDim.z;
    const unsigned w = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
    const unsigned per = nw / 8, rem = nw % 8, xcd = w % 8;
    const unsigned t = xcd * per + (xcd < rem ? xcd : rem) + w / 8;
    const int m0 = (int)((t / nx) % ny) * XT;
    const int n0 = (int)(t % nx) * XT;
    const int bz = (int)(t / (nx * ny));
    const int b = bz / g.ksplit;
    const int kc = bz - b * g.ksplit;
    const int kbeg = kc * g.kchunk;
    const int kend = min(g.K, kbeg + g.kchunk);

    // A value (m, k) at A.p + 2 (m rs + k cs); B value (k, n) at B.p + 2 (k rs + n cs)
    const XPat pa = xpat(tid, g.A.cs == 1), pb = xpat(tid, g.B.rs == 1);
    const float* Ab = g.A.p + 2 * ((long)b * g.sA + (long)(m0 + pa.r0) * g.A.rs + (long)pa.k0 * g.A.cs);
    const long Aj = 2 * ((long)pa.dr * g.A.rs + (long)pa.dk * g.A.cs), Ak = 2 * (long)g.A.cs;
    const float* Bb = g.B.p + 2 * ((long)b * g.sB + (long)(n0 + pb.r0) * g.B.cs + (long)pb.k0 * g.B.rs);
    const long Bj = 2 * ((long)pb.dr * g.B.cs + (long)pb.dk * g.B.rs), Bk = 2 * (long)g.B.rs;
    const float sa = g.A.conj ? -1.0f : 1.0f, sb = g.B.conj ? -1.0f : 1.0f;
    float* Cp = g.C.p + 2 * (long)b * g.sC;

    v4f cr[WM][WM], ci[WM][WM];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WM; ++j) {
            cr[i][j] = (v4f){0, 0, 0, 0};
            ci[i][j] = (v4f){0, 0, 0, 0};
        }

    const int li = lane & 15;
    const int lk = lane >> 4;

    float2 va[XL], vb[XL];
    auto fetch = [&](int k0) {
        const float* ap = Ab + (long)k0 * Ak;
        const float* bp = Bb + (long)k0 * Bk;
#pragma unroll
        for (int j = 0; j < XL; ++j) {
            va[j] = make_float2(0.0f, 0.0f);
            if (m0 + pa.r0 + j * pa.dr < g.M && k0 + pa.k0 + j * pa.dk < kend)
                va[j] = *(const float2*)(ap + j * Aj);
        }
#pragma unroll
        for (int j = 0; j < XL; ++j) {
            vb[j] = make_float2(0.0f, 0.0f);
            if (n0 + pb.r0 + j * pb.dr < g.N && k0 + pb.k0 + j * pb.dk < kend)
                vb[j] = *(const float2*)(bp + j * Bj);
        }
    };
    if (kbeg < kend) fetch(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += XK) {
#pragma unroll
        for (int j = 0; j < XL; ++j) {
            const int r = pa.r0 + j * pa.dr, k = pa.k0 + j * pa.dk;
            const unsigned re = split_bf16(va[j].x), im = split_bf16(sa * va[j].y);
            sA[0][r][k] = (unsigned short)re;
            sA[1][r][k] = (unsigned short)(re >> 16);
            sA[2][r][k] = (unsigned short)im;
            sA[3][r][k] = (unsigned short)(im >> 16);
        }
#pragma unroll
        for (int j = 0; j < XL; ++j) {
            const int r = pb.r0 + j * pb.dr, k = pb.k0 + j * pb.dk;
            const unsigned re = split_bf16(vb[j].x), im = split_bf16(sb * vb[j].y);
            sB[0][r][k] = (unsigned short)re;
            sB[1][r][k] = (unsigned short)(re >> 16);
            sB[2][r][k] = (unsigned short)im;
            sB[3][r][k] = (unsigned short)(im >> 16);
        }
        __syncthreads();
        if (k0 + XK < kend) fetch(k0 + XK);
        v8us bb[WM][4];
#pragma unroll
        for (int j = 0; j < WM; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) bb[j][q] = *(const v8us*)&sB[q][wc * WQ + j * 16 + li][8 * lk];
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            v8us a[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] = *(const v8us*)&sA[q][wr * WQ + i * 16 + li][8 * lk];
            const v8us nih = a[2] ^ (unsigned short)0x8000, nil = a[3] ^ (unsigned short)0x8000;
#pragma unroll
            for (int j = 0; j < WM; ++j) {
                // the small terms first
                cr[i][j] = mfma_bf16(a[1], bb[j][0], cr[i][j]);
                cr[i][j] = mfma_bf16(a[0], bb[j][1], cr[i][j]);
                cr[i][j] = mfma_bf16(nil, bb[j][2], cr[i][j]);
                cr[i][j] = mfma_bf16(nih, bb[j][3], cr[i][j]);
                cr[i][j] = mfma_bf16(a[0], bb[j][0], cr[i][j]);
                cr[i][j] = mfma_bf16(nih, bb[j][2], cr[i][j]);
                ci[i][j] = mfma_bf16(a[1], bb[j][2], ci[i][j]);
                ci[i][j] = mfma_bf16(a[0], bb[j][3], ci[i][j]);
                ci[i][j] = mfma_bf16(a[3], bb[j][0], ci[i][j]);
                ci[i][j] = mfma_bf16(a[2], bb[j][1], ci[i][j]);
                ci[i][j] = mfma_bf16(a[0], bb[j][2], ci[i][j]);
                ci[i][j] = mfma_bf16(a[2], bb[j][0], ci[i][j]);
            }
        }
        __syncthreads();
    }

    // epilogue as in cgemm_kernel (FP32 accumulator layout: rows 4 (lane / 16) + r)
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WM; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wr * WQ + i * 16 + 4 * lk + r;
                const int gn = n0 + wc * WQ + j * 16 + li;
                if (gm >= g.M || gn >= g.N) continue;
                const double xr = (double)cr[i][j][r], xi = (double)ci[i][j][r];
                const double vr = g.ar * xr - g.ai * xi;
                const double vi = g.ar * xi + g.ai * xr;
                if (g.part) {
                    float* pp = g.part + 2 * (((long)kc * g.batch + b) * g.M * (long)g.N + (long)gm * g.N + gn);
                    pp[0] = (float)vr;
                    pp[1] = (float)vi;
                } else {
                    const long off = 2 * ((long)gm * g.C.rs + (long)gn * g.C.cs);
                    double or_ = 0.0, oi = 0.0;
                    if (g.br != 0.0 || g.bi != 0.0) {
                        const double cr0 = (double)Cp[off];
                        const double ci0 = g.C.conj ? -(double)Cp[off + 1] : (double)Cp[off + 1];
                        or_ = g.br * cr0 - g.bi * ci0;
                        oi = g.br * ci0 + g.bi * cr0;
                    }
                    const double wr_ = vr + or_;
                    const double wi_ = vi + oi;
                    Cp[off] = (float)wr_;
                    Cp[off + 1] = (float)(g.C.conj ? -wi_ : wi_);
                }
            }
}

// FP32 products of large outputs: the 128 x 128 workgroup tile and the load pattern of the
// split-BF16 kernel, with the FP32 16x16x4 MFMA (four real products per complex k-step).  A
// k-tile of 32 then costs each SIMD 16 tiles x 8 steps x 4 MFMAs x 32 cycles of matrix core,
// against 32 KB of operands per workgroup and one LDS staging, which the 64 x 64 kernel pays
// for a quarter of the work.  LDS planes [row of A or column of B][k] with rows of 34 floats:
// the 32 lanes that a 16x16x4 read serves at once (16 rows at 2 k) land on 32 distinct banks.
constexpr int FPAD = 2;
__global__ __launch_bounds__(256) void cgemm_f32_big_kernel(GemmArgs<float> g) {
    constexpr int WM = 4, WQ = 16 * WM;
    __shared__ float sAr[XT][XK + FPAD], sAi[XT][XK + FPAD];
    __shared__ float sBr[XT][XK + FPAD], sBi[XT][XK + FPAD];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1;
    const int wc = wave & 1;
    const unsigned nx = gridDim.x, ny = gridDim.y;
    const unsigned nw = nx * ny * gridDim.z;
    const unsigned w = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
    const unsigned per = nw / 8, rem = nw % 8, xcd = w % 8;
    const unsigned t = xcd * per + (xcd < rem ? xcd : rem) + w / 8;
    const int m0 = (int)((t / nx) % ny) * XT;
    const int n0 = (int)(t % nx) * XT;
    const int bz = (int)(t / (nx * ny));
    const int b = bz / g.ksplit;
    const int kc = bz - b * g.ksplit;
    const int kbeg = kc * g.kchunk;
    const int kend = min(g.K, kbeg + g.kchunk);

    const XPat pa = xpat(tid, g.A.cs == 1), pb = xpat(tid, g.B.rs == 1);
    const float* Ab = g.A.p + 2 * ((long)b * g.sA + (long)(m0 + pa.r0) * g.A.rs + (long)pa.k0 * g.A.cs);
    const long Aj = 2 * ((long)pa.dr * g.A.rs + (long)pa.dk * g.A.cs), Ak = 2 * (long)g.A.cs;
    const float* Bb = g.B.p + 2 * ((long)b * g.sB + (long)(n0 + pb.r0) * g.B.cs + (long)pb.k0 * g.B.rs);
    const long Bj = 2 * ((long)pb.dr * g.B.cs + (long)pb.dk * g.B.rs), Bk = 2 * (long)g.B.rs;
    const float sa = g.A.conj ? -1.0f : 1.0f, sb = g.B.conj ? -1.0f : 1.0f;
    float* Cp = g.C.p + 2 * (long)b * g.sC;

    v4f cr[WM][WM], ci[WM][WM];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WM; ++j) {
            cr[i][j] = (v4f){0, 0, 0, 0};
            ci[i][j] = (v4f){0, 0, 0, 0};
        }
    const int li = lane & 15;
    const int lk = lane >> 4;

    float2 va[XL], vb[XL];
    auto fetch = [&](int k0) {
        const float* ap = Ab + (long)k0 * Ak;
        const float* bp = Bb + (long)k0 * Bk;
#pragma unroll
        for (int j = 0; j < XL; ++j) {
            va[j] = make_float2(0.0f, 0.0f);
            if (m0 + pa.r0 + j * pa.dr < g.M && k0 + pa.k0 + j * pa.dk < kend)
                va[j] = *(const float2*)(ap + j * Aj);
        }
#pragma unroll
        for (int j = 0; j < XL; ++j) {
            vb[j] = make_float2(0.0f, 0.0f);
            if (n0 + pb.r0 + j * pb.dr < g.N && k0 + pb.k0 + j * pb.dk < kend)
                vb[j] = *(const float2*)(bp + j * Bj);
        }
    };
    if (kbeg < kend) fetch(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += XK) {
#pragma unroll
        for (int j = 0; j < XL; ++j) {
            const int r = pa.r0 + j * pa.dr, k = pa.k0 + j * pa.dk;
            sAr[r][k] = va[j].x;
            sAi[r][k] = sa * va[j].y;
        }
#pragma unroll
        for (int j = 0; j < XL; ++j) {
            const int r = pb.r0 + j * pb.dr, k = pb.k0 + j * pb.dk;
            sBr[r][k] = vb[j].x;
            sBi[r][k] = sb * vb[j].y;
        }
        __syncthreads();
        if (k0 + XK < kend) fetch(k0 + XK);
#pragma unroll 2
        for (int kk = 0; kk < XK; kk += 4) {
            float br[WM], bi[WM];
#pragma unroll
            for (int j = 0; j < WM; ++j) {
                br[j] = sBr[wc * WQ + j * 16 + li][kk + lk];
                bi[j] = sBi[wc * WQ + j * 16 + li][kk + lk];
            }
#pragma unroll
            for (int i = 0; i < WM; ++i) {
                const float ar = sAr[wr * WQ + i * 16 + li][kk + lk];
                const float ai = sAi[wr * WQ + i * 16 + li][kk + lk];
                const float nai = -ai;
#pragma unroll
                for (int j = 0; j < WM; ++j) {
                    cr[i][j] = mfma16(ar, br[j], cr[i][j]);
                    cr[i][j] = mfma16(nai, bi[j], cr[i][j]);
                    ci[i][j] = mfma16(ar, bi[j], ci[i][j]);
                    ci[i][j] = mfma16(ai, br[j], ci[i][j]);
                }
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WM; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wr * WQ + i * 16 + 4 * lk + r;
                const int gn = n0 + wc * WQ + j * 16 + li;
                if (gm >= g.M || gn >= g.N) continue;
                const double xr = (double)cr[i][j][r], xi = (double)ci[i][j][r];
                const double vr = g.ar * xr - g.ai * xi;
                const double vi = g.ar * xi + g.ai * xr;
                if (g.part) {
                    float* pp = g.part + 2 * (((long)kc * g.batch + b) * g.M * (long)g.N + (long)gm * g.N + gn);
                    pp[0] = (float)vr;
                    pp[1] = (float)vi;
                } else {
                    const long off = 2 * ((long)gm * g.C.rs + (long)gn * g.C.cs);
                    double or_ = 0.0, oi = 0.0;
                    if (g.br != 0.0 || g.bi != 0.0) {
                        const double cr0 = (double)Cp[off];
                        const double ci0 = g.C.conj ? -(double)Cp[off + 1] : (double)Cp[off + 1];
                        or_ = g.br * cr0 - g.bi * ci0;
                        oi = g.br * ci0 + g.bi * cr0;
                    }
                    const double wr_ = vr + or_;
                    const double wi_ = vi + oi;
                    Cp[off] = (float)wr_;
                    Cp[off + 1] = (float)(g.C.conj ? -wi_ : wi_);
                }
            }
}

// FP64 products of large outputs: 128 x 64 workgroup tiles (each wave 64 x 32: 4 x 2 MFMA
// 16x16x4 FP64 tiles, whose accumulators fill 128 AGPRs; a square 64 x 64 wave tile would
// need all 256), the load pattern of the FP32 kernel above.  A k-tile of 32 then costs each
// SIMD 8 tiles x 8 steps x 4 MFMAs x 64 cycles, twice the 64 x 64 kernel's, against 1.5 times
// its operands.  LDS rows of 33 doubles.
constexpr int DM = 128, DN = 64;
__global__ __launch_bounds__(256) void cgemm_f64_big_kernel(GemmArgs<double> g) {
    constexpr int TM = 4, TN = 2, WQM = 16 * TM, WQN = 16 * TN;
    constexpr int LA = DM * XK / 256, LB = DN * XK / 256;
    __shared__ double sAr[DM][XK + 1], sAi[DM][XK + 1];
    __shared__ double sBr[DN][XK + 1], sBi[DN][XK + 1];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1;
    const int wc = wave & 1;
    const unsigned nx = gridDim.x, ny = gridDim.y;
    const unsigned nw = nx * ny * gridDim.z;
    const unsigned w = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
    const unsigned per = nw / 8, rem = nw % 8, xcd = w % 8;
    const unsigned t = xcd * per + (xcd < rem ? xcd : rem) + w / 8;
    const int m0 = (int)((t / nx) % ny) * DM;
    const int n0 = (int)(t % nx) * DN;
    const int bz = (int)(t / (nx * ny));
    const int b = bz / g.ksplit;
    const int kc = bz - b * g.ksplit;
    const int kbeg = kc * g.kchunk;
    const int kend = min(g.K, kbeg + g.kchunk);

    const XPat pa = xpat<DM>(tid, g.A.cs == 1), pb = xpat<DN>(tid, g.B.rs == 1);
    const double* Ab = g.A.p + 2 * ((long)b * g.sA + (long)(m0 + pa.r0) * g.A.rs + (long)pa.k0 * g.A.cs);
    const long Aj = 2 * ((long)pa.dr * g.A.rs + (long)pa.dk * g.A.cs), Ak = 2 * (long)g.A.cs;
    const double* Bb = g.B.p + 2 * ((long)b * g.sB + (long)(n0 + pb.r0) * g.B.cs + (long)pb.k0 * g.B.rs);
    const long Bj = 2 * ((long)pb.dr * g.B.cs + (long)pb.dk * g.B.rs), Bk = 2 * (long)g.B.rs;
    const double sa = g.A.conj ? -1.0 : 1.0, sb = g.B.conj ? -1.0 : 1.0;
    double* Cp = g.C.p + 2 * (long)b * g.sC;

    v4d cr[TM][TN], ci[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            cr[i][j] = (v4d){0, 0, 0, 0};
            ci[i][j] = (v4d){0, 0, 0, 0};
        }
    const int li = lane & 15;
    const int lk = lane >> 4;

    double2 va[LA], vb[LB];
    auto fetch = [&](int k0) {
        const double* ap = Ab + (long)k0 * Ak;
        const double* bp = Bb + (long)k0 * Bk;
#pragma unroll
        for (int j = 0; j < LA; ++j) {
            va[j] = make_double2(0.0, 0.0);
            if (m0 + pa.r0 + j * pa.dr < g.M && k0 + pa.k0 + j * pa.dk < kend)
                va[j] = *(const double2*)(ap + j * Aj);
        }
#pragma unroll
        for (int j = 0; j < LB; ++j) {
            vb[j] = make_double2(0.0, 0.0);
            if (n0 + pb.r0 + j * pb.dr < g.N && k0 + pb.k0 + j * pb.dk < kend)
                vb[j] = *(const double2*)(bp + j * Bj);
        }
    };
    if (kbeg < kend) fetch(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += XK) {
#pragma unroll
        for (int j = 0; j < LA; ++j) {
            const int r = pa.r0 + j * pa.dr, k = pa.k0 + j * pa.dk;
            sAr[r][k] = va[j].x;
            sAi[r][k] = sa * va[j].y;
        }
#pragma unroll
        for (int j = 0; j < LB; ++j) {
            const int r = pb.r0 + j * pb.dr, k = pb.k0 + j * pb.dk;
            sBr[r][k] = vb[j].x;
            sBi[r][k] = sb * vb[j].y;
        }
        __syncthreads();
        if (k0 + XK < kend) fetch(k0 + XK);
#pragma unroll 2
        for (int kk = 0; kk < XK; kk += 4) {
            double br[TN], bi[TN];
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                br[j] = sBr[wc * WQN + j * 16 + li][kk + lk];
                bi[j] = sBi[wc * WQN + j * 16 + li][kk + lk];
            }
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const double ar = sAr[wr * WQM + i * 16 + li][kk + lk];
                const double ai = sAi[wr * WQM + i * 16 + li][kk + lk];
                const double nai = -ai;
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    cr[i][j] = mfma16(ar, br[j], cr[i][j]);
                    cr[i][j] = mfma16(nai, bi[j], cr[i][j]);
                    ci[i][j] = mfma16(ar, bi[j], ci[i][j]);
                    ci[i][j] = mfma16(ai, br[j], ci[i][j]);
                }
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wr * WQM + i * 16 + acc_row(0.0, lk, r);
                const int gn = n0 + wc * WQN + j * 16 + li;
                if (gm >= g.M || gn >= g.N) continue;
                const double xr = cr[i][j][r], xi = ci[i][j][r];
                const double vr = g.ar * xr - g.ai * xi;
                const double vi = g.ar * xi + g.ai * xr;
                if (g.part) {
                    double* pp = g.part + 2 * (((long)kc * g.batch + b) * g.M * (long)g.N + (long)gm * g.N + gn);
                    pp[0] = vr;
                    pp[1] = vi;
                } else {
                    const long off = 2 * ((long)gm * g.C.rs + (long)gn * g.C.cs);
                    double or_ = 0.0, oi = 0.0;
                    if (g.br != 0.0 || g.bi != 0.0) {
                        const double cr0 = Cp[off];
                        const double ci0 = g.C.conj ? -Cp[off + 1] : Cp[off + 1];
                        or_ = g.br * cr0 - g.bi * ci0;
                        oi = g.br * ci0 + g.bi * cr0;
                    }
                    const double wr_ = vr + or_;
                    const double wi_ = vi + oi;
                    Cp[off] = wr_;
                    Cp[off + 1] = g.C.conj ? -wi_ : wi_;
                }
            }
}

// C = beta C + sum over the ks k-chunks of the partial products, added in chunk order (FP64
// sums), one thread per output element of every batch.
template <typename T>
__global__ void csplit_reduce_kernel(const T* __restrict__ part, int ks, int batch, int M, int N, CView<T> C,
                                     long sC, double br, double bi) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long mn = (long)M * N;
    if (idx >= mn * batch) return;
    const int b = (int)(idx / mn);
    const long e = idx - (long)b * mn;
    const int m = (int)(e / N), n = (int)(e - (long)(e / N) * N);
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < ks; ++k) {
        const T* pp = part + 2 * (((long)k * batch + b) * mn + e);
        sr += (double)pp[0];
        si += (double)pp[1];
    }
    T* Cp = C.p + 2 * (long)b * sC;
    const long off = 2 * ((long)m * C.rs + (long)n * C.cs);
    if (br != 0.0 || bi != 0.0) {
        const double cr = (double)Cp[off];
        const double ci = C.conj ? -(double)Cp[off + 1] : (double)Cp[off + 1];
        sr += br * cr - bi * ci;
        si += br * ci + bi * cr;
    }
    Cp[off] = (T)sr;
    Cp[off + 1] = (T)(C.conj ? -si : si);
}

template <typename T>
size_t split_bytes(int M, int N, int batch, int ks) {
    return (size_t)ks * batch * (size_t)M * N * 2 * sizeof(T);
}

// Launch plan: block tile wm = 4 (128 x 128; FP64 128 x 64), 2 (64 x 64) or 1 (32 x 32), and the
// k range split ks ways.
struct Plan {
    int wm, ks;
};

// Workgroup tile of a plan: (32 wm) x (32 wm), except FP64 wm = 4: 128 x 64.
void tile_dims(bool fp64, int wm, int& bm, int& bn) {
    bm = 32 * wm;
    bn = (fp64 && wm == 4) ? 64 : 32 * wm;
}

int tiles_of(int M, int N, int batch, int wm, bool fp64 = false) {
    int bm, bn;
    tile_dims(fp64, wm, bm, bn);
    return ((M + bm - 1) / bm) * ((N + bn - 1) / bn) * batch;
}

// k extent of one chunk when the k range is split about ks ways (a multiple of BK)
int chunk_of(int K, int ks) { return (((K + ks - 1) / ks + BK - 1) / BK) * BK; }

// Estimated time (us) of a plan.  Matrix-core time: a workgroup spends 64 wm^2 cycles (FP64;
// 32 for FP32) per unit of k on its compute unit, and the workgroups run in rounds of 256, one
// per compute unit (a unit that holds two shares its matrix cores between them).  Operand
// traffic: every workgroup reads a (32 wm) x chunk tile of A and of B, at ~16 TB/s from L2
// and the memory-side cache, counted at a quarter weight (it mostly overlaps the matrix work;
// it decides between plans of equal matrix time).  A split adds its partial tiles, written and
// read back by the reduce launch (~4 TB/s), and ~5 us of fixed cost; every launch ~2 us.
// The split-BF16 kernel (x3) spends 12 MFMAs of 16 cycles per 16x16 tile and k-step of 32.
// Launch plan: block tile (32 wm)^2.
double plan_cost(int M, int N, int K, int batch, bool fp64, Plan p, bool x3 = false) {
    const double tsz = fp64 ? 8.0 : 4.0;
    int bm, bn;
    tile_dims(fp64, p.wm, bm, bn);
    const double W = (double)tiles_of(M, N, batch, p.wm, fp64) * p.ks;
    const int chunk = p.ks > 1 ? chunk_of(K, p.ks) : K;
    // per unit of k a 16x16 tile costs 64 (FP64), 32 (FP32) or 6 (split-BF16) cycles, but a
    // k-step of 32 takes at least the k-loop's own latency (the next tile's loads, the LDS
    // round trip, two barriers), about 2048 cycles: the matrix work of a 32 x 32 FP64 tile.
    // FP32 32 x 32 tiles are bound by it (measured per launch on the M3 products: slower than
    // FP64's when planned at half the cost), the larger tiles by their matrix work.
    const double cyc = std::max((x3 ? 6.0 : fp64 ? 64.0 : 32.0) * (bm / 32) * (bn / 32), 64.0) * chunk;
    const double mfma_us = std::ceil(W / 256.0) * cyc / 2400.0;
    const double bytes = W * chunk * (double)(bm + bn) * 2.0 * tsz;
    const double part_us = p.ks > 1 ? 2.0 * W * (double)bm * bn * 2.0 * tsz / 4e6 : 0.0;
    return mfma_us + 0.25 * bytes / 16e6 + part_us + 2.0 + (p.ks > 1 ? 5.0 : 0.0);
}

// wm_max = 1 restricts the plan to 32 x 32 tiles (the kernel with operand transforms needs
// more registers than two waves per SIMD allow at 64 x 64)
// x3: the split-BF16 kernel (128 x 128 tile, wm = 4)
Plan plan_of(int M, int N, int K, int batch, bool fp64, int wm_max = 2, int ks_max = 64, bool x3 = false) {
    if (x3) wm_max = 4;   // the split-BF16 kernel has only the 128 x 128 tile
    else if (wm_max == 2) wm_max = 4;   // plain products may take the large tile too
    Plan best{wm_max, 1};
    double best_t = plan_cost(M, N, K, batch, fp64, best, x3);
    for (int wm = wm_max; wm >= (x3 ? 4 : 1); wm /= 2)   // tiles of 128, 64, 32
        for (int ks = 1; ks <= ks_max; ks *= 2) {
            if (ks > 1 && K < 2 * BK) break;
            const int k_eff = ks > 1 ? (K + chunk_of(K, ks) - 1) / chunk_of(K, ks) : 1;
            if (ks > 1 && k_eff < 2) continue;
            const Plan p{wm, k_eff};
            const double t = plan_cost(M, N, K, batch, fp64, p, x3);
            if (t < 0.97 * best_t) {
                best = p;
                best_t = t;
            }
        }
    return best;
}

// One product with the plan's tile size and k split (ks = 1: no split).
template <typename T>
hipError_t cgemm_launch(hipStream_t s, int M, int N, int K, cd alpha, CView<T> A, CView<T> B, cd beta, CView<T> C,
                        int batch, long sA, long sB, long sC, Plan plan, ProfSink* prof,
                        const GemmOpts& opt = GemmOpts()) {
    GemmArgs<T> g;
    g.M = M;
    g.N = N;
    g.K = K < 0 ? 0 : K;
    g.batch = batch;
    g.A = A;
    g.B = B;
    g.C = C;
    g.sA = sA;
    g.sB = sB;
    g.sC = sC;
    g.ar = alpha.re;
    g.ai = alpha.im;
    g.br = beta.re;
    g.bi = beta.im;
    g.part = nullptr;
    g.bshift = (opt.b_scale != 1.0 || opt.b_diag != 0.0) ? 1 : 0;
    g.bsc = opt.b_scale;
    g.bdg = opt.b_diag;
    g.bcol = opt.b_col;
    g.ksplit = 1;
    g.kchunk = ((g.K + BK - 1) / BK) * BK;
    if (g.kchunk == 0) g.kchunk = BK;
    int ks = plan.ks;
    if (ks >= 2) {
        const int chunk = chunk_of(g.K, ks);
        ks = (g.K + chunk - 1) / chunk;
        // the partials need ks M N complex per batch in the caller's workspace; without room the
        // product runs unsplit (the same result, computed by fewer workgroups)
        if (ks >= 2 && split_bytes<T>(M, N, batch, ks) <= opt.ws_bytes && opt.ws) {
            g.ksplit = ks;
            g.kchunk = chunk;
            g.part = (T*)opt.ws;
        }
    }
    int bm, bn;
    tile_dims(std::is_same<T, double>::value, plan.wm, bm, bn);
    dim3 grid((N + bn - 1) / bn, (M + bm - 1) / bm, batch * g.ksplit);   // plan.wm = 4: the large tile
    if (getenv("MPDO_DEBUG_GEMM"))
        fprintf(stderr, "[mpdo gemm] %s M %d N %d K %d batch %d tile %dx%d ksplit %d chunk %d%s\n",
                sizeof(T) == 8 ? "f64" : (opt.split_bf16 ? "bf16x3" : "f32"), M, N, K, batch, bm, bn, g.ksplit, g.kchunk,
                g.bshift || g.bcol ? " transforms" : "");
    // With a profiling sink the kernel is launched with an event pair attached to it
    // (hipExtLaunchKernelGGL stamps the kernel's own start and end), so the recorded time is
    // kernel execution alone, as for the k-split sums that follow.
    hipEvent_t ka = nullptr, kb = nullptr;
    const bool timed = prof && prof->kernel_events(PF_GEMM, &ka, &kb);
#define MPDO_GEMM_GO(K)                                                                 \
    do {                                                                                \
        if (timed)                                                                      \
            hipExtLaunchKernelGGL(K, grid, dim3(256), 0, s, ka, kb, 0u, g);              \
        else                                                                            \
            hipLaunchKernelGGL(K, grid, dim3(256), 0, s, g);                            \
    } while (0)
    const bool tf = g.bshift || g.bcol;
    bool big = false;   // the large-tile kernels (plan.wm = 4, plain operands)
    if constexpr (std::is_same<T, float>::value) {
        big = !tf && plan.wm == 4;
        if (big && opt.split_bf16) MPDO_GEMM_GO(cgemm_x3_kernel);
        else if (big) MPDO_GEMM_GO(cgemm_f32_big_kernel);
    } else {
        big = !tf && plan.wm == 4;
        if (big) MPDO_GEMM_GO(cgemm_f64_big_kernel);
    }
    if (big) {
    } else if (plan.wm == 2) {
        if (tf)
            MPDO_GEMM_GO((cgemm_kernel<T, 2, 1>));
        else
            MPDO_GEMM_GO((cgemm_kernel<T, 2, 0>));
    } else {
        if (tf)
            MPDO_GEMM_GO((cgemm_kernel<T, 1, 1>));
        else
            MPDO_GEMM_GO((cgemm_kernel<T, 1, 0>));
    }
#undef MPDO_GEMM_GO
    // algorithmic: 8 flop per complex multiply-add; A, B read and C written once (and read
    // when beta != 0)
    const double flop = 8.0 * M * (double)N * K * batch;
    const double bytes = 2.0 * sizeof(T) * batch *
                         ((double)M * K + (double)K * N + (double)M * N * ((beta.re != 0 || beta.im != 0) ? 2 : 1));
    if (timed) prof->kernel_done(PF_GEMM, ka, kb, flop, bytes);
    if (g.part) {
        const long tot = (long)M * N * batch;
        const dim3 rg((unsigned)((tot + 255) / 256));
        hipEvent_t ra = nullptr, rb = nullptr;
        if (prof && prof->kernel_events(PF_SPLIT_SUM, &ra, &rb)) {
            hipExtLaunchKernelGGL(csplit_reduce_kernel<T>, rg, dim3(256), 0, s, ra, rb, 0u, (const T*)g.part, g.ksplit,
                                  batch, M, N, C, sC, beta.re, beta.im);
            // the partials read once, C written (and read when beta != 0)
            prof->kernel_done(PF_SPLIT_SUM, ra, rb, 2.0 * tot * g.ksplit,
                              2.0 * sizeof(T) * tot * (g.ksplit + ((beta.re != 0 || beta.im != 0) ? 2 : 1)));
        } else {
            hipLaunchKernelGGL(csplit_reduce_kernel<T>, rg, dim3(256), 0, s, (const T*)g.part, g.ksplit, batch, M, N, C,
                               sC, beta.re, beta.im);
        }
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- autotuner of the plan
// Shapes are bucketed by the powers of two of M, N, K, the batch and the precision.  With
// tuning on (environment MPDO_GEMM_AUTOTUNE=1), the first product of a bucket with beta = 0
// (the output then does not depend on its old contents) is run with each candidate plan on
// its stream between HIP events, the fastest is cached for the bucket, and the product is run
// once more with it; later products of the bucket use the cached plan.  With tuning off, or
// with beta != 0, the cost model above decides.  The cache is shared by all threads.
struct TuneKey {
    int m, n, k, batch, fp64;
    bool operator==(const TuneKey& o) const {
        return m == o.m && n == o.n && k == o.k && batch == o.batch && fp64 == o.fp64;
    }
};
struct TuneHash {
    size_t operator()(const TuneKey& t) const {
        return (((size_t)t.m * 131 + t.n) * 131 + t.k) * 131 + (size_t)t.batch * 2 + t.fp64;
    }
};
std::mutex g_tune_mutex;
std::unordered_map<TuneKey, Plan, TuneHash> g_tune;

int log2_bucket(long x) {
    int b = 0;
    while ((1L << b) < x) ++b;
    return b;
}

bool autotune_on() {
    const char* e = getenv("MPDO_GEMM_AUTOTUNE");
    return e && atoi(e) != 0;
}

template <typename T>
Plan tune_plan(hipStream_t s, int M, int N, int K, cd alpha, CView<T> A, CView<T> B, cd beta, CView<T> C,
               int batch, long sA, long sB, long sC, const GemmOpts& opt, int ks_max) {
    const bool fp64 = std::is_same<T, double>::value;
    const TuneKey key{log2_bucket(M), log2_bucket(N), log2_bucket(K), log2_bucket(batch), fp64 ? 1 : 0};
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) return it->second;
    }
    const Plan h = plan_of(M, N, K, batch, fp64, 2, ks_max);
    Plan cands[24];
    int nc = 0;
    cands[nc++] = h;
    for (int wm = 4; wm >= 1; wm /= 2)
        for (int ks = 1; ks <= ks_max && nc < 24; ks *= 2) {
            if (ks > 1 && ks > K / 64) break;
            if (!(wm == h.wm && ks == h.ks)) cands[nc++] = Plan{wm, ks};
        }
    Plan best = h;
    float best_ms = 1e30f;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return h;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return h;
    }
    for (int i = 0; i < nc; ++i) {
        // one untimed run, then one timed
        if (cgemm_launch<T>(s, M, N, K, alpha, A, B, beta, C, batch, sA, sB, sC, cands[i], nullptr, opt) != hipSuccess)
            continue;
        (void)hipEventRecord(e0, s);
        (void)cgemm_launch<T>(s, M, N, K, alpha, A, B, beta, C, batch, sA, sB, sC, cands[i], nullptr, opt);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) continue;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < best_ms) {
            best_ms = ms;
            best = cands[i];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    g_tune[key] = best;
    return best;
}

}  // namespace

template <typename T>
hipError_t cgemm_ex(hipStream_t s, int M, int N, int K, cd alpha, CView<T> A, CView<T> B, cd beta, CView<T> C,
                    const GemmOpts& opt, ProfSink* prof, int batch, long sA, long sB, long sC) {
    if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
    const int k = K < 0 ? 0 : K;
    const bool plain = opt.b_scale == 1.0 && opt.b_diag == 0.0 && !opt.b_col;
    // the largest k split whose partials fit the workspace
    int ks_max = 1;
    while (ks_max < 64 && opt.ws && split_bytes<T>(M, N, batch, 2 * ks_max) <= opt.ws_bytes) ks_max *= 2;
    const bool x3 = std::is_same<T, float>::value && opt.split_bf16 && plain;
    Plan plan = plan_of(M, N, k, batch, std::is_same<T, double>::value, plain ? 2 : 1, ks_max, x3);
    if (plain && !x3 && autotune_on() && beta.re == 0.0 && beta.im == 0.0 && K >= 128)
        plan = tune_plan<T>(s, M, N, k, alpha, A, B, beta, C, batch, sA, sB, sC, opt, ks_max);
    return cgemm_launch<T>(s, M, N, k, alpha, A, B, beta, C, batch, sA, sB, sC, plan, prof, opt);
}

template <typename T>
hipError_t cgemm(hipStream_t s, int M, int N, int K, cd alpha, CView<T> A, CView<T> B, cd beta,
                 CView<T> C, int batch, long sA, long sB, long sC, ProfSink* prof) {
    return cgemm_ex<T>(s, M, N, K, alpha, A, B, beta, C, GemmOpts(), prof, batch, sA, sB, sC);
}

int gemm_tuned_buckets() {
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    return (int)g_tune.size();
}

template hipError_t cgemm<double>(hipStream_t, int, int, int, cd, CView<double>, CView<double>, cd,
                                  CView<double>, int, long, long, long, ProfSink*);
template hipError_t cgemm<float>(hipStream_t, int, int, int, cd, CView<float>, CView<float>, cd,
                                 CView<float>, int, long, long, long, ProfSink*);
template hipError_t cgemm_ex<double>(hipStream_t, int, int, int, cd, CView<double>, CView<double>, cd,
                                     CView<double>, const GemmOpts&, ProfSink*, int, long, long, long);
template hipError_t cgemm_ex<float>(hipStream_t, int, int, int, cd, CView<float>, CView<float>, cd, CView<float>,
                                    const GemmOpts&, ProfSink*, int, long, long, long);

}  // namespace mpdo
