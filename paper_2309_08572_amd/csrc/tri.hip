// Hermitian eigensolver for Gram matrices of order up to TRI_MAX in FP64 (gfx950), restricted to
// the eigenpairs one deflation level of the split accepts.
//
//   tri_reduce_*       Householder reduction H = Q T Q^H to a real symmetric
//                      tridiagonal T (complex reflectors chosen so the off-diagonal is real);
//                      the reflectors are copied to contiguous rows for the back-transform
//   tri_top_kernel     one wave: the largest eigenvalue by multisection of Sturm counts, the
//                      level's threshold and the number m of accepted eigenvalues
//   tri_eval_kernel    one wave per accepted eigenvalue: multisection (64 shifts per pass)
//   tri_vec_kernel     one wave per accepted eigenvalue: inverse iteration on T, factors in LDS
//   tri_mgs_kernel     modified Gram-Schmidt inside clusters of eigenvalues closer than
//                      1e-12 ||T|| (one wave per cluster)
//   tri_back_kernel    independent workgroups of 8 columns: V = Q Z for the m vectors
//
// Grids are sized for the cap on the host and exit early past the accepted count, which lives
// on the device, so the launches need no host synchronisation.
#include <float.h>
#include <math.h>

#include "common.h"
#include "tri.h"

namespace mpdo {

namespace {

constexpr int TB = 1024;      // threads of the one-workgroup kernels
constexpr int NW = TB / 64;   // waves
constexpr int BK_COLS = 4;    // columns per back-transform workgroup (LDS: (BK_COLS + 1) x 16 TRI_MAX + 64 KB)
constexpr int BK_THREADS = 256;
constexpr int BK_LANES = BK_THREADS / BK_COLS;   // lanes per column (one wave)
static_assert(BK_LANES == 64, "one wave per back-transform column");
constexpr double EPS = 2.220446049250313e-16;

// x from another lane of the same row of 16 (DPP; every source lane is in the row, so with all
// lanes active no lane keeps the placeholder 0)
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Reductions over the 64 lanes of a wave (all lanes active), returned to every lane.  Inside
// each row of 16 lanes: quad swaps (xor 1, xor 2), then the half-row mirror (lane i with 7 - i)
// and the row mirror (i with 15 - i), register moves with no LDS round trip; then two
// cross-row shuffles.  Each step combines the same two values in either order, so every lane
// ends with the same bits.
template <class Op>
__device__ __forceinline__ double wave_reduce(double x, Op op) {
    x = op(x, dpp_mov<0xB1>(x));    // quad_perm [1,0,3,2]
    x = op(x, dpp_mov<0x4E>(x));    // quad_perm [2,3,0,1]
    x = op(x, dpp_mov<0x141>(x));   // row_half_mirror
    x = op(x, dpp_mov<0x140>(x));   // row_mirror
    x = op(x, __shfl_xor(x, 16, 64));
    x = op(x, __shfl_xor(x, 32, 64));
    return x;
}
struct SumOp {
    __device__ double operator()(double a, double b) const { return a + b; }
};
struct MaxOp {
    __device__ double operator()(double a, double b) const { return fmax(a, b); }
};
struct MinOp {
    __device__ double operator()(double a, double b) const { return fmin(a, b); }
};
__device__ __forceinline__ double wave_sum(double x) { return wave_reduce(x, SumOp()); }
__device__ __forceinline__ double wave_max(double x) { return wave_reduce(x, MaxOp()); }
__device__ __forceinline__ double wave_min(double x) { return wave_reduce(x, MinOp()); }

// sums of a and b over a workgroup of NWV waves, returned to every thread (red: 2 * NWV doubles)
template <int NWV = NW>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        red[2 * w] = a;
        red[2 * w + 1] = b;
    }
    __syncthreads();
    double sa = 0.0, sb = 0.0;
    for (int k = 0; k < NWV; ++k) {
        sa += red[2 * k];
        sb += red[2 * k + 1];
    }
    __syncthreads();
    a = sa;
    b = sb;
}

// max of a and min of b over the workgroup
__device__ __forceinline__ void block_maxmin(double& a, double& b, double* red) {
    a = wave_max(a);
    b = wave_min(b);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        red[2 * w] = a;
        red[2 * w + 1] = b;
    }
    __syncthreads();
    double sa = red[0], sb = red[1];
    for (int k = 1; k < NW; ++k) {
        sa = fmax(sa, red[2 * k]);
        sb = fmin(sb, red[2 * k + 1]);
    }
    __syncthreads();
    a = sa;
    b = sb;
}

// ------------------------------------------------------------------ reduction, orders > RMAX
// H (n x n complex, row-major, leading dimension ld) is overwritten.  Outputs: dg[0..n) and
// off[0..n-1) (T), tau[j] (complex) and refl row j = v_j (length n-1-j, v_j[0] = 1) of
// H_j = I - tau_j v_j v_j^H acting on rows j+1..n-1, so that H = H_0 ... H_{n-2} T (...)^H;
// trace[0] = sum of the diagonal of H.
//
// The trailing matrix does not fit on chip above RMAX, and one workgroup streaming it through
// L2 once per column is bound by that one compute unit.  So each column is a launch over many
// workgroups (tri_col_kernel below), the rows of the trailing matrix split between their waves
// (ROWS_PER_WAVE rows at a time).
constexpr int RW = 256;                 // threads of the multi-workgroup reduction kernels
constexpr int RWV = RW / 64;
constexpr int ROWS_PER_WAVE = 1;
constexpr int COL_CHUNK = 12;           // columns per lane whose loads tri_col_kernel issues together
constexpr int MAX_RGROUPS = 256;

int reduce_groups(int m) {
    const int g = (m + RWV * ROWS_PER_WAVE - 1) / (RWV * ROWS_PER_WAVE);
    return g < 1 ? 1 : (g > MAX_RGROUPS ? MAX_RGROUPS : g);
}

// Hermitian part (average of the two triangles, real diagonal), rows spread over the grid
__global__ __launch_bounds__(RW) void tri_herm_kernel(double* __restrict__ H, int ld, int n) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int x = blockIdx.x * RWV + w; x < n; x += gridDim.x * RWV)
        for (int y = x + lane; y < n; y += 64) {
            double* a = H + 2 * ((long)x * ld + y);
            if (y == x) {
                a[1] = 0.0;
                continue;
            }
            double* b = H + 2 * ((long)y * ld + x);
            const double r = 0.5 * (a[0] + b[0]), im = 0.5 * (a[1] - b[1]);
            a[0] = r;
            a[1] = im;
            b[0] = r;
            b[1] = -im;
        }
}

__global__ __launch_bounds__(RW) void tri_trace_kernel(const double* __restrict__ H, int ld, int n,
                                                       double* __restrict__ trace) {
    __shared__ double red[2 * RWV];
    double tr = 0.0, unused = 0.0;
    for (int i = threadIdx.x; i < n; i += RW) tr += H[2 * ((long)i * ld + i)];
    block_sum2<RWV>(tr, unused, red);
    if (threadIdx.x == 0) trace[0] = tr;
}


// 1/q from the hardware reciprocal and one Newton step (the Sturm count tolerates a last-bit
// difference from IEEE division; |q| >= pivmin keeps q normal)
__device__ __forceinline__ double rcp_nr(double q) {
    double r = __builtin_amdgcn_rcp(q);
    const double e = fma(-q, r, 1.0);
    return fma(r, e, r);
}
// 1/q to a few ulp (two Newton steps) for 1e-290 <= |q| <= 1e290; outside that range the
// hardware estimate can overflow or flush, and callers divide instead (pivot_rcp)
__device__ __forceinline__ double rcp_nr2(double q) {
    double r = __builtin_amdgcn_rcp(q);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double e = fma(-q, r, 1.0);
        r = fma(r, e, r);
    }
    return r;
}

__device__ __forceinline__ double pivot_rcp(double q) {
    const double a = fabs(q);
    return (a >= 1e-290 && a <= 1e290) ? rcp_nr2(q) : 1.0 / q;
}

// On-chip reduction for orders <= RMAX.  The lower triangle is cut into 8 x 8 tiles (diagonal
// tiles stored in full); a group of 8 lanes owns RS tiles, lane k row k of each (8 complex
// values, slot q holding column q ^ k of the tile): RS_REG tiles in registers, the rest in
// LDS, so no matrix element leaves the chip until the reflectors are written.  v and w live in LDS at absolute indices with zeros over
// the reduced part, so the arithmetic needs no masks.  Per column one pass over the tiles:
// the previous column's rank-2 update in place, then the Hermitian matvec with the updated
// values (row sums in registers, column sums and row totals by LDS f64 atomics).
constexpr int RB = 512;        // threads: 2 waves per SIMD leave 256 registers per lane
constexpr int RNW = RB / 64;
constexpr int RT = 8;
constexpr int RG = RB / RT;    // 64 tile groups
constexpr int RS_REG = 3;      // tiles per group in registers
constexpr int RS_LDS = 2;      // tiles per group in LDS
constexpr int RS = RS_REG + RS_LDS;
constexpr int RMAX = 192;      // 24 tile rows: 300 lower tiles <= RG * RS = 320
static_assert((RMAX / RT) * (RMAX / RT + 1) / 2 <= RG * RS, "tiles of the largest order must fit");

struct RedLds {
    double tr[RS_LDS][RT][RB];   // LDS tiles, [slot][column][lane]
    double ti[RS_LDS][RT][RB];
    double vabs[2 * RMAX];       // column j below the diagonal, all earlier updates applied (absolute rows)
    double raw[2 * RMAX];        // column j + 1 as the tiles hold it during step j (update j not applied)
    double v[2][2 * RMAX];       // Householder vectors of columns j and j - 1 (by parity; absolute
                                 // rows, zero outside the block)
    double pabs[2 * RMAX];       // A22 v, accumulated by the tiles' atomics (cleared after use)
    double wv[2 * RMAX];         // w of the last rank-2 update
    double red[2 * RNW];         // per-wave partials of v^H A22 v (written before the matvec barrier)
    double red2[2 * RNW];        // per-wave partials of the next column's norm
};

// Per-wave partial of a workgroup sum into red[w]; after the next barrier collect() returns the
// sum to every thread.  red must not be written again before every thread has passed a later
// barrier.
__device__ __forceinline__ void publish(double a, double* red) {
    a = wave_sum(a);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
}
template <int NWV>
__device__ __forceinline__ double collect(const double* red) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NWV; ++q) s += red[q];
    return s;
}

__device__ __forceinline__ bool tile_live(int I, int J, int j) {
    return I >= 0 && RT * I + RT - 1 > j && RT * J + RT - 1 > j;
}

// column j of the tile row held by this lane -> vabs, and the diagonal entry -> dg[j]
template <class TileRow>
__device__ __forceinline__ void tile_extract(const TileRow& x, int I, int J, int j, int k, int n, double* vabs,
                                             double* dg, double& x2) {
    if (I < 0 || J != j / RT) return;
    const int r = RT * I + k, jq = (j - RT * (j / RT)) ^ k;   // the slot of column j
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int q = 0; q < RT; ++q)
        if (q == jq) {
            a = x.re(q);
            b = x.im(q);
        }
    if (r == j) dg[j] = a;
    if (r > j && r < n) {
        vabs[2 * r] = a;
        vabs[2 * r + 1] = b;
        if (r > j + 1) x2 += a * a + b * b;
    }
}

// Householder vector entry c of column j: 1 at j + 1, (sr + i si) x_c below it (x = column j in
// vabs), 0 above and past n
__device__ __forceinline__ void hh_entry(const double* vabs, int c, int j, int n, double sr, double si,
                                         double& vr, double& vi) {
    vr = 0.0;
    vi = 0.0;
    if (c == j + 1) {
        vr = 1.0;
    } else if (c > j + 1 && c < n) {
        const double xr = vabs[2 * c], xi = vabs[2 * c + 1];
        vr = xr * sr - xi * si;
        vi = xr * si + xi * sr;
    }
}

// p += A22 v over one tile.  Row sums of the tile row stay in the lane.  For an off-diagonal
// tile the lane also forms its row's share of every mirrored column, conj(A_rc) v_r, in the
// slot of that column, and the group of 8 lanes reduce-scatters the 8 column sums so that
// lane k ends with column 8J + k.  Because slot q of lane k holds column q ^ k, the partner
// k ^ m of an exchange holds the same column in slot q ^ m, so every lane sends the same
// registers: the half-row mirror (k <-> k ^ 7) adds slots 7..4 into 0..3, the quad
// permutations (k ^ 2, then k ^ 1) slots 2, 3 into 0, 1 and slot 1 into 0, which then holds
// column 0 ^ k = k.  14 double moves and no selects per tile.  Two atomics per lane per tile
// follow, none of them to the same address within a group.  This lane's share of v^H A22 v
// (real: A22 is Hermitian) goes to vav: conj(v_r) times the row sum, and for an off-diagonal
// tile conj(v_c) times the column sum the lane receives.  All 8 lanes of a group hold the
// same tile, so they are active together, as the moves need.
template <class TileRow>
__device__ __forceinline__ void tile_matvec(TileRow& x, int I, int J, int k, const double* v, double* pabs,
                                            double& vav) {
    __builtin_amdgcn_sched_barrier(0);   // keep one tile's operands live at a time
    const int r = RT * I + k;
    const double vrr = v[2 * r], vri = v[2 * r + 1];
    double rr = 0.0, ri = 0.0;
    double ar[RT], ai[RT];
#pragma unroll
    for (int q = 0; q < RT; ++q) {
        const int c = RT * J + (q ^ k);
        const double vcr = v[2 * c], vci = v[2 * c + 1];
        const double hr = x.re(q), hi = x.im(q);
        rr += hr * vcr - hi * vci;
        ri += hr * vci + hi * vcr;
        ar[q] = hr * vrr + hi * vri;   // conj(A_rc) v_r
        ai[q] = hr * vri - hi * vrr;
    }
    if (I != J) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ar[q] += dpp_mov<0x141>(ar[7 - q]);   // row_half_mirror: lane k ^ 7, slot q ^ 7
            ai[q] += dpp_mov<0x141>(ai[7 - q]);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            ar[q] += dpp_mov<0x4E>(ar[q + 2]);    // quad_perm [2,3,0,1]: lane k ^ 2, slot q ^ 2
            ai[q] += dpp_mov<0x4E>(ai[q + 2]);
        }
        ar[0] += dpp_mov<0xB1>(ar[1]);            // quad_perm [1,0,3,2]: lane k ^ 1, slot 1
        ai[0] += dpp_mov<0xB1>(ai[1]);
        const int c = RT * J + k;
        atomicAdd(&pabs[2 * c], ar[0]);
        atomicAdd(&pabs[2 * c + 1], ai[0]);
        vav += v[2 * c] * ar[0] + v[2 * c + 1] * ai[0];
    }
    atomicAdd(&pabs[2 * r], rr);
    atomicAdd(&pabs[2 * r + 1], ri);
    vav += vrr * rr + vri * ri;
    __builtin_amdgcn_sched_barrier(0);
}

// A -= v w^H + w v^H on this lane's tile row
template <class TileRow>
__device__ __forceinline__ void tile_update(TileRow& x, int I, int J, int k, const double* vabs, const double* wabs) {
    __builtin_amdgcn_sched_barrier(0);
    const int r = RT * I + k;
    const double vr = vabs[2 * r], vi = vabs[2 * r + 1], wr = wabs[2 * r], wi = wabs[2 * r + 1];
#pragma unroll
    for (int q = 0; q < RT; ++q) {
        const int c = RT * J + (q ^ k);
        const double vcr = vabs[2 * c], vci = vabs[2 * c + 1], wcr = wabs[2 * c], wci = wabs[2 * c + 1];
        x.set(q, x.re(q) - (vr * wcr + vi * wci + wr * vcr + wi * vci),
              x.im(q) - (vi * wcr - vr * wci + wi * vcr - wr * vci));
    }
    __builtin_amdgcn_sched_barrier(0);
}

// The previous column's update A -= vp wp^H + wp vp^H on this lane's tile row, and then, when
// mv, p += A v over the updated tile exactly as tile_matvec does: one pass over the tile per
// column instead of an update pass and a product pass.
template <class TileRow>
__device__ __forceinline__ void tile_update_matvec(TileRow& x, int I, int J, int k, const double* vp,
                                                   const double* wp, const double* v, double* pabs, double& vav,
                                                   bool mv) {
    __builtin_amdgcn_sched_barrier(0);
    const int r = RT * I + k;
    const double pr = vp[2 * r], pi = vp[2 * r + 1], qr = wp[2 * r], qi = wp[2 * r + 1];
    const double vrr = v[2 * r], vri = v[2 * r + 1];
    double rr = 0.0, ri = 0.0;
    double ar[RT], ai[RT];
#pragma unroll
    for (int q = 0; q < RT; ++q) {
        const int c = RT * J + (q ^ k);
        const double pcr = vp[2 * c], pci = vp[2 * c + 1], qcr = wp[2 * c], qci = wp[2 * c + 1];
        const double hr = x.re(q) - (pr * qcr + pi * qci + qr * pcr + qi * pci);
        const double hi = x.im(q) - (pi * qcr - pr * qci + qi * pcr - qr * pci);
        x.set(q, hr, hi);
        const double vcr = v[2 * c], vci = v[2 * c + 1];
        rr += hr * vcr - hi * vci;
        ri += hr * vci + hi * vcr;
        ar[q] = hr * vrr + hi * vri;   // conj(A_rc) v_r
        ai[q] = hr * vri - hi * vrr;
    }
    if (mv) {
        if (I != J) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                ar[q] += dpp_mov<0x141>(ar[7 - q]);
                ai[q] += dpp_mov<0x141>(ai[7 - q]);
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                ar[q] += dpp_mov<0x4E>(ar[q + 2]);
                ai[q] += dpp_mov<0x4E>(ai[q + 2]);
            }
            ar[0] += dpp_mov<0xB1>(ar[1]);
            ai[0] += dpp_mov<0xB1>(ai[1]);
            const int c = RT * J + k;
            atomicAdd(&pabs[2 * c], ar[0]);
            atomicAdd(&pabs[2 * c + 1], ai[0]);
            vav += v[2 * c] * ar[0] + v[2 * c + 1] * ai[0];
        }
        atomicAdd(&pabs[2 * r], rr);
        atomicAdd(&pabs[2 * r + 1], ri);
        vav += vrr * rr + vri * ri;
    }
    __builtin_amdgcn_sched_barrier(0);
}

// column col (rows col.. of this lane's tile row) -> raw, unchanged
template <class TileRow>
__device__ __forceinline__ void tile_extract_raw(const TileRow& x, int I, int J, int col, int k, int n, double* raw) {
    if (I < 0 || J != col / RT) return;
    const int r = RT * I + k, jq = (col - RT * (col / RT)) ^ k;
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int q = 0; q < RT; ++q)
        if (q == jq) {
            a = x.re(q);
            b = x.im(q);
        }
    if (r >= col && r < n) {
        raw[2 * r] = a;
        raw[2 * r + 1] = b;
    }
}

// a lane's row of one tile: in registers, or in LDS ([column][lane] planes)
struct RegRow {
    double (&r)[RT];
    double (&i)[RT];
    __device__ double re(int q) const { return r[q]; }
    __device__ double im(int q) const { return i[q]; }
    __device__ void set(int q, double a, double b) {
        r[q] = a;
        i[q] = b;
    }
};
struct LdsRow {
    double (*r)[RB];
    double (*i)[RB];
    int lane;
    __device__ double re(int q) const { return r[q][lane]; }
    __device__ double im(int q) const { return i[q][lane]; }
    __device__ void set(int q, double a, double b) {
        r[q][lane] = a;
        i[q][lane] = b;
    }
};

__global__ __launch_bounds__(RB) void tri_reduce_reg_kernel(const double* __restrict__ H, int ld, int n,
                                                            double* __restrict__ dg, double* __restrict__ off,
                                                            double* __restrict__ tau, double* __restrict__ refl,
                                                            double* __restrict__ trace) {
    __shared__ RedLds L;
    const int tid = threadIdx.x;
    const int g = tid >> 3, k = tid & 7;
    const int NT = (n + RT - 1) / RT, NTT = NT * (NT + 1) / 2;
    int tI[RS], tJ[RS];
    double ar[RS_REG][RT], ai[RS_REG][RT];
    double tr = 0.0;
#pragma unroll
    for (int s = 0; s < RS; ++s) {
        // Tiles in column-major order (J, then I): a tile stops being live after column
        // 8J + 7, so the 8 groups of a wave get 8 consecutive tiles of this order in each
        // slot and go idle together; consecutive batches go to different waves.
        const int b = s * RNW + (g >> 3);
        const int t = b * RT + (g & 7);
        int I = -1, J = 0;
        if (t < NTT) {
            int c0 = 0;
            while (c0 + (NT - J) <= t) {
                c0 += NT - J;
                ++J;
            }
            I = J + (t - c0);
        }
        tI[s] = I;
        tJ[s] = J;
        __builtin_amdgcn_sched_barrier(0);
        const int r = RT * I + k;
        double xr[RT], xi[RT];
#pragma unroll
        for (int q = 0; q < RT; ++q) {
            const int c = RT * J + (q ^ k);   // slot q holds column q ^ k
            xr[q] = 0.0;
            xi[q] = 0.0;
            if (I >= 0 && r < n && c < n) {
                // Hermitian part: (H_rc + conj(H_cr)) / 2
                const double* a = H + 2 * ((long)r * ld + c);
                const double* b = H + 2 * ((long)c * ld + r);
                xr[q] = 0.5 * (a[0] + b[0]);
                xi[q] = 0.5 * (a[1] - b[1]);
                if (r == c) {
                    xi[q] = 0.0;
                    tr += xr[q];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < RT; ++q) {
            if (s < RS_REG) {
                ar[s < RS_REG ? s : 0][q] = xr[q];
                ai[s < RS_REG ? s : 0][q] = xi[q];
            } else {
                L.tr[s - RS_REG][q][tid] = xr[q];
                L.ti[s - RS_REG][q][tid] = xi[q];
            }
        }
    }
    for (int i = tid; i < 2 * RMAX; i += RB) {
        L.vabs[i] = 0.0;
        L.raw[i] = 0.0;
        L.v[0][i] = 0.0;
        L.v[1][i] = 0.0;
        L.pabs[i] = 0.0;
        L.wv[i] = 0.0;
    }
    {
        double unused = 0.0;
        block_sum2<RNW>(tr, unused, L.red);
        if (tid == 0) trace[0] = tr;
    }
    // column 0 below the diagonal -> vabs, dg[0]; the squared norm below the subdiagonal -> red2
    {
        double x2 = 0.0;
#pragma unroll
        for (int s = 0; s < RS_REG; ++s) tile_extract(RegRow{ar[s], ai[s]}, tI[s], tJ[s], 0, k, n, L.vabs, dg, x2);
#pragma unroll
        for (int s = 0; s < RS_LDS; ++s)
            tile_extract(LdsRow{L.tr[s], L.ti[s], tid}, tI[RS_REG + s], tJ[RS_REG + s], 0, k, n, L.vabs, dg, x2);
        publish(x2, L.red2);
        __syncthreads();
    }

    // Three barriers per column.  Step j: (1) every thread forms column j's reflector from the
    // corrected column in vabs and its norm; v_j goes to LDS.  (2) One pass over the tiles applies
    // column j - 1's rank-2 update (held back from step j - 1) and accumulates p = A22 v_j and
    // v_j^H A22 v_j with the updated values; the tiles' column j + 1 is copied to raw.  (3) w_j =
    // tau p - (|tau|^2 / 2)(v^H A22 v) v, and column j + 1 corrected for update j (O(n): each
    // thread recomputes w_{j+1}), with its norm.  p^H v = conj(tau) v^H A22 v, so w needs no
    // reduction of its own.  The last update is never applied to the tiles (nothing reads them).
    for (int j = 0; j < n - 1; ++j) {
        // Tile coordinates are laundered each column so that the compiler recomputes the
        // LDS column addresses instead of keeping 40 of them live across the loop.
#pragma unroll
        for (int s = 0; s < RS; ++s) {
            asm volatile("" : "+v"(tI[s]));
            asm volatile("" : "+v"(tJ[s]));
        }
        const double x2 = collect<RNW>(L.red2);
        // every thread forms the reflector scalars itself (same inputs, same result)
        double tr_ = 0.0, ti_ = 0.0, sr = 0.0, si = 0.0;
        {
            const double arr = L.vabs[2 * (j + 1)], aii = L.vabs[2 * (j + 1) + 1];
            double beta;
            if (x2 == 0.0 && aii == 0.0) {
                beta = arr;
            } else {
                // IEEE divisions: |alpha - beta|^2 underflows for columns below ~1e-154, where
                // a hardware reciprocal would overflow
                beta = -copysign(sqrt(arr * arr + aii * aii + x2), arr);
                tr_ = (beta - arr) / beta;
                ti_ = -aii / beta;
                const double dr = arr - beta, di = aii, den = dr * dr + di * di;
                sr = dr / den;
                si = -di / den;
            }
            if (tid == 0) {
                off[j] = beta;
                tau[2 * j] = tr_;
                tau[2 * j + 1] = ti_;
            }
        }
        const bool reflect = tr_ != 0.0 || ti_ != 0.0;   // the same in every thread
        double* vc = L.v[j & 1];
        const double* vp = L.v[(j & 1) ^ 1];
        // p at row j (read by every thread in step j - 1 after its product) is cleared here, a
        // barrier after those reads and before this step's product accumulates into p
        if (tid == 0) {
            L.pabs[2 * j] = 0.0;
            L.pabs[2 * j + 1] = 0.0;
        }
        // v (absolute rows: 1 at j + 1, (sr + i si) x below, 0 elsewhere) and reflector row j
        for (int i = tid; i < RMAX; i += RB) {
            double vr, vi;
            hh_entry(L.vabs, i, j, n, sr, si, vr, vi);
            vc[2 * i] = vr;
            vc[2 * i + 1] = vi;
            if (i > j && i < n) {
                refl[2 * ((long)j * n + (i - j - 1))] = vr;
                refl[2 * ((long)j * n + (i - j - 1)) + 1] = vi;
            }
        }
        __syncthreads();
        // update j - 1, then p = A22 v_j (tau applied below) and this thread's share of v^H A22 v;
        // column j + 1 of the updated tiles -> raw
        double vav = 0.0;
#pragma unroll
        for (int s = 0; s < RS_REG; ++s) {
            RegRow x{ar[s], ai[s]};
            if (tile_live(tI[s], tJ[s], j - 1)) tile_update_matvec(x, tI[s], tJ[s], k, vp, L.wv, vc, L.pabs, vav, reflect);
            tile_extract_raw(x, tI[s], tJ[s], j + 1, k, n, L.raw);
        }
#pragma unroll
        for (int s = 0; s < RS_LDS; ++s) {
            LdsRow x{L.tr[s], L.ti[s], tid};
            if (tile_live(tI[RS_REG + s], tJ[RS_REG + s], j - 1))
                tile_update_matvec(x, tI[RS_REG + s], tJ[RS_REG + s], k, vp, L.wv, vc, L.pabs, vav, reflect);
            tile_extract_raw(x, tI[RS_REG + s], tJ[RS_REG + s], j + 1, k, n, L.raw);
        }
        publish(vav, L.red);
        __syncthreads();
        // w = tau p - (|tau|^2 / 2)(v^H A22 v) v; clear p; column j + 1 with update j applied
        // (a_i -= v_i conj(w_{j+1}) + w_i conj(v_{j+1})) -> vabs, dg[j + 1], its norm below the
        // subdiagonal -> red2
        double x2n = 0.0;
        {
            const double h = 0.5 * (tr_ * tr_ + ti_ * ti_) * collect<RNW>(L.red);
            const int j1 = j + 1;
            double w1r = 0.0, w1i = 0.0;
            if (reflect) {
                const double p1r = L.pabs[2 * j1], p1i = L.pabs[2 * j1 + 1];
                w1r = tr_ * p1r - ti_ * p1i - h * vc[2 * j1];
                w1i = tr_ * p1i + ti_ * p1r - h * vc[2 * j1 + 1];
            }
            const double v1r = vc[2 * j1], v1i = vc[2 * j1 + 1];
            for (int i = tid; i < RMAX; i += RB) {
                double wr = 0.0, wi = 0.0;
                const double vr = vc[2 * i], vi = vc[2 * i + 1];
                if (reflect && i > j && i < n) {
                    const double pr0 = L.pabs[2 * i], pi0 = L.pabs[2 * i + 1];
                    wr = tr_ * pr0 - ti_ * pi0 - h * vr;
                    wi = tr_ * pi0 + ti_ * pr0 - h * vi;
                }
                L.wv[2 * i] = wr;
                L.wv[2 * i + 1] = wi;
                // p is cleared for the next product, except at row j + 1: every thread read
                // that entry above, and a later wave may not have yet (the next step clears it)
                if (i != j1) {
                    L.pabs[2 * i] = 0.0;
                    L.pabs[2 * i + 1] = 0.0;
                }
                if (i >= j1 && i < n) {
                    // v_i conj(w1) + w_i conj(v1)
                    const double cr = vr * w1r + vi * w1i + wr * v1r + wi * v1i;
                    const double ci = vi * w1r - vr * w1i + wi * v1r - wr * v1i;
                    const double ar_ = L.raw[2 * i] - cr, ai_ = L.raw[2 * i + 1] - ci;
                    if (i == j1) {
                        dg[j1] = ar_;
                    } else {
                        L.vabs[2 * i] = ar_;
                        L.vabs[2 * i + 1] = ai_;
                        if (i > j1 + 1) x2n += ar_ * ar_ + ai_ * ai_;
                    }
                }
            }
        }
        publish(x2n, L.red2);
        __syncthreads();
    }
}

// One launch per column for orders above RMAX (column j = 0 .. n-1; j = n - 1 only finishes).
// The rank-2 update of column j - 1 is deferred into launch j and fused with the matrix-vector
// product of column j, so the trailing matrix is read and written once per column:
//   1. every workgroup loads v and p = tau A v of column j - 1 (double buffers, by column
//      parity), forms w = p - (tau/2)(p^H v) v, and computes the updated row j itself (O(n));
//      row j is never written back (no later column reads it), so no workgroup waits for
//      another;
//   2. every workgroup forms the Householder vector of column j from that row (the same
//      arithmetic in the same order, so all agree); workgroup 0 writes dg[j], off[j], tau[j],
//      the reflector row and v;
//   3. each wave applies A -= v w^H + w v^H (column j - 1) to its rows j+1.. of the trailing
//      matrix and, in the same pass over the columns, accumulates p = tau A v of column j for
//      those rows; a lane re-reads only entries it wrote itself.
// The arithmetic is that of applying each column's rank-2 update before the next column's
// product (same formulas, same summation order); only the launch boundaries move.
// vbuf and pbuf hold two vectors of n complex entries each (4 n doubles).
__global__ __launch_bounds__(RW) void tri_col_kernel(double* __restrict__ H, int ld, int n, int j,
                                                     double* __restrict__ dg, double* __restrict__ off,
                                                     double* __restrict__ tau, double* __restrict__ refl,
                                                     double* __restrict__ vbuf, double* __restrict__ pbuf) {
    __shared__ double vp[2 * TRI_MAX];   // v of column j - 1, rows j .. n-1
    __shared__ double wp[2 * TRI_MAX];   // w of column j - 1, rows j .. n-1
    __shared__ double rw[2 * TRI_MAX];   // updated row j, columns j .. n-1
    __shared__ double v[2 * TRI_MAX];    // v of column j, rows j+1 .. n-1
    __shared__ double red[2 * RWV];
    __shared__ double sc[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int mp = n - j;       // rows j .. n-1
    const int m = n - j - 1;    // rows j+1 .. n-1
    const double* vprev = vbuf + 2 * (size_t)n * ((j + 1) & 1);
    const double* pprev = pbuf + 2 * (size_t)n * ((j + 1) & 1);
    double* vcur = vbuf + 2 * (size_t)n * (j & 1);
    double* pcur = pbuf + 2 * (size_t)n * (j & 1);
    bool upd = false;
    if (j > 0) {
        const double tr_ = tau[2 * (j - 1)], ti_ = tau[2 * (j - 1) + 1];
        upd = tr_ != 0.0 || ti_ != 0.0;   // the same in every workgroup
        if (upd) {
            double hr = 0.0, hi = 0.0;
            for (int i = tid; i < mp; i += RW) {
                const double vr = vprev[2 * i], vi = vprev[2 * i + 1], pr = pprev[2 * i], pi = pprev[2 * i + 1];
                vp[2 * i] = vr;
                vp[2 * i + 1] = vi;
                wp[2 * i] = pr;
                wp[2 * i + 1] = pi;
                hr += pr * vr + pi * vi;
                hi += pr * vi - pi * vr;
            }
            block_sum2<RWV>(hr, hi, red);   // its barriers also publish vp, wp
            const double a2r = -0.5 * (tr_ * hr - ti_ * hi), a2i = -0.5 * (tr_ * hi + ti_ * hr);
            for (int i = tid; i < mp; i += RW) {
                const double vr = vp[2 * i], vi = vp[2 * i + 1];
                wp[2 * i] += a2r * vr - a2i * vi;
                wp[2 * i + 1] += a2r * vi + a2i * vr;
            }
            __syncthreads();
        }
    }
    // row j, columns j .. n-1, with column j - 1's update applied (relative row 0 of its block)
    for (int c = tid; c < mp; c += RW) {
        const double* h = H + 2 * ((long)j * ld + (j + c));
        double a = h[0], b = h[1];
        if (upd) {
            const double vr = vp[0], vi = vp[1], wr = wp[0], wi = wp[1];
            const double vcr = vp[2 * c], vci = vp[2 * c + 1], wcr = wp[2 * c], wci = wp[2 * c + 1];
            a -= vr * wcr + vi * wci + wr * vcr + wi * vci;
            b -= vi * wcr - vr * wci + wi * vcr - wr * vci;
        }
        rw[2 * c] = a;
        rw[2 * c + 1] = b;
    }
    __syncthreads();
    if (m <= 0) {   // last column: only its diagonal entry remains
        if (blockIdx.x == 0 && tid == 0) dg[j] = rw[0];
        return;
    }
    // x = column j below the diagonal = conj(row j right of the diagonal): x_i = conj(rw[i + 1])
    double x2 = 0.0, unused = 0.0;
    for (int i = tid; i < m; i += RW)
        if (i > 0) x2 += rw[2 * (i + 1)] * rw[2 * (i + 1)] + rw[2 * (i + 1) + 1] * rw[2 * (i + 1) + 1];
    block_sum2<RWV>(x2, unused, red);
    if (tid == 0) {
        const double ar = rw[2], ai = -rw[3];
        double beta, tr_ = 0.0, ti_ = 0.0, sr = 0.0, si = 0.0;
        if (x2 == 0.0 && ai == 0.0) {
            beta = ar;   // already reduced: H_j = I
        } else {
            beta = -copysign(sqrt(ar * ar + ai * ai + x2), ar);
            tr_ = (beta - ar) / beta;
            ti_ = -ai / beta;
            const double dr = ar - beta, di = ai, den = dr * dr + di * di;   // 1/(alpha - beta)
            sr = dr / den;
            si = -di / den;
        }
        sc[0] = tr_;
        sc[1] = ti_;
        sc[2] = sr;
        sc[3] = si;
        if (blockIdx.x == 0) {
            off[j] = beta;
            tau[2 * j] = tr_;
            tau[2 * j + 1] = ti_;
            dg[j] = rw[0];
        }
    }
    __syncthreads();
    const double tr_ = sc[0], ti_ = sc[1], sr = sc[2], si = sc[3];
    for (int i = tid; i < m; i += RW) {
        double vr = 1.0, vi = 0.0;
        if (i > 0) {
            const double xr = rw[2 * (i + 1)], xi = -rw[2 * (i + 1) + 1];
            vr = xr * sr - xi * si;
            vi = xr * si + xi * sr;
        }
        v[2 * i] = vr;
        v[2 * i + 1] = vi;
        if (blockIdx.x == 0) {
            refl[2 * ((long)j * n + i)] = vr;
            refl[2 * ((long)j * n + i) + 1] = vi;
            vcur[2 * i] = vr;
            vcur[2 * i + 1] = vi;
        }
    }
    __syncthreads();
    // rows j+1 .. n-1 of this workgroup: apply column j - 1's update (relative index + 1 in its
    // vectors), store, and accumulate tau A v of column j
    const long base = (long)(j + 1) * ld + (j + 1);
    const int nw = gridDim.x * RWV;
    for (int r0 = ROWS_PER_WAVE * (blockIdx.x * RWV + w); r0 < m; r0 += ROWS_PER_WAVE * nw) {
        double ar[ROWS_PER_WAVE], ai[ROWS_PER_WAVE];
#pragma unroll
        for (int q = 0; q < ROWS_PER_WAVE; ++q) ar[q] = ai[q] = 0.0;
        // columns in chunks of COL_CHUNK per lane: the chunk's loads are all issued before its
        // stores (written in that order, so they cannot be reordered), so a chunk waits for
        // one memory latency rather than one per column
        for (int cb = 0; cb < m; cb += 64 * COL_CHUNK) {
            double2 x[COL_CHUNK][ROWS_PER_WAVE];
#pragma unroll
            for (int t = 0; t < COL_CHUNK; ++t) {
                const int c = cb + 64 * t + lane;
#pragma unroll
                for (int q = 0; q < ROWS_PER_WAVE; ++q) {
                    const int r = r0 + q;
                    x[t][q] = make_double2(0.0, 0.0);
                    if (r < m && c < m) x[t][q] = *(const double2*)(H + 2 * (base + (long)r * ld + c));
                }
            }
#pragma unroll
            for (int t = 0; t < COL_CHUNK; ++t) {
                const int c = cb + 64 * t + lane;
                if (c >= m) continue;
                const double vcr = v[2 * c], vci = v[2 * c + 1];
                double pvr = 0.0, pvi = 0.0, pwr = 0.0, pwi = 0.0;
                if (upd) {
                    pvr = vp[2 * (c + 1)];
                    pvi = vp[2 * (c + 1) + 1];
                    pwr = wp[2 * (c + 1)];
                    pwi = wp[2 * (c + 1) + 1];
                }
#pragma unroll
                for (int q = 0; q < ROWS_PER_WAVE; ++q) {
                    const int r = r0 + q;
                    if (r < m) {
                        double hr = x[t][q].x, hi = x[t][q].y;
                        if (upd) {
                            const double vr = vp[2 * (r + 1)], vi = vp[2 * (r + 1) + 1];
                            const double wr = wp[2 * (r + 1)], wi = wp[2 * (r + 1) + 1];
                            hr -= vr * pwr + vi * pwi + wr * pvr + wi * pvi;
                            hi -= vi * pwr - vr * pwi + wi * pvr - wr * pvi;
                            *(double2*)(H + 2 * (base + (long)r * ld + c)) = make_double2(hr, hi);
                        }
                        ar[q] += hr * vcr - hi * vci;
                        ai[q] += hr * vci + hi * vcr;
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < ROWS_PER_WAVE; ++q) {
            const double qr = wave_sum(ar[q]), qi = wave_sum(ai[q]);
            if (lane == 0 && r0 + q < m) {
                pcur[2 * (r0 + q)] = tr_ * qr - ti_ * qi;
                pcur[2 * (r0 + q) + 1] = tr_ * qi + ti_ * qr;
            }
        }
    }
}

// ------------------------------------------------------------------ eigenvalues / vectors
// number of eigenvalues of T below x (Sturm sequence in ratio form with the LAPACK pivot guard)
__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int c = q < 0.0;
    for (int i = 1; i < n; ++i) {
        q = (d[i] - x) - e2[i - 1] * rcp_nr(q);
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
    }
    return c;
}

__device__ __forceinline__ double bis_tol(double lo, double hi, double tnorm) {
    return 2.0 * EPS * fmax(fabs(lo), fabs(hi)) + EPS * tnorm;
}

// A workgroup of MS_WAVES waves (one per SIMD) narrows [lo, hi] around the eigenvalue of
// ascending index idx (count(lo) <= idx < count(hi)) with 64 MS_WAVES shifts per pass, one per
// lane (8 bits per pass); every thread returns the same bracket.  A Sturm count is a chain of
// dependent steps, so one wave per SIMD runs it at the chain's latency and the extra waves
// buy bits per pass at no cost in pass time (one wave: 6 bits per pass).
constexpr int MS_WAVES = 4;
constexpr int MS_THREADS = 64 * MS_WAVES;
__device__ void block_multisect(const double* d, const double* e2, int n, int idx, double pivmin, double tnorm,
                                double& lo, double& hi, double* red) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int it = 0; it < 24; ++it) {
        if (hi - lo <= bis_tol(lo, hi, tnorm)) break;   // the same in every thread
        const double h = (hi - lo) / (double)(MS_THREADS + 1);
        const double x = lo + (double)(tid + 1) * h;
        const int c = sturm_count(d, e2, n, x, pivmin);
        double nlo = wave_max(c <= idx ? x : lo), nhi = wave_min(c <= idx ? hi : x);
        if (lane == 0) {
            red[2 * w] = nlo;
            red[2 * w + 1] = nhi;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < MS_WAVES; ++q) {
            nlo = fmax(nlo, red[2 * q]);
            nhi = fmin(nhi, red[2 * q + 1]);
        }
        lo = nlo;
        hi = nhi;
        __syncthreads();   // red is rewritten in the next pass
    }
}

__device__ __forceinline__ unsigned hash32(unsigned x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// par[] written by tri_top_kernel and read by the later kernels
enum { P_TNORM = 0, P_PIVMIN = 1, P_TOP = 2, P_THR = 3, P_COUNT = 8 };

// One workgroup: Gershgorin bounds, the largest eigenvalue, the level's threshold t and the
// accepted count m (cnt[0]); st as spectrum_cut writes it.
__global__ __launch_bounds__(MS_THREADS) void tri_top_kernel(const double* __restrict__ dg, const double* __restrict__ off,
                                                     int n, int level, double floor2, double noise, double tau_rel,
                                                     int cap, const double* __restrict__ trace,
                                                     double* __restrict__ st, int* __restrict__ cnt,
                                                     double* __restrict__ par) {
    __shared__ double d[TRI_MAX], e2[TRI_MAX], red[4 * MS_WAVES];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double gmax = -INFINITY, gmin = INFINITY, e2max = 0.0, dmax = -INFINITY;
    for (int i = tid; i < n; i += MS_THREADS) {
        const double di = dg[i];
        const double el = i > 0 ? fabs(off[i - 1]) : 0.0, er = i < n - 1 ? fabs(off[i]) : 0.0;
        d[i] = di;
        e2[i] = i < n - 1 ? off[i] * off[i] : 0.0;
        gmax = fmax(gmax, di + el + er);
        gmin = fmin(gmin, di - el - er);
        e2max = fmax(e2max, e2[i]);
        dmax = fmax(dmax, di);
    }
    gmax = wave_max(gmax);
    gmin = wave_min(gmin);
    e2max = wave_max(e2max);
    dmax = wave_max(dmax);
    if (lane == 0) {
        red[4 * w] = gmax;
        red[4 * w + 1] = gmin;
        red[4 * w + 2] = e2max;
        red[4 * w + 3] = dmax;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MS_WAVES; ++q) {
        gmax = fmax(gmax, red[4 * q]);
        gmin = fmin(gmin, red[4 * q + 1]);
        e2max = fmax(e2max, red[4 * q + 2]);
        dmax = fmax(dmax, red[4 * q + 3]);
    }
    __syncthreads();
    const double tnorm = fmax(fabs(gmin), fabs(gmax));
    const double pivmin = DBL_MIN * fmax(1.0, e2max);
    double lo = dmax, hi = gmax + EPS * tnorm + pivmin;   // count(lo) <= n-1 < count(hi)
    block_multisect(d, e2, n, n - 1, pivmin, tnorm, lo, hi, red);
    if (tid == 0) {
        const double lmax = 0.5 * (lo + hi);
        const double st0 = level == 0 ? lmax : st[0];
        double t = floor2 * st0;
        if (noise * lmax > t) t = noise * lmax;
        if (tau_rel * lmax > t) t = tau_rel * lmax;
        int m = 0;
        if (lmax > 0.0) {
            m = n - sturm_count(d, e2, n, t, pivmin);
            if (m > cap) m = cap;
            if (m < 0) m = 0;
        }
        if (level == 0) {
            st[0] = lmax;
            st[4] = trace[0];
        }
        st[1 + level] = t;
        cnt[0] = m;
        par[P_TNORM] = tnorm;
        par[P_PIVMIN] = pivmin;
        par[P_TOP] = hi;
        par[P_THR] = t;
    }
}

// Workgroup k < m: eigenvalue k (descending) by multisection on [t, top].
__global__ __launch_bounds__(MS_THREADS) void tri_eval_kernel(const double* __restrict__ dg, const double* __restrict__ off,
                                                      int n, const int* __restrict__ cnt,
                                                      const double* __restrict__ par, double* __restrict__ evals,
                                                      double* __restrict__ sig, double* __restrict__ inv) {
    __shared__ double d[TRI_MAX], e2[TRI_MAX], red[2 * MS_WAVES];
    const int k = blockIdx.x, tid = threadIdx.x;
    if (k >= cnt[0]) return;
    for (int i = tid; i < n; i += MS_THREADS) {
        d[i] = dg[i];
        e2[i] = i < n - 1 ? off[i] * off[i] : 0.0;
    }
    __syncthreads();
    double lo = par[P_THR], hi = par[P_TOP];
    block_multisect(d, e2, n, n - 1 - k, par[P_PIVMIN], par[P_TNORM], lo, hi, red);
    if (tid == 0) {
        const double lk = 0.5 * (lo + hi);
        evals[k] = lk;
        const double sk = sqrt(fmax(lk, 0.0));
        if (sig) sig[k] = sk;
        if (inv) inv[k] = sk > 0.0 ? 1.0 / sk : 0.0;
    }
}

// Wave k < m: eigenvector k of T by three steps of inverse iteration.  The first pass factors
// T - lambda_k I (LU with partial pivoting between neighbouring rows) fused with its forward
// solve and keeps the multipliers, the row swaps and the reciprocal pivots in the wave's LDS;
// the later passes only substitute.  Z row k (length n) receives the unit vector.
__global__ __launch_bounds__(64) void tri_vec_kernel(const double* __restrict__ dg, const double* __restrict__ off,
                                                     int n, const int* __restrict__ cnt,
                                                     const double* __restrict__ par,
                                                     const double* __restrict__ evals, double* __restrict__ Z) {
    __shared__ double d[TRI_MAX], e[TRI_MAX], u0[TRI_MAX], u1[TRI_MAX], u2[TRI_MAX], yv[TRI_MAX], z[TRI_MAX],
        fm[TRI_MAX];
    __shared__ unsigned char sw[TRI_MAX];
    const int k = blockIdx.x, lane = threadIdx.x;
    if (k >= cnt[0]) return;
    for (int i = lane; i < n; i += 64) {
        d[i] = dg[i];
        e[i] = i < n - 1 ? off[i] : 0.0;
        z[i] = (double)(hash32((unsigned)(i * 7919 + k * 104729 + 17)) >> 8) * (2.0 / 16777216.0) - 1.0;
    }
    __syncthreads();
    const double lk = evals[k];
    const double tnorm = par[P_TNORM];
    const double tiny = EPS * tnorm > 0.0 ? EPS * tnorm : DBL_MIN;
    for (int iter = 0; iter < 3; ++iter) {
        if (lane == 0) {
            double y = z[0];
            if (iter == 0) {
                double p0 = d[0] - lk, p1 = n > 1 ? e[0] : 0.0;
                for (int i = 0; i < n - 1; ++i) {
                    const double sub = e[i], nd = d[i + 1] - lk, ns = (i + 1 < n - 1) ? e[i + 1] : 0.0;
                    const double xn = z[i + 1];
                    if (fabs(p0) >= fabs(sub)) {
                        if (p0 == 0.0) p0 = tiny;
                        const double r0 = pivot_rcp(p0);
                        const double mlt = fabs(p0) >= 1e-290 ? sub * r0 : sub / p0;
                        fm[i] = mlt;
                        sw[i] = 0;
                        u0[i] = r0;
                        u1[i] = p1;
                        u2[i] = 0.0;
                        yv[i] = y;
                        p0 = nd - mlt * p1;
                        p1 = ns;
                        y = xn - mlt * y;
                    } else {
                        const double r0 = pivot_rcp(sub);
                        const double mlt = fabs(sub) >= 1e-290 ? p0 * r0 : p0 / sub;
                        fm[i] = mlt;
                        sw[i] = 1;
                        u0[i] = r0;
                        u1[i] = nd;
                        u2[i] = ns;
                        yv[i] = xn;
                        const double np0 = p1 - mlt * nd;
                        p1 = -mlt * ns;
                        p0 = np0;
                        y = y - mlt * xn;
                    }
                }
                if (p0 == 0.0) p0 = tiny;
                u0[n - 1] = pivot_rcp(p0);
            } else {
                for (int i = 0; i < n - 1; ++i) {
                    const double xn = z[i + 1];
                    if (sw[i] == 0) {
                        yv[i] = y;
                        y = xn - fm[i] * y;
                    } else {
                        yv[i] = xn;
                        y = y - fm[i] * xn;
                    }
                }
            }
            double z1 = y * u0[n - 1], z2 = 0.0;
            z[n - 1] = z1;
            for (int i = n - 2; i >= 0; --i) {
                const double z0 = (yv[i] - u1[i] * z1 - u2[i] * z2) * u0[i];
                z[i] = z0;
                z2 = z1;
                z1 = z0;
            }
        }
        __syncthreads();
        double s = 0.0;
        for (int i = lane; i < n; i += 64) s += z[i] * z[i];
        s = wave_sum(s);
        const double sc = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
        for (int i = lane; i < n; i += 64) z[i] *= sc;
        __syncthreads();
    }
    for (int i = lane; i < n; i += 64) Z[(long)k * n + i] = z[i];
}

// Clusters of eigenvalues closer than 1e-12 ||T|| (inverse iteration leaves their vectors at
// arbitrary angles inside the cluster): modified Gram-Schmidt, one wave per cluster.  Vectors of
// different clusters are orthogonal to about eps ||T|| / gap <= 2e-4.
__global__ __launch_bounds__(TB) void tri_mgs_kernel(int n, const int* __restrict__ cnt,
                                                     const double* __restrict__ par,
                                                     const double* __restrict__ evals, double* __restrict__ Z) {
    __shared__ int cstart[TRI_MAX + 1];
    __shared__ int ncl;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m = cnt[0];
    if (m < 2) return;
    if (tid == 0) {
        const double gap = 1e-12 * par[P_TNORM];
        int nc = 0;
        cstart[nc++] = 0;
        for (int k = 1; k < m; ++k)
            if (evals[k - 1] - evals[k] >= gap) cstart[nc++] = k;
        cstart[nc] = m;
        ncl = nc;
    }
    __syncthreads();
    const int nc = ncl;
    for (int ci = w; ci < nc; ci += NW) {
        const int c0 = cstart[ci], c1 = cstart[ci + 1];
        if (c1 - c0 < 2) continue;
        for (int j = c0; j < c1; ++j) {
            double* zj = Z + (long)j * n;
            for (int pq = c0; pq < j; ++pq) {
                const double* zp = Z + (long)pq * n;
                double s = 0.0;
                for (int i = lane; i < n; i += 64) s += zp[i] * zj[i];
                s = wave_sum(s);
                for (int i = lane; i < n; i += 64) zj[i] -= s * zp[i];
            }
            double s = 0.0;
            for (int i = lane; i < n; i += 64) s += zj[i] * zj[i];
            s = wave_sum(s);
            const double sc = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
            for (int i = lane; i < n; i += 64) zj[i] *= sc;
        }
    }
}

// ------------------------------------------------------------------ back-transform
// V[:, k] = H_0 ... H_{n-2} z_k for k < cnt[0]; workgroup b owns columns [BK_COLS b, BK_COLS (b+1)),
// one wave per column.  Reflectors are staged through LDS in chunks of R = BK_CH / (2 (n-1))
// (slot stride 2 (n-1) doubles): the next chunk is loaded into registers while the current one
// is applied, so the latency of a global load is paid once per chunk, and the waves apply a
// chunk with no barrier between its reflectors (each touches only its own column).
constexpr int BK_CH = 4096;   // doubles per chunk buffer
__global__ __launch_bounds__(BK_THREADS) void tri_back_kernel(const double* __restrict__ refl,
                                                              const double* __restrict__ tau, int n,
                                                              const double* __restrict__ Z,
                                                              const int* __restrict__ cnt, double* __restrict__ V,
                                                              int ldv) {
    constexpr int PF = BK_CH / BK_THREADS;   // doubles per thread per chunk
    __shared__ double zb[BK_COLS][2 * TRI_MAX];
    __shared__ double vb[2][BK_CH];
    __shared__ double tl[2 * TRI_MAX];
    const int m = cnt[0];
    const int k0 = blockIdx.x * BK_COLS;
    if (k0 >= m) return;
    const int kc = min(BK_COLS, m - k0);
    const int tid = threadIdx.x;
    for (int i = tid; i < 2 * (n - 1); i += BK_THREADS) tl[i] = tau[i];
    for (int idx = tid; idx < BK_COLS * n; idx += BK_THREADS) {
        const int c = idx / n, i = idx - c * n;
        zb[c][2 * i] = c < kc ? Z[(long)(k0 + c) * n + i] : 0.0;
        zb[c][2 * i + 1] = 0.0;
    }
    const int c = tid / BK_LANES, part = tid % BK_LANES;
    const int S = 2 * (n - 1);
    const int R = S > 0 ? BK_CH / S : 1;   // >= 2 since n <= TRI_MAX
    // reflector j occupies refl[2 j n .. 2 j n + 2 (n-1-j)); chunk of jhi holds jhi, jhi-1, ...
    double pf[PF];
    auto fetch = [&](int jhi) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int idx = tid + q * BK_THREADS;
            const int r = S > 0 ? idx / S : 0, o = idx - r * S, j = jhi - r;
            pf[q] = (S > 0 && r < R && j >= 0 && o < 2 * (n - 1 - j)) ? refl[2L * j * n + o] : 0.0;
        }
    };
    int buf = 0;
    fetch(n - 2);
    for (int jhi = n - 2; jhi >= 0; jhi -= R) {
#pragma unroll
        for (int q = 0; q < PF; ++q) vb[buf][tid + q * BK_THREADS] = pf[q];
        fetch(jhi - R);
        __syncthreads();
        for (int r = 0; r < R && jhi - r >= 0; ++r) {
            const int j = jhi - r, L = n - 1 - j;
            const double tr = tl[2 * j], ti = tl[2 * j + 1];
            if (tr == 0.0 && ti == 0.0) continue;
            // s = v^H z[j+1..]
            double sr = 0.0, si = 0.0;
            const double* zc = &zb[c][2 * (j + 1)];
            const double* vv = &vb[buf][r * S];
            for (int i = part; i < L; i += BK_LANES) {
                const double vr = vv[2 * i], vi = vv[2 * i + 1], zr = zc[2 * i], zi = zc[2 * i + 1];
                sr += vr * zr + vi * zi;
                si += vr * zi - vi * zr;
            }
            sr = wave_sum(sr);
            si = wave_sum(si);
            // z -= tau s v
            const double fr = tr * sr - ti * si, fi = tr * si + ti * sr;
            double* zw = &zb[c][2 * (j + 1)];
            for (int i = part; i < L; i += BK_LANES) {
                const double vr = vv[2 * i], vi = vv[2 * i + 1];
                zw[2 * i] -= fr * vr - fi * vi;
                zw[2 * i + 1] -= fr * vi + fi * vr;
            }
        }
        buf ^= 1;
    }
    __syncthreads();
    for (int idx = tid; idx < n * kc; idx += BK_THREADS) {
        const int i = idx / kc, cc = idx - i * kc;
        V[2 * ((long)i * ldv + k0 + cc)] = zb[cc][2 * i];
        V[2 * ((long)i * ldv + k0 + cc) + 1] = zb[cc][2 * i + 1];
    }
}

}  // namespace

size_t tri_work_bytes(int n) {
    if (n > TRI_MAX) n = TRI_MAX;
    size_t b = 0;
    b += (size_t)n * sizeof(double) * 4;          // dg, off, tau (complex)
    b += 64 * sizeof(double);                     // trace
    b += P_COUNT * sizeof(double);                // par
    b += (size_t)n * n * 2 * sizeof(double);      // reflector rows
    b += (size_t)n * n * sizeof(double);          // Z
    b += (size_t)n * 8 * sizeof(double);          // v and p of the multi-workgroup reduction (two each)
    return b + 1024;
}

hipError_t eigh_top(hipStream_t s, int n, double* H, int ldh, int level, double floor2, double noise, double tau,
                    int cap, double* st, int* cnt, double* evals, double* sig, double* inv, double* V, int ldv,
                    void* work, ProfSink* prof) {
    if (n < 1 || n > TRI_MAX || cap < 0) return hipErrorInvalidValue;
    if (cap > n) cap = n;
    char* w = (char*)work;
    double* dg = (double*)w;
    double* off = dg + n;
    double* tv = off + n;
    double* trace = tv + 2 * n;
    double* par = trace + 64;
    double* refl = par + P_COUNT;
    double* Z = refl + (size_t)n * n * 2;
    double* vbuf = Z + (size_t)n * n;
    double* pbuf = vbuf + 4 * (size_t)n;
    const double nn = (double)n;
    if (prof) prof->begin(s, PF_TRI_REDUCE);
    if (n <= RMAX)
        hipLaunchKernelGGL(tri_reduce_reg_kernel, dim3(1), dim3(RB), 0, s, H, ldh, n, dg, off, tv, refl, trace);
    else
    {
        hipLaunchKernelGGL(tri_herm_kernel, dim3(reduce_groups(n)), dim3(RW), 0, s, H, ldh, n);
        hipLaunchKernelGGL(tri_trace_kernel, dim3(1), dim3(RW), 0, s, H, ldh, n, trace);
        // one launch per column; the last one applies column n - 2's update to dg[n - 1]
        for (int j = 0; j < n; ++j)
            hipLaunchKernelGGL(tri_col_kernel, dim3(reduce_groups(n - j - 1)), dim3(RW), 0, s, H, ldh, n, j, dg, off,
                               tv, refl, vbuf, pbuf);
    }
    // Hermitian tridiagonal reduction: 16/3 n^3 real flop; the matrix is read and rewritten
    // once per column
    if (prof) prof->end(s, PF_TRI_REDUCE, 16.0 / 3.0 * nn * nn * nn, 16.0 * nn * nn * 2.0);
    if (prof) prof->begin(s, PF_TRI_SOLVE);
    hipLaunchKernelGGL(tri_top_kernel, dim3(1), dim3(MS_THREADS), 0, s, dg, off, n, level, floor2, noise, tau, cap, trace,
                       st, cnt, par);
    if (cap > 0) {
        hipLaunchKernelGGL(tri_eval_kernel, dim3(cap), dim3(MS_THREADS), 0, s, dg, off, n, cnt, par, evals, sig, inv);
        hipLaunchKernelGGL(tri_vec_kernel, dim3(cap), dim3(64), 0, s, dg, off, n, cnt, par, evals, Z);
        hipLaunchKernelGGL(tri_mgs_kernel, dim3(1), dim3(TB), 0, s, n, cnt, par, evals, Z);
    }
    if (prof) prof->end(s, PF_TRI_SOLVE, 0.0, 0.0);
    if (cap > 0) {
        if (prof) prof->begin(s, PF_TRI_BACK);
        hipLaunchKernelGGL(tri_back_kernel, dim3((cap + BK_COLS - 1) / BK_COLS), dim3(BK_THREADS), 0, s, refl, tv, n,
                           Z, cnt, V, ldv);
        // n reflectors applied to at most cap vectors: 8 n^2 cap flop (bound, the count is on
        // the device)
        if (prof) prof->end(s, PF_TRI_BACK, 8.0 * nn * nn * cap, 16.0 * nn * nn);
    }
    return hipGetLastError();
}

}  // namespace mpdo
