// Pulse-level two-atom channel (gfx950, FP64): Trotterised Lindblad evolution of the basis
// inputs |a><b| of a pair of atoms through one laser pulse (Sec. II; Sec. III.A).
//
//   pulse_drive_kernel   one thread per step: the single-atom propagator exp(-i tau H) on the
//                        {|1>, |r>} block in closed form (the other levels are untouched)
//   pulse_evolve_kernel  one workgroup per (time segment, basis input |a><b|), one thread per entry of the
//                        pair's density matrix (d^4 <= 256), the matrix held in LDS through all
//                        steps.  Per step two passes, each ended by a barrier:
//                          1. dissipators of both atoms and the blockade phase, entry-wise:
//                             an entry keeps a decay/dephasing factor and, on a sink's diagonal,
//                             receives the r-r entry it is fed from;
//                          2. conjugation by u (x) u, u mixing only |1> and |r>: at most 16
//                             terms per entry.
//                        The per-step coefficients are staged in LDS, CHUNK steps at a time
//                        (one coalesced load per chunk instead of a dependent load per step).
//   segment products     the steps are cut into up to MAX_SEG consecutive segments whose
//                        channels are built concurrently (d^4 basis inputs alone give one
//                        workgroup per compute unit, too few to hide the per-step barriers);
//                        the segment channels are then multiplied in time order, pairwise in a
//                        tree, by the library's complex FP64 matrix-core GEMM.
//
// Dissipators in closed form (each is the exact exponential of its generator).  Decay r -> j
// with rate k_j = gamma b_j: rho_rr *= e_j, rho_jj += (1 - e_j) rho_rr, coherences with one r
// index *= sqrt(e_j), e_j = exp(-k_j tau); applied for j = 0, 1, dark in that order, the step
// keeps E = e_0 e_1 e_dark of rho_rr and moves (1 - e_0), e_0 (1 - e_1), e_0 e_1 (1 - e_dark)
// of it to 0, 1, dark.  Dephasing multiplies rho_01 by exp(-g^2 tau) and a coherence between a
// qubit level and r or dark by exp(-g^2 tau / 4), g = gamma_deph; populations stay.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "../../include/mpdo_pulse.h"
#include "gemm.h"

// Scratch of the allocation-free entry point (mpdo_pulse_channel_noalloc): one fixed block per
// device, which every call on that device reuses (calls that overlap on one device race) and
// which stays allocated until the process ends.  Host code never uses the name itself, only the
// address hipGetSymbolAddress returns for the current device.  Nothing in it must start at
// zero: every kernel and product writes all of its part before reading it.
constexpr size_t PULSE_SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) char scratch[PULSE_SCRATCH_BYTES];

namespace {

constexpr int LR = 2;      // Rydberg level
constexpr int LDARK = 3;   // dark level (d = 4)
constexpr int EVOLVE_THREADS = 256;
constexpr int CHUNK = 256;   // steps whose drive coefficients are staged in LDS at a time
constexpr int MAX_SEG = 16;  // time segments built concurrently
constexpr int SEG_MIN_STEPS = 512;

thread_local std::string g_err;

// per step: u11, u1r (= ur1), urr as re/im pairs
__global__ __launch_bounds__(256) void pulse_drive_kernel(const double* __restrict__ om, const double* __restrict__ de,
                                                          int n, double tau, double* __restrict__ tab) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double O = om[k], D = de[k];
    // exp(-i tau M), M = [[0, O/2], [O/2, D]] on (|1>, |r>):
    //   = exp(-i tau D/2) [cos(w tau) I - i sin(w tau)/w (M - D/2 I)],  w = sqrt(O^2 + D^2) / 2
    const double w = 0.5 * sqrt(O * O + D * D);
    const double c = cos(w * tau);
    const double s = w > 0.0 ? sin(w * tau) / w : tau;
    const double pr = cos(0.5 * D * tau), pi = -sin(0.5 * D * tau);
    // a11 = c + i s D/2, a1r = -i s O/2, arr = c - i s D/2; u = phase * a
    const double a11r = c, a11i = 0.5 * s * D;
    const double a1ri = -0.5 * s * O;
    const double arrr = c, arri = -0.5 * s * D;
    double* t = tab + 6 * (long)k;
    t[0] = pr * a11r - pi * a11i;
    t[1] = pr * a11i + pi * a11r;
    t[2] = -pi * a1ri;
    t[3] = pr * a1ri;
    t[4] = pr * arrr - pi * arri;
    t[5] = pr * arri + pi * arrr;
}

struct SiteNoise {
    double sqrtE;      // survival of one r index per step
    double tr[4];      // transfer into level j's population (0 for non-sinks)
    double dq;         // dephasing of a 0-1 coherence
    double dh;         // dephasing of a qubit / (r or dark) coherence
};

__device__ inline double site_factor(const SiteNoise& z, int x, int y) {
    double f = 1.0;
    if (x == LR) f *= z.sqrtE;
    if (y == LR) f *= z.sqrtE;
    const bool qx = x < 2, qy = y < 2;
    if (qx && qy && x != y) f *= z.dq;
    else if (qx != qy) f *= z.dh;
    return f;
}

__device__ inline double sink_fraction(const SiteNoise& z, int l) {
    return l == 0 ? z.tr[0] : l == 1 ? z.tr[1] : l == LDARK ? z.tr[3] : 0.0;
}

template <int DL>
__global__ __launch_bounds__(EVOLVE_THREADS) void pulse_evolve_kernel(const double* __restrict__ tab, int n,
                                                                      int nseg, double tau, double blockade,
                                                                      SiteNoise z, double* __restrict__ out) {
    constexpr int DIM = DL * DL;   // pair Hilbert dimension
    constexpr int NE = DIM * DIM;  // entries of rho = basis inputs = superoperator order
    static_assert(NE <= EVOLVE_THREADS, "one thread per entry");
    __shared__ double sr[2][NE], si[2][NE];
    __shared__ double ut[6 * CHUNK];
    const int col = blockIdx.x;
    const int seg = blockIdx.y;
    const int k0 = (int)((long)seg * n / nseg), k1 = (int)((long)(seg + 1) * n / nseg);
    out += 2 * (long)seg * NE * NE;
    const int a = col / DIM, b = col - (col / DIM) * DIM;
    const int t = threadIdx.x;
    const bool act = t < NE;
    const int x = act ? t / DIM : 0, y = act ? t - (t / DIM) * DIM : 0;
    const int x1 = x / DL, x2 = x - (x / DL) * DL, y1 = y / DL, y2 = y - (y / DL) * DL;
    if (act) {
        sr[0][t] = (x == a && y == b) ? 1.0 : 0.0;
        si[0][t] = 0.0;
    }
    // pass-1 constants
    const double f1 = site_factor(z, x1, y1), f2 = site_factor(z, x2, y2);
    const double t1 = (x1 == y1) ? sink_fraction(z, x1) : 0.0, t2 = (x2 == y2) ? sink_fraction(z, x2) : 0.0;
    const int src1 = (LR * DL + x2) * DIM + (LR * DL + y2);
    const int src2 = (x1 * DL + LR) * DIM + (y1 * DL + LR);
    const int src12 = (LR * DL + LR) * DIM + (LR * DL + LR);
    const int rr = LR * DL + LR;
    const double bph = -tau * blockade * ((x == rr ? 1.0 : 0.0) - (y == rr ? 1.0 : 0.0));
    const double bc = cos(bph), bs = sin(bph);
    // pass-2 partners: a level l in {1, r} mixes with both levels of the pair, any other level
    // only with itself.  Partner p of l is level 1 (p = 0) or r (p = 1) and its coefficient is
    // u_{l,partner}, stored at slot 0 (u11), 1 (u1r = ur1) or 2 (urr) of the step's table;
    // slot -1 is the identity.
    const bool m1x = x1 == 1 || x1 == LR, m2x = x2 == 1 || x2 == LR;
    const bool m1y = y1 == 1 || y1 == LR, m2y = y2 == 1 || y2 == LR;
    const int nx1 = m1x ? 2 : 1, nx2 = m2x ? 2 : 1, ny1 = m1y ? 2 : 1, ny2 = m2y ? 2 : 1;
    int px1[2], px2[2], py1[2], py2[2], sx1[2], sx2[2], sy1[2], sy2[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const int lev = p == 0 ? 1 : LR;
        px1[p] = m1x ? lev : x1;
        px2[p] = m2x ? lev : x2;
        py1[p] = m1y ? lev : y1;
        py2[p] = m2y ? lev : y2;
        sx1[p] = m1x ? (x1 == 1 ? p : 1 + p) : -1;
        sx2[p] = m2x ? (x2 == 1 ? p : 1 + p) : -1;
        sy1[p] = m1y ? (y1 == 1 ? p : 1 + p) : -1;
        sy2[p] = m2y ? (y2 == 1 ? p : 1 + p) : -1;
    }
    __syncthreads();
    for (int k = k0; k < k1; ++k) {
        const int kc = (k - k0) % CHUNK;
        if (kc == 0) {
            // the previous chunk's last pass-2 reads of ut ended at the barrier below
            const int m = min(CHUNK, k1 - k);
            for (int i = threadIdx.x; i < 6 * m; i += EVOLVE_THREADS) ut[i] = tab[6 * (long)k + i];
        }
        // ---- pass 1: dissipators of both atoms, then the blockade phase (buffer 0 -> 1)
        if (act) {
            double vr = f1 * f2 * sr[0][t], vi = f1 * f2 * si[0][t];
            if (t1 != 0.0) {
                vr += t1 * f2 * sr[0][src1];
                vi += t1 * f2 * si[0][src1];
            }
            if (t2 != 0.0) {
                vr += f1 * t2 * sr[0][src2];
                vi += f1 * t2 * si[0][src2];
            }
            if (t1 != 0.0 && t2 != 0.0) {
                vr += t1 * t2 * sr[0][src12];
                vi += t1 * t2 * si[0][src12];
            }
            sr[1][t] = bc * vr - bs * vi;
            si[1][t] = bc * vi + bs * vr;
        }
        __syncthreads();
        // ---- pass 2: rho <- (u (x) u) rho (u (x) u)^+ (buffer 1 -> 0)
        if (act) {
            const double* u = ut + 6 * kc;
            double accr = 0.0, acci = 0.0;
#pragma unroll
            for (int p1 = 0; p1 < 2; ++p1) {
                if (p1 >= nx1) continue;
                const double c1r = sx1[p1] < 0 ? 1.0 : u[2 * sx1[p1]], c1i = sx1[p1] < 0 ? 0.0 : u[2 * sx1[p1] + 1];
#pragma unroll
                for (int p2 = 0; p2 < 2; ++p2) {
                    if (p2 >= nx2) continue;
                    const double c2r = sx2[p2] < 0 ? 1.0 : u[2 * sx2[p2]], c2i = sx2[p2] < 0 ? 0.0 : u[2 * sx2[p2] + 1];
                    const double cxr = c1r * c2r - c1i * c2i, cxi = c1r * c2i + c1i * c2r;
                    const int xs = px1[p1] * DL + px2[p2];
#pragma unroll
                    for (int q1 = 0; q1 < 2; ++q1) {
                        if (q1 >= ny1) continue;
                        // conj(u) on the bra side
                        const double d1r = sy1[q1] < 0 ? 1.0 : u[2 * sy1[q1]];
                        const double d1i = sy1[q1] < 0 ? 0.0 : -u[2 * sy1[q1] + 1];
#pragma unroll
                        for (int q2 = 0; q2 < 2; ++q2) {
                            if (q2 >= ny2) continue;
                            const double d2r = sy2[q2] < 0 ? 1.0 : u[2 * sy2[q2]];
                            const double d2i = sy2[q2] < 0 ? 0.0 : -u[2 * sy2[q2] + 1];
                            const double dyr = d1r * d2r - d1i * d2i, dyi = d1r * d2i + d1i * d2r;
                            const double cr = cxr * dyr - cxi * dyi, ci = cxr * dyi + cxi * dyr;
                            const int e = xs * DIM + (py1[q1] * DL + py2[q2]);
                            const double vr = sr[1][e], vi = si[1][e];
                            accr += cr * vr - ci * vi;
                            acci += cr * vi + ci * vr;
                        }
                    }
                }
            }
            sr[0][t] = accr;
            si[0][t] = acci;
        }
        __syncthreads();
    }
    if (act) {
        // per-atom layout: row (x1 d + y1) D2 + (x2 d + y2), column likewise from (a, b)
        const int a1 = a / DL, a2 = a - (a / DL) * DL, b1 = b / DL, b2 = b - (b / DL) * DL;
        const long row = (long)(x1 * DL + y1) * DIM + (x2 * DL + y2);
        const long cidx = (long)(a1 * DL + b1) * DIM + (a2 * DL + b2);
        out[2 * (row * NE + cidx)] = sr[0][t];
        out[2 * (row * NE + cidx) + 1] = si[0][t];
    }
}

bool finite_all(const double* p, long n) {
    for (long i = 0; i < n; ++i)
        if (!isfinite(p[i])) return false;
    return true;
}

mpdo_status fail(mpdo_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

// Device buffers of one call: step samples (2 n), per-step drive table (6 n), the segment
// channels (nseg) and the pairwise products (ceil(nseg / 2)), each channel ne^2 complex.
struct PulseBufs {
    double *samp, *tab, *out, *tmp;
};

struct PulseSizes {
    int ne, nseg;
    size_t samp_b, tab_b, one_b;
    size_t total() const {   // one block of scratch, every part 256-byte aligned
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        return al(samp_b) + al(tab_b) + al(one_b * nseg) + al(one_b * ((nseg + 1) / 2));
    }
};

PulseSizes pulse_sizes(int d, int n) {
    PulseSizes z;
    z.ne = d * d * d * d;
    z.nseg = std::max(1, std::min(MAX_SEG, n / SEG_MIN_STEPS));
    z.samp_b = 2 * (size_t)n * sizeof(double);
    z.tab_b = 6 * (size_t)n * sizeof(double);
    z.one_b = 2 * (size_t)z.ne * z.ne * sizeof(double);
    return z;
}

mpdo_status check_params(const mpdo_pulse_params* p, const double* omega, const double* delta, double* superop) {
    if (!p || !omega || !delta || !superop) return fail(MPDO_E_ARG, "null pointer");
    const int d = p->d, n = p->n_steps;
    if (d != 3 && d != 4) return fail(MPDO_E_ARG, "d must be 3 or 4");
    if (n < 1) return fail(MPDO_E_ARG, "n_steps must be >= 1");
    const double rates[7] = {p->tau, p->blockade, p->gamma_diss, p->branch[0], p->branch[1], p->branch[2],
                             p->gamma_deph};
    if (!finite_all(rates, 7)) return fail(MPDO_E_ARG, "non-finite parameter");
    if (!(p->tau > 0.0)) return fail(MPDO_E_ARG, "tau must be > 0");
    if (p->gamma_diss < 0.0 || p->branch[0] < 0.0 || p->branch[1] < 0.0 || p->branch[2] < 0.0)
        return fail(MPDO_E_ARG, "negative rate or branch ratio");
    if (d == 3 && p->branch[2] != 0.0) return fail(MPDO_E_ARG, "a dark branch needs d = 4");
    if (!finite_all(omega, n) || !finite_all(delta, n)) return fail(MPDO_E_ARG, "non-finite pulse sample");
    return MPDO_OK;
}

// The channel of one pulse into superop (host), computed in the device buffers B (validated
// parameters; the sizes of B follow pulse_sizes(d, n_steps)).
mpdo_status pulse_run(const mpdo_pulse_params* p, const double* omega, const double* delta, double* superop,
                      hipStream_t s, const PulseBufs& B) {
    const int d = p->d, n = p->n_steps;
    const double tau = p->tau;
    SiteNoise z{};
    const double e0 = exp(-p->gamma_diss * p->branch[0] * tau);
    const double e1 = exp(-p->gamma_diss * p->branch[1] * tau);
    const double ed = exp(-p->gamma_diss * p->branch[2] * tau);
    z.sqrtE = sqrt(e0 * e1 * ed);
    z.tr[0] = 1.0 - e0;
    z.tr[1] = e0 * (1.0 - e1);
    z.tr[2] = 0.0;
    z.tr[3] = d == 4 ? e0 * e1 * (1.0 - ed) : 0.0;
    const double g2 = p->gamma_deph * p->gamma_deph;
    z.dq = exp(-g2 * tau);
    z.dh = exp(-0.25 * g2 * tau);

    const PulseSizes zs = pulse_sizes(d, n);
    const int ne = zs.ne, nseg = zs.nseg;
    hipError_t e = hipMemcpyAsync(B.samp, omega, n * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(B.samp + n, delta, n * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(pulse_drive_kernel, dim3((n + 255) / 256), dim3(256), 0, s, B.samp, B.samp + n, n, tau,
                           B.tab);
        if (d == 4)
            hipLaunchKernelGGL(pulse_evolve_kernel<4>, dim3(ne, nseg), dim3(EVOLVE_THREADS), 0, s, B.tab, n, nseg,
                               tau, p->blockade, z, B.out);
        else
            hipLaunchKernelGGL(pulse_evolve_kernel<3>, dim3(ne, nseg), dim3(EVOLVE_THREADS), 0, s, B.tab, n, nseg,
                               tau, p->blockade, z, B.out);
        e = hipGetLastError();
    }
    // product of the segment channels in time order: S = S_{nseg-1} ... S_1 S_0, pairwise
    double* cur = B.out;
    double* nxt = B.tmp;
    int cnt = nseg;
    const long one = (long)ne * ne;   // complex elements of one channel
    while (e == hipSuccess && cnt > 1) {
        const int pairs = cnt / 2;
        e = mpdo::cgemm<double>(s, ne, ne, ne, mpdo::cd{1.0, 0.0}, mpdo::view<double>(cur + 2 * one, ne, 1),
                                mpdo::view<double>(cur, ne, 1), mpdo::cd{0.0, 0.0}, mpdo::view<double>(nxt, ne, 1),
                                pairs, 2 * one, 2 * one, one);
        if (e == hipSuccess && (cnt & 1))
            e = hipMemcpyAsync(nxt + 2 * one * pairs, cur + 2 * one * (cnt - 1), zs.one_b, hipMemcpyDeviceToDevice, s);
        cnt = pairs + (cnt & 1);
        std::swap(cur, nxt);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(superop, cur, zs.one_b, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(MPDO_E_DEVICE, std::string("HIP error: ") + hipGetErrorString(e));
    return MPDO_OK;
}

constexpr int PULSE_MAX_DEVICES = 64;
char* g_scratch_ptr[PULSE_MAX_DEVICES] = {nullptr};   // device address of scratch, per device
std::mutex g_scratch_mu;

// The device address of this device's scratch (looked up once per device, with it current).
mpdo_status scratch_of_device(char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(MPDO_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= PULSE_MAX_DEVICES) return fail(MPDO_E_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(MPDO_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = (char*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return MPDO_OK;
}

}  // namespace

extern "C" mpdo_status mpdo_pulse_channel(const mpdo_pulse_params* p, const double* omega, const double* delta,
                                          double* superop, void* hip_stream) {
    mpdo_status st = check_params(p, omega, delta, superop);
    if (st != MPDO_OK) return st;
    const PulseSizes zs = pulse_sizes(p->d, p->n_steps);
    PulseBufs B{nullptr, nullptr, nullptr, nullptr};
    if (hipMalloc(&B.samp, zs.samp_b) != hipSuccess || hipMalloc(&B.tab, zs.tab_b) != hipSuccess ||
        hipMalloc(&B.out, zs.one_b * zs.nseg) != hipSuccess ||
        hipMalloc(&B.tmp, zs.one_b * ((zs.nseg + 1) / 2)) != hipSuccess) {
        st = fail(MPDO_E_NOMEM, "device allocation failed");
    } else {
        st = pulse_run(p, omega, delta, superop, (hipStream_t)hip_stream, B);
    }
    if (B.samp) (void)hipFree(B.samp);
    if (B.tab) (void)hipFree(B.tab);
    if (B.out) (void)hipFree(B.out);
    if (B.tmp) (void)hipFree(B.tmp);
    if (st == MPDO_OK) g_err.clear();
    return st;
}

extern "C" mpdo_status mpdo_pulse_channel_noalloc(const mpdo_pulse_params* p, const double* omega,
                                                  const double* delta, double* superop, void* hip_stream) {
    mpdo_status st = check_params(p, omega, delta, superop);
    if (st != MPDO_OK) return st;
    const PulseSizes zs = pulse_sizes(p->d, p->n_steps);
    if (zs.total() > PULSE_SCRATCH_BYTES)
        return fail(MPDO_E_ARG, "n_steps too large for the fixed scratch of mpdo_pulse_channel_noalloc (" +
                                    std::to_string(zs.total()) + " bytes needed, " +
                                    std::to_string(PULSE_SCRATCH_BYTES) + " available)");
    char* base = nullptr;
    st = scratch_of_device(&base);
    if (st != MPDO_OK) return st;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    PulseBufs B;
    B.samp = (double*)base;
    B.tab = (double*)(base + al(zs.samp_b));
    B.out = (double*)(base + al(zs.samp_b) + al(zs.tab_b));
    B.tmp = (double*)(base + al(zs.samp_b) + al(zs.tab_b) + al(zs.one_b * zs.nseg));
    st = pulse_run(p, omega, delta, superop, (hipStream_t)hip_stream, B);
    if (st == MPDO_OK) g_err.clear();
    return st;
}

extern "C" const char* mpdo_pulse_last_error(void) { return g_err.c_str(); }
