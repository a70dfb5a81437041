// libmpdo host side: the C ABI of include/mpdo.h and the orchestration of one two-site
// update of the vectorised density-operator MPO with Purity-Preserving Truncation.
//
// Update of atoms (i, i+1) (Sec. III.A, Fig. (ansatzes)c; Sec. III.D):
//  1. single-atom channels queued on i and i+1 are folded into the two-site superoperator;
//  2. the canonical centre is moved onto {i, i+1} (every site left of i a left isometry,
//     every site right of i+1 a right isometry) by orthonormal-basis moves;
//  3. theta = S . (A_i A_{i+1}) is split.  When the gate's operator-Schmidt rank r makes
//     r * chi_mid smaller than the side being orthonormalised, theta is never formed: the
//     split works on the factor pair theta = M_L M_R, M_L = [X_k A_i], M_R = [Y_k A_{i+1}];
//     otherwise theta is formed with two matrix-core products (merge, then gate);
//  4. Schmidt vectors come from FP64 Hermitian eigensolves of Gram matrices with
//     residual deflation levels, so values far below sqrt(eps) of the largest are resolved;
//  5. the spectrum is cut to chi (and the relative cutoff) and PPT rescales the kept
//     values on the device (Eqs. (xiformula), (ppt));
//  6. the isometric factor and the rescaled centre factor become the new site tensors.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mpdo.h"
#include "common.h"
#include "chol.h"
#include "eig.h"
#include "pchol.h"
#include "tri.h"
#include "gemm.h"
#include "kernels.h"

using namespace mpdo;
typedef std::complex<double> zc;

namespace {

constexpr double EPS64 = 2.220446049250313e-16;
constexpr double EPS32 = 1.1920928955078125e-07;
constexpr int MAX_FACTOR_RANK = 16;   // operator-Schmidt terms kept in LDS by phys_* kernels
constexpr int EIG_MAX_SWEEPS = 40;
constexpr int EIG_JACOBI_MAX = 32;   // largest order eig_cut gives to the Jacobi solver
// Range bases whose exact construction would need an eigenproblem above TRI_MAX are found by
// block subspace iteration on theta theta^H: SUB_OVER extra directions beyond chi, at most
// SUB_ITERS passes, stopping once the captured weight ||Q^H theta||_F^2 grows by less than the
// tolerance (relative; FP64 1e-10, FP32 1e-6), far below the weight a chi-cut discards there.
constexpr int SUB_OVER = 256;
constexpr int SUB_ITERS = 8;
// largest block the subspace iteration orthonormalises by shifted Cholesky QR
constexpr int CHOL_MAX = 2048;

// Order above which a split uses the subspace iteration: TRI_MAX, or MPDO_SUBSPACE_MIN_ORDER
// from the environment (lower values let tests run the subspace path where the exact path
// also works).
int subspace_min_order() {
    const char* e = getenv("MPDO_SUBSPACE_MIN_ORDER");
    const int v = e ? atoi(e) : 0;
    return v > 0 ? std::min(v, TRI_MAX) : TRI_MAX;
}

struct Fail {
    mpdo_status st;
    std::string msg;
    bool retry = false;   // an update that failed this way may be recomputed once
};

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) throw Fail{MPDO_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
    } while (0)

inline cd C1() { return cd{1.0, 0.0}; }
inline cd C0() { return cd{0.0, 0.0}; }
inline cd Cr(double x) { return cd{x, 0.0}; }

// 64-bit lookup key of a byte range: four independent multiply-xorshift lanes over 8-byte
// words, the tail byte by byte.  Only a key: every cache hit is confirmed by comparing the data.
uint64_t hash_bytes(const void* p, size_t n, uint64_t seed) {
    const unsigned char* b = (const unsigned char*)p;
    uint64_t h[4] = {seed, seed ^ 0x9E3779B97F4A7C15ull, seed ^ 0xC2B2AE3D27D4EB4Full, seed ^ 0x165667B19E3779F9ull};
    size_t i = 0;
    for (; i + 32 <= n; i += 32)
        for (int l = 0; l < 4; ++l) {
            uint64_t w;
            memcpy(&w, b + i + 8 * l, 8);
            h[l] = (h[l] ^ w) * 0x9E3779B97F4A7C15ull;
            h[l] ^= h[l] >> 29;
        }
    uint64_t r = h[0] ^ (h[1] * 3) ^ (h[2] * 5) ^ (h[3] * 7) ^ n;
    for (; i < n; ++i) r = (r ^ b[i]) * 0x100000001B3ull;
    r ^= r >> 31;
    return r * 0xBF58476D1CE4E5B9ull;
}

// ---------------------------------------------------------------------- device arena
struct Arena {
    char* base = nullptr;
    size_t cap = 0, used = 0;
    template <typename X>
    X* take(size_t count) {
        size_t bytes = ((count * sizeof(X)) + 255) & ~(size_t)255;
        if (used + bytes > cap) throw Fail{MPDO_E_NOMEM, "workspace exhausted"};
        X* p = (X*)(base + used);
        used += bytes;
        return p;
    }
};

// ---------------------------------------------------------------------- scratch of one precision
template <typename T>
struct Scratch {
    int nmax = 0;        // largest matrix side handled
    T *bA, *bB, *bT1, *bQ, *bK, *bC, *bR, *bU, *bB2, *bG, *bW, *bVT, *bQ2, *bK2, *bU2;
    double *Gd, *Vd, *evals, *sig, *inv, *st, *sums, *lvec, *rvec, *tl, *tr, *fac, *pout, *sc, *vtmp, *vtmp2;
    double* odev;   // ||Q||_F^2 and non-finite count of recent orthonormal bases (64 pairs)
    double* sqp;    // partial sums of sumsq (2 SUMSQ_MAX_BLOCKS)
    unsigned* sqc;  // arrival counter of sumsq (0 between calls)
    int* cnt;
    void* eigwork;
    void* skw;           // partial tiles of k-split products (GemmOpts::ws)
    size_t skw_bytes;
    double* cholw;       // Cholesky QR: shift and diagonal-block inverses (order <= CHOL_MAX)
    double* pcw;         // pivoted-Cholesky range bases: Cholesky columns and pivot-block inverse

    // k-split workspace: eight n_max^2 complex outputs, capped at 128 MiB
    static size_t split_ws_bytes(int nmax) {
        const size_t b = (size_t)8 * nmax * nmax * 2 * sizeof(T);
        return std::max((size_t)1 << 20, std::min(b, (size_t)128 << 20));
    }
    static size_t bytes(int nmax) {
        const size_t n2 = (size_t)nmax * nmax * 2;
        size_t b = 0;
        b += 15 * (n2 * sizeof(T) + 256);
        b += 2 * (n2 * sizeof(double) + 256);
        b += 14 * ((size_t)nmax * 2 * sizeof(double) + 256) + 4096 + 2048;
        b += 2 * SUMSQ_MAX_BLOCKS * sizeof(double) + 256 + 256;   // sumsq partials and counter
        b += eigh_work_bytes(nmax) + 256;
        b += split_ws_bytes(nmax) + 256;
        b += chol_work_doubles(CHOL_MAX) * sizeof(double) + 256;
        b += pchol_work_doubles(nmax) * sizeof(double) + 256;
        return b;
    }
    void carve(Arena& a, int n) {
        nmax = n;
        const size_t n2 = (size_t)n * n * 2;
        bA = a.take<T>(n2);
        bB = a.take<T>(n2);
        bT1 = a.take<T>(n2);
        bQ = a.take<T>(n2);
        bK = a.take<T>(n2);
        bC = a.take<T>(n2);
        bR = a.take<T>(n2);
        bU = a.take<T>(n2);
        bB2 = a.take<T>(n2);
        bG = a.take<T>(n2);
        bW = a.take<T>(n2);
        bQ2 = a.take<T>(n2);
        bK2 = a.take<T>(n2);
        bU2 = a.take<T>(n2);
        Gd = a.take<double>(n2);
        Vd = a.take<double>(n2);
        bVT = std::is_same<T, double>::value ? (T*)Vd : a.take<T>(n2);
        evals = a.take<double>((size_t)n * 2);
        sig = a.take<double>((size_t)n * 2);
        inv = a.take<double>((size_t)n * 2);
        lvec = a.take<double>((size_t)n * 2);
        rvec = a.take<double>((size_t)n * 2);
        tl = a.take<double>((size_t)n * 2);
        tr = a.take<double>((size_t)n * 2);
        fac = a.take<double>((size_t)n * 2);
        vtmp = a.take<double>((size_t)n * 2);
        vtmp2 = a.take<double>((size_t)n * 2);
        st = a.take<double>(64);
        sums = a.take<double>(64);
        pout = a.take<double>(64);
        sc = a.take<double>(64);
        odev = a.take<double>(128);
        sqp = a.take<double>(2 * SUMSQ_MAX_BLOCKS);
        sqc = a.take<unsigned>(64);
        cnt = a.take<int>(64);
        eigwork = (void*)a.take<char>(eigh_work_bytes(n));
        skw_bytes = split_ws_bytes(n);
        skw = (void*)a.take<char>(skw_bytes);
        cholw = a.take<double>(chol_work_doubles(CHOL_MAX));
        pcw = a.take<double>(pchol_work_doubles(n));
    }
};

// HIP-event timing of kernel families on the context's stream.
struct EventProf : public ProfSink {
    struct Rec {
        hipEvent_t a, b;
        int fam;
        double flop, bytes;
    };
    std::vector<hipEvent_t> pool;
    std::vector<Rec> recs;
    hipEvent_t cur = nullptr;
    int cur_fam = -1;
    unsigned mask = ~0u;   // families recorded (bit f)
    unsigned stride = 1;   // stamped kernels: one launch in `stride` of each family recorded
    unsigned long seen[PF_COUNT] = {0};
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void begin(hipStream_t s, int fam) override {
        if (!((mask >> fam) & 1u)) return;
        cur = get();
        cur_fam = fam;
        if (cur) (void)hipEventRecord(cur, s);
    }
    void end(hipStream_t s, int fam, double flop, double bytes) override {
        if (!((mask >> fam) & 1u) || !cur) return;
        hipEvent_t b = get();
        if (!b) return;
        (void)hipEventRecord(b, s);
        recs.push_back(Rec{cur, b, fam, flop, bytes});
        cur = nullptr;
    }
    bool kernel_events(int fam, hipEvent_t* a, hipEvent_t* b) override {
        if (!((mask >> fam) & 1u)) return false;
        if (seen[fam]++ % stride != 0) return false;
        *a = get();
        *b = get();
        if (*a && *b) return true;
        if (*a) pool.push_back(*a);
        if (*b) pool.push_back(*b);
        return false;
    }
    void kernel_done(int fam, hipEvent_t a, hipEvent_t b, double flop, double bytes) override {
        recs.push_back(Rec{a, b, fam, flop, bytes});
    }
    void amend(int fam, double flop, double bytes) override {
        for (auto r = recs.rbegin(); r != recs.rend(); ++r)
            if (r->fam == fam) {
                r->flop = flop;
                r->bytes = bytes;
                return;
            }
    }
    // families x (launches, ms, flop, bytes); returns events to the pool
    void collect(double* acc) {
        for (auto& r : recs) {
            float ms = 0.f;
            (void)hipEventSynchronize(r.b);
            (void)hipEventElapsedTime(&ms, r.a, r.b);
            double* o = acc + 4 * r.fam;
            o[0] += 1.0;
            o[1] += ms;
            o[2] += r.flop;
            o[3] += r.bytes;
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        recs.clear();
    }
    ~EventProf() override {
        for (auto& r : recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

struct GateFactor {
    int r = 0;
    double* X = nullptr;   // r x D2 x D2 (device)
    double* Y = nullptr;
};

// A two-site map as an update applies it: the caller's input folded with the single-atom maps
// queued on the two atoms, with its operator-Schmidt factors.  Keyed by exactly what determines
// it (input bytes and queued maps), so repeated gates skip the host-side build, fold and
// factorisation.
struct FoldEntry {
    uint64_t id = 0, h = 0, used = 0;
    int kind = 0;                  // 0: superoperator given, 1: Kraus set given
    std::vector<double> in;        // the caller's input as given
    bool ida = true, idb = true;   // nothing queued on atom i / atom i+1
    std::vector<zc> pa, pb;        // the queued maps otherwise
    GateFactor gf;                 // X, Y null: the update takes the explicit path
    std::vector<zc> S;             // the folded superoperator (read by the explicit path)
};
constexpr int FOLD_CACHE_MAX = 64;

// Two-site map that depends on the classes carried by the pair's outer bonds (crosstalk gate):
// the left bond is na consecutive blocks, block alpha at offset lo[alpha] with ln[alpha]
// indices, the right bond nb blocks (ro, rn); block (alpha, beta) of theta receives the
// D2^2 x D2^2 superoperator G[4 alpha + beta] (device, working precision).
template <typename T>
struct BlockGate {
    int na = 1, nb = 1;
    int lo[4] = {0}, ln[4] = {0}, ro[4] = {0}, rn[4] = {0};
    const T* G[16] = {nullptr};
};

}  // namespace

// ====================================================================== context
struct mpdo_ctx_s {
    mpdo_config cfg{};
    int N = 0, d = 0, D2 = 0, chi = 0;
    bool fp32 = false;            // site data and products in FP32 (MPDO_FP32, MPDO_BF16X3)
    bool x3 = false;              // MPDO_BF16X3: the theta products by split-BF16 matrix-core products
    double cutoff = 1e-14;
    hipStream_t st = nullptr;
    std::string err;
    bool poisoned = false;
    long retries = 0;             // updates recomputed after a failed basis check
    bool ready = false;

    // memory
    char* ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    Arena arena;

    // chain
    std::vector<void*> site;      // N site buffers (T), capacity chi*D2*chi
    std::vector<void*> spare;     // 2 spare buffers
    std::vector<int> dims;        // dims[j]: bond between j-1 and j; dims[0] = dims[N] = 1
    int centre = 0;
    int dir = 1;
    std::vector<std::vector<zc>> pending;   // D2 x D2 superoperator queued per atom
    std::vector<char> pend_id;
    double* ovec = nullptr;       // N x D2 complex: trace vector of each atom
    double* Lv = nullptr;         // (N+1) x chi complex
    double* Rv = nullptr;
    int lvalid = 0, rvalid = 0;
    double* Sdev = nullptr;       // D2^2 x D2^2 superoperator (FP64)
    void* SdevT = nullptr;        // same in the working precision
    double* xg = nullptr;         // crosstalk block superoperators (16 x D2^4 complex FP64), on first use
    void* xgT = nullptr;          // the same in the working precision (FP32 mode)
    std::vector<double> xg_src;   // what the blocks in xg were built from (reused when it repeats)
    double* hbuf = nullptr;       // pinned host buffer
    int* hint = nullptr;

    Scratch<double> sd;           // FP64 scratch (all work in FP64 mode; eigen/PPT always)
    Scratch<float> sf;            // FP32 scratch (FP32 mode)
    Scratch<double> sg;           // small FP64 scratch for gate factorisation (D2^2)
    std::vector<FoldEntry> fcache;    // folded two-site maps (at most FOLD_CACHE_MAX)
    uint64_t fclock = 0, fnext = 1;
    uint64_t sdev_id = 0;            // entry whose superoperator is in Sdev / SdevT (0: none)
    const std::vector<zc>* Scur = nullptr;   // host copy of the current update's superoperator
    uint64_t Scur_id = 0;
    std::vector<double*> gslots;     // free device slots for operator-Schmidt factors
    std::unique_ptr<EventProf> prof;   // non-null while measurement is on
    double prof_acc[4 * PF_COUNT] = {0};
    double* obuf = nullptr;       // operator vectors of one expectation term (N x D2)
    double* o2buf = nullptr;      // second-order operators of one term (N x D2 x D2 complex, in T)

    size_t site_cap() const { return (size_t)chi * D2 * chi * 2; }  // in T elements
    size_t tsize() const { return fp32 ? sizeof(float) : sizeof(double); }
};

static thread_local std::string g_create_err;

namespace mpdo {
// Sets the calling thread's context-free message (mpdo_last_error(NULL)); the batch runner
// passes a worker's failure on to the thread that called it.
void set_thread_error(const std::string& msg) { g_create_err = msg; }
}  // namespace mpdo

namespace {

// ====================================================================== generic helpers
template <typename T>
CView<T> V(T* p, long rs, long cs, int conj = 0) {
    return view<T>(p, rs, cs, conj);
}

template <typename T>
struct Engine {
    mpdo_ctx_s& c;
    Scratch<T>& s;
    hipStream_t st;
    int eig_calls = 0;
    int sub_iters = 0;   // subspace-iteration passes of the current update
    // Where the last split found the largest discarded Schmidt value: >= 0, its index in s.sig;
    // -1, the cut was not made by the chi cap (everything discarded lies below the cutoff or
    // the rounding floor); -2 - level, the cap was met with the next value below the threshold
    // of that deflation level (s.st[1 + level], an eigenvalue bound).
    int cut_next = -1;
    bool theta_check = false;   // sc[4..5] (||theta||^2, non-finite count) awaits the next orth_verify

    Engine(mpdo_ctx_s& ctx, Scratch<T>& sc) : c(ctx), s(sc), st(ctx.st) {}

    T* site(int j) { return (T*)c.site[j]; }
    double eps() const { return std::is_same<T, double>::value ? EPS64 : EPS32; }

    void sync() { HIPCHK(hipStreamSynchronize(st)); }

    // the superoperator of the current update into Sdev / SdevT, unless it is there already
    void load_superop() {
        if (!c.Scur) throw Fail{MPDO_E_STATE, "no superoperator for the explicit update"};
        if (c.sdev_id == c.Scur_id) return;
        const int m2 = c.D2 * c.D2;
        HIPCHK(hipMemcpyAsync(c.Sdev, c.Scur->data(), c.Scur->size() * sizeof(zc), hipMemcpyHostToDevice, st));
        if (c.fp32)
            HIPCHK((geam<double, float>(st, m2, m2, C1(), V<double>(c.Sdev, m2, 1), C0(),
                                        V<float>((float*)c.SdevT, m2, 1))));
        sync();
        c.sdev_id = c.Scur_id;
    }

    int read_int(const int* dp) {
        HIPCHK(hipMemcpyAsync(c.hint, dp, sizeof(int), hipMemcpyDeviceToHost, st));
        sync();
        return c.hint[0];
    }
    void read_doubles(const double* dp, int n, double* out) {
        HIPCHK(hipMemcpyAsync(c.hbuf, dp, n * sizeof(double), hipMemcpyDeviceToHost, st));
        sync();
        memcpy(out, c.hbuf, n * sizeof(double));
    }
    // two device arrays (na + nb <= 64 doubles) with one synchronisation; one copy when they lie
    // within 1024 doubles of each other (the small result slots of a scratch do)
    void read_doubles2(const double* da, int na, double* oa, const double* db, int nb, double* ob) {
        const double* lo = std::min(da, db);
        const double* hi = std::max(da + na, db + nb);
        if (hi - lo <= 1024) {
            HIPCHK(hipMemcpyAsync(c.hbuf, lo, (size_t)(hi - lo) * sizeof(double), hipMemcpyDeviceToHost, st));
            sync();
            memcpy(oa, c.hbuf + (da - lo), na * sizeof(double));
            memcpy(ob, c.hbuf + (db - lo), nb * sizeof(double));
            return;
        }
        HIPCHK(hipMemcpyAsync(c.hbuf, da, na * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(c.hbuf + na, db, nb * sizeof(double), hipMemcpyDeviceToHost, st));
        sync();
        memcpy(oa, c.hbuf, na * sizeof(double));
        memcpy(ob, c.hbuf + na, nb * sizeof(double));
    }

    ProfSink* ps() { return c.prof.get(); }

    // product options carrying this scratch's k-split workspace (deterministic split sums)
    GemmOpts wso() const {
        GemmOpts o;
        o.ws = s.skw;
        o.ws_bytes = s.skw_bytes;
        return o;
    }
    // the same for products with theta (its merge, the gate, the subspace iteration's
    // applications): split-BF16 products in MPDO_BF16X3 mode
    GemmOpts xo() const {
        GemmOpts o = wso();
        o.split_bf16 = c.x3;
        return o;
    }
    void gemm(int M, int N, int K, cd a, CView<T> A, CView<T> B, cd b, CView<T> C_, int batch = 1, long sA = 0,
              long sB = 0, long sC = 0) {
        HIPCHK(cgemm_ex<T>(st, M, N, K, a, A, B, b, C_, wso(), ps(), batch, sA, sB, sC));
    }
    // a product with theta (xo())
    void gemm_x(int M, int N, int K, cd a, CView<T> A, CView<T> B, cd b, CView<T> C_) {
        HIPCHK(cgemm_ex<T>(st, M, N, K, a, A, B, b, C_, xo(), ps()));
    }
    // C = A (B diag(f)) for a device array f of N real factors
    void gemm_cols(int M, int N, int K, CView<T> A, CView<T> B, const double* f, CView<T> C_) {
        GemmOpts o = wso();
        o.b_col = f;
        HIPCHK(cgemm_ex<T>(st, M, N, K, C1(), A, B, C0(), C_, o, ps()));
    }

    // Gram G = F^H F (c x c) of the n x c view F, into the FP64 eigen buffer (dense, ld c)
    void gram_cols(CView<T> F, int n, int cc) {
        if (std::is_same<T, double>::value) {
            gemm(cc, cc, n, C1(), adj(F), F, C0(), V<T>((T*)s.Gd, cc, 1));
        } else {
            gemm(cc, cc, n, C1(), adj(F), F, C0(), V<T>(s.bG, cc, 1));
            HIPCHK((geam<T, double>(st, cc, cc, C1(), V<T>(s.bG, cc, 1), C0(), V<double>(s.Gd, cc, 1))));
        }
    }

    // eigen-decomposition of the Gram in s.Gd (order n): s.evals, s.Vd (ld n); s.bVT gets
    // the eigenvectors in T
    void eig(int n) {
        int sw = 0;
        HIPCHK(eigh(st, n, s.Gd, n, s.Vd, n, s.evals, s.eigwork, EIG_MAX_SWEEPS, &sw, c.hint, ps(), eps()));
        ++eig_calls;
        if (sw >= EIG_MAX_SWEEPS) throw Fail{MPDO_E_NUMERIC, "Jacobi eigensolver did not converge"};
        if (!std::is_same<T, double>::value)
            HIPCHK((geam<double, T>(st, n, n, C1(), V<double>(s.Vd, n, 1), C0(), V<T>(s.bVT, n, 1))));
    }

    // Eigenpairs of the Gram in s.Gd (order n) that a deflation level accepts (the rule of
    // spectrum_cut): returns the accepted count; s.sig/s.inv style outputs go to sig/inv, the
    // eigenvectors to columns [0, count) of s.Vd (ld n) and s.bVT.  Orders above EIG_JACOBI_MAX
    // up to TRI_MAX use the tridiagonal solver, which computes only the accepted pairs; smaller
    // orders the one-workgroup Jacobi solver (a round of it costs about 1 us of barriers and
    // LDS latency whatever the order, and a sweep has n - 1 rounds, so from order ~32 on the
    // tridiagonal route is faster: orders 33..48 took 400 us by Jacobi, about 170 us this way).
    int eig_cut(int n, int level, double floor2, double noise, double tau, int cap, double* sig, double* inv) {
        int acc;
        if (n > EIG_JACOBI_MAX && n <= TRI_MAX) {
            HIPCHK(eigh_top(st, n, s.Gd, n, level, floor2, noise, tau, cap, s.st, s.cnt, s.evals, sig, inv, s.Vd, n,
                            s.eigwork, ps()));
            ++eig_calls;
            acc = read_int(s.cnt);
            if (!std::is_same<T, double>::value && acc > 0)
                HIPCHK((geam<double, T>(st, n, acc, C1(), V<double>(s.Vd, n, 1), C0(), V<T>(s.bVT, n, 1))));
        } else if (n <= EIG_JACOBI_MAX) {
            // one workgroup solves to convergence; its sweep count is read together with the
            // accepted count, in one synchronisation
            HIPCHK(eigh(st, n, s.Gd, n, s.Vd, n, s.evals, s.eigwork, EIG_MAX_SWEEPS, nullptr, c.hint, ps(), eps()));
            ++eig_calls;
            if (!std::is_same<T, double>::value)
                HIPCHK((geam<double, T>(st, n, n, C1(), V<double>(s.Vd, n, 1), C0(), V<T>(s.bVT, n, 1))));
            HIPCHK(spectrum_cut(st, s.evals, n, level, floor2, noise, tau, cap, s.st, s.cnt, sig, inv));
            HIPCHK(hipMemcpyAsync(c.hint, s.cnt, sizeof(int), hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(c.hint + 1, eigh_sweep_counter(s.eigwork, n), sizeof(int), hipMemcpyDeviceToHost,
                                  st));
            sync();
            if (c.hint[1] >= EIG_MAX_SWEEPS) throw Fail{MPDO_E_NUMERIC, "Jacobi eigensolver did not converge"};
            acc = c.hint[0];
        } else {
            eig(n);
            HIPCHK(spectrum_cut(st, s.evals, n, level, floor2, noise, tau, cap, s.st, s.cnt, sig, inv));
            acc = read_int(s.cnt);
        }
        return acc;
    }

    // relative eigenvalue noise of a Gram matrix of order n formed in this precision
    double noise_of(int n) const { return std::max(64.0, 4.0 * n) * eps(); }

    // Every orthonormal basis the split builds is checked: ||Q||_F^2 of its q columns is reduced
    // on the device (orth_check) and compared with q at the end of the update (orth_verify, one
    // read for all of them).  A basis off by more than 1e-9 (FP64) or 1e-3 (FP32), or with
    // non-finite entries, means the eigenvectors it came from were not accurate enough for the
    // range refinement and Newton-Schulz steps: the update fails with E_NUMERIC instead of
    // writing a wrong state.  MPDO_DEBUG_CHECKS=1 prints every check to stderr.
    static constexpr int NCHK = 64;
    int nchk = 0;
    int chk_q[NCHK], chk_order[NCHK], chk_level[NCHK];
    const char* chk_stage[NCHK];
    void orth_check(const char* stage, T* Q, long ldq, int n, int q, int level, int order) {
        if (q <= 0) return;
        if (nchk == NCHK) orth_verify();
        HIPCHK(sumsq<T>(st, V<T>(Q, ldq, 1), n, q, s.odev + 2 * nchk, s.sqp, s.sqc));
        chk_q[nchk] = q;
        chk_order[nchk] = order;
        chk_level[nchk] = level;
        chk_stage[nchk] = stage;
        ++nchk;
    }
    void orth_verify() {
        const bool dbg = getenv("MPDO_DEBUG_CHECKS") != nullptr;
        if (nchk == 0 && !theta_check) return;
        const int m = nchk;
        nchk = 0;
        double buf[2 * NCHK], th[2] = {0.0, 0.0};
        if (theta_check) {
            // ||theta||^2 and the non-finite count of the merged tensor (sc[4..5]) in the same copy
            read_doubles2(s.odev, 2 * std::max(m, 1), buf, s.sc + 4, 2, th);
            theta_check = false;
            if (th[1] != 0.0) throw Fail{MPDO_E_NUMERIC, "non-finite entries in the merged tensor"};
        } else {
            read_doubles(s.odev, 2 * m, buf);
        }
        const double tol = std::is_same<T, double>::value ? 1e-9 : 1e-3;
        for (int k = 0; k < m; ++k) {
            const double dev = buf[2 * k] / chk_q[k] - 1.0;
            if (dbg)
                fprintf(stderr, "[mpdo check] %s level %d order %d cols %d |Q|^2/q - 1 = %.3e nonfinite %g\n",
                        chk_stage[k], chk_level[k], chk_order[k], chk_q[k], dev, buf[2 * k + 1]);
            if (buf[2 * k + 1] != 0.0 || !(fabs(dev) <= tol)) {
                char msg[256];
                snprintf(msg, sizeof(msg),
                         "orthonormal basis lost accuracy in the split (%s, level %d, order %d, %d columns: "
                         "|Q|^2/q - 1 = %.3e, non-finite %g)",
                         chk_stage[k], chk_level[k], chk_order[k], chk_q[k], dev, buf[2 * k + 1]);
                throw Fail{MPDO_E_NUMERIC, msg, true};
            }
        }
    }

    // Newton-Schulz steps after each range refinement.  A step maps a deviation E = X^H X - I to
    // about -3/4 E^2, and the refined columns start within ~1e-3 of orthonormal (about
    // eps lambda_max / lambda_j), so two steps reach the basis check's bar; the two-site update
    // takes two (an even count also leaves the result in place), and three, or four when an
    // update is recomputed after a failed check, elsewhere.
    int ns_iters = 3;
    // Range bases by pivoted Cholesky (orth2).  On for the first computation of a two-site
    // update; a recomputation after a failed basis check takes the Gram eigendecomposition.
    bool orth_pchol = false;

    // Newton-Schulz: make the n x q columns of Q (view, dense storage in buffer with ld) orthonormal,
    // X <- X (3/2 I - 1/2 X^H X), alternating between Q and the scratch bW (ld q)
    void ns_orth(T* Q, long ldq, int n, int q, int iters) {
        T* cur = Q;
        long ldc = ldq;
        for (int it = 0; it < iters; ++it) {
            gemm(q, q, n, C1(), adj(V<T>(cur, ldc, 1)), V<T>(cur, ldc, 1), C0(), V<T>(s.bG, q, 1));
            T* nxt = cur == Q ? s.bW : Q;
            const long ldn = cur == Q ? (long)q : ldq;
            GemmOpts o = wso();
            o.b_scale = -0.5;
            o.b_diag = 1.5;
            HIPCHK(cgemm_ex<T>(st, n, q, q, C1(), V<T>(cur, ldc, 1), V<T>(s.bG, q, 1), C0(), V<T>(nxt, ldn, 1), o,
                               ps()));
            cur = nxt;
            ldc = ldn;
        }
        if (cur != Q) HIPCHK((geam<T, T>(st, n, q, C1(), V<T>(cur, ldc, 1), C0(), V<T>(Q, ldq, 1))));
    }

    // Orthonormal basis of range(F) for the n x cc view F, up to three Gram levels: level 0
    // takes the well-conditioned directions (lambda > 1e-10 lambda_max in FP64, 1e-5 in FP32),
    // each further level the residual F - Q Q^H F down to the cutoff or the residual's rounding
    // floor, so that F = Q K holds to rounding.  With orth_pchol (orders <= PCHOL_MAX) a level
    // takes the columns of a pivoted Cholesky factorisation of its Gram instead of accepted
    // eigenvectors: the same contract (F = Q K to rounding, Q orthonormal, checked), at the
    // cost of the accepted pivots instead of a tridiagonal reduction of order cc.
    // Q: n x q written to Qb (ld cc); K = Q^H F: q x cc written to Kb (ld cc).  Uses bT1.
    int orth2(CView<T> F, int n, int cc, T* Qb, T* Kb) {
        const double e = eps();
        const int qmax = std::min(n, cc);
        const double tau0 = std::is_same<T, double>::value ? 1e-10 : 1e-5;
        // deeper levels stop at the residual's rounding floor (8 eps ||F||_F, set after
        // level 0 as a fraction of lambda_max): content above it is kept so that F = Q K
        // holds to rounding whatever the later cut of the product
        double floor2 = 0.0, fro2 = 0.0;
        CView<T> R = F;
        int q = 0;
        const bool f64 = std::is_same<T, double>::value;
        const bool pc = orth_pchol && cc <= PCHOL_MAX;
        // FP32 pivots stop at 1e-5 of a level's trace (the Cholesky QR error grows as eps32 / rel),
        // so it takes a fourth level to reach the depth three eigen levels reach
        const int nlev = pc && !f64 ? 4 : 3;
        for (int lev = 0; lev < nlev; ++lev) {
            gram_cols(R, n, cc);
            int acc;
            if (pc) {
                // pivots while the Schur-complement diagonal exceeds rel * trace: the chosen
                // columns' squared condition number stays near 1/rel, so the Cholesky QR basis
                // starts within ~1e-5 (FP64) or ~1e-3 (FP32) of orthonormal.  FP64: 1e-10 at
                // level 0, 1e-12 on the residual levels, which reach the rounding floor in three
                // levels; FP32: 1e-5 (level 0: at least the Gram's rounding noise)
                const double rel = lev == 0 ? std::max(tau0, noise_of(cc)) : (f64 ? 1e-12 : tau0);
                HIPCHK(pchol_basis<T>(st, s.Gd, cc, cc, lev, lev == 0 ? 0.0 : floor2, rel, lev == 0 ? qmax : qmax - q,
                                      s.st, s.cnt, s.pcw, s.bVT, cc, ps()));
                acc = read_int(s.cnt);
                if (ps()) ps()->amend(PF_PCHOL, pchol_flop(cc, acc), pchol_bytes(cc, acc));
            } else {
                acc = lev == 0 ? eig_cut(cc, 0, 0.0, noise_of(cc), tau0, qmax, nullptr, s.inv)
                               : eig_cut(cc, lev, floor2, 4096.0 * e, 0.0, qmax - q, nullptr, s.inv);
            }
            if (acc <= 0) break;
            // new columns R W (pivoted Cholesky: W = P L11^{-H}; eigenvectors: W diag(lambda^-1/2)),
            // made orthogonal to the earlier ones
            T* Qn = Qb + 2 * q;
            if (pc)
                gemm(n, acc, cc, C1(), R, V<T>(s.bVT, cc, 1), C0(), V<T>(Qn, cc, 1));
            else
                gemm_cols(n, acc, cc, R, V<T>(s.bVT, cc, 1), s.inv, V<T>(Qn, cc, 1));
            if (q > 0) {
                gemm(q, acc, n, C1(), adj(V<T>(Qb, cc, 1)), V<T>(Qn, cc, 1), C0(), V<T>(s.bG, acc, 1));
                gemm(n, acc, q, Cr(-1.0), V<T>(Qb, cc, 1), V<T>(s.bG, acc, 1), C1(), V<T>(Qn, cc, 1));
            }
            ns_orth(Qn, cc, n, acc, ns_iters);
            orth_check("orth2", Qn, cc, n, acc, lev, cc);
            gemm(acc, cc, n, C1(), adj(V<T>(Qn, cc, 1)), F, C0(), V<T>(Kb + 2 * (long)q * cc, cc, 1));
            q += acc;
            if (q >= qmax || lev == nlev - 1) break;
            // residual F - Q K, projected out of range(Q) a second time (its rounding inside
            // range(Q), ~eps sqrt(q) ||F||, would otherwise return as deep-level directions that
            // the projection of the new columns leaves short and nearly dependent); stop once
            // nothing above the cutoff is left
            HIPCHK((geam<T, T>(st, n, cc, C1(), F, C0(), V<T>(s.bT1, cc, 1))));
            gemm(n, cc, q, Cr(-1.0), V<T>(Qb, cc, 1), V<T>(Kb, cc, 1), C1(), V<T>(s.bT1, cc, 1));
            gemm(q, cc, n, C1(), adj(V<T>(Qb, cc, 1)), V<T>(s.bT1, cc, 1), C0(), V<T>(s.bW, cc, 1));
            gemm(n, cc, q, Cr(-1.0), V<T>(Qb, cc, 1), V<T>(s.bW, cc, 1), C1(), V<T>(s.bT1, cc, 1));
            if (pc) {
                // no read here: the next level's pivots are tested against the floor
                // 64 eps^2 ||F||_F^2 on the device (level 0 left trace(G) = ||F||_F^2 in st[0]
                // and st[4]), and a residual below it gives no pivot
                floor2 = 64.0 * e * e;
                R = V<T>(s.bT1, cc, 1);
                continue;
            }
            HIPCHK(sumsq<T>(st, V<T>(s.bT1, cc, 1), n, cc, s.sums, s.sqp, s.sqc));
            double sums[2], st5[5];
            read_doubles2(s.sums, 2, sums, s.st, 5, st5);
            if (lev == 0) {
                fro2 = st5[4];
                floor2 = st5[0] > 0.0 ? 64.0 * e * e * fro2 / st5[0] : 0.0;
            }
            if (!(sums[0] > 64.0 * e * e * fro2)) break;
            R = V<T>(s.bT1, cc, 1);
        }
        return q;
    }

    // Orthonormal basis of range(Y) for an n x m block (n >= m, m <= CHOL_MAX) whose condition
    // number is below ~1/eps64, by shifted Cholesky QR (one pass with the shift, two without):
    // Gram products, 64-wide Cholesky blocks and block triangular solves, no eigenproblem.  The
    // passes run in FP64 (an FP32 block is widened first and the basis rounded back, so FP32
    // rounding of Y only adds noise directions far below its cut).  Y (ld m) is overwritten; Q
    // (n x m, ld m) receives the basis.  Returns false when a pivot broke down or the result is
    // not orthonormal (a block too close to rank deficiency): the caller then uses orth2 on the
    // input, recomputed.
    bool orth_chol(T* Y, int n, int m, T* Q) {
        if (m > CHOL_MAX || m > n || m < 1) return false;
        const bool f64 = std::is_same<T, double>::value;
        double* Yd = f64 ? (double*)Y : s.Gd;
        double* Qd = f64 ? (double*)Q : s.Vd;
        double* G = f64 ? s.Gd : (double*)s.bG;
        double* L = f64 ? s.Vd : (double*)s.bW;
        if (!f64) HIPCHK((geam<T, double>(st, n, m, C1(), V<T>(Y, m, 1), C0(), V<double>(Yd, m, 1))));
        int* flag = s.cnt + 32;
        HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), st));
        const double coef = 11.0 * ((double)n * m + (double)m * (m + 1)) * EPS64;
        double* in = Yd;
        double* out = Qd;
        for (int pass = 0; pass < 3; ++pass) {
            HIPCHK(cgemm_ex<double>(st, m, m, n, C1(), adj(V<double>(in, m, 1)), V<double>(in, m, 1), C0(),
                                    V<double>(G, m, 1), wso(), ps()));
            HIPCHK(cholesky_lower(st, G, m, m, pass == 0 ? coef : 0.0, L, m, s.cholw, flag, wso(), ps()));
            HIPCHK(trsm_right_lower_adj(st, in, m, n, m, L, m, s.cholw, out, m, wso(), ps()));
            std::swap(in, out);
        }
        // an odd number of passes leaves the basis in Qd
        if (!f64) HIPCHK((geam<double, T>(st, n, m, C1(), V<double>(Qd, m, 1), C0(), V<T>(Q, m, 1))));
        HIPCHK(sumsq<T>(st, V<T>(Q, m, 1), n, m, s.sums, s.sqp, s.sqc));
        HIPCHK(hipMemcpyAsync(c.hint, flag, sizeof(int), hipMemcpyDeviceToHost, st));
        double w[2];
        read_doubles(s.sums, 2, w);
        const double tol = f64 ? 1e-12 : 1e-5;
        const bool ok = c.hint[0] == 0 && w[1] == 0.0 && fabs(w[0] / m - 1.0) <= tol;
        if (getenv("MPDO_DEBUG_CHECKS"))
            fprintf(stderr, "[mpdo check] cholqr order %d cols %d |Q|^2/q - 1 = %.3e breakdown %d -> %s\n", n, m,
                    w[0] / m - 1.0, c.hint[0], ok ? "ok" : "orth2");
        return ok;
    }

    // Orthonormal basis Q (na x q) of the dominant left singular subspace of the na x nb view
    // Th (theta), for splits whose exact range basis would need an eigenproblem above TRI_MAX
    // (the saturated regime: theta up to 8192 x 8192 of rank 4608).  Block subspace iteration
    // from a seeded random block of m = min(chi + SUB_OVER, na, nb) columns: Q = orth(theta X);
    // then repeatedly Z = orth(theta^H Q), Q = orth(theta Z).  Every block is orthonormalised
    // by orth2 (eigenproblems of order <= m), so a block never spans more than the
    // sigma_max / sigma_j of one application and directions down to orth2's rounding floor
    // survive.  Stops when ||Q^H theta||_F^2, the weight of theta captured by Q, grows by less
    // than the tolerance, or at once when m reaches min(na, nb) (one pass then spans
    // range(theta)).  The later cut keeps at most chi directions of this basis, so what the
    // basis misses lies below the truncation; PPT still reads ||theta||_F^2 and tr(rho) of
    // the whole theta.
    // Outputs: Q -> Qout (ld ldq), Q^H theta -> Kout (q x nb, ld ldk).
    int subspace_basis(CView<T> Th, int na, int nb, int chi, uint64_t seed, T* Qout, long ldq, T* Kout, long ldk) {
        const int rank_bound = std::min(na, nb);
        const int m = std::min(chi + SUB_OVER, rank_bound);
        const double tol = std::is_same<T, double>::value ? 1e-10 : 1e-6;
        T* X = s.bR;     // nb x cols: random start block, then orth(theta^H Q)
        T* Y = s.bC;     // na x cols
        T* Qt = s.bQ2;   // orth2's basis of Y (ld cols)
        T* Kt = s.bK2;   // orth2's coefficients (unused)
        T* Cq = s.bU2;   // Q^H theta (q x nb, ld nb)
        HIPCHK(fill_random<T>(st, V<T>(X, m, 1), nb, m, seed));
        gemm_x(na, m, nb, C1(), Th, V<T>(X, m, 1), C0(), V<T>(Y, m, 1));
        int cols = m, q = 0;
        double w_old = -1.0;
        for (int it = 0;; ++it) {
            // Y = theta X (X: the start block, then Z): shifted Cholesky QR, or orth2 where the
            // block is too close to rank deficiency for it
            if (orth_chol(Y, na, cols, Qt)) {
                q = cols;
            } else {
                gemm_x(na, cols, nb, C1(), Th, V<T>(X, cols, 1), C0(), V<T>(Y, cols, 1));
                q = orth2(V<T>(Y, cols, 1), na, cols, Qt, Kt);
            }
            if (q <= 0) return 0;
            gemm_x(q, nb, na, C1(), adj(V<T>(Qt, cols, 1)), Th, C0(), V<T>(Cq, nb, 1));
            ++sub_iters;
            if (m >= rank_bound) break;
            HIPCHK(sumsq<T>(st, V<T>(Cq, nb, 1), q, nb, s.sums, s.sqp, s.sqc));
            double w[2];
            read_doubles(s.sums, 2, w);
            if (w[1] != 0.0) throw Fail{MPDO_E_NUMERIC, "non-finite entries in the subspace iteration"};
            if ((w_old >= 0.0 && w[0] - w_old <= tol * w[0]) || it + 1 >= SUB_ITERS) break;
            w_old = w[0];
            // Z = orth(theta^H Q) (nb x z), then Y = theta Z
            HIPCHK((geam<T, T>(st, nb, q, C1(), adj(V<T>(Cq, nb, 1)), C0(), V<T>(Kt, q, 1))));
            int z = q;
            if (!orth_chol(Kt, nb, q, X)) z = orth2(adj(V<T>(Cq, nb, 1)), nb, q, X, Kt);
            if (z <= 0) return 0;
            gemm_x(na, z, nb, C1(), Th, V<T>(X, q, 1), C0(), V<T>(Y, z, 1));
            cols = z;
        }
        HIPCHK((geam<T, T>(st, na, q, C1(), V<T>(Qt, cols, 1), C0(), V<T>(Qout, ldq, 1))));
        HIPCHK((geam<T, T>(st, q, nb, C1(), V<T>(Cq, nb, 1), C0(), V<T>(Kout, ldk, 1))));
        return q;
    }

    // Left split of the a x b view F: U (a x kept) into Ub (ld chi_cap), Schmidt values in
    // s.sig, B = U^H F (kept x b) into Bb (ld b).  Up to three deflation levels.
    int split_left(CView<T> F, int a, int b, int chi, T* Ub, long ldu, T* Bb) {
        const double e = eps();
        int kacc = 0;
        cut_next = -1;
        double rfloor = 0.0;   // residual rounding floor 8 eps ||F||_F, as a fraction of lambda_max
        CView<T> R = F;
        for (int lev = 0; lev < 3; ++lev) {
            // H = R R^H (a x a)
            if (std::is_same<T, double>::value) {
                gemm(a, a, b, C1(), R, adj(R), C0(), V<T>((T*)s.Gd, a, 1));
            } else {
                gemm(a, a, b, C1(), R, adj(R), C0(), V<T>(s.bG, a, 1));
                HIPCHK((geam<T, double>(st, a, a, C1(), V<T>(s.bG, a, 1), C0(), V<double>(s.Gd, a, 1))));
            }
            // level 0 accepts lambda > 1e-6 lambda_max (sigma > 1e-3 sigma_max); what lies below is
            // resolved by the residual levels with a smaller backward error
            const double tau = (lev == 0) ? 1e-6 : 0.0;
            // one pair beyond the chi cap is asked for: when it is accepted, the cap decides the
            // cut at this level and its value is the largest discarded Schmidt value, left in
            // s.sig[chi] (the gap at the cut; ties there make the truncated state non-unique)
            const int cap = chi - kacc;
            const int accd = eig_cut(a, lev, std::max(c.cutoff * c.cutoff, rfloor), noise_of(a), tau,
                                     std::min(cap + 1, a), s.sig + kacc, s.inv);
            const int acc = std::min(accd, cap);
            if (accd > cap) cut_next = kacc + acc;
            else if (kacc + acc >= chi) cut_next = -2 - lev;   // capped, next value below the level threshold
            if (acc <= 0) break;
            T* Vn = Ub + 2 * kacc;   // columns kacc.. of U
            // Eigenvectors of R R^H lean out of range(R) by about eps lambda_max / lambda_j; the
            // next residual would carry that lean as directions of size eps sigma_max^2 / sigma_j
            // and the cut would keep them as spurious Schmidt values.  One pass
            // V <- R (R^H V) diag(1/lambda) puts the columns back into range(R) to rounding.
            gemm_cols(b, acc, a, adj(R), V<T>(s.bVT, a, 1), s.inv, V<T>(s.bT1, acc, 1));
            gemm_cols(a, acc, b, R, V<T>(s.bT1, acc, 1), s.inv, V<T>(Vn, ldu, 1));
            if (kacc > 0) {
                gemm(kacc, acc, a, C1(), adj(V<T>(Ub, ldu, 1)), V<T>(Vn, ldu, 1), C0(), V<T>(s.bG, acc, 1));
                gemm(a, acc, kacc, Cr(-1.0), V<T>(Ub, ldu, 1), V<T>(s.bG, acc, 1), C1(), V<T>(Vn, ldu, 1));
            }
            ns_orth(Vn, ldu, a, acc, ns_iters);
            orth_check("split", Vn, ldu, a, acc, lev, a);
            kacc += acc;
            if (kacc >= chi || kacc >= a || lev == 2) break;
            // residual R = F - U (U^H F), projected twice (as in orth2); Bb is rebuilt at the end
            gemm(kacc, b, a, C1(), adj(V<T>(Ub, ldu, 1)), F, C0(), V<T>(Bb, b, 1));
            HIPCHK((geam<T, T>(st, a, b, C1(), F, C0(), V<T>(s.bR, b, 1))));
            gemm(a, b, kacc, Cr(-1.0), V<T>(Ub, ldu, 1), V<T>(Bb, b, 1), C1(), V<T>(s.bR, b, 1));
            gemm(kacc, b, a, C1(), adj(V<T>(Ub, ldu, 1)), V<T>(s.bR, b, 1), C0(), V<T>(Bb, b, 1));
            gemm(a, b, kacc, Cr(-1.0), V<T>(Ub, ldu, 1), V<T>(Bb, b, 1), C1(), V<T>(s.bR, b, 1));
            HIPCHK(sumsq<T>(st, V<T>(s.bR, b, 1), a, b, s.sums, s.sqp, s.sqc));
            double sums[2], st5[5];
            read_doubles2(s.sums, 2, sums, s.st, 5, st5);
            // the residual R = F - U U^H F carries rounding of about eps ||F||_F: values below
            // 8 eps ||F||_F are not spectrum
            if (lev == 0 && st5[0] > 0.0) rfloor = 64.0 * e * e * st5[4] / st5[0];
            if (!(sums[0] > std::max(c.cutoff * c.cutoff, rfloor) * st5[0])) break;
            R = V<T>(s.bR, b, 1);
        }
        if (kacc == 0) return 0;
        gemm(kacc, b, a, C1(), adj(V<T>(Ub, ldu, 1)), F, C0(), V<T>(Bb, b, 1));
        return kacc;
    }

    // Left singular vectors of the a x b view F without an eigenproblem larger than
    // min(a, b): a tall F is first compressed to an orthonormal basis Q of its range
    // (Gram of the short side), F = Q K, and the split runs on the q x b core K.
    // U (a x kept) -> Uout (ld kept), B = U^H F (kept x b) -> s.bB2, values in s.sig.
    int svd_left(CView<T> F, int a, int b, int chi, T* Uout) {
        if (a > b) {
            const int q = orth2(F, a, b, s.bQ2, s.bK2);
            if (q <= 0) return 0;
            const int kept = split_left(V<T>(s.bK2, b, 1), q, b, chi, s.bU, c.chi, s.bB2);
            if (kept <= 0) return 0;
            gemm(a, kept, q, C1(), V<T>(s.bQ2, b, 1), V<T>(s.bU, c.chi, 1), C0(), V<T>(Uout, kept, 1));
            return kept;
        }
        const int kept = split_left(F, a, b, chi, s.bU, c.chi, s.bB2);
        if (kept > 0)
            HIPCHK((geam<T, T>(st, a, kept, C1(), V<T>(s.bU, c.chi, 1), C0(), V<T>(Uout, kept, 1))));
        return kept;
    }

    // ------------------------------------------------------------ trace vectors
    double* Lv(int j) { return c.Lv + (size_t)j * c.chi * 2; }
    double* Rv(int j) { return c.Rv + (size_t)j * c.chi * 2; }

    double tbytes(int j) const { return 2.0 * sizeof(T) * c.dims[j] * (double)c.D2 * c.dims[j + 1]; }
    void ensureL(int i) {
        for (int j = c.lvalid; j < i; ++j) {
            if (ps()) ps()->begin(st, PF_TRANSFER);
            HIPCHK(transfer_left<T>(st, site(j), c.dims[j], c.D2, c.dims[j + 1], Lv(j), c.ovec + 2 * j * c.D2,
                                    Lv(j + 1)));
            if (ps()) ps()->end(st, PF_TRANSFER, 8.0 * c.dims[j] * (double)c.D2 * c.dims[j + 1], tbytes(j));
        }
        if (i > c.lvalid) c.lvalid = i;
    }
    void ensureR(int i) {
        for (int j = c.rvalid - 1; j >= i; --j) {
            if (ps()) ps()->begin(st, PF_TRANSFER);
            HIPCHK(transfer_right<T>(st, site(j), c.dims[j], c.D2, c.dims[j + 1], Rv(j + 1), c.ovec + 2 * j * c.D2,
                                     Rv(j)));
            if (ps()) ps()->end(st, PF_TRANSFER, 8.0 * c.dims[j] * (double)c.D2 * c.dims[j + 1], tbytes(j));
        }
        if (i < c.rvalid) c.rvalid = i;
    }
    void site_changed(int j) {
        c.lvalid = std::min(c.lvalid, j);
        c.rvalid = std::max(c.rvalid, j + 1);
    }

    // ------------------------------------------------------------ canonical moves
    void swap_site(int j, int spare_idx) { std::swap(c.site[j], c.spare[spare_idx]); }

    // site j <- P applied on its physical index (P: D2 x D2 device matrix, row = new index)
    void apply_phys(int j, const T* P) {
        const int cl = c.dims[j], cr = c.dims[j + 1], D2 = c.D2;
        gemm(D2, cr, D2, C1(), V<T>((T*)P, D2, 1), V<T>(site(j), cr, 1), C0(), V<T>((T*)c.spare[0], cr, 1), cl, 0,
             (long)D2 * cr, (long)D2 * cr);
        swap_site(j, 0);
        site_changed(j);
    }
    // site j enlarged by class_expand (mode, ncls); the caller updates the bond dimension
    void expand(int j, int mode, int ncls, const EtaClass& cls) {
        HIPCHK(class_expand<T>(st, site(j), c.dims[j], c.D2, c.dims[j + 1], mode, ncls, cls, (T*)c.spare[0]));
        swap_site(j, 0);
        site_changed(j);
    }

    void move_right(int j) {
        const int cl = c.dims[j], cr = c.dims[j + 1], cr2 = c.dims[j + 2];
        const int n = cl * c.D2;
        CView<T> F = V<T>(site(j), cr, 1);
        const int q = orth2(F, n, cr, s.bQ, s.bK);
        if (q <= 0) throw Fail{MPDO_E_NUMERIC, "zero site tensor"};
        T* nq = (T*)c.spare[0];
        HIPCHK((geam<T, T>(st, n, q, C1(), V<T>(s.bQ, cr, 1), C0(), V<T>(nq, q, 1))));
        T* nx = (T*)c.spare[1];
        const int m2 = c.D2 * cr2;
        gemm(q, m2, cr, C1(), V<T>(s.bK, cr, 1), V<T>(site(j + 1), m2, 1), C0(), V<T>(nx, m2, 1));
        swap_site(j, 0);
        swap_site(j + 1, 1);
        c.dims[j + 1] = q;
        site_changed(j);
        site_changed(j + 1);
        c.centre = j + 1;
    }

    void move_left(int j) {
        const int cl = c.dims[j], cr = c.dims[j + 1], cl0 = c.dims[j - 1];
        const int m = c.D2 * cr;
        // site_j^H = Q K  (m x cl view of the adjoint)
        CView<T> F = adj(V<T>(site(j), m, 1));
        const int q = orth2(F, m, cl, s.bQ, s.bK);
        if (q <= 0) throw Fail{MPDO_E_NUMERIC, "zero site tensor"};
        T* nq = (T*)c.spare[0];
        HIPCHK((geam<T, T>(st, q, m, C1(), adj(V<T>(s.bQ, cl, 1)), C0(), V<T>(nq, m, 1))));
        T* nx = (T*)c.spare[1];
        const int n0 = cl0 * c.D2;
        gemm(n0, q, cl, C1(), V<T>(site(j - 1), cl, 1), adj(V<T>(s.bK, cl, 1)), C0(), V<T>(nx, q, 1));
        swap_site(j, 0);
        swap_site(j - 1, 1);
        c.dims[j] = q;
        site_changed(j);
        site_changed(j - 1);
        c.centre = j - 1;
    }

    // ------------------------------------------------------------ the two-site update
    void update(int i, const GateFactor* gf, int chi, mpdo_trunc_info* info, const BlockGate<T>* bg = nullptr) {
        eig_calls = 0;
        sub_iters = 0;
        const int D2 = c.D2;
        if (c.centre < i) c.dir = 1;
        else if (c.centre > i + 1) c.dir = -1;
        while (c.centre < i) move_right(c.centre);
        while (c.centre > i + 1) move_left(c.centre);
        const int dir = c.dir;
        const int cl = c.dims[i], cm = c.dims[i + 1], cr = c.dims[i + 2];
        const int nL = cl * D2, nR = D2 * cr;
        ensureL(i);
        ensureR(i + 2);
        // trace vectors over the two sides: lvec = L_i (x) vec(I), rvec = vec(I) (x) R_{i+2}
        // (the atoms' queued maps were folded into the gate, so their trace vector is vec(I))
        HIPCHK(kron_vec(st, Lv(i), cl, c.ovec + 2 * (size_t)c.N * D2, D2, s.lvec));
        HIPCHK(kron_vec(st, c.ovec + 2 * (size_t)c.N * D2, D2, Rv(i + 2), cr, s.rvec));

        const int na = dir > 0 ? nL : nR;
        const int nb = dir > 0 ? nR : nL;
        const int r = gf ? gf->r : 0;
        // The factored split needs an exact range basis of M_L (eigenproblems of order r chi_mid).
        // Where that order is above the subspace switch, theta is formed instead: the subspace
        // iteration then runs on theta itself (one product per application instead of two), and
        // ||theta||_F^2 and tr(rho), which PPT reads (Eq. (xiformula)), are those of the whole
        // merged tensor, not of the part the subspace captures.
        const bool factored = !bg && gf && r <= MAX_FACTOR_RANK && (long)r * cm < (long)na &&
                              (long)r * cm <= (long)subspace_min_order();
        int kept = 0;
        double n2 = 0.0;
        T* Left = nullptr;   // new site i  (nL x kept), unscaled
        T* Right = nullptr;  // new site i+1 (kept x nR), unscaled
        T* outL = (T*)c.spare[0];
        T* outR = (T*)c.spare[1];
        if (factored) {
            const int k = r * cm;
            // M_L (nL x k) in bA, M_R (k x nR) in bB
            if (ps()) ps()->begin(st, PF_PHYS);
            HIPCHK(phys_left<T>(st, site(i), cl, D2, cm, gf->X, r, s.bA));
            HIPCHK(phys_right<T>(st, site(i + 1), cm, D2, cr, gf->Y, r, s.bB));
            if (ps())
                ps()->end(st, PF_PHYS, 8.0 * D2 * (double)D2 * r * cm * (cl + cr),
                          2.0 * sizeof(T) * ((double)cl * D2 * cm + (double)cm * D2 * cr) * (1.0 + r));
            CView<T> ML = V<T>(s.bA, k, 1), MR = V<T>(s.bB, nR, 1);
            // tr rho = (lvec^T M_L)(M_R rvec)
            HIPCHK(gemv_left<T>(st, ML, nL, k, s.lvec, s.vtmp));
            HIPCHK(gemv_left<T>(st, trans(MR), nR, k, s.rvec, s.vtmp2));
            HIPCHK(dot(st, s.vtmp, s.vtmp2, k, s.sc));
            CView<T> Fa = dir > 0 ? ML : adj(MR);
            CView<T> Fb = dir > 0 ? MR : adj(ML);
            const int q = orth2(Fa, na, k, s.bQ, s.bK);
            if (q <= 0) throw Fail{MPDO_E_NUMERIC, "merged tensor vanished"};
            // core C = K Fb (q x nb)
            gemm(q, nb, k, C1(), V<T>(s.bK, k, 1), Fb, C0(), V<T>(s.bC, nb, 1));
            // ||theta||^2 (= ||C||^2) and its non-finite count stay in sc[4..5] for PPT
            HIPCHK(sumsq<T>(st, V<T>(s.bC, nb, 1), q, nb, s.sc + 4, s.sqp, s.sqc));
            theta_check = true;   // its non-finite count is read with the basis checks
            kept = svd_left(V<T>(s.bC, nb, 1), q, nb, chi, s.bU2);
            if (kept <= 0) throw Fail{MPDO_E_NUMERIC, "empty spectrum"};
            if (dir > 0) {
                gemm(nL, kept, q, C1(), V<T>(s.bQ, k, 1), V<T>(s.bU2, kept, 1), C0(), V<T>(outL, kept, 1));
                HIPCHK((geam<T, T>(st, kept, nR, C1(), V<T>(s.bB2, nR, 1), C0(), V<T>(outR, nR, 1))));
            } else {
                // new site i+1 = U^H = Uc^H Q^H ; new site i = B^H
                gemm(kept, nR, q, C1(), adj(V<T>(s.bU2, kept, 1)), adj(V<T>(s.bQ, k, 1)), C0(), V<T>(outR, nR, 1));
                HIPCHK((geam<T, T>(st, nL, kept, C1(), adj(V<T>(s.bB2, nL, 1)), C0(), V<T>(outL, kept, 1))));
            }
        } else {
            // explicit theta: merge then gate
            const int m2 = D2 * D2;
            ProfRename th(ps(), PF_GEMM, PF_THETA);
            ProfSink* tps = ps() ? &th : nullptr;
            HIPCHK(cgemm_ex<T>(st, nL, nR, cm, C1(), V<T>(site(i), cm, 1), V<T>(site(i + 1), nR, 1), C0(),
                               V<T>(s.bT1, nR, 1), xo(), tps));
            if (bg) {
                // theta[l][eta eta'][r] as cl blocks of m2 x cr: block (alpha, beta) = rows
                // l in [lo, lo + ln) of alpha, columns r in [ro, ro + rn) of beta
                for (int a = 0; a < bg->na; ++a)
                    for (int b = 0; b < bg->nb; ++b) {
                        if (bg->ln[a] <= 0 || bg->rn[b] <= 0) continue;
                        const long off = 2 * ((long)bg->lo[a] * m2 * cr + (long)bg->ro[b]);
                        HIPCHK(cgemm_ex<T>(st, m2, bg->rn[b], m2, C1(), V<T>((T*)bg->G[4 * a + b], m2, 1),
                                           V<T>(s.bT1 + off, cr, 1), C0(), V<T>(s.bA + off, cr, 1), xo(), tps,
                                           bg->ln[a], 0, (long)m2 * cr, (long)m2 * cr));
                    }
            } else {
                load_superop();
                HIPCHK(cgemm_ex<T>(st, m2, cr, m2, C1(), V<T>((T*)c.SdevT, m2, 1), V<T>(s.bT1, cr, 1), C0(),
                                   V<T>(s.bA, cr, 1), xo(), tps, cl, 0, (long)m2 * cr, (long)m2 * cr));
            }
            CView<T> Th = V<T>(s.bA, nR, 1);
            HIPCHK(gemv_left<T>(st, trans(Th), nR, nL, s.rvec, s.vtmp));   // theta rvec
            HIPCHK(dot(st, s.lvec, s.vtmp, nL, s.sc));
            HIPCHK(sumsq<T>(st, Th, nL, nR, s.sc + 4, s.sqp, s.sqc));
            theta_check = true;   // its non-finite count is read with the basis checks
            CView<T> Fa = dir > 0 ? Th : adj(Th);
            if (std::min(na, nb) > subspace_min_order()) {
                // range basis by subspace iteration, then the exact split of the q x nb core
                const int q = subspace_basis(Fa, na, nb, chi, 0x5EED0000ull + (uint64_t)i, s.bQ, nb, s.bK, nb);
                if (q <= 0) throw Fail{MPDO_E_NUMERIC, "merged tensor vanished"};
                kept = svd_left(V<T>(s.bK, nb, 1), q, nb, chi, s.bU2);
                if (kept <= 0) throw Fail{MPDO_E_NUMERIC, "empty spectrum"};
                gemm(na, kept, q, C1(), V<T>(s.bQ, nb, 1), V<T>(s.bU2, kept, 1), C0(), V<T>(s.bR, kept, 1));
                HIPCHK((geam<T, T>(st, na, kept, C1(), V<T>(s.bR, kept, 1), C0(), V<T>(s.bU2, kept, 1))));
            } else {
                kept = svd_left(Fa, na, nb, chi, s.bU2);
            }
            if (kept <= 0) throw Fail{MPDO_E_NUMERIC, "empty spectrum"};
            if (dir > 0) {
                HIPCHK((geam<T, T>(st, nL, kept, C1(), V<T>(s.bU2, kept, 1), C0(), V<T>(outL, kept, 1))));
                HIPCHK((geam<T, T>(st, kept, nR, C1(), V<T>(s.bB2, nR, 1), C0(), V<T>(outR, nR, 1))));
            } else {
                HIPCHK((geam<T, T>(st, kept, nR, C1(), adj(V<T>(s.bU2, kept, 1)), C0(), V<T>(outR, nR, 1))));
                HIPCHK((geam<T, T>(st, nL, kept, C1(), adj(V<T>(s.bB2, nL, 1)), C0(), V<T>(outL, kept, 1))));
            }
        }
        Left = outL;
        Right = outR;
        // Schmidt values as the norms of the rows of B = U^H theta: with them |Lambda'|^2 and
        // T'.Lambda' equal ||theta||^2 and tr(rho) up to rounding whatever the accuracy of
        // the Gram eigenvalues, so PPT is the identity when nothing is cut
        HIPCHK(row_norms<T>(st, V<T>(s.bB2, nb, 1), kept, nb, s.sig));
        // trace factors of the kept Schmidt pairs and PPT
        HIPCHK(gemv_left<T>(st, V<T>(Left, kept, 1), nL, kept, s.lvec, s.tl));
        HIPCHK(gemv_left<T>(st, trans(V<T>(Right, nR, 1)), nR, kept, s.rvec, s.tr));
        // sc[0..1] holds tr(rho) from the dot, sc[4] = ||theta||^2: PPT reads both on the device
        HIPCHK(ppt(st, s.sig, s.tl, s.tr, s.sc, kept, c.cfg.ppt, c.cfg.renorm_trace, s.fac, s.pout));
        if (dir > 0)
            HIPCHK(scale_rows<T>(st, Right, kept, nR, nR, s.fac));
        else
            HIPCHK(scale_cols<T>(st, V<T>(Left, kept, 1), nL, kept, s.fac));
        orth_verify();   // before the new sites are committed
        swap_site(i, 0);
        swap_site(i + 1, 1);
        c.dims[i + 1] = kept;
        site_changed(i);
        site_changed(i + 1);
        c.centre = dir > 0 ? i + 1 : i;
        if (info) {
            double po[16], sg[2], nn[2];
            read_doubles2(s.pout, 13, po, s.sc + 4, 2, nn);
            n2 = nn[0];
            read_doubles(s.sig, 1, sg);
            double smin = 0.0;
            read_doubles(s.sig + (kept - 1), 1, &smin);
            info->bond = i;
            info->chi_l = cl;
            info->chi_mid = cm;
            info->chi_r = cr;
            info->kept = kept;
            info->path = factored ? 1 : 0;
            info->eig_calls = eig_calls;
            info->ppt_feasible = (int)po[3];
            info->trace_before = po[0];
            info->trace_after = po[10];
            info->xi_before = po[1];
            info->xi_after = po[11];
            info->ppt_theta = po[2];
            info->discarded_weight = n2 > 0.0 ? std::max(0.0, 1.0 - po[7] / n2) : 0.0;
            info->max_abs_imag_t = po[0] != 0.0 ? po[6] / fabs(po[0]) : po[6];
            info->sigma_max = sg[0];
            info->sigma_min_kept = smin;
            // the largest discarded Schmidt value: from the level whose chi cap made the cut,
            // else bounded by that level's threshold (an eigenvalue of the Gram), else below the
            // cutoff (reported as 0)
            double snext = 0.0;
            if (cut_next >= 0) {
                read_doubles(s.sig + cut_next, 1, &snext);
            } else if (cut_next <= -2) {
                double st4[4];
                read_doubles(s.st, 4, st4);
                snext = sqrt(std::max(0.0, st4[1 + (-2 - cut_next)]));
            }
            info->sigma_next = snext;
            info->sigma_gap_at_cut = smin - snext;
            info->sigma_next_exact = cut_next >= 0 ? 1 : 0;
        }
    }
};

// ====================================================================== host math
std::vector<zc> superop_from_kraus_2(const double* kraus, int nk, int d) {
    const int D2 = d * d, m = D2 * D2;
    std::vector<zc> S((size_t)m * m, zc(0, 0));
    for (int q = 0; q < nk; ++q) {
        const zc* K = (const zc*)(kraus + (size_t)q * 2 * D2 * D2);   // (d^2 x d^2) on (a,b),(s,t)
        for (int a = 0; a < d; ++a)
            for (int ap = 0; ap < d; ++ap)
                for (int b = 0; b < d; ++b)
                    for (int bp = 0; bp < d; ++bp) {
                        const int row = (a * d + ap) * D2 + (b * d + bp);
                        for (int s_ = 0; s_ < d; ++s_)
                            for (int sp = 0; sp < d; ++sp)
                                for (int t = 0; t < d; ++t)
                                    for (int tp = 0; tp < d; ++tp) {
                                        const int col = (s_ * d + sp) * D2 + (t * d + tp);
                                        const zc k1 = K[(a * d + b) * D2 + (s_ * d + t)];
                                        const zc k2 = K[(ap * d + bp) * D2 + (sp * d + tp)];
                                        S[(size_t)row * m + col] += k1 * std::conj(k2);
                                    }
                    }
    }
    return S;
}

// Superoperator of rho -> Kk rho Kb^+ on two atoms (Kk, Kb: d^2 x d^2 on sigma_i d + sigma_{i+1}),
// in the layout of superop_from_kraus_2 (which sums this over Kk = Kb = K)
std::vector<zc> superop_pair(const zc* Kk, const zc* Kb, int d) {
    const int D2 = d * d, m = D2 * D2;
    std::vector<zc> S((size_t)m * m);
    for (int a = 0; a < d; ++a)
        for (int ap = 0; ap < d; ++ap)
            for (int b = 0; b < d; ++b)
                for (int bp = 0; bp < d; ++bp) {
                    const int row = (a * d + ap) * D2 + (b * d + bp);
                    for (int s_ = 0; s_ < d; ++s_)
                        for (int sp = 0; sp < d; ++sp)
                            for (int t = 0; t < d; ++t)
                                for (int tp = 0; tp < d; ++tp) {
                                    const int col = (s_ * d + sp) * D2 + (t * d + tp);
                                    S[(size_t)row * m + col] =
                                        Kk[(a * d + b) * D2 + (s_ * d + t)] * std::conj(Kb[(ap * d + bp) * D2 + (sp * d + tp)]);
                                }
                }
    return S;
}

std::vector<zc> superop_from_kraus_1(const double* kraus, int nk, int d) {
    const int D2 = d * d;
    std::vector<zc> S((size_t)D2 * D2, zc(0, 0));
    for (int q = 0; q < nk; ++q) {
        const zc* K = (const zc*)(kraus + (size_t)q * 2 * d * d);
        for (int a = 0; a < d; ++a)
            for (int ap = 0; ap < d; ++ap)
                for (int s_ = 0; s_ < d; ++s_)
                    for (int sp = 0; sp < d; ++sp)
                        S[(size_t)(a * d + ap) * D2 + (s_ * d + sp)] += K[a * d + s_] * std::conj(K[ap * d + sp]);
    }
    return S;
}

double cptp_defect(const double* kraus, int nk, int dim) {
    std::vector<zc> acc((size_t)dim * dim, zc(0, 0));
    for (int q = 0; q < nk; ++q) {
        const zc* K = (const zc*)(kraus + (size_t)q * 2 * dim * dim);
        for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b) {
                zc sacc(0, 0);
                for (int k = 0; k < dim; ++k) sacc += std::conj(K[k * dim + a]) * K[k * dim + b];
                acc[(size_t)a * dim + b] += sacc;
            }
    }
    double dmax = 0.0;
    for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b) dmax = std::max(dmax, std::abs(acc[(size_t)a * dim + b] - zc(a == b ? 1 : 0, 0)));
    return dmax;
}

bool all_finite(const double* p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// ====================================================================== context plumbing
size_t workspace_for(const mpdo_config& cfg) {
    const int D2 = cfg.d * cfg.d;
    const int nmax = cfg.chi_max * D2;
    const bool f32 = cfg.precision != MPDO_FP64;
    const size_t tsz = f32 ? sizeof(float) : sizeof(double);
    size_t b = 0;
    const size_t site = (size_t)cfg.chi_max * D2 * cfg.chi_max * 2 * tsz + 256;
    b += (size_t)(cfg.n_sites + 2) * site;
    b += (size_t)(cfg.n_sites + 1) * D2 * 2 * sizeof(double) + 256;          // ovec (+ vec(I))
    b += 2 * ((size_t)(cfg.n_sites + 1) * cfg.chi_max * 2 * sizeof(double) + 256);  // Lv, Rv
    b += (size_t)D2 * D2 * D2 * D2 * 2 * (sizeof(double) + tsz) + 512;       // superoperator
    b += Scratch<double>::bytes(f32 ? 64 : nmax);
    if (f32) b += Scratch<float>::bytes(nmax);
    b += Scratch<double>::bytes(D2 * D2);
    b += (size_t)128 * (MAX_FACTOR_RANK * D2 * D2 * 2 * sizeof(double) + 256);   // gate factor slots
    b += (size_t)cfg.n_sites * D2 * 2 * sizeof(double) + 256;                       // expectation operators
    b += (size_t)cfg.n_sites * D2 * D2 * 2 * sizeof(double) + 256;                  // second-order operators
    return b + (1 << 20);
}

void set_err(mpdo_ctx ctx, const Fail& f) {
    ctx->err = f.msg;
    if (f.st == MPDO_E_DEVICE || f.st == MPDO_E_NUMERIC) ctx->poisoned = true;
}

void alloc_state(mpdo_ctx c) {
    const size_t need = workspace_for(c->cfg);
    if (!c->ws) {
        void* p = nullptr;
        if (hipMalloc(&p, need) != hipSuccess) throw Fail{MPDO_E_NOMEM, "hipMalloc of the workspace failed"};
        c->ws = (char*)p;
        c->ws_bytes = need;
        c->own_ws = true;
    }
    c->arena.base = c->ws;
    c->arena.cap = c->ws_bytes;
    c->arena.used = 0;
    const size_t tsz = c->tsize();
    const size_t scap = c->site_cap();
    c->site.resize(c->N);
    for (int j = 0; j < c->N; ++j) c->site[j] = c->arena.take<char>(scap * tsz);
    c->spare.resize(2);
    for (int j = 0; j < 2; ++j) c->spare[j] = c->arena.take<char>(scap * tsz);
    c->ovec = c->arena.take<double>((size_t)(c->N + 1) * c->D2 * 2);
    c->Lv = c->arena.take<double>((size_t)(c->N + 1) * c->chi * 2);
    c->Rv = c->arena.take<double>((size_t)(c->N + 1) * c->chi * 2);
    const int m2 = c->D2 * c->D2;
    c->Sdev = c->arena.take<double>((size_t)m2 * m2 * 2);
    c->SdevT = c->fp32 ? (void*)c->arena.take<float>((size_t)m2 * m2 * 2) : (void*)c->Sdev;
    const int nmax = c->chi * c->D2;
    c->sd.carve(c->arena, c->fp32 ? 64 : nmax);
    if (c->fp32) c->sf.carve(c->arena, nmax);
    c->sg.carve(c->arena, m2);
    // sumsq arrival counters start at 0 (every call leaves them 0)
    HIPCHK(hipMemsetAsync(c->sd.sqc, 0, 64 * sizeof(unsigned), c->st));
    if (c->fp32) HIPCHK(hipMemsetAsync(c->sf.sqc, 0, 64 * sizeof(unsigned), c->st));
    HIPCHK(hipMemsetAsync(c->sg.sqc, 0, 64 * sizeof(unsigned), c->st));
    c->gslots.clear();
    c->fcache.clear();
    c->sdev_id = 0;
    c->Scur = nullptr;
    for (int q = 0; q < 128; ++q) c->gslots.push_back(c->arena.take<double>((size_t)MAX_FACTOR_RANK * m2 * 2));
    c->obuf = c->arena.take<double>((size_t)c->N * c->D2 * 2);
    c->o2buf = c->arena.take<double>((size_t)c->N * c->D2 * c->D2 * 2);
    if (!c->hbuf) {
        if (hipHostMalloc((void**)&c->hbuf, 1 << 16) != hipSuccess) throw Fail{MPDO_E_NOMEM, "pinned buffer"};
        if (hipHostMalloc((void**)&c->hint, 256) != hipSuccess) throw Fail{MPDO_E_NOMEM, "pinned buffer"};
    }
    c->ready = true;
}

void upload(mpdo_ctx c, void* dst, const void* src, size_t bytes) {
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
}

void set_ovec(mpdo_ctx c, int j) {
    // trace vector of atom j: o = P_j^T vec(I)
    const int D2 = c->D2, d = c->d;
    std::vector<zc> o(D2, zc(0, 0));
    for (int eta = 0; eta < D2; ++eta) {
        zc acc(0, 0);
        for (int a = 0; a < d; ++a) {
            const int r = a * d + a;
            acc += c->pend_id[j] ? zc(r == eta ? 1 : 0, 0) : c->pending[j][(size_t)r * D2 + eta];
        }
        o[eta] = acc;
    }
    upload(c, c->ovec + 2 * (size_t)j * D2, o.data(), D2 * sizeof(zc));
}

void release_entry(mpdo_ctx c, size_t k) {
    FoldEntry& e = c->fcache[k];
    if (e.gf.X) {
        c->gslots.push_back(e.gf.X);
        c->gslots.push_back(e.gf.Y);
    }
    if (e.id == c->sdev_id) c->sdev_id = 0;
    c->fcache.erase(c->fcache.begin() + (long)k);
}

// index of the least recently used entry (only among those holding factor slots if asked)
long lru_entry(mpdo_ctx c, bool with_slots) {
    long k = -1;
    for (size_t q = 0; q < c->fcache.size(); ++q) {
        if (with_slots && !c->fcache[q].gf.X) continue;
        if (k < 0 || c->fcache[q].used < c->fcache[(size_t)k].used) k = (long)q;
    }
    return k;
}

// operator-Schmidt factors of the (D2^2 x D2^2) superoperator S: S = sum_k X_k (x) Y_k
GateFactor factorize(mpdo_ctx c, const std::vector<zc>& S) {
    const int D2 = c->D2, m2 = D2 * D2;
    // reshuffle R[(a,c),(b,e)] = S[(a,b),(c,e)]
    std::vector<zc> R((size_t)m2 * m2);
    for (int a = 0; a < D2; ++a)
        for (int b = 0; b < D2; ++b)
            for (int cc = 0; cc < D2; ++cc)
                for (int e = 0; e < D2; ++e)
                    R[(size_t)(a * D2 + cc) * m2 + (b * D2 + e)] = S[(size_t)(a * D2 + b) * m2 + (cc * D2 + e)];
    Scratch<double>& g = c->sg;
    upload(c, g.bA, R.data(), R.size() * sizeof(zc));
    Engine<double> E(*c, g);
    const int r = E.orth2(V<double>(g.bA, m2, 1), m2, m2, g.bQ, g.bK);
    E.orth_verify();
    GateFactor gf;
    gf.r = r;
    if (r > MAX_FACTOR_RANK || r <= 0) {
        gf.X = gf.Y = nullptr;
    } else {
        // free the least recently used factors until a slot pair is available
        while (c->gslots.size() < 2) {
            const long k = lru_entry(c, true);
            if (k < 0) throw Fail{MPDO_E_NOMEM, "no slot for gate factors"};
            release_entry(c, (size_t)k);
        }
        gf.X = c->gslots.back();
        c->gslots.pop_back();
        gf.Y = c->gslots.back();
        c->gslots.pop_back();
        // X[k][(a,c)] = Q[(a,c), k]   (Q: m2 x r, ld m2);  Y[k][(b,e)] = K[k][(b,e)]
        HIPCHK((geam<double, double>(c->st, r, m2, C1(), trans(V<double>(g.bQ, m2, 1)), C0(),
                                     V<double>(gf.X, m2, 1))));
        HIPCHK((geam<double, double>(c->st, r, m2, C1(), V<double>(g.bK, m2, 1), C0(), V<double>(gf.Y, m2, 1))));
    }
    return gf;
}

// S <- S (P_i (x) P_{i+1}) for the single-atom maps queued on atoms i and i+1
void fold_pending(mpdo_ctx c, int i, std::vector<zc>& S) {
    const int D2 = c->D2, m2 = D2 * D2;
    std::vector<zc> P((size_t)m2 * m2, zc(0, 0));
    for (int a = 0; a < D2; ++a)
        for (int b = 0; b < D2; ++b)
            for (int cc = 0; cc < D2; ++cc)
                for (int e = 0; e < D2; ++e) {
                    const zc pa = c->pend_id[i] ? zc(a == cc ? 1 : 0, 0) : c->pending[i][(size_t)a * D2 + cc];
                    const zc pb = c->pend_id[i + 1] ? zc(b == e ? 1 : 0, 0) : c->pending[i + 1][(size_t)b * D2 + e];
                    P[(size_t)(a * D2 + b) * m2 + (cc * D2 + e)] = pa * pb;
                }
    std::vector<zc> out((size_t)m2 * m2, zc(0, 0));
    for (int r = 0; r < m2; ++r)
        for (int k = 0; k < m2; ++k) {
            const zc sv = S[(size_t)r * m2 + k];
            if (sv == zc(0, 0)) continue;
            for (int col = 0; col < m2; ++col) out[(size_t)r * m2 + col] += sv * P[(size_t)k * m2 + col];
        }
    S.swap(out);
}

// The folded map of an update on atoms (i, i+1): from the cache when the same input meets the
// same queued maps again, otherwise built (from the Kraus set if kind == 1), folded, factorised
// and cached.  Returns the entry's index in the cache.
size_t folded_map(mpdo_ctx c, int i, int kind, const double* in, size_t n_in, int n_kraus) {
    const int D2 = c->D2;
    const size_t pbytes = (size_t)D2 * D2 * sizeof(zc);
    const bool ida = c->pend_id[i] != 0, idb = c->pend_id[i + 1] != 0;
    uint64_t h = hash_bytes(in, n_in * sizeof(double), 0x51ull + (uint64_t)kind);
    h = hash_bytes(ida ? nullptr : c->pending[i].data(), ida ? 0 : pbytes, h ^ 0xA1ull);
    h = hash_bytes(idb ? nullptr : c->pending[i + 1].data(), idb ? 0 : pbytes, h ^ 0xB2ull);
    for (size_t k = 0; k < c->fcache.size(); ++k) {
        FoldEntry& e = c->fcache[k];
        if (e.h != h || e.kind != kind || e.in.size() != n_in || e.ida != ida || e.idb != idb) continue;
        if (memcmp(e.in.data(), in, n_in * sizeof(double)) != 0) continue;
        if (!ida && memcmp(e.pa.data(), c->pending[i].data(), pbytes) != 0) continue;
        if (!idb && memcmp(e.pb.data(), c->pending[i + 1].data(), pbytes) != 0) continue;
        e.used = ++c->fclock;
        return k;
    }
    std::vector<zc> S;
    if (kind == 1) {
        S = superop_from_kraus_2(in, n_kraus, c->d);
    } else {
        S.resize(n_in / 2);
        memcpy(S.data(), in, n_in * sizeof(double));
    }
    if (!ida || !idb) fold_pending(c, i, S);
    while ((int)c->fcache.size() >= FOLD_CACHE_MAX) release_entry(c, (size_t)lru_entry(c, false));
    FoldEntry e;
    e.gf = factorize(c, S);   // may release entries to free factor slots
    e.id = c->fnext++;
    e.h = h;
    e.used = ++c->fclock;
    e.kind = kind;
    e.in.assign(in, in + n_in);
    e.ida = ida;
    e.idb = idb;
    if (!ida) e.pa = c->pending[i];
    if (!idb) e.pb = c->pending[i + 1];
    e.S.swap(S);
    c->fcache.push_back(std::move(e));
    return c->fcache.size() - 1;
}

// MPDO_ORTH_EIG=1 builds every range basis from Gram eigenvectors (no pivoted Cholesky).
static bool use_pchol() {
    const char* v = getenv("MPDO_ORTH_EIG");
    return !(v && atoi(v) != 0);
}

template <typename T>
void do_update(mpdo_ctx c, int i, int kind, const double* in, size_t n_in, int n_kraus, int chi,
               mpdo_trunc_info* info) {
    const FoldEntry& e = c->fcache[folded_map(c, i, kind, in, n_in, n_kraus)];
    const GateFactor gf = e.gf;
    if (!c->pend_id[i] || !c->pend_id[i + 1]) {   // the queued maps are now part of the update
        c->pend_id[i] = c->pend_id[i + 1] = 1;
        set_ovec(c, i);
        set_ovec(c, i + 1);
        c->lvalid = std::min(c->lvalid, i);
        c->rvalid = std::max(c->rvalid, i + 2);
    }
    c->Scur = &e.S;   // loaded to the device only if the update takes the explicit path
    c->Scur_id = e.id;
    // A failed basis check is raised before the pair's new sites are written (the canonical
    // moves before it keep rho exactly), so the update can be recomputed from the same sites;
    // it is, once, and a second failure is returned.
    for (int attempt = 0;; ++attempt) {
        try {
            if (c->fp32) {
                Engine<float> E(*c, c->sf);
                E.ns_iters = attempt ? 4 : 2;
                E.orth_pchol = attempt == 0 && use_pchol();
                E.update(i, gf.X ? &gf : nullptr, chi, info);
            } else {
                Engine<double> E(*c, c->sd);
                E.ns_iters = attempt ? 4 : 2;
                E.orth_pchol = attempt == 0 && use_pchol();
                E.update(i, gf.X ? &gf : nullptr, chi, info);
            }
            if (info) info->retried = attempt;
            c->retries += attempt;
            return;
        } catch (const Fail& f) {
            if (!f.retry || attempt > 0) throw;
            if (getenv("MPDO_DEBUG_CHECKS") || getenv("MPDO_DEBUG_FAILURES"))
                fprintf(stderr, "[mpdo] recomputing update %d: %s\n", i, f.msg.c_str());
        }
    }
}

// Crosstalk gate of the pair (i, i+1) (noise-free, Sec. II "MPO form of the noisy CZ gate with
// crosstalk"): U = sum_ab P^a_{i-1} (x) u[a + 2b] (x) P^b_{i+2}, P^1 the Rydberg projector.  On
// the vectorised index eta = sigma d + sigma' of a neighbour the projectors pick the class
// alpha = [sigma = r] + 2 [sigma' = r]; the superoperator is block diagonal in the two
// neighbours' classes, with block u[a + 2b] (x) conj(u[a' + 2b']).  Steps:
//  1. the centre moves to the pair; queued maps of the neighbours are applied to their sites,
//     those of the pair are folded into the blocks;
//  2. each neighbour is split on its bond by the class of its physical index and
//     orthonormalised class by class; the factors go into the pair, so the pair's outer bonds
//     carry the class while the neighbours are isometries;
//  3. the pair update applies block (alpha, beta) to its part of theta; theta is then rho's
//     coefficient matrix in orthonormal bases, so the cut to chi_max and PPT are those of an
//     ordinary update;
//  4. canonical moves across both neighbour bonds compress them to their Schmidt ranks
//     (range bases; nothing above the rounding floor is cut).
// The class-split neighbour bonds (4x) must fit chi_max.
template <typename T>
void do_crosstalk(mpdo_ctx c, Engine<T>& E, int i, int ryd, const double* u4, mpdo_trunc_info* info) {
    const int d = c->d, D2 = c->D2, m2 = D2 * D2, N = c->N;
    const bool left = i >= 1, right = i + 2 <= N - 1;
    const int na = left ? 4 : 1, nb = right ? 4 : 1;
    if ((long)na * c->dims[i] > c->chi || (long)nb * c->dims[i + 2] > c->chi)
        throw Fail{MPDO_E_ARG, "crosstalk gate: four times a neighbour bond exceeds chi_max"};
    EtaClass cls;
    for (int e = 0; e < EtaClass::MAXD2; ++e) cls.c[e] = 0;
    for (int e = 0; e < D2; ++e) cls.c[e] = ((e / d) == ryd ? 1 : 0) + ((e % d) == ryd ? 2 : 0);
    // block superoperators with the pair's queued maps folded in
    const size_t blk = (size_t)m2 * m2;
    if (!c->xg) {
        if (hipMalloc((void**)&c->xg, 16 * blk * sizeof(zc)) != hipSuccess) throw Fail{MPDO_E_NOMEM, "crosstalk blocks"};
        if (c->fp32 && hipMalloc(&c->xgT, 16 * blk * 2 * sizeof(float)) != hipSuccess)
            throw Fail{MPDO_E_NOMEM, "crosstalk blocks"};
    }
    // The blocks depend on the unitaries, the Rydberg level, the chain-end shape and the maps
    // queued on the pair: the last set stays on the device and is rebuilt only when these differ.
    std::vector<double> src(u4, u4 + (size_t)4 * m2 * 2);
    src.push_back(ryd);
    src.push_back(na);
    src.push_back(nb);
    for (int j : {i, i + 1}) {
        src.push_back(c->pend_id[j]);
        if (!c->pend_id[j])
            src.insert(src.end(), (const double*)c->pending[j].data(), (const double*)c->pending[j].data() + 2 * D2 * D2);
    }
    if (src != c->xg_src) {
        const zc* U = (const zc*)u4;
        std::vector<zc> all(16 * blk, zc(0, 0));
        for (int al = 0; al < na; ++al)
            for (int be = 0; be < nb; ++be) {
                const int a = al & 1, ap = al >> 1, b = be & 1, bp = be >> 1;
                std::vector<zc> S = superop_pair(U + (size_t)(a + 2 * b) * m2, U + (size_t)(ap + 2 * bp) * m2, d);
                if (!c->pend_id[i] || !c->pend_id[i + 1]) fold_pending(c, i, S);
                std::copy(S.begin(), S.end(), all.begin() + (size_t)(4 * al + be) * blk);
            }
        c->xg_src.clear();   // a failed upload leaves no stale tag
        upload(c, c->xg, all.data(), all.size() * sizeof(zc));
        if (c->fp32)
            HIPCHK((geam<double, float>(c->st, 16 * m2, m2, C1(), V<double>(c->xg, m2, 1), C0(),
                                        V<float>((float*)c->xgT, m2, 1))));
        c->xg_src.swap(src);
    }
    BlockGate<T> bg;
    bg.na = na;
    bg.nb = nb;
    for (int q = 0; q < 16; ++q) {
        if (c->fp32)
            bg.G[q] = (const T*)((float*)c->xgT + 2 * (size_t)q * blk);
        else
            bg.G[q] = (const T*)(c->xg + 2 * (size_t)q * blk);
    }
    // 1. centre to the pair; queued maps
    if (c->centre < i) c->dir = 1;
    else if (c->centre > i + 1) c->dir = -1;
    while (c->centre < i) E.move_right(c->centre);
    while (c->centre > i + 1) E.move_left(c->centre);
    for (int j : {i - 1, i + 2}) {
        if (j < 0 || j >= N || c->pend_id[j]) continue;
        std::vector<zc> P = c->pending[j];
        upload(c, c->Sdev, P.data(), P.size() * sizeof(zc));   // Sdev as staging; its cache tag is cleared
        c->sdev_id = 0;
        if (c->fp32) {
            HIPCHK((geam<double, float>(c->st, D2, D2, C1(), V<double>(c->Sdev, D2, 1), C0(),
                                        V<float>((float*)c->SdevT, D2, 1))));
            E.apply_phys(j, (const T*)c->SdevT);
        } else {
            E.apply_phys(j, (const T*)c->Sdev);
        }
        c->pend_id[j] = 1;
        set_ovec(c, j);
    }
    if (!c->pend_id[i] || !c->pend_id[i + 1]) {   // folded into the blocks above
        c->pend_id[i] = c->pend_id[i + 1] = 1;
        set_ovec(c, i);
        set_ovec(c, i + 1);
    }
    // 2. absorb the neighbours class by class.  Left: the class-split site i-1 (its bond
    //    (alpha, r)) has column blocks on disjoint physical rows, so orthonormalising each block
    //    alone, F_alpha = Q_alpha K_alpha, gives a left isometry [Q_0 .. Q_3] whose bond keeps
    //    the class; K_alpha goes into site i (whose left bond was the replicated (alpha, l)).
    //    Right: the same with the rows of the class-split site i+2.
    const int c1 = c->dims[i], c3 = c->dims[i + 2];
    if (left) {
        const int c0 = c->dims[i - 1], cm = c->dims[i + 1];
        const int n = c0 * D2, w = D2 * cm;
        HIPCHK(class_expand<T>(c->st, (T*)c->site[i - 1], c0, D2, c1, 0, 4, cls, E.s.bR));
        T* tq = E.s.bU2;               // the Q blocks side by side, ld 4 c1
        T* nnext = (T*)c->spare[1];    // new site i: q x w, block alpha at rows [oa, oa + qa)
        int q = 0;
        for (int al = 0; al < 4; ++al) {
            const int qb = E.orth2(V<T>(E.s.bR + 2 * (long)al * c1, 4L * c1, 1), n, c1, E.s.bQ, E.s.bK);
            bg.lo[al] = q;
            bg.ln[al] = qb;
            if (qb > 0) {
                HIPCHK((geam<T, T>(c->st, n, qb, C1(), V<T>(E.s.bQ, c1, 1), C0(), V<T>(tq + 2 * (long)q, 4L * c1, 1))));
                E.gemm(qb, w, c1, C1(), V<T>(E.s.bK, c1, 1), V<T>((T*)c->site[i], w, 1), C0(),
                       V<T>(nnext + 2 * (long)q * w, w, 1));
            }
            q += qb;
        }
        if (q <= 0) throw Fail{MPDO_E_NUMERIC, "crosstalk: left neighbour vanished"};
        HIPCHK((geam<T, T>(c->st, n, q, C1(), V<T>(tq, 4L * c1, 1), C0(), V<T>((T*)c->spare[0], q, 1))));
        E.swap_site(i - 1, 0);
        E.swap_site(i, 1);
        c->dims[i] = q;
        E.site_changed(i - 1);
        E.site_changed(i);
    } else {
        bg.lo[0] = 0;
        bg.ln[0] = c1;
    }
    if (right) {
        const int c5 = c->dims[i + 3];
        const int n = D2 * c5;
        const int h = c->dims[i + 1] * D2;   // site i+1 as an h x c3 matrix
        // site i+2 class-split on its left bond: rows (beta, l), l < c3, as a (4 c3) x n matrix
        HIPCHK(class_expand<T>(c->st, (T*)c->site[i + 2], c3, D2, c5, 3, 4, cls, E.s.bR));
        T* nsite = (T*)c->spare[0];   // new site i+2: p x n, block beta at rows [ob, ob + pb)
        T* tk = E.s.bU2;              // new site i+1 blocks side by side, ld 4 c3
        int p = 0;
        for (int be = 0; be < 4; ++be) {
            // G_beta^H = Q K (Q: n x pb, K: pb x c3), so G_beta = K^H Q^H
            const int pbk = E.orth2(adj(V<T>(E.s.bR + 2 * (long)be * c3 * n, n, 1)), n, c3, E.s.bQ, E.s.bK);
            bg.ro[be] = p;
            bg.rn[be] = pbk;
            if (pbk > 0) {
                HIPCHK((geam<T, T>(c->st, pbk, n, C1(), adj(V<T>(E.s.bQ, c3, 1)), C0(),
                                   V<T>(nsite + 2 * (long)p * n, n, 1))));
                E.gemm(h, pbk, c3, C1(), V<T>((T*)c->site[i + 1], c3, 1), adj(V<T>(E.s.bK, c3, 1)), C0(),
                       V<T>(tk + 2 * (long)p, 4L * c3, 1));
            }
            p += pbk;
        }
        if (p <= 0) throw Fail{MPDO_E_NUMERIC, "crosstalk: right neighbour vanished"};
        HIPCHK((geam<T, T>(c->st, h, p, C1(), V<T>(tk, 4L * c3, 1), C0(), V<T>((T*)c->spare[1], p, 1))));
        E.swap_site(i + 2, 0);
        E.swap_site(i + 1, 1);
        c->dims[i + 2] = p;
        E.site_changed(i + 1);
        E.site_changed(i + 2);
    } else {
        bg.ro[0] = 0;
        bg.rn[0] = c3;
    }
    // 3. the pair update with the block superoperators: the outer sites are isometries whose
    //    bonds carry the classes, so theta is rho's coefficient matrix in orthonormal bases and
    //    the cut to chi_max and PPT are those of an ordinary update
    E.update(i, nullptr, c->chi, info, &bg);
    // 4. compress the neighbour bonds to their Schmidt ranks.  After the update the chain is in
    //    canonical form around the centre (i or i+1; the absorbed neighbours are isometries),
    //    and a move orthonormalises a site whose far side is isometric: moving to a neighbour
    //    and back across both neighbour bonds compresses each exactly.  The nearer side first.
    auto to = [&](int target) {
        while (c->centre < target) E.move_right(c->centre);
        while (c->centre > target) E.move_left(c->centre);
    };
    const bool right_first = c->centre > i;
    if (right_first) {
        if (right) to(i + 2);
        if (left) to(i - 1);
    } else {
        if (left) to(i - 1);
        if (right) to(i + 2);
    }
    E.orth_verify();
}

mpdo_status guard(mpdo_ctx c) {
    if (!c) return MPDO_E_ARG;
    if (c->poisoned) {
        c->err = "context poisoned by an earlier device or numeric failure";
        return MPDO_E_STATE;
    }
    return MPDO_OK;
}

}  // namespace

template <typename T>
static Scratch<T>& scratch_of(mpdo_ctx c);
template <>
Scratch<double>& scratch_of<double>(mpdo_ctx c) {
    return c->sd;
}
template <>
Scratch<float>& scratch_of<float>(mpdo_ctx c) {
    return c->sf;
}

template <typename T>
static void expect_impl(mpdo_ctx c, int n_terms, const int* first, const int* len, const double* ops, int normalize,
                        double* out) {
    Scratch<T>& s = scratch_of<T>(c);
    Engine<T> E(*c, s);
    const int D2 = c->D2, d = c->d;
    E.ensureL(c->N);
    size_t opos = 0;
    double* res = s.pout;   // 2 doubles per term, staged in chunks
    std::vector<double> all((size_t)n_terms * 2);
    int t0 = 0;
    const int chunk = 16;
    while (t0 < n_terms) {
        const int t1 = std::min(n_terms, t0 + chunk);
        for (int t = t0; t < t1; ++t) {
            const int f = first[t], m = len[t];
            // operator vectors o = P^T vec(O^T)
            std::vector<zc> o((size_t)m * D2);
            for (int u = 0; u < m; ++u) {
                const zc* O = (const zc*)(ops + (opos + (size_t)u * d * d) * 2);
                const int j = f + u;
                for (int eta = 0; eta < D2; ++eta) {
                    zc acc(0, 0);
                    for (int a = 0; a < d; ++a)
                        for (int b = 0; b < d; ++b) {
                            const zc v = O[b * d + a];   // vec(O^T)[a d + b] = O[b][a]
                            if (v == zc(0, 0)) continue;
                            const int r = a * d + b;
                            acc += (c->pend_id[j] ? zc(r == eta ? 1 : 0, 0) : c->pending[j][(size_t)r * D2 + eta]) * v;
                        }
                    o[(size_t)u * D2 + eta] = acc;
                }
            }
            opos += (size_t)m * d * d;
            HIPCHK(hipMemcpyAsync(c->obuf, o.data(), o.size() * sizeof(zc), hipMemcpyHostToDevice, c->st));
            E.ensureR(f + m);
            HIPCHK((geam<double, double>(c->st, 1, c->dims[f], C1(), V<double>(E.Lv(f), 0, 1), C0(),
                                         V<double>(s.vtmp, 0, 1))));
            double* x = s.vtmp;
            double* y = s.vtmp2;
            for (int u = 0; u < m; ++u) {
                const int j = f + u;
                HIPCHK(transfer_left<T>(c->st, E.site(j), c->dims[j], D2, c->dims[j + 1], x, c->obuf + 2 * (size_t)u * D2,
                                        y));
                std::swap(x, y);
            }
            HIPCHK(dot(c->st, x, E.Rv(f + m), c->dims[f + m], res + 2 * (t - t0)));
            HIPCHK(hipStreamSynchronize(c->st));   // obuf is reused by the next term
        }
        E.read_doubles(res, 2 * (t1 - t0), all.data() + 2 * t0);
        t0 = t1;
    }
    double trv[2] = {1.0, 0.0};
    if (normalize) E.read_doubles(E.Lv(c->N), 2, trv);
    for (int t = 0; t < n_terms; ++t) {
        zc v(all[2 * t], all[2 * t + 1]);
        if (normalize) v /= zc(trv[0], trv[1]);
        out[2 * t] = v.real();
        out[2 * t + 1] = v.imag();
    }
}

// Second-order expectation (Fig. 6c): E2 = sum vec(rho)[eta] vec(rho)[eta'] prod_j M_j[eta_j, eta'_j]
// with the given M_j on atoms f..f+m-1 and vec(I) vec(I)^T (both copies traced) elsewhere, so the
// environments outside the term are outer products of the cached trace vectors.  An atom's
// queued single-atom maps P enter as M' = P^T M P.  Per atom three complex GEMMs:
//   T1[eta][l'][r]  = sum_l  L[l][l'] A[l][eta][r]                 (batch over eta)
//   T2[l'][eta'][r] = sum_eta M'[eta][eta'] T1[eta][l'][r]           (batch over l')
//   L'[r][r']       = sum_{l',eta'} T2[l'][eta'][r] A[l'][eta'][r']
template <typename T>
static void expect2_impl(mpdo_ctx c, int n_terms, const int* first, const int* len, const double* ops, int normalize,
                         double* out) {
    Scratch<T>& s = scratch_of<T>(c);
    Engine<T> E(*c, s);
    const int D2 = c->D2;
    E.ensureL(c->N);
    std::vector<double> all((size_t)n_terms * 2);
    size_t opos = 0;
    T* Mdev = (T*)c->o2buf;
    for (int t = 0; t < n_terms; ++t) {
        const int f = first[t], m = len[t];
        // M' = P^T M P per atom, in T
        std::vector<T> Mh((size_t)m * D2 * D2 * 2);
        for (int u = 0; u < m; ++u) {
            const int j = f + u;
            const zc* M = (const zc*)(ops + (opos + (size_t)u * D2 * D2) * 2);
            std::vector<zc> MP((size_t)D2 * D2, zc(0, 0));   // M P
            for (int a = 0; a < D2; ++a)
                for (int b = 0; b < D2; ++b) {
                    zc acc(0, 0);
                    for (int q = 0; q < D2; ++q) {
                        const zc pq = c->pend_id[j] ? zc(q == b ? 1 : 0, 0) : c->pending[j][(size_t)q * D2 + b];
                        acc += M[(size_t)a * D2 + q] * pq;
                    }
                    MP[(size_t)a * D2 + b] = acc;
                }
            for (int a = 0; a < D2; ++a)
                for (int b = 0; b < D2; ++b) {
                    zc acc(0, 0);
                    for (int q = 0; q < D2; ++q) {
                        const zc pq = c->pend_id[j] ? zc(q == a ? 1 : 0, 0) : c->pending[j][(size_t)q * D2 + a];
                        acc += pq * MP[(size_t)q * D2 + b];
                    }
                    Mh[2 * ((size_t)u * D2 * D2 + (size_t)a * D2 + b)] = (T)acc.real();
                    Mh[2 * ((size_t)u * D2 * D2 + (size_t)a * D2 + b) + 1] = (T)acc.imag();
                }
        }
        opos += (size_t)m * D2 * D2;
        HIPCHK(hipMemcpyAsync(Mdev, Mh.data(), Mh.size() * sizeof(T), hipMemcpyHostToDevice, c->st));
        E.ensureR(f + m);
        T* L = s.bA;
        T* L2 = s.bT1;
        T* T1 = s.bB;
        T* T2 = s.bC;
        HIPCHK(outer<T>(c->st, E.Lv(f), c->dims[f], L));
        for (int u = 0; u < m; ++u) {
            const int j = f + u, cl = c->dims[j], cr = c->dims[j + 1];
            const T* A = E.site(j);
            const T* Mj = Mdev + 2 * (size_t)u * D2 * D2;
            E.gemm(cl, cr, cl, C1(), V<T>(L, 1, cl), V<T>((T*)A, (long)D2 * cr, 1), C0(), V<T>(T1, cr, 1), D2, 0, cr,
                   (long)cl * cr);
            E.gemm(D2, cr, D2, C1(), V<T>((T*)Mj, 1, D2), V<T>(T1, (long)cl * cr, 1), C0(), V<T>(T2, cr, 1), cl, 0, cr,
                   (long)D2 * cr);
            E.gemm(cr, cr, cl * D2, C1(), V<T>(T2, 1, cr), V<T>((T*)A, cr, 1), C0(), V<T>(L2, cr, 1));
            std::swap(L, L2);
        }
        HIPCHK(bilinear<T>(c->st, L, c->dims[f + m], E.Rv(f + m), s.pout + 2 * (t % 16)));
        if (t % 16 == 15 || t == n_terms - 1) {
            const int t0 = t - (t % 16);
            E.read_doubles(s.pout, 2 * (t - t0 + 1), all.data() + 2 * t0);
        } else {
            HIPCHK(hipStreamSynchronize(c->st));   // Mdev is rewritten by the next term
        }
    }
    zc tr2(1, 0);
    if (normalize) {
        double trv[2];
        E.read_doubles(E.Lv(c->N), 2, trv);
        tr2 = zc(trv[0], trv[1]) * zc(trv[0], trv[1]);
    }
    for (int t = 0; t < n_terms; ++t) {
        zc v(all[2 * t], all[2 * t + 1]);
        if (normalize) v /= tr2;
        out[2 * t] = v.real();
        out[2 * t + 1] = v.imag();
    }
}

// The product kernels on host operands (mpdo_cgemm): device copies in T, one cgemm_ex on the
// null stream, the result back in complex128.
template <typename T>
void run_cgemm(bool x3, int M, int N, int K, const double* alpha, const double* A, int op_a, const double* B,
               int op_b, const double* beta, double* C, int split_k) {
    struct Buf {
        void* p = nullptr;
        ~Buf() {
            if (p) (void)hipFree(p);
        }
    } dA, dB, dC, ws;
    auto up = [](Buf& d, const double* h, long n) {
        std::vector<T> t((size_t)2 * n);
        for (long i = 0; i < 2 * n; ++i) t[i] = (T)h[i];
        if (hipMalloc(&d.p, sizeof(T) * (size_t)std::max(2 * n, 2L)) != hipSuccess)
            throw Fail{MPDO_E_NOMEM, "device allocation failed"};
        if (n > 0 && hipMemcpy(d.p, t.data(), sizeof(T) * 2 * n, hipMemcpyHostToDevice) != hipSuccess)
            throw Fail{MPDO_E_DEVICE, "copy to the device failed"};
    };
    up(dA, A, (long)M * K);
    up(dB, B, (long)K * N);
    up(dC, C, (long)M * N);
    // op 0: stored as op(X) row-major; 1: stored transposed; 2: stored transposed, conjugated
    const CView<T> va = op_a == 0 ? view<T>((T*)dA.p, K, 1) : view<T>((T*)dA.p, 1, M, op_a == 2);
    const CView<T> vb = op_b == 0 ? view<T>((T*)dB.p, N, 1) : view<T>((T*)dB.p, 1, K, op_b == 2);
    GemmOpts o;
    o.split_bf16 = x3;
    if (split_k) {
        o.ws_bytes = std::min((size_t)64 * M * N * 2 * sizeof(T), (size_t)256 << 20);
        if (hipMalloc(&ws.p, o.ws_bytes) != hipSuccess) throw Fail{MPDO_E_NOMEM, "device allocation failed"};
        o.ws = ws.p;
    }
    if (cgemm_ex<T>(0, M, N, K, cd{alpha[0], alpha[1]}, va, vb, cd{beta[0], beta[1]}, view<T>((T*)dC.p, N, 1), o) !=
            hipSuccess ||
        hipDeviceSynchronize() != hipSuccess)
        throw Fail{MPDO_E_DEVICE, "product kernel failed"};
    std::vector<T> t((size_t)2 * M * N);
    if (M * (long)N > 0 && hipMemcpy(t.data(), dC.p, sizeof(T) * t.size(), hipMemcpyDeviceToHost) != hipSuccess)
        throw Fail{MPDO_E_DEVICE, "copy to the host failed"};
    for (size_t i = 0; i < t.size(); ++i) C[i] = (double)t[i];
}

// The split's eigensolver on a host matrix (mpdo_eigh): the order dispatch of Engine::eig_cut
// for orders up to TRI_MAX, on the null stream, with device buffers of its own.
void run_eigh(int n, const double* H, double tau, int cap, int* m, double* evals, double* V) {
    struct Buf {
        void* p = nullptr;
        ~Buf() {
            if (p) (void)hipFree(p);
        }
    } dH, dV, dl, dst, dcnt, dw;
    struct Pinned {
        int* p = nullptr;
        ~Pinned() {
            if (p) (void)hipHostFree(p);
        }
    } hint;
    const size_t n2 = (size_t)n * n;
    auto alloc = [](Buf& b, size_t bytes) {
        if (hipMalloc(&b.p, std::max(bytes, (size_t)256)) != hipSuccess) throw Fail{MPDO_E_NOMEM, "device allocation failed"};
    };
    alloc(dH, n2 * 2 * sizeof(double));
    alloc(dV, n2 * 2 * sizeof(double));
    alloc(dl, (size_t)n * sizeof(double));
    alloc(dst, 64 * sizeof(double));
    alloc(dcnt, 64 * sizeof(int));
    alloc(dw, std::max(eigh_work_bytes(n), tri_work_bytes(n)));
    if (hipHostMalloc((void**)&hint.p, 4 * sizeof(int)) != hipSuccess) throw Fail{MPDO_E_NOMEM, "pinned allocation failed"};
    if (hipMemcpy(dH.p, H, n2 * 2 * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(dst.p, 0, 64 * sizeof(double)) != hipSuccess || hipMemset(dcnt.p, 0, 64 * sizeof(int)) != hipSuccess)
        throw Fail{MPDO_E_DEVICE, "copy to the device failed"};
    double* Hd = (double*)dH.p;
    double* Vd = (double*)dV.p;
    double* lam = (double*)dl.p;
    double* st = (double*)dst.p;
    int* cnt = (int*)dcnt.p;
    if (n <= EIG_JACOBI_MAX) {
        int sw = 0;
        if (eigh(0, n, Hd, n, Vd, n, lam, dw.p, EIG_MAX_SWEEPS, &sw, hint.p) != hipSuccess)
            throw Fail{MPDO_E_DEVICE, "eigensolver launch failed"};
        if (sw >= EIG_MAX_SWEEPS) throw Fail{MPDO_E_NUMERIC, "Jacobi eigensolver did not converge"};
        if (spectrum_cut(0, lam, n, 0, 0.0, 0.0, tau, cap, st, cnt, nullptr, nullptr) != hipSuccess)
            throw Fail{MPDO_E_DEVICE, "spectrum cut launch failed"};
    } else {
        if (eigh_top(0, n, Hd, n, 0, 0.0, 0.0, tau, cap, st, cnt, lam, nullptr, nullptr, Vd, n, dw.p) != hipSuccess)
            throw Fail{MPDO_E_DEVICE, "eigensolver launch failed"};
    }
    if (hipDeviceSynchronize() != hipSuccess) throw Fail{MPDO_E_DEVICE, "eigensolver failed"};
    int acc = 0;
    if (hipMemcpy(&acc, cnt, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        throw Fail{MPDO_E_DEVICE, "copy to the host failed"};
    if (acc < 0 || acc > cap) throw Fail{MPDO_E_NUMERIC, "accepted count out of range"};
    *m = acc;
    if (acc == 0) return;
    std::vector<double> v(n2 * 2);
    if (hipMemcpy(evals, lam, (size_t)acc * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(v.data(), Vd, n2 * 2 * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        throw Fail{MPDO_E_DEVICE, "copy to the host failed"};
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < acc; ++j) {
            V[2 * ((size_t)i * cap + j)] = v[2 * ((size_t)i * n + j)];
            V[2 * ((size_t)i * cap + j) + 1] = v[2 * ((size_t)i * n + j) + 1];
        }
}

// ====================================================================== C ABI
extern "C" {

mpdo_status mpdo_create(const mpdo_config* cfg, mpdo_ctx* out) {
    if (!cfg || !out) {
        g_create_err = "null argument";
        return MPDO_E_ARG;
    }
    *out = nullptr;
    if (cfg->n_sites < 2 || cfg->d < 2 || cfg->d > 4 || cfg->chi_max < 1 || cfg->chi_max > 1024 ||
        (cfg->precision != MPDO_FP64 && cfg->precision != MPDO_FP32 && cfg->precision != MPDO_BF16X3) ||
        cfg->cutoff_rel < 0.0 ||
        !(cfg->cutoff_rel < 1.0)) {
        g_create_err = "config out of range";
        return MPDO_E_ARG;
    }
    mpdo_ctx c = new mpdo_ctx_s();
    c->cfg = *cfg;
    c->N = cfg->n_sites;
    c->d = cfg->d;
    c->D2 = cfg->d * cfg->d;
    c->chi = cfg->chi_max;
    c->fp32 = cfg->precision != MPDO_FP64;
    c->x3 = cfg->precision == MPDO_BF16X3;
    // default relative cutoff: the rounding floor of the working precision's products
    c->cutoff = cfg->cutoff_rel > 0.0 ? cfg->cutoff_rel : (c->fp32 ? 1e-6 : 1e-14);
    c->st = (hipStream_t)cfg->hip_stream;
    c->dims.assign(c->N + 1, 1);
    c->pending.assign(c->N, std::vector<zc>());
    c->pend_id.assign(c->N, 1);
    *out = c;
    return MPDO_OK;
}

mpdo_status mpdo_destroy(mpdo_ctx c) {
    if (!c) return MPDO_E_ARG;
    if (c->st || c->ready) (void)hipStreamSynchronize(c->st);
    if (c->own_ws && c->ws) (void)hipFree(c->ws);
    if (c->xg) (void)hipFree(c->xg);
    if (c->xgT) (void)hipFree(c->xgT);
    if (c->hbuf) (void)hipHostFree(c->hbuf);
    if (c->hint) (void)hipHostFree(c->hint);
    delete c;
    return MPDO_OK;
}

size_t mpdo_workspace_bytes(const mpdo_config* cfg) {
    if (!cfg || cfg->d < 2 || cfg->d > 4 || cfg->chi_max < 1 || cfg->n_sites < 2) return 0;
    return workspace_for(*cfg);
}

mpdo_status mpdo_bind_workspace(mpdo_ctx c, void* dev, size_t bytes) {
    if (!c || !dev) return MPDO_E_ARG;
    if (c->ws) {
        c->err = "device memory already in use";
        return MPDO_E_STATE;
    }
    if (bytes < workspace_for(c->cfg)) {
        c->err = "workspace smaller than mpdo_workspace_bytes";
        return MPDO_E_NOMEM;
    }
    c->ws = (char*)dev;
    c->ws_bytes = bytes;
    c->own_ws = false;
    return MPDO_OK;
}

mpdo_status mpdo_init_product_state(mpdo_ctx c, const double* rho_sites) {
    mpdo_status g = guard(c);
    if (g != MPDO_OK) return g;
    if (!rho_sites) {
        c->err = "null rho_sites";
        return MPDO_E_ARG;
    }
    const int d = c->d, D2 = c->D2;
    if (!all_finite(rho_sites, (size_t)c->N * D2 * 2)) {
        c->err = "non-finite rho entry";
        return MPDO_E_ARG;
    }
    try {
        if (!c->ready) alloc_state(c);
        std::vector<double> norms(c->N);
        double prod = 1.0;
        for (int j = 0; j < c->N; ++j) {
            double s2 = 0.0;
            for (int e = 0; e < D2 * 2; ++e) s2 += rho_sites[(size_t)j * D2 * 2 + e] * rho_sites[(size_t)j * D2 * 2 + e];
            norms[j] = sqrt(s2);
            if (!(norms[j] > 0.0)) {
                c->err = "zero site density matrix";
                return MPDO_E_ARG;
            }
            if (j > 0) prod *= norms[j];
        }
        // sites j >= 1 normalised (right isometries); site 0 carries the norm (centre)
        for (int j = 0; j < c->N; ++j) {
            const double f = (j == 0) ? prod : 1.0 / norms[j];
            std::vector<double> hostv(D2 * 2);
            for (int e = 0; e < D2 * 2; ++e) hostv[e] = rho_sites[(size_t)j * D2 * 2 + e] * f;
            if (c->fp32) {
                std::vector<float> hf(D2 * 2);
                for (int e = 0; e < D2 * 2; ++e) hf[e] = (float)hostv[e];
                upload(c, c->site[j], hf.data(), hf.size() * sizeof(float));
            } else {
                upload(c, c->site[j], hostv.data(), hostv.size() * sizeof(double));
            }
        }
        c->dims.assign(c->N + 1, 1);
        c->centre = 0;
        c->dir = 1;
        c->pend_id.assign(c->N, 1);
        c->pending.assign(c->N, std::vector<zc>());
        // vec(I) per atom, plus one spare slot N holding vec(I)
        std::vector<zc> o((size_t)(c->N + 1) * D2, zc(0, 0));
        for (int j = 0; j <= c->N; ++j)
            for (int a = 0; a < d; ++a) o[(size_t)j * D2 + a * d + a] = zc(1, 0);
        upload(c, c->ovec, o.data(), o.size() * sizeof(zc));
        std::vector<zc> one(1, zc(1, 0));
        upload(c, c->Lv, one.data(), sizeof(zc));
        upload(c, c->Rv + (size_t)c->N * c->chi * 2, one.data(), sizeof(zc));
        c->lvalid = 0;
        c->rvalid = c->N;
    } catch (const Fail& f) {
        set_err(c, f);
        return f.st;
    }
    return MPDO_OK;
}

static mpdo_status gate_common(mpdo_ctx c, int site, int kind, const double* in, size_t n_in, int n_kraus, int chi,
                               mpdo_trunc_info* info) {
    try {
        if (c->fp32)
            do_update<float>(c, site, kind, in, n_in, n_kraus, chi, info);
        else
            do_update<double>(c, site, kind, in, n_in, n_kraus, chi, info);
    } catch (const Fail& f) {
        set_err(c, f);
        return f.st;
    }
    return MPDO_OK;
}

mpdo_status mpdo_apply_gate(mpdo_ctx c, int site, const double* superop, mpdo_trunc_info* info) {
    mpdo_status g = guard(c);
    if (g != MPDO_OK) return g;
    if (!c->ready) {
        c->err = "state not initialised";
        return MPDO_E_STATE;
    }
    if (site < 0 || site > c->N - 2 || !superop) {
        c->err = "site out of range or null superoperator";
        return MPDO_E_ARG;
    }
    const int m2 = c->D2 * c->D2;
    if (!all_finite(superop, (size_t)m2 * m2 * 2)) {
        c->err = "non-finite superoperator entry";
        return MPDO_E_ARG;
    }
    return gate_common(c, site, 0, superop, (size_t)m2 * m2 * 2, 0, c->chi, info);
}

mpdo_status mpdo_apply_gate_kraus(mpdo_ctx c, int site, int n_kraus, const double* kraus, mpdo_trunc_info* info) {
    mpdo_status g = guard(c);
    if (g != MPDO_OK) return g;
    if (!c->ready) {
        c->err = "state not initialised";
        return MPDO_E_STATE;
    }
    const int dim = c->d * c->d;
    if (site < 0 || site > c->N - 2 || n_kraus < 1 || !kraus) {
        c->err = "bad site or Kraus set";
        return MPDO_E_ARG;
    }
    if (!all_finite(kraus, (size_t)n_kraus * dim * dim * 2)) {
        c->err = "non-finite Kraus entry";
        return MPDO_E_ARG;
    }
    if (cptp_defect(kraus, n_kraus, dim) > 1e-10) {
        c->err = "Kraus set is not trace preserving";
        return MPDO_E_ARG;
    }
    return gate_common(c, site, 1, kraus, (size_t)n_kraus * dim * dim * 2, n_kraus, c->chi, info);
}

mpdo_status mpdo_apply_gate_crosstalk(mpdo_ctx c, int site, int rydberg, const double* u4, mpdo_trunc_info* info) {
    mpdo_status g = guard(c);
    if (g != MPDO_OK) return g;
    if (!c->ready) {
        c->err = "state not initialised";
        return MPDO_E_STATE;
    }
    const int dim = c->d * c->d;
    if (site < 0 || site > c->N - 2 || rydberg < 0 || rydberg >= c->d || !u4) {
        c->err = "bad site, Rydberg level or null unitaries";
        return MPDO_E_ARG;
    }
    if (!all_finite(u4, (size_t)4 * dim * dim * 2)) {
        c->err = "non-finite unitary entry";
        return MPDO_E_ARG;
    }
    for (int q = 0; q < 4; ++q)
        if (cptp_defect(u4 + (size_t)q * dim * dim * 2, 1, dim) > 1e-10) {
            c->err = "crosstalk pair gate is not unitary";
            return MPDO_E_ARG;
        }
    try {
        if (c->fp32) {
            Engine<float> E(*c, c->sf);
            do_crosstalk<float>(c, E, site, rydberg, u4, info);
        } else {
            Engine<double> E(*c, c->sd);
            do_crosstalk<double>(c, E, site, rydberg, u4, info);
        }
    } catch (const Fail& f) {
        set_err(c, f);
        return f.st;
    }
    return MPDO_OK;
}

mpdo_status mpdo_apply_channel(mpdo_ctx c, int site, int n_kraus, const double* kraus) {
    mpdo_status g = guard(c);
    if (g != MPDO_OK) return g;
    if (!c->ready) {
        c->err = "state not initialised";
        return MPDO_E_STATE;
    }
    if (site < 0 || site >= c->N || n_kraus < 1 || !kraus) {
        c->err = "bad site or Kraus set";
        return MPDO_E_ARG;
    }
    if (!all_finite(kraus, (size_t)n_kraus * c->d * c->d * 2)) {
        c->err = "non-finite Kraus entry";
        return MPDO_E_ARG;
    }
    if (cptp_defect(kraus, n_kraus, c->d) > 1e-10) {
        c->err = "Kraus set is not trace preserving";
        return MPDO_E_ARG;
    }
    const int D2 = c->D2;
    std::vector<zc> S1 = superop_from_kraus_1(kraus, n_kraus, c->d);
    if (c->pend_id[site]) {
        c->pending[site] = S1;
    } else {
        std::vector<zc> out((size_t)D2 * D2, zc(0, 0));
        for (int a = 0; a < D2; ++a)
            for (int k = 0; k < D2; ++k)
                for (int b = 0; b < D2; ++b)
                    out[(size_t)a * D2 + b] += S1[(size_t)a * D2 + k] * c->pending[site][(size_t)k * D2 + b];
        c->pending[site].swap(out);
    }
    c->pend_id[site] = 0;
    try {
        set_ovec(c, site);
    } catch (const Fail& f) {
        set_err(c, f);
        return f.st;
    }
    c->lvalid = std::min(c->lvalid, site);
    c->rvalid = std::max(c->rvalid, site + 1);
    return MPDO_OK;
}

mpdo_status mpdo_truncate(mpdo_ctx c, int bond, int chi, mpdo_trunc_info* info) {
    mpdo_status g = guard(c);
    if (g != MPDO_OK) return g;
    if (!c->ready) {
        c->err = "state not initialised";
        return MPDO_E_STATE;
    }
    if (bond < 0 || bond > c->N - 2 || chi < 1 || chi > c->chi) {
        c->err = "bad bond or chi";
        return MPDO_E_ARG;
    }
    const int m2 = c->D2 * c->D2;
    std::vector<double> S((size_t)m2 * m2 * 2, 0.0);
    for (int a = 0; a < m2; ++a) S[((size_t)a * m2 + a) * 2] = 1.0;
    return gate_common(c, bond, 0, S.data(), S.size(), 0, chi, info);
}

mpdo_status mpdo_expect(mpdo_ctx c, int n_terms, const int* first_site, const int* n_sites_in_term, const double* ops,
                        int normalize, double* out) {
    mpdo_status g = guard(c);
    if (g != MPDO_OK) return g;
    if (!c->ready) {
        c->err = "state not initialised";
        return MPDO_E_STATE;
    }
    if (n_terms < 0 || (n_terms > 0 && (!first_site || !n_sites_in_term || !ops || !out))) {
        c->err = "null argument";
        return MPDO_E_ARG;
    }
    size_t nops = 0;
    for (int t = 0; t < n_terms; ++t) {
        if (n_sites_in_term[t] < 1 || first_site[t] < 0 || first_site[t] + n_sites_in_term[t] > c->N) {
            c->err = "term out of range";
            return MPDO_E_ARG;
        }
        nops += n_sites_in_term[t];
    }
    if (!all_finite(ops, nops * c->d * c->d * 2)) {
        c->err = "non-finite operator entry";
        return MPDO_E_ARG;
    }
    try {
        if (c->fp32)
            expect_impl<float>(c, n_terms, first_site, n_sites_in_term, ops, normalize, out);
        else
            expect_impl<double>(c, n_terms, first_site, n_sites_in_term, ops, normalize, out);
    } catch (const Fail& f) {
        set_err(c, f);
        return f.st;
    }
    return MPDO_OK;
}

mpdo_status mpdo_expect2(mpdo_ctx c, int n_terms, const int* first_site, const int* n_sites_in_term,
                         const double* ops, int normalize, double* out) {
    mpdo_status g = guard(c);
    if (g != MPDO_OK) return g;
    if (!c->ready) {
        c->err = "state not initialised";
        return MPDO_E_STATE;
    }
    if (n_terms < 0 || (n_terms > 0 && (!first_site || !n_sites_in_term || !ops || !out))) {
        c->err = "null argument";
        return MPDO_E_ARG;
    }
    size_t nops = 0;
    for (int t = 0; t < n_terms; ++t) {
        if (n_sites_in_term[t] < 1 || first_site[t] < 0 || first_site[t] + n_sites_in_term[t] > c->N) {
            c->err = "term out of range";
            return MPDO_E_ARG;
        }
        nops += n_sites_in_term[t];
    }
    if (!all_finite(ops, nops * c->D2 * c->D2 * 2)) {
        c->err = "non-finite operator entry";
        return MPDO_E_ARG;
    }
    try {
        if (c->fp32)
            expect2_impl<float>(c, n_terms, first_site, n_sites_in_term, ops, normalize, out);
        else
            expect2_impl<double>(c, n_terms, first_site, n_sites_in_term, ops, normalize, out);
    } catch (const Fail& f) {
        set_err(c, f);
        return f.st;
    }
    return MPDO_OK;
}

mpdo_status mpdo_trace(mpdo_ctx c, double* out) {
    mpdo_status g = guard(c);
    if (g != MPDO_OK) return g;
    if (!c->ready || !out) {
        c->err = "state not initialised or null output";
        return c->ready ? MPDO_E_ARG : MPDO_E_STATE;
    }
    try {
        if (c->fp32) {
            Engine<float> E(*c, c->sf);
            E.ensureL(c->N);
            E.read_doubles(E.Lv(c->N), 2, out);
        } else {
            Engine<double> E(*c, c->sd);
            E.ensureL(c->N);
            E.read_doubles(E.Lv(c->N), 2, out);
        }
    } catch (const Fail& f) {
        set_err(c, f);
        return f.st;
    }
    return MPDO_OK;
}

mpdo_status mpdo_bond_dims(mpdo_ctx c, int* out) {
    if (!c || !out) return MPDO_E_ARG;
    for (int j = 0; j < c->N - 1; ++j) out[j] = c->dims[j + 1];
    return MPDO_OK;
}

mpdo_status mpdo_get_site(mpdo_ctx c, int site, double* out, int* shape) {
    mpdo_status g = guard(c);
    if (g != MPDO_OK) return g;
    if (!c->ready || site < 0 || site >= c->N || !shape) {
        c->err = "bad site";
        return MPDO_E_ARG;
    }
    shape[0] = c->dims[site];
    shape[1] = c->D2;
    shape[2] = c->dims[site + 1];
    if (!out) return MPDO_OK;
    const size_t n = (size_t)shape[0] * shape[1] * shape[2] * 2;
    try {
        if (c->fp32) {
            std::vector<float> tmp(n);
            HIPCHK(hipMemcpyAsync(tmp.data(), c->site[site], n * sizeof(float), hipMemcpyDeviceToHost, c->st));
            HIPCHK(hipStreamSynchronize(c->st));
            for (size_t e = 0; e < n; ++e) out[e] = tmp[e];
        } else {
            HIPCHK(hipMemcpyAsync(out, c->site[site], n * sizeof(double), hipMemcpyDeviceToHost, c->st));
            HIPCHK(hipStreamSynchronize(c->st));
        }
    } catch (const Fail& f) {
        set_err(c, f);
        return f.st;
    }
    return MPDO_OK;
}

mpdo_status mpdo_set_state(mpdo_ctx c, const int* bond_dims, const double* sites, int centre) {
    mpdo_status g = guard(c);
    if (g != MPDO_OK) return g;
    if (!bond_dims || !sites || centre < -1 || centre >= c->N) {
        c->err = "set_state: null pointer or centre out of range";
        return MPDO_E_ARG;
    }
    std::vector<int> dims(c->N + 1, 1);
    size_t total = 0;
    for (int j = 0; j + 1 < c->N; ++j) {
        if (bond_dims[j] < 1 || bond_dims[j] > c->chi) {
            c->err = "set_state: bond dimension outside [1, chi_max]";
            return MPDO_E_ARG;
        }
        dims[j + 1] = bond_dims[j];
    }
    for (int j = 0; j < c->N; ++j) total += (size_t)dims[j] * c->D2 * dims[j + 1] * 2;
    if (!all_finite(sites, total)) {
        c->err = "set_state: non-finite entry";
        return MPDO_E_ARG;
    }
    try {
        if (!c->ready) {
            // ovec and the trace-vector ends as for a product state, then the sites below
            std::vector<double> rho((size_t)c->N * c->D2 * 2, 0.0);
            for (int j = 0; j < c->N; ++j) rho[(size_t)j * c->D2 * 2] = 1.0;
            const mpdo_status st0 = mpdo_init_product_state(c, rho.data());
            if (st0 != MPDO_OK) return st0;
        }
        size_t off = 0;
        for (int j = 0; j < c->N; ++j) {
            const size_t n = (size_t)dims[j] * c->D2 * dims[j + 1] * 2;
            if (c->fp32) {
                std::vector<float> hf(n);
                for (size_t e = 0; e < n; ++e) hf[e] = (float)sites[off + e];
                upload(c, c->site[j], hf.data(), n * sizeof(float));
            } else {
                upload(c, c->site[j], sites + off, n * sizeof(double));
            }
            off += n;
        }
        HIPCHK(hipStreamSynchronize(c->st));
        c->dims = dims;
        c->pend_id.assign(c->N, 1);
        c->pending.assign(c->N, std::vector<zc>());
        c->lvalid = 0;
        c->rvalid = c->N;
        c->dir = 1;
        if (centre >= 0) {
            c->centre = centre;
        } else {
            // sweep the centre from atom 0 to atom N-1: range-basis moves keep rho exactly
            c->centre = 0;
            if (c->fp32) {
                Engine<float> E(*c, c->sf);
                for (int j = 0; j + 1 < c->N; ++j) E.move_right(j);
                E.orth_verify();
            } else {
                Engine<double> E(*c, c->sd);
                for (int j = 0; j + 1 < c->N; ++j) E.move_right(j);
                E.orth_verify();
            }
        }
    } catch (const Fail& f) {
        set_err(c, f);
        return f.st;
    }
    return MPDO_OK;
}

mpdo_status mpdo_move_centre(mpdo_ctx c, int site) {
    mpdo_status g = guard(c);
    if (g != MPDO_OK) return g;
    if (!c->ready || site < 0 || site >= c->N) {
        c->err = "move_centre: no state or site out of range";
        return MPDO_E_ARG;
    }
    try {
        if (c->fp32) {
            Engine<float> E(*c, c->sf);
            while (c->centre < site) E.move_right(c->centre);
            while (c->centre > site) E.move_left(c->centre);
            E.orth_verify();
        } else {
            Engine<double> E(*c, c->sd);
            while (c->centre < site) E.move_right(c->centre);
            while (c->centre > site) E.move_left(c->centre);
            E.orth_verify();
        }
    } catch (const Fail& f) {
        set_err(c, f);
        return f.st;
    }
    return MPDO_OK;
}

mpdo_status mpdo_canonical_centre(mpdo_ctx c, int* out) {
    mpdo_status g = guard(c);
    if (g != MPDO_OK) return g;
    if (!out || !c->ready) {
        c->err = "canonical_centre: null pointer or no state";
        return MPDO_E_ARG;
    }
    out[0] = c->centre;
    out[1] = c->dir;
    return MPDO_OK;
}

mpdo_status mpdo_synchronize(mpdo_ctx c) {
    if (!c) return MPDO_E_ARG;
    if (hipStreamSynchronize(c->st) != hipSuccess) {
        c->err = "stream synchronisation failed";
        c->poisoned = true;
        return MPDO_E_DEVICE;
    }
    return MPDO_OK;
}

mpdo_status mpdo_profile_enable(mpdo_ctx c, int enable) {
    if (!c) return MPDO_E_ARG;
    if (enable) {
        c->prof.reset(new EventProf());
        for (double& x : c->prof_acc) x = 0.0;
    } else if (c->prof) {
        c->prof->collect(c->prof_acc);
        c->prof.reset();
    }
    return MPDO_OK;
}

mpdo_status mpdo_profile_enable_mask(mpdo_ctx c, unsigned family_mask) {
    if (!c) return MPDO_E_ARG;
    if (c->prof) {
        c->prof->collect(c->prof_acc);
        c->prof.reset();
    }
    if (family_mask) {
        EventProf* p = new EventProf();
        p->mask = family_mask;
        c->prof.reset(p);
        for (double& x : c->prof_acc) x = 0.0;
    }
    return MPDO_OK;
}

mpdo_status mpdo_profile_stride(mpdo_ctx c, int stride) {
    if (!c || stride < 1) return MPDO_E_ARG;
    if (c->prof) {
        c->prof->stride = (unsigned)stride;
        for (auto& x : c->prof->seen) x = 0;
    }
    return MPDO_OK;
}

mpdo_status mpdo_profile_read(mpdo_ctx c, double* out, int n_families) {
    if (!c || !out || n_families < 0) return MPDO_E_ARG;
    if (c->prof) c->prof->collect(c->prof_acc);
    const int nf = std::min(n_families, (int)PF_COUNT);
    for (int f = 0; f < nf; ++f)
        for (int q = 0; q < 4; ++q) out[4 * f + q] = c->prof_acc[4 * f + q];
    return MPDO_OK;
}

mpdo_status mpdo_cgemm(int precision, int M, int N, int K, const double* alpha, const double* A, int op_a,
                       const double* B, int op_b, const double* beta, double* C, int split_k) {
    if (M < 0 || N < 0 || K < 0 || !alpha || !beta || (M * (long)N > 0 && !C) || (M * (long)K > 0 && !A) ||
        (K * (long)N > 0 && !B) || op_a < 0 || op_a > 2 || op_b < 0 || op_b > 2 ||
        (precision != MPDO_FP64 && precision != MPDO_FP32 && precision != MPDO_BF16X3) ||
        (long)M * K > (1L << 28) || (long)K * N > (1L << 28) || (long)M * N > (1L << 28)) {
        g_create_err = "bad product arguments";
        return MPDO_E_ARG;
    }
    try {
        if (precision == MPDO_FP64) run_cgemm<double>(false, M, N, K, alpha, A, op_a, B, op_b, beta, C, split_k);
        else run_cgemm<float>(precision == MPDO_BF16X3, M, N, K, alpha, A, op_a, B, op_b, beta, C, split_k);
    } catch (const Fail& f) {
        g_create_err = f.msg;
        return f.st;
    }
    return MPDO_OK;
}

mpdo_status mpdo_eigh(int n, const double* H, double tau, int cap, int* m, double* evals, double* V) {
    if (n < 1 || n > TRI_MAX || cap < 0 || cap > n || !(tau >= 0.0) || !H || !m || !evals || (cap > 0 && !V)) {
        g_create_err = "bad eigensolver arguments";
        return MPDO_E_ARG;
    }
    *m = 0;
    if (cap == 0) return MPDO_OK;
    try {
        run_eigh(n, H, tau, cap, m, evals, V);
    } catch (const Fail& f) {
        g_create_err = f.msg;
        return f.st;
    }
    return MPDO_OK;
}

const char* mpdo_last_error(mpdo_ctx c) { return c ? c->err.c_str() : g_create_err.c_str(); }

const char* mpdo_version(void) { return "libmpdo 0.1 (HIP, gfx950)"; }

}  // extern "C"
