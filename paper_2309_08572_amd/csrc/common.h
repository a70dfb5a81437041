// Shared device/host definitions for libmpdo (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpdo {

// A strided complex matrix view: element (r, c) sits at p[2 * (r * rs + c * cs)]
// (interleaved re, im).  conj = 1 reads the complex conjugate.
template <typename T>
struct CView {
    T* p;
    long rs;
    long cs;
    int conj;
};

template <typename T>
__host__ __device__ inline CView<T> view(T* p, long rs, long cs, int conj = 0) {
    CView<T> v;
    v.p = p;
    v.rs = rs;
    v.cs = cs;
    v.conj = conj;
    return v;
}

// Hermitian adjoint of a view: (r, c) -> conj((c, r)).
template <typename T>
__host__ __device__ inline CView<T> adj(CView<T> v) {
    CView<T> w;
    w.p = v.p;
    w.rs = v.cs;
    w.cs = v.rs;
    w.conj = !v.conj;
    return w;
}

template <typename T>
__host__ __device__ inline CView<T> trans(CView<T> v) {
    CView<T> w;
    w.p = v.p;
    w.rs = v.cs;
    w.cs = v.rs;
    w.conj = v.conj;
    return w;
}

struct cd {
    double re, im;
};

// Kernel families timed by the profiling sink.
enum ProfFamily { PF_GEMM = 0, PF_EIG_PAIR = 1, PF_EIG_ROT = 2, PF_EIG_SMALL = 3, PF_PHYS = 4,
                  PF_TRANSFER = 5, PF_OTHER = 6, PF_TRI_REDUCE = 7, PF_TRI_SOLVE = 8, PF_TRI_BACK = 9,
                  PF_THETA = 10, PF_PCHOL = 11, PF_SPLIT_SUM = 12, PF_COUNT = 13 };

// Receives begin/end marks around kernel launches when measurement is on (else null).
struct ProfSink {
    virtual void begin(hipStream_t s, int family) = 0;
    virtual void end(hipStream_t s, int family, double flop, double bytes) = 0;
    // replaces the work of the last launch recorded for family (once the host knows it)
    virtual void amend(int family, double flop, double bytes) {}
    // An event pair for one kernel that the caller launches with hipExtLaunchKernelGGL, which
    // stamps the kernel's own start and end (no dispatch time in between); false when the
    // family is not recorded.  kernel_done records the pair with the launch's work.
    virtual bool kernel_events(int family, hipEvent_t* a, hipEvent_t* b) { return false; }
    virtual void kernel_done(int family, hipEvent_t a, hipEvent_t b, double flop, double bytes) {}
    virtual ~ProfSink() {}
};

// Forwards to another sink with one family renamed (e.g. the GEMMs that form theta, timed
// apart from the other products).
struct ProfRename : public ProfSink {
    ProfSink* to;
    int from_fam, to_fam;
    ProfRename(ProfSink* t, int f, int g) : to(t), from_fam(f), to_fam(g) {}
    void begin(hipStream_t s, int family) override { to->begin(s, family == from_fam ? to_fam : family); }
    void end(hipStream_t s, int family, double flop, double bytes) override {
        to->end(s, family == from_fam ? to_fam : family, flop, bytes);
    }
    void amend(int family, double flop, double bytes) override {
        to->amend(family == from_fam ? to_fam : family, flop, bytes);
    }
    bool kernel_events(int family, hipEvent_t* a, hipEvent_t* b) override {
        return to->kernel_events(family == from_fam ? to_fam : family, a, b);
    }
    void kernel_done(int family, hipEvent_t a, hipEvent_t b, double flop, double bytes) override {
        to->kernel_done(family == from_fam ? to_fam : family, a, b, flop, bytes);
    }
};

}  // namespace mpdo
