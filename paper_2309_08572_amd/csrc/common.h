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

}  // namespace mpdo
