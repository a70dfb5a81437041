// Surrogate MLP on gfx950: FP32 parameters and activations, BF16 matrix-core products with
// FP32 accumulation, hand-written forward, backward and Adam kernels.
//
// Network: h_0 = x; z_l = h_l W_l^T + b_l; h_{l+1} = tanh(z_l) for hidden layers, y = z_{L-1}.
// Loss: mean squared error over batch and outputs.  Parameters packed as W_0 (row-major,
// out x in), b_0, W_1, b_1, ...
//
//   sgemm_bf16_kernel   C = alpha op(A) op(B) + beta C on 64 x 64 tiles, k-step 32; operands
//                       rounded to BF16 (nearest even) when staged in LDS; 4 waves, each a
//                       32 x 32 quadrant of 2 x 2 MFMA 16x16x16 tiles; strided views carry the
//                       transposes of the forward and backward products
//   bias_act_kernel     z + b, tanh for hidden layers
//   mse_grad_kernel     d loss / d y and the per-block loss partials
//   tanh_back_kernel    dz = dh (1 - h^2)
//   colsum_kernel       bias gradients
//   adam_kernel         bias-corrected Adam on the packed parameters
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/mpdo_mlp.h"

namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

struct RV {   // read view: element (i, j) at p[i rs + j cs]
    const float* p;
    long rs, cs;
};

constexpr int GB = 64;   // tile rows / columns
constexpr int GK = 32;   // k-step

__device__ __forceinline__ unsigned short to_bf16(float f) {
    const unsigned u = __float_as_uint(f);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);   // round to nearest even
}

__global__ __launch_bounds__(256) void sgemm_bf16_kernel(int M, int N, int K, float alpha, RV A, RV B, float beta,
                                                         float* __restrict__ C, long ldc) {
    __shared__ unsigned short sA[GB][GK + 4];
    __shared__ unsigned short sB[GK][GB + 4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
    const int m0 = blockIdx.y * GB, n0 = blockIdx.x * GB;
    const bool a_kfast = A.cs == 1, b_nfast = B.cs == 1;
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
        for (int q = 0; q < (GB * GK) / 256; ++q) {
            const int e = tid + 256 * q;
            const int m = a_kfast ? e / GK : e % GB, k = a_kfast ? e % GK : e / GB;
            const int gm = m0 + m, gk = k0 + k;
            const float v = (gm < M && gk < K) ? A.p[(long)gm * A.rs + (long)gk * A.cs] : 0.f;
            sA[m][k] = to_bf16(v);
        }
#pragma unroll
        for (int q = 0; q < (GB * GK) / 256; ++q) {
            const int e = tid + 256 * q;
            const int n = b_nfast ? e % GB : e / GK, k = b_nfast ? e / GB : e % GK;
            const int gn = n0 + n, gk = k0 + k;
            const float v = (gn < N && gk < K) ? B.p[(long)gk * B.rs + (long)gn * B.cs] : 0.f;
            sB[k][n] = to_bf16(v);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; kk += 16) {
            s4 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) a[i][j] = (short)sA[wr * 32 + i * 16 + li][kk + 4 * lk + j];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) b[i][j] = (short)sB[kk + 4 * lk + j][wc * 32 + i * 16 + li];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // lane holds column li and rows 4 lk + r of each 16 x 16 tile
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wr * 32 + i * 16 + 4 * lk + r, gn = n0 + wc * 32 + j * 16 + li;
                if (gm >= M || gn >= N) continue;
                float v = alpha * acc[i][j][r];
                if (beta != 0.f) v += beta * C[(long)gm * ldc + gn];
                C[(long)gm * ldc + gn] = v;
            }
}

__global__ void bias_act_kernel(float* __restrict__ Z, const float* __restrict__ b, int rows, int cols, int act) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)rows * cols) return;
    const float v = Z[idx] + b[idx % cols];
    Z[idx] = act ? tanhf(v) : v;
}

// dy = 2 (y - t) / (rows cols); part[block] = sum of (y - t)^2 over the block's entries
__global__ void mse_grad_kernel(const float* __restrict__ y, const float* __restrict__ t, long n, float scale,
                                float* __restrict__ dy, float* __restrict__ part) {
    __shared__ float s[256];
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    float e = 0.f;
    if (idx < n) {
        const float r = y[idx] - t[idx];
        dy[idx] = 2.f * r * scale;
        e = r * r;
    }
    s[threadIdx.x] = e;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void tanh_back_kernel(float* __restrict__ dh, const float* __restrict__ h, long n) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const float v = h[idx];
    dh[idx] *= 1.f - v * v;
}

// out[c] = sum_r X[r][c]
__global__ void colsum_kernel(const float* __restrict__ X, int rows, int cols, float* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int r = 0; r < rows; ++r) s += X[(long)r * cols + c];
    out[c] = s;
}

__global__ void fill_kernel(float* __restrict__ p, long n, float v) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) p[idx] = v;
}

__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, long n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const float gi = g[idx];
    const float mi = b1 * m[idx] + (1.f - b1) * gi;
    const float vi = b2 * v[idx] + (1.f - b2) * gi * gi;
    m[idx] = mi;
    v[idx] = vi;
    w[idx] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline unsigned nblk(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

struct mpdo_mlp_s {
    int L = 0;                     // layers
    std::vector<int> w;            // widths, L + 1
    int max_batch = 0;
    hipStream_t st = nullptr;
    long np = 0;                   // parameter count
    std::vector<long> woff, boff;  // offsets of W_l and b_l in the packed vector
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
    std::vector<float*> h;         // h_0 .. h_L (max_batch x w_l)
    float *t = nullptr, *dA = nullptr, *dB = nullptr, *part = nullptr, *wout = nullptr;
    float* hpin = nullptr;         // pinned host staging
    long adam_step = 0;
    std::string err;
};

namespace {

struct MlpFail {
    mpdo_status st;
    std::string msg;
};

#define MLPCHK(x)                                                                   \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) throw MlpFail{MPDO_E_DEVICE, hipGetErrorString(e_)};  \
    } while (0)

void gemm(mpdo_mlp n, int M, int N, int K, float alpha, RV A, RV B, float beta, float* C, long ldc) {
    if (M <= 0 || N <= 0) return;
    dim3 grid((N + GB - 1) / GB, (M + GB - 1) / GB);
    hipLaunchKernelGGL(sgemm_bf16_kernel, grid, dim3(256), 0, n->st, M, N, K, alpha, A, B, beta, C, ldc);
    MLPCHK(hipGetLastError());
}

void upload(mpdo_mlp n, float* dst, const float* src, long count) {
    MLPCHK(hipMemcpyAsync(dst, src, count * sizeof(float), hipMemcpyHostToDevice, n->st));
}

void download(mpdo_mlp n, float* dst, const float* src, long count) {
    MLPCHK(hipMemcpyAsync(dst, src, count * sizeof(float), hipMemcpyDeviceToHost, n->st));
    MLPCHK(hipStreamSynchronize(n->st));
}

// forward pass of `batch` rows whose inputs are already in h[0]; outputs land in h[L]
void forward(mpdo_mlp n, int batch) {
    for (int l = 0; l < n->L; ++l) {
        const int in = n->w[l], out = n->w[l + 1];
        // z = h_l W_l^T: B operand W^T is (in x out), element (k, j) = W[j][k]
        gemm(n, batch, out, in, 1.f, RV{n->h[l], in, 1}, RV{n->params + n->woff[l], 1, in}, 0.f, n->h[l + 1], out);
        hipLaunchKernelGGL(bias_act_kernel, dim3(nblk((long)batch * out)), dim3(256), 0, n->st, n->h[l + 1],
                           n->params + n->boff[l], batch, out, l < n->L - 1 ? 1 : 0);
        MLPCHK(hipGetLastError());
    }
}

// backward pass from dz of the output layer (in dA); writes grads; leaves d loss / d x in the
// last used buffer when want_dx (returned)
float* backward(mpdo_mlp n, int batch, bool want_params, bool want_dx) {
    float* dz = n->dA;
    float* dh = n->dB;
    for (int l = n->L - 1; l >= 0; --l) {
        const int in = n->w[l], out = n->w[l + 1];
        if (want_params) {
            // dW = dz^T h_l : A = dz^T (out x batch), element (i, k) = dz[k][i]
            gemm(n, out, in, batch, 1.f, RV{dz, 1, out}, RV{n->h[l], in, 1}, 0.f, n->grads + n->woff[l], in);
            hipLaunchKernelGGL(colsum_kernel, dim3(nblk(out)), dim3(256), 0, n->st, dz, batch, out,
                               n->grads + n->boff[l]);
            MLPCHK(hipGetLastError());
        }
        if (l > 0 || want_dx) {
            // dh = dz W_l (batch x in)
            gemm(n, batch, in, out, 1.f, RV{dz, out, 1}, RV{n->params + n->woff[l], in, 1}, 0.f, dh, in);
            if (l > 0) {
                hipLaunchKernelGGL(tanh_back_kernel, dim3(nblk((long)batch * in)), dim3(256), 0, n->st, dh, n->h[l],
                                   (long)batch * in);
                MLPCHK(hipGetLastError());
            }
            std::swap(dz, dh);
        }
    }
    return dz;
}

// loss of the batch already forwarded against targets in t; d loss / d y -> dA
float loss_grad_out(mpdo_mlp n, int batch) {
    const int out = n->w[n->L];
    const long cnt = (long)batch * out;
    const unsigned nb = nblk(cnt);
    hipLaunchKernelGGL(mse_grad_kernel, dim3(nb), dim3(256), 0, n->st, n->h[n->L], n->t, cnt, 1.f / (float)cnt,
                       n->dA, n->part);
    MLPCHK(hipGetLastError());
    download(n, n->hpin, n->part, nb);
    double s = 0.0;
    for (unsigned i = 0; i < nb; ++i) s += n->hpin[i];
    return (float)(s / (double)cnt);
}

mpdo_status guard(mpdo_mlp n, int batch) {
    if (!n) return MPDO_E_ARG;
    if (batch < 1 || batch > n->max_batch) {
        n->err = "batch out of range";
        return MPDO_E_ARG;
    }
    return MPDO_OK;
}

bool finite(const float* p, long cnt) {
    for (long i = 0; i < cnt; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace

extern "C" {

size_t mpdo_mlp_param_count(int n_layers, const int* widths) {
    if (n_layers < 1 || !widths) return 0;
    size_t c = 0;
    for (int l = 0; l < n_layers; ++l) c += (size_t)widths[l + 1] * widths[l] + widths[l + 1];
    return c;
}

mpdo_status mpdo_mlp_create(int n_layers, const int* widths, int max_batch, void* hip_stream, mpdo_mlp* out) {
    if (!out || !widths || n_layers < 1 || n_layers > 16 || max_batch < 1 || max_batch > (1 << 20))
        return MPDO_E_ARG;
    for (int l = 0; l <= n_layers; ++l)
        if (widths[l] < 1 || widths[l] > 4096) return MPDO_E_ARG;
    mpdo_mlp n = new mpdo_mlp_s();
    n->L = n_layers;
    n->w.assign(widths, widths + n_layers + 1);
    n->max_batch = max_batch;
    n->st = (hipStream_t)hip_stream;
    long pos = 0;
    for (int l = 0; l < n_layers; ++l) {
        n->woff.push_back(pos);
        pos += (long)widths[l + 1] * widths[l];
        n->boff.push_back(pos);
        pos += widths[l + 1];
    }
    n->np = pos;
    int wmax = 0;
    for (int x : n->w) wmax = wmax > x ? wmax : x;
    bool ok = true;
    auto take = [&](float** p, long cnt) {
        if (hipMalloc((void**)p, (size_t)cnt * sizeof(float)) != hipSuccess) ok = false;
    };
    take(&n->params, pos);
    take(&n->grads, pos);
    take(&n->m, pos);
    take(&n->v, pos);
    n->h.assign(n_layers + 1, nullptr);
    for (int l = 0; l <= n_layers; ++l) take(&n->h[l], (long)max_batch * widths[l]);
    take(&n->t, (long)max_batch * widths[n_layers]);
    take(&n->dA, (long)max_batch * wmax);
    take(&n->dB, (long)max_batch * wmax);
    take(&n->part, (long)nblk((long)max_batch * widths[n_layers]) + 1);
    take(&n->wout, widths[n_layers]);
    const size_t pin = (size_t)std::max<long>((long)max_batch * wmax, pos) * sizeof(float);
    if (hipHostMalloc((void**)&n->hpin, pin) != hipSuccess) ok = false;
    if (!ok) {
        mpdo_mlp_destroy(n);
        return MPDO_E_NOMEM;
    }
    hipLaunchKernelGGL(fill_kernel, dim3(nblk(pos)), dim3(256), 0, n->st, n->m, pos, 0.f);
    hipLaunchKernelGGL(fill_kernel, dim3(nblk(pos)), dim3(256), 0, n->st, n->v, pos, 0.f);
    hipLaunchKernelGGL(fill_kernel, dim3(nblk(pos)), dim3(256), 0, n->st, n->params, pos, 0.f);
    if (hipStreamSynchronize(n->st) != hipSuccess) {
        mpdo_mlp_destroy(n);
        return MPDO_E_DEVICE;
    }
    *out = n;
    return MPDO_OK;
}

mpdo_status mpdo_mlp_destroy(mpdo_mlp n) {
    if (!n) return MPDO_E_ARG;
    if (n->st) (void)hipStreamSynchronize(n->st);
    else (void)hipDeviceSynchronize();
    float* bufs[] = {n->params, n->grads, n->m, n->v, n->t, n->dA, n->dB, n->part, n->wout};
    for (float* p : bufs)
        if (p) (void)hipFree(p);
    for (float* p : n->h)
        if (p) (void)hipFree(p);
    if (n->hpin) (void)hipHostFree(n->hpin);
    delete n;
    return MPDO_OK;
}

mpdo_status mpdo_mlp_set_params(mpdo_mlp n, const float* params) {
    if (!n || !params) return MPDO_E_ARG;
    if (!finite(params, n->np)) {
        n->err = "non-finite parameter";
        return MPDO_E_ARG;
    }
    try {
        upload(n, n->params, params, n->np);
        hipLaunchKernelGGL(fill_kernel, dim3(nblk(n->np)), dim3(256), 0, n->st, n->m, n->np, 0.f);
        hipLaunchKernelGGL(fill_kernel, dim3(nblk(n->np)), dim3(256), 0, n->st, n->v, n->np, 0.f);
        MLPCHK(hipGetLastError());
        MLPCHK(hipStreamSynchronize(n->st));
        n->adam_step = 0;
    } catch (const MlpFail& f) {
        n->err = f.msg;
        return f.st;
    }
    return MPDO_OK;
}

mpdo_status mpdo_mlp_get_params(mpdo_mlp n, float* params) {
    if (!n || !params) return MPDO_E_ARG;
    try {
        download(n, n->hpin, n->params, n->np);
        memcpy(params, n->hpin, n->np * sizeof(float));
    } catch (const MlpFail& f) {
        n->err = f.msg;
        return f.st;
    }
    return MPDO_OK;
}

mpdo_status mpdo_mlp_forward(mpdo_mlp n, int batch, const float* x, float* y) {
    mpdo_status g = guard(n, batch);
    if (g != MPDO_OK) return g;
    if (!x || !y || !finite(x, (long)batch * n->w[0])) {
        n->err = "null or non-finite input";
        return MPDO_E_ARG;
    }
    try {
        upload(n, n->h[0], x, (long)batch * n->w[0]);
        forward(n, batch);
        const long cnt = (long)batch * n->w[n->L];
        download(n, n->hpin, n->h[n->L], cnt);
        memcpy(y, n->hpin, cnt * sizeof(float));
    } catch (const MlpFail& f) {
        n->err = f.msg;
        return f.st;
    }
    return MPDO_OK;
}

mpdo_status mpdo_mlp_loss_grad(mpdo_mlp n, int batch, const float* x, const float* t, float* loss, float* grads) {
    mpdo_status g = guard(n, batch);
    if (g != MPDO_OK) return g;
    if (!x || !t || !loss || !finite(x, (long)batch * n->w[0]) || !finite(t, (long)batch * n->w[n->L])) {
        n->err = "null or non-finite input";
        return MPDO_E_ARG;
    }
    try {
        upload(n, n->h[0], x, (long)batch * n->w[0]);
        upload(n, n->t, t, (long)batch * n->w[n->L]);
        forward(n, batch);
        *loss = loss_grad_out(n, batch);
        backward(n, batch, true, false);
        if (grads) {
            download(n, n->hpin, n->grads, n->np);
            memcpy(grads, n->hpin, n->np * sizeof(float));
        }
    } catch (const MlpFail& f) {
        n->err = f.msg;
        return f.st;
    }
    return MPDO_OK;
}

mpdo_status mpdo_mlp_train_step(mpdo_mlp n, int batch, const float* x, const float* t, float lr, float* loss) {
    mpdo_status g = guard(n, batch);
    if (g != MPDO_OK) return g;
    if (!x || !t || !finite(x, (long)batch * n->w[0]) || !finite(t, (long)batch * n->w[n->L]) || !(lr > 0.f)) {
        n->err = "null or non-finite input, or lr <= 0";
        return MPDO_E_ARG;
    }
    try {
        upload(n, n->h[0], x, (long)batch * n->w[0]);
        upload(n, n->t, t, (long)batch * n->w[n->L]);
        forward(n, batch);
        const float l = loss_grad_out(n, batch);
        if (loss) *loss = l;
        backward(n, batch, true, false);
        ++n->adam_step;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.f - powf(b1, (float)n->adam_step), c2 = 1.f - powf(b2, (float)n->adam_step);
        hipLaunchKernelGGL(adam_kernel, dim3(nblk(n->np)), dim3(256), 0, n->st, n->params, n->grads, n->m, n->v,
                           n->np, lr, b1, b2, 1e-8f, c1, c2);
        MLPCHK(hipGetLastError());
    } catch (const MlpFail& f) {
        n->err = f.msg;
        return f.st;
    }
    return MPDO_OK;
}

mpdo_status mpdo_mlp_input_grad(mpdo_mlp n, int batch, const float* x, const float* w_out, float* y, float* dx) {
    mpdo_status g = guard(n, batch);
    if (g != MPDO_OK) return g;
    if (!x || !w_out || !dx || !finite(x, (long)batch * n->w[0]) || !finite(w_out, n->w[n->L])) {
        n->err = "null or non-finite input";
        return MPDO_E_ARG;
    }
    try {
        const int out = n->w[n->L], in = n->w[0];
        upload(n, n->h[0], x, (long)batch * in);
        forward(n, batch);
        // dz of the output layer: w_out in every row
        std::vector<float> rows((size_t)batch * out);
        for (int b = 0; b < batch; ++b)
            for (int k = 0; k < out; ++k) rows[(size_t)b * out + k] = w_out[k];
        upload(n, n->dA, rows.data(), (long)batch * out);
        MLPCHK(hipStreamSynchronize(n->st));   // rows is host memory of this frame
        float* d = backward(n, batch, false, true);
        if (y) {
            download(n, n->hpin, n->h[n->L], (long)batch * out);
            memcpy(y, n->hpin, (size_t)batch * out * sizeof(float));
        }
        download(n, n->hpin, d, (long)batch * in);
        memcpy(dx, n->hpin, (size_t)batch * in * sizeof(float));
    } catch (const MlpFail& f) {
        n->err = f.msg;
        return f.st;
    }
    return MPDO_OK;
}

const char* mpdo_mlp_last_error(mpdo_mlp n) { return n ? n->err.c_str() : "null handle"; }

}  // extern "C"
