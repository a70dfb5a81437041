// Batched execution of independent circuits: a native worker pool over the C ABI.
//
// Each worker thread owns one HIP stream and a slice of the device workspace; it takes
// circuits from a shared atomic counter over a list ordered by estimated cost, largest first
// (bond cap, then the number of two-site updates; so circuits of one bond cap run together and
// the long ones do not start last), builds a context for the circuit on its stream,
// applies the circuit's Kraus maps in order (two-site updates with PPT, queued single-atom
// maps), evaluates the observables and records them.  Circuits share no state, so the
// latency-bound kernels of different circuits (Jacobi rounds, small GEMMs) fill the GPU
// together.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <string.h>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mpdo.h"

namespace mpdo {
void set_thread_error(const std::string& msg);
}

namespace {

bool circuit_ok(const mpdo_circuit& c) {
    if (c.n_sites < 2 || c.d < 2 || c.d > 4 || c.chi_max < 1 || c.chi_max > 1024 || c.n_ops < 0 || c.n_terms < 0)
        return false;
    if (!c.rho0 || (c.n_ops > 0 && (!c.op_kind || !c.op_site || !c.op_set || !c.set_count || !c.set_offset ||
                                    !c.kraus)))
        return false;
    if (c.n_terms > 0 && (!c.term_first || !c.term_len || !c.term_ops || !c.out)) return false;
    return true;
}

mpdo_config config_of(const mpdo_circuit& c, void* stream) {
    mpdo_config cfg;
    memset(&cfg, 0, sizeof(cfg));
    cfg.n_sites = c.n_sites;
    cfg.d = c.d;
    cfg.chi_max = c.chi_max;
    cfg.precision = c.precision;
    cfg.cutoff_rel = 0.0;
    cfg.ppt = c.ppt;
    cfg.renorm_trace = 0;
    cfg.hip_stream = stream;
    return cfg;
}

// Relative cost of a circuit: two-site updates times the cube of its bond cap (an update's
// products and eigenproblems grow with the third power of the bond dimension).
double cost_of(const mpdo_circuit& c) {
    long two = 0;
    for (int k = 0; k < c.n_ops; ++k) two += c.op_kind[k] == 0;
    const double chi = (double)c.chi_max;
    return (double)two * chi * chi * chi;
}

// The first failure of a batch and its message (passed to the calling thread's
// mpdo_last_error(NULL) when the batch returns).
struct FirstError {
    std::mutex mu;
    std::string msg;
    void note(int circuit, const char* what) {
        std::lock_guard<std::mutex> lk(mu);
        if (msg.empty()) msg = "circuit " + std::to_string(circuit) + ": " + (what ? what : "");
    }
};

mpdo_status run_one(mpdo_circuit& c, hipStream_t stream, char* ws, size_t ws_bytes, int index, FirstError& fe) {
    mpdo_config cfg = config_of(c, (void*)stream);
    mpdo_ctx ctx = nullptr;
    mpdo_status st = mpdo_create(&cfg, &ctx);
    if (st != MPDO_OK) {
        fe.note(index, mpdo_last_error(nullptr));
        return st;
    }
    st = mpdo_bind_workspace(ctx, ws, ws_bytes);
    if (st == MPDO_OK) st = mpdo_init_product_state(ctx, c.rho0);
    int k = 0;
    for (; st == MPDO_OK && k < c.n_ops; ++k) {
        const int set = c.op_set[k];
        const double* K = c.kraus + 2 * c.set_offset[set];
        if (c.op_kind[k] == 0)
            st = mpdo_apply_gate_kraus(ctx, c.op_site[k], c.set_count[set], K, nullptr);
        else
            st = mpdo_apply_channel(ctx, c.op_site[k], c.set_count[set], K);
    }
    // MPDO_DEBUG_FAILURES=1: the message of a failed circuit (the context and its message end here)
    if (st != MPDO_OK && getenv("MPDO_DEBUG_FAILURES"))
        fprintf(stderr, "[mpdo batch] circuit failed at op %d of %d (site %d): status %d: %s\n", k - 1, c.n_ops,
                k > 0 ? c.op_site[k - 1] : -1, (int)st, mpdo_last_error(ctx));
    if (st == MPDO_OK && c.n_terms > 0)
        st = mpdo_expect(ctx, c.n_terms, c.term_first, c.term_len, c.term_ops, 1, c.out);
    if (st == MPDO_OK && c.out_trace) st = mpdo_trace(ctx, c.out_trace);
    if (st == MPDO_OK && c.out_bonds) st = mpdo_bond_dims(ctx, c.out_bonds);
    if (st != MPDO_OK) fe.note(index, mpdo_last_error(ctx));
    mpdo_destroy(ctx);
    return st;
}

}  // namespace

extern "C" {

size_t mpdo_batch_workspace_bytes(const mpdo_circuit* circuits, int n_circuits) {
    size_t mx = 0;
    for (int i = 0; i < n_circuits; ++i) {
        if (!circuit_ok(circuits[i])) continue;
        mpdo_config cfg = config_of(circuits[i], nullptr);
        const size_t b = mpdo_workspace_bytes(&cfg);
        if (b > mx) mx = b;
    }
    return (mx + 4095) & ~(size_t)4095;
}

mpdo_status mpdo_run_batch(mpdo_circuit* circuits, int n_circuits, int n_workers, void* device_workspace,
                           size_t workspace_bytes) {
    if (!circuits || n_circuits < 0 || n_workers < 1 || n_workers > 64) return MPDO_E_ARG;
    for (int i = 0; i < n_circuits; ++i)
        if (!circuit_ok(circuits[i])) return MPDO_E_ARG;
    if (n_circuits == 0) return MPDO_OK;
    if (n_workers > n_circuits) n_workers = n_circuits;
    const size_t per = mpdo_batch_workspace_bytes(circuits, n_circuits);
    char* base = (char*)device_workspace;
    bool own = false;
    if (!base) {
        void* p = nullptr;
        if (hipMalloc(&p, per * (size_t)n_workers) != hipSuccess) return MPDO_E_NOMEM;
        base = (char*)p;
        own = true;
    } else if (workspace_bytes < per * (size_t)n_workers) {
        return MPDO_E_NOMEM;
    }
    int device = 0;
    (void)hipGetDevice(&device);
    std::vector<int> order(n_circuits);
    std::vector<double> cost(n_circuits);
    for (int i = 0; i < n_circuits; ++i) {
        order[i] = i;
        cost[i] = cost_of(circuits[i]);
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (circuits[a].chi_max != circuits[b].chi_max) return circuits[a].chi_max > circuits[b].chi_max;
        return cost[a] > cost[b];
    });
    FirstError fe;
    auto run_on = [&](int i, hipStream_t stream, char* ws) {
        const auto t0 = std::chrono::steady_clock::now();
        circuits[i].status = run_one(circuits[i], stream, ws, per, i, fe);
        const auto t1 = std::chrono::steady_clock::now();
        circuits[i].seconds = std::chrono::duration<double>(t1 - t0).count();
    };
    // The smallest circuit runs alone in the calling thread before the workers start, so the
    // library's first use in the process (the runtime loading its code objects, per-thread
    // runtime state) is not made by many threads at once.
    const int first = order.back();
    order.pop_back();
    {
        hipStream_t s0 = nullptr;
        if (hipStreamCreateWithFlags(&s0, hipStreamNonBlocking) != hipSuccess) {
            fe.note(first, "stream creation failed");
            circuits[first].status = MPDO_E_DEVICE;
        } else {
            run_on(first, s0, base);
            (void)hipStreamDestroy(s0);
        }
    }
    const int n_rest = (int)order.size();
    std::atomic<int> next(0);
    std::vector<std::thread> pool;
    for (int w = 0; w < std::min(n_workers, std::max(n_rest, 1)); ++w) {
        pool.emplace_back([&, w]() {
            (void)hipSetDevice(device);
            hipStream_t stream = nullptr;
            if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) stream = nullptr;
            char* ws = base + per * (size_t)w;
            for (;;) {
                const int q = next.fetch_add(1);
                if (q >= n_rest) break;
                const int i = order[q];
                if (stream) {
                    run_on(i, stream, ws);
                } else {
                    fe.note(i, "stream creation failed");
                    circuits[i].status = MPDO_E_DEVICE;
                }
            }
            if (stream) (void)hipStreamDestroy(stream);
        });
    }
    for (auto& t : pool) t.join();
    if (own) (void)hipFree(base);
    for (int i = 0; i < n_circuits; ++i)
        if (circuits[i].status != MPDO_OK) {
            mpdo::set_thread_error(fe.msg);
            return (mpdo_status)circuits[i].status;
        }
    return MPDO_OK;
}

}  // extern "C"
