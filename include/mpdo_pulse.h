/* Pulse-level two-atom gate: the channel of one laser pulse on a pair of neutral atoms,
 * integrated from the Lindblad master equation (Sec. II, Eqs. (LME_Hamiltonian),
 * (LME_Single_Site), (LME)) by Trotterised time steps (Sec. III.A, "MPO form of the noisy CZ
 * gate"), ready for mpdo_apply_gate.
 *
 * Levels per atom: 0, 1, r (index 2) and, for d = 4, a dark level (index 3).  Both atoms see
 * the same pulse:
 *   H_p(t) = H(t) (x) I + I (x) H(t) + B |rr><rr|,  H(t) = Omega(t)/2 (|r><1| + h.c.) + Delta(t) |r><r|;
 *   jump operators per atom: sqrt(gamma_diss b_j) |j><r| for j = 0, 1, dark, and
 *   gamma_deph / sqrt(2) (|0><0| - |1><1|).
 * The pulse is cut into n_steps steps of length tau.  Each step applies to rho, in this order:
 * the exact exponential of every jump operator's dissipator (atom 1: decay to 0, to 1, to dark,
 * dephasing; then atom 2), the blockade phase exp(-i tau B |rr><rr|), and the single-atom
 * propagators exp(-i tau H) with Omega and Delta sampled once per step (the caller passes the
 * values at the middle of each step).  The channel is the product of the steps in time order;
 * every factor is completely positive and trace preserving, and the Trotter error is first
 * order in tau.  Units are the caller's: rates and frequencies in radians per time unit of tau.
 *
 * Output layout: superop is D2^2 x D2^2 complex (D2 = d*d), interleaved re/im, row-major, row
 * index eta_1 * D2 + eta_2 with eta = sigma * d + sigma' per atom: exactly the input of
 * mpdo_apply_gate for the bond (site, site + 1), atom 1 = site.
 *
 * The call computes on the GPU (one workgroup per basis input |a><b|, the pair's density matrix
 * held on chip through all steps), allocates and frees its own device buffers, runs on
 * hip_stream (may be null: the default stream) and returns after the result is on the host.
 * Status codes as in mpdo.h:
 *   MPDO_E_ARG     d not 3 or 4, n_steps < 1, tau <= 0, a negative rate or branch ratio, a dark
 *                  branch with d = 3, a null pointer or a non-finite value;
 *   MPDO_E_NOMEM   a device allocation failed;
 *   MPDO_E_DEVICE  a HIP error.
 * mpdo_pulse_last_error() describes the calling thread's last failure. */
#ifndef MPDO_PULSE_H
#define MPDO_PULSE_H

#include "mpdo.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpdo_pulse_params {
    int d;              /* levels per atom: 3 or 4 */
    int n_steps;        /* time steps */
    double tau;         /* step length */
    double blockade;    /* B */
    double gamma_diss;  /* Rydberg dissipation rate */
    double branch[3];   /* b_0, b_1, b_dark */
    double gamma_deph;  /* dephasing amplitude */
} mpdo_pulse_params;

/* omega, delta: n_steps values each (host), Omega and Delta at the middle of each step. */
mpdo_status mpdo_pulse_channel(const mpdo_pulse_params* params, const double* omega,
                               const double* delta, double* superop, void* hip_stream);

/* As mpdo_pulse_channel, for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the call makes no hipMalloc,
 * hipFree or other allocating call.  Its device buffers are carved from one fixed scratch block
 * of 32 MiB per device (a static device array, resident from the library's load until the
 * process ends), which limits n_steps to 131072 for d = 4 and 484917 for d = 3; a larger
 * n_steps returns MPDO_E_ARG with the bytes needed, before any device work.  Every call on a
 * device shares that device's block: calls that overlap on one device (two host threads, or
 * two streams with work in flight) race and give wrong results, so serialise them.  Inputs
 * and outputs are as in mpdo_pulse_channel (host arrays, copied in and out on hip_stream);
 * the call returns after the result is on the host.  Other status codes as above. */
mpdo_status mpdo_pulse_channel_noalloc(const mpdo_pulse_params* params, const double* omega,
                                       const double* delta, double* superop, void* hip_stream);

const char* mpdo_pulse_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
