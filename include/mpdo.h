/*
 * mpdo.h -- C ABI of libmpdo: the two-site update of a vectorised density-operator MPO
 * with Purity-Preserving Truncation, on one AMD Instinct MI355X (gfx950).
 *
 * Paper: "Simulating Large One-Dimensional Neutral Atom Quantum Systems" (arXiv 2309.08572).
 *
 * State (Sec. III, Eq. (MPO) and "MPO form of the noisy CZ gate"): rho over N atoms of d
 * levels is a chain of site tensors A_j[l][eta][r], complex, row-major, l slowest, with the
 * vectorised physical index eta = sigma*d + sigma' (D2 = d*d values) and bond dimensions
 * chi_l, chi_r <= chi_max.  Superoperators act on eta: a Kraus map rho -> sum K rho K^+
 * is sum K (x) conj(K) in this basis.
 *
 * Conventions for every call
 *  - Host arrays are copied before the call returns; the caller keeps ownership.
 *  - Complex numbers are interleaved pairs of doubles (re, im), row-major.
 *  - Device state belongs to the context.  Work is enqueued on the context's HIP stream;
 *    calls that return host data (expect, trace, a non-null info, bond_dims, get_site)
 *    synchronise that stream.
 *  - Every call returns a status and never throws.  mpdo_last_error() returns the message
 *    of the last failure.  After MPDO_E_NUMERIC or MPDO_E_DEVICE the context is poisoned
 *    and later calls return MPDO_E_STATE.  An infeasible PPT cut is not an error: it falls
 *    back to theta = 0 (end of Sec. III.D) and is reported in mpdo_trunc_info.
 *  - A context is not re-entrant; use one context per stream.
 *
 * Numerical safeguards of the two-site update (apply_gate, apply_gate_kraus, truncate)
 *  - Every orthonormal basis built by the split (range bases, Schmidt vectors) is checked
 *    before the new sites are written: ||Q||_F^2 must equal its column count to 1e-9 (FP64)
 *    or 1e-3 (FP32) with no non-finite entry.  The check runs before the pair's new sites are
 *    written; an update that fails it is recomputed once from the same sites, and a second
 *    failure returns MPDO_E_NUMERIC ("orthonormal basis lost accuracy", naming the basis)
 *    instead of committing a wrong state.
 *  - Products whose k range is split over workgroups add their partial tiles in a fixed order,
 *    so a call gives the same result bits on every run.
 *  - Splits whose exact range basis would need a Hermitian eigenproblem above order 1024
 *    (the saturated chi = 512 regime) form theta explicitly, build the basis of its dominant
 *    left singular subspace by block subspace iteration (chi + 256 directions, stopped when
 *    the captured weight changes by less than 1e-10 of itself) and split its core exactly;
 *    the weight it misses lies below the chi cut.  tr(rho) and ||theta||_F^2, which PPT
 *    reads (Eq. (xiformula)), are taken from the whole theta.
 *
 * Environment (read at each use)
 *   MPDO_DEBUG_CHECKS=1         print every orthonormality check and block-Jacobi sweep count
 *                               to stderr
 *   MPDO_SUBSPACE_MIN_ORDER=n   use the subspace iteration above order n (< 1024) instead of
 *                               1024, for testing it where the exact split also runs
 *   MPDO_GEMM_AUTOTUNE=1        time the launch plan (tile size and k split) of each GEMM
 *                               shape bucket on first use and keep the fastest (default: a
 *                               cost model of matrix-core time per compute unit)
 *   MPDO_JACOBI_INNER_SWEEPS=k  sweeps of each 32 x 32 pair problem per round of the block
 *                               Jacobi solver (orders above 1024; default 1)
 */
#ifndef MPDO_H
#define MPDO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpdo_ctx_s* mpdo_ctx;

typedef enum {
    MPDO_OK = 0,
    MPDO_E_ARG = 1,         /* bad index, size, pointer, non-finite or non-CPTP input   */
    MPDO_E_STATE = 2,       /* context poisoned or not initialised                       */
    MPDO_E_NOMEM = 3,       /* device allocation failed or workspace too small          */
    MPDO_E_DEVICE = 4,      /* a HIP call failed                                         */
    MPDO_E_NUMERIC = 5,     /* NaN/Inf in a merged tensor or the eigensolver diverged   */
    MPDO_E_UNSUPPORTED = 6  /* a size beyond the compiled limits                         */
} mpdo_status;

typedef enum {
    MPDO_FP64 = 0,          /* every contraction and Gram product in FP64 (MFMA f64)     */
    MPDO_FP32 = 1,          /* contractions and Gram products on FP32 MFMA with FP32
                               accumulation; eigensolve, PPT and observables in FP64     */
    MPDO_BF16X3 = 2         /* as MPDO_FP32 (FP32 site data), but the products with the
                               merged tensor theta (the merge, the gate, the saturated
                               split's subspace iteration) split each FP32 operand into
                               two BF16 terms and form three BF16 matrix-core products
                               with FP32 accumulation: an elementary product carries a
                               relative error below 2^-15 instead of 2^-24.  Gram
                               products, projections and the rest stay in FP32.          */
} mpdo_precision;

typedef struct {
    int n_sites;            /* N >= 2                                                    */
    int d;                  /* levels per atom, 2..4 (D2 = d*d <= 16)                    */
    int chi_max;            /* bond-dimension cap, 1..1024                               */
    int precision;          /* mpdo_precision                                            */
    double cutoff_rel;      /* drop Schmidt values below cutoff_rel * largest; 0 -> 1e-14
                               (MPDO_FP64) or 1e-6 (MPDO_FP32, MPDO_BF16X3)            */
    int ppt;                /* 1: Purity-Preserving Truncation (Sec. III.D); 0: plain cut */
    int renorm_trace;       /* 1: rescale the cut spectrum so tr(rho) is unchanged       */
    void* hip_stream;       /* hipStream_t to enqueue on; NULL = the null stream         */
} mpdo_config;

typedef struct {
    int bond;               /* left site of the updated pair                             */
    int chi_l, chi_mid, chi_r;  /* bond dimensions around the pair before the update     */
    int kept;               /* new bond dimension                                        */
    int path;               /* 0: theta formed explicitly; 1: factored through the gate's
                               operator-Schmidt decomposition                            */
    int eig_calls;          /* Hermitian eigensolves this update made                    */
    int ppt_feasible;       /* 0 when |T'| < |T| cos(phi) and theta = 0 was used         */
    double trace_before;    /* tr(rho) = sum T_i Lambda_i before the cut                 */
    double trace_after;     /* tr(rho) after the cut and PPT                             */
    double xi_before;       /* tr(rho^2)/tr(rho)^2 before the cut                        */
    double xi_after;        /* the same after the cut and PPT                            */
    double ppt_theta;       /* angle theta of Eq. (xiformula)                            */
    double discarded_weight;/* 1 - sum_kept Lambda^2 / |Lambda|^2                        */
    double max_abs_imag_t;  /* largest |Im T'_i Lambda'_i| relative to |tr rho|          */
    double sigma_max;       /* largest Schmidt value                                     */
    double sigma_min_kept;  /* smallest kept Schmidt value                               */
    double sigma_next;      /* largest discarded Schmidt value: exact (to the Gram
                               eigenvalue's accuracy, ~sqrt(eps) sigma_max) when the chi
                               cap made the cut at a deflation level that resolved it;
                               otherwise an upper bound from that level's acceptance
                               threshold; 0 when the cut was not made by chi (everything
                               dropped lies below cutoff_rel or the rounding floor)      */
    double sigma_gap_at_cut;/* sigma_min_kept - sigma_next.  Where it is ~0 (a tie at
                               the cut) the truncated state is not unique (Sec. III.A
                               cuts the least significant values; the paper does not say
                               how ties are broken): results may differ from another
                               correct implementation by the weight of the tied pair    */
    int sigma_next_exact;   /* 1 when sigma_next is the resolved value, 0 for a bound    */
    int retried;            /* 1 when the update was recomputed after a failed basis
                               check (see the safeguards above), else 0                 */
} mpdo_trunc_info;

/* Create a context for a chain described by cfg.  Allocates nothing on the device until
 * mpdo_bind_workspace or mpdo_init_product_state (which allocates with hipMalloc when no
 * workspace is bound).  E_ARG for sizes out of range. */
mpdo_status mpdo_create(const mpdo_config* cfg, mpdo_ctx* out);

/* Release the context and any device memory it allocated itself. */
mpdo_status mpdo_destroy(mpdo_ctx ctx);

/* Device bytes the context needs for cfg (site tensors at chi_max plus scratch). */
size_t mpdo_workspace_bytes(const mpdo_config* cfg);

/* Hand the context a caller-owned device buffer of `bytes` (>= mpdo_workspace_bytes) that
 * stays alive until mpdo_destroy.  Must precede mpdo_init_product_state.  E_NOMEM if too
 * small, E_STATE if device memory is already in use. */
mpdo_status mpdo_bind_workspace(mpdo_ctx ctx, void* device_ptr, size_t bytes);

/* Initial product state rho = (x)_j rho_j (Sec. IV: |+_X> on every atom).
 * rho_sites: n_sites * d * d complex (host), rho_j row-major.  Each site becomes a
 * 1 x D2 x 1 tensor; the canonical centre is site 0.  Clears pending channels. */
mpdo_status mpdo_init_product_state(mpdo_ctx ctx, const double* rho_sites);

/* Two-site update (Sec. III.A "MPO form of the noisy CZ gate"; Fig. (ansatzes)c;
 * Fig. (mpo_mpdo_update_comparisons)a): apply the channel `superop` to atoms
 * (site, site+1), split the merged tensor, cut to chi_max and apply PPT (Sec. III.D,
 * Eqs. (xiformula), (ppt)).  superop: D2^2 x D2^2 complex (host), row index
 * eta_site*D2 + eta_{site+1}.  Channels queued on the two atoms by mpdo_apply_channel act
 * first.  info may be NULL.  E_ARG for site outside [0, N-2] or non-finite entries. */
mpdo_status mpdo_apply_gate(mpdo_ctx ctx, int site, const double* superop,
                            mpdo_trunc_info* info);

/* As mpdo_apply_gate, for a two-atom Kraus map: kraus holds n_kraus operators of
 * d^2 x d^2 complex (host) on the index sigma_site*d + sigma_{site+1}.  E_ARG if
 * sum K^+ K differs from the identity by more than 1e-10. */
mpdo_status mpdo_apply_gate_kraus(mpdo_ctx ctx, int site, int n_kraus, const double* kraus,
                                  mpdo_trunc_info* info);

/* Pulse-level gate of atoms (site, site+1) with nearest-neighbour Rydberg crosstalk (Sec. II,
 * "MPO form of the noisy CZ gate with crosstalk"; noise-free, as the paper simulates it):
 * rho -> U rho U^+ with U = sum_{a,b in {0,1}} P^a_{site-1} (x) u[a + 2b] (x) P^b_{site+2},
 * P^1 = |rydberg><rydberg| and P^0 = I - P^1 on the neighbour.  u4: four pair unitaries of
 * d^2 x d^2 complex (host, index sigma_site*d + sigma_{site+1}), u4[a + 2b] being the pulse
 * with the detunings of atoms site and site+1 shifted by a*B and b*B.  At an end of the chain
 * the missing neighbour contributes a = 0 (or b = 0) only.  Channels queued on the four atoms
 * act first.  The neighbours are class-split on their bonds (the classes of their
 * vectorised index under the projectors) and orthonormalised class by class into the pair,
 * so their bonds keep the class and grow at most four-fold; the pair's merged tensor receives
 * u[a + 2b] (x) conj(u[a' + 2b']) block by block and is split, cut to chi_max and corrected
 * by PPT like any two-site update (info describes that update); canonical sweeps over the
 * four atoms then compress the neighbour bonds to their Schmidt ranks.  Needs four times each
 * neighbour bond within chi_max (one time at a chain end).  The first call allocates 16 D2^4
 * complex FP64 (plus an FP32 copy in FP32 mode) with hipMalloc, freed by mpdo_destroy.  E_ARG
 * for site outside [0, N-2], rydberg outside [0, d), non-finite or non-unitary (by more than
 * 1e-10) entries, or a neighbour bond whose four-fold exceeds chi_max (nothing is changed). */
mpdo_status mpdo_apply_gate_crosstalk(mpdo_ctx ctx, int site, int rydberg, const double* u4,
                                      mpdo_trunc_info* info);

/* Single-atom channel (Sec. II noise; Sec. IV mixer): n_kraus operators of d x d complex
 * (host).  The map is queued on the atom and enters the next two-site update that touches
 * it (maps on different atoms commute), or the next expectation.  E_ARG if not trace
 * preserving within 1e-10. */
mpdo_status mpdo_apply_channel(mpdo_ctx ctx, int site, int n_kraus, const double* kraus);

/* Cut bond (bond, bond+1) to at most chi (<= chi_max) with PPT: the two-site update with
 * the identity superoperator.  Queued channels on the two atoms are applied first. */
mpdo_status mpdo_truncate(mpdo_ctx ctx, int bond, int chi, mpdo_trunc_info* info);

/* Linear observables by transfer matrices (Sec. III.E; Eq. (tfim_hamiltonian)):
 * term t is the product of n_sites_in_term[t] single-atom operators on consecutive atoms
 * starting at first_site[t]; ops holds all of them concatenated, d x d complex each (host).
 * out[2t], out[2t+1] = re, im of tr(rho O_t), divided by tr(rho) when normalize != 0.
 * Queued channels are applied to the operators (Heisenberg picture). */
mpdo_status mpdo_expect(mpdo_ctx ctx, int n_terms, const int* first_site,
                        const int* n_sites_in_term, const double* ops, int normalize,
                        double* out);

/* Second-order observables, i.e. linear functions of rho (x) rho, by doubled transfer
 * matrices (Fig. 6c; Sec. III.E).  Examples are the purity, the collision probability
 * (Sec. III.F) and the second Renyi entropy of a block of atoms.
 *
 * Term t covers the consecutive atoms first_site[t] .. first_site[t] + n_sites_in_term[t] - 1.
 * For each atom j of the term, ops holds one D2 x D2 complex matrix M_j (D2 = d^2), row-major
 * [eta][eta'] with eta = sigma d + sigma'.  The terms' matrices are concatenated in order, on
 * the host, and are copied before the call returns.  Atoms outside the term are traced out in
 * both copies.
 *
 * out[2t], out[2t+1] receive the real and imaginary parts of
 *     sum_{eta, eta'} vec(rho)[eta] vec(rho)[eta'] prod_j M_j[eta_j, eta'_j],
 * divided by tr(rho)^2 when normalize != 0.  Queued channels P on an atom enter as P^T M P.
 *
 * Per atom this costs three complex GEMMs of order D2 chi^3.  The call synchronises the stream.
 * Errors: MPDO_E_ARG for a term out of range, a null pointer or a non-finite entry;
 * MPDO_E_STATE before the state is initialised. */
mpdo_status mpdo_expect2(mpdo_ctx ctx, int n_terms, const int* first_site,
                         const int* n_sites_in_term, const double* ops, int normalize,
                         double* out);

/* tr(rho): out[0], out[1] = re, im. */
mpdo_status mpdo_trace(mpdo_ctx ctx, double* out);

/* Current bond dimensions: out[j] for bond (j, j+1), j < N-1. */
mpdo_status mpdo_bond_dims(mpdo_ctx ctx, int* out);

/* Copy site tensor j to the host as complex128 [chi_l][D2][chi_r] (queued channels not
 * applied); shape[0..2] receives its dimensions.  out may be NULL to query the shape. */
mpdo_status mpdo_get_site(mpdo_ctx ctx, int site, double* out, int* shape);

/* Replace the chain by the caller's site tensors (Sec. III, Eq. (MPO)), for instance the state
 * of another context of the same chain read back with mpdo_get_site, possibly in the other
 * precision.  bond_dims: N-1 bond dimensions (bond j between atoms j and j+1), each in
 * [1, chi_max].  sites: the N tensors concatenated, each complex [chi_l][D2][chi_r] (host,
 * interleaved doubles), converted to the working precision.  centre >= 0: the caller vouches
 * that every site left of `centre` is a left isometry and every site right of it a right
 * isometry (the mixed canonical form of Sec. III.A that PPT relies on; mpdo_canonical_centre
 * returns it for a context's own state).  centre = -1: the library brings the chain into that
 * form itself by range-basis moves from atom 0 to atom N-1 (rho is kept to rounding; nothing
 * is cut) and the centre ends on atom N-1.  Queued single-atom channels are cleared.
 * E_ARG for a null pointer, a bond outside [1, chi_max], a non-finite entry or centre
 * outside [-1, N-1]. */
mpdo_status mpdo_set_state(mpdo_ctx ctx, const int* bond_dims, const double* sites, int centre);

/* out[0]: the atom holding the canonical centre; out[1]: +1 or -1, the direction of the last
 * sweep (the side of the pair the centre moves to after the next update). */
mpdo_status mpdo_canonical_centre(mpdo_ctx ctx, int* out);

/* Move the canonical centre to atom `site` (the canonisation identities of Sec. III.A) by
 * range-basis moves across the bonds in between: every site passed becomes a left (moving
 * right) or right (moving left) isometry.  rho is kept: a move drops only directions below the
 * rounding floor of the working precision (1e-14 relative in FP64; in FP32 the floor of FP32
 * products, so an FP32 move can shrink a bond that carries values below it).  E_ARG for a site
 * outside [0, N-1] or before a state exists. */
mpdo_status mpdo_move_centre(mpdo_ctx ctx, int site);

/* ---------------------------------------------------------------- batches of circuits
 * Many independent circuits (QAOA angle sets x noise rates, of uneven N and chi): each is
 * an ordered list of Kraus maps applied to a product state, then linear observables.
 * Circuits share nothing, so they run concurrently (Sec. IV studies sweep parameters as
 * independent simulations). */
typedef struct {
    int n_sites, d, chi_max, precision, ppt;
    int n_ops;
    const int* op_kind;        /* per operation: 0 = two-atom map on (site, site+1), 1 = one atom */
    const int* op_site;
    const int* op_set;         /* index of its Kraus set                                         */
    const int* set_count;      /* operators in each set                                          */
    const long* set_offset;    /* offset of each set in kraus, in complex numbers               */
    const double* kraus;       /* complex operators, d^2 x d^2 (two-atom) or d x d (one atom)   */
    const double* rho0;        /* n_sites * d * d complex: the initial product state            */
    int n_terms;               /* observables as in mpdo_expect, normalised by tr(rho)          */
    const int* term_first;
    const int* term_len;
    const double* term_ops;
    double* out;               /* 2 * n_terms: re, im                                            */
    double* out_trace;         /* 2: tr(rho)                                                     */
    int* out_bonds;            /* n_sites - 1 final bond dimensions (may be NULL)               */
    int status;                /* set by mpdo_run_batch: mpdo_status of this circuit            */
    double seconds;            /* set by mpdo_run_batch: wall time of this circuit on its worker */
} mpdo_circuit;

/* Device bytes one worker needs to run any circuit of the batch (the largest circuit). */
size_t mpdo_batch_workspace_bytes(const mpdo_circuit* circuits, int n_circuits);

/* Run n_circuits circuits on n_workers host threads, each with its own HIP stream and
 * context (default stream priority), taking circuits from a shared queue ordered by bond cap
 * and then by estimated cost (two-site updates x chi_max^3), largest first; the kernels of
 * different circuits overlap on the GPU.  The smallest circuit runs first, alone, in the
 * calling thread, so that the library's first use in a process is not made by many threads
 * at once.  device_workspace: NULL (the library allocates n_workers *
 * mpdo_batch_workspace_bytes with hipMalloc) or a caller buffer of at least that size.
 * Per-circuit failures are reported in circuits[i].status; the call returns MPDO_E_ARG for
 * bad arguments and otherwise the first failing circuit's status, with the message of the
 * first failure in mpdo_last_error(NULL) ("circuit i: ..."). */
mpdo_status mpdo_run_batch(mpdo_circuit* circuits, int n_circuits, int n_workers, void* device_workspace,
                           size_t workspace_bytes);

/* Kernel families reported by mpdo_profile_read, in this order. */
enum {
    MPDO_PROF_GEMM = 0,        /* complex matrix-core GEMM (theta, Gram, projections, rebuild);
                                  timed by the kernel's own start and end stamps            */
    MPDO_PROF_EIG_PAIR = 1,    /* Jacobi: 32 x 32 pair eigenproblems in LDS                    */
    MPDO_PROF_EIG_ROTATE = 2,  /* Jacobi: pair rotations applied to block rows and columns     */
    MPDO_PROF_EIG_SMALL = 3,   /* Jacobi: whole matrix of order <= 64 in one workgroup         */
    MPDO_PROF_PHYS = 4,        /* gate factors applied to the physical index of a site         */
    MPDO_PROF_TRANSFER = 5,    /* transfer-matrix steps of trace / expectation vectors         */
    MPDO_PROF_OTHER = 6,
    MPDO_PROF_TRI_REDUCE = 7,  /* Householder reduction to tridiagonal form (one workgroup)    */
    MPDO_PROF_TRI_SOLVE = 8,   /* bisection + inverse iteration for the accepted eigenpairs    */
    MPDO_PROF_TRI_BACK = 9,    /* back-transformation of the accepted eigenvectors             */
    MPDO_PROF_THETA = 10,      /* the theta contraction: the merge and gate products that form
                                  theta explicitly (GEMM kernel, timed apart from family 0)    */
    MPDO_PROF_PCHOL = 11,      /* pivoted Cholesky of a Gram matrix for a range basis (one
                                  workgroup)                                                   */
    MPDO_PROF_SPLIT_SUM = 12,  /* the k-split GEMMs' partial sums, added in chunk order (own
                                  start and end stamps like family 0)                          */
    MPDO_PROF_FAMILIES = 13
};

/* Measurement switch (instrumentation, not part of the method): with enable = 1 the
 * context records a HIP event pair around every launch of the families above on its
 * stream and clears earlier totals; enable = 0 stops recording (totals are kept).  For the
 * GEMM families (0, 10, 12) the pair is attached to the kernel itself (hipExtLaunchKernelGGL),
 * so their milliseconds are kernel execution time; for the others a pair brackets the
 * family's launches and also holds their dispatch. */
mpdo_status mpdo_profile_enable(mpdo_ctx ctx, int enable);

/* As mpdo_profile_enable(ctx, 1), recording only the families whose bit (1u << f) is set in
 * family_mask: an event pair costs host time at every launch it brackets, so a measurement of
 * one family's kernels leaves the rest of the stream as it runs unmeasured.  family_mask = 0
 * stops recording. */
mpdo_status mpdo_profile_enable_mask(mpdo_ctx ctx, unsigned family_mask);

/* Sampling of the stamped families (0, 10, 12) while recording: only every stride-th launch
 * of each is stamped and counted (the first of each family since this call), so a measurement
 * of the many short product kernels costs the stream little; the totals then hold the sampled
 * launches, whose average stands for the family's.  stride = 1 stamps every launch (the
 * default of each mpdo_profile_enable / _mask call).  E_ARG for stride < 1; no effect while
 * nothing is recorded. */
mpdo_status mpdo_profile_stride(mpdo_ctx ctx, int stride);

/* Totals since the last mpdo_profile_enable(ctx, 1): out[4 f + 0..3] = launches,
 * milliseconds, algorithmic flop and algorithmic bytes of family f, for f < n_families.
 * Synchronises the stream. */
mpdo_status mpdo_profile_read(mpdo_ctx ctx, double* out, int n_families);

/* Block until all work of the context has finished. */
mpdo_status mpdo_synchronize(mpdo_ctx ctx);

/* The FP64 Hermitian eigensolver that replaces the SVD in the split of Sec. III.A (the
 * spectrum is cut to the largest Schmidt values, Sec. III.A and III.D), on a host matrix, so
 * that tests can check it element by element here: the eigenpairs of the Hermitian part of H
 * that one deflation level of the update accepts, i.e. the largest eigenvalues above
 * tau * lambda_max (and above 0), at most cap of them, through the update's own kernels and
 * order dispatch: one-workgroup Jacobi for n <= 32; for 33 <= n <= 1024 the Householder
 * tridiagonal reduction, multisection for the accepted eigenvalues, inverse iteration with
 * Gram-Schmidt inside clusters closer than 1e-12 ||T|| and the back-transformation.
 * H: host complex128 n x n, row-major, interleaved (re, im), read only.  Outputs: *m = the
 * accepted count; evals[0..m) descending; V: host complex128 n x cap, row-major, whose columns
 * 0..m) receive the unit eigenvectors (the other columns are left as they are).  Eigenvectors
 * are unique up to a phase (and within a subspace of equal eigenvalues).  Synchronous on the
 * null stream of the current device; allocates and frees its device buffers.  E_ARG for
 * n < 1 or n > 1024, cap < 0 or cap > n, tau < 0 or NaN, or a null pointer; E_NOMEM /
 * E_DEVICE for a failed allocation or HIP call; E_NUMERIC if Jacobi does not converge
 * (message: mpdo_last_error(NULL)). */
mpdo_status mpdo_eigh(int n, const double* H, double tau, int cap, int* m, double* evals, double* V);

/* C = alpha op(A) op(B) + beta C on the library's matrix-core product kernels: every
 * contraction of the update (the merge and gate of Sec. III.A, Fig. 2(c); the Gram products
 * and rebuilds that replace the SVD) runs through them, and tests check them element by
 * element here.  precision: a value of mpdo_precision; FP32 and BF16X3 round the operands to
 * FP32 first.  A, B, C: host complex128 (interleaved re, im), row-major.  op_a = 0: A is M x K
 * and op(A) = A; 1: A is K x M and op(A) = A^T; 2: A is K x M and op(A) = A^H.  op_b the same
 * with B K x N (op 0) or N x K (1, 2).  C is M x N, read when beta != 0 and overwritten.
 * alpha, beta: complex scalars (2 doubles).  split_k = 1 lends the product a workspace for
 * k-split partial sums (added in a fixed order), 0 runs k unsplit.  Synchronous on the null
 * stream of the current device; allocates and frees its device copies.  E_ARG for a negative
 * size, a null pointer, an unknown op or precision, or an operand above 2^28 elements;
 * E_NOMEM / E_DEVICE for a failed allocation or HIP call (message: mpdo_last_error(NULL)). */
mpdo_status mpdo_cgemm(int precision, int M, int N, int K, const double* alpha, const double* A, int op_a,
                       const double* B, int op_b, const double* beta, double* C, int split_k);

/* Message of the last failed call on ctx (or of mpdo_create when ctx is NULL). */
const char* mpdo_last_error(mpdo_ctx ctx);

/* Library build string (compiler, target). */
const char* mpdo_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MPDO_H */
