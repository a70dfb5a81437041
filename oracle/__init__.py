"""CPU oracle for the noisy neutral-atom density-operator simulator (arXiv 2309.08572).

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library may import, call, link or run
anything in this package; only the test-suite, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the GPU path.  The only module both
sides read is ``workloads`` (seeded numbers, no arithmetic of the method).

Modules
-------
channels    vectorisation of rho, superoperators of Kraus maps and unitaries
            (Sec. III.A), the QAOA gate / noise model (Sec. IV, Eq. (tfim_model)).
dense       exact dense density matrix (d^N x d^N), evolved by the same Kraus maps.
mpo         plain FP64 vectorised density-operator MPO: merge -> SVD -> cut -> PPT
            (Sec. III.A, Fig. (ansatzes)c; Sec. III.D), canonical centre by QR
            (Sec. III.A, canonisation identities), transfer-matrix expectations.
ppt         the Purity-Preserving Truncation on vectors (Sec. III.D, Eqs. (xiformula)
            and (ppt); App. B).
statevector pure-state QAOA for the noiseless pins (Eq. (tfim_model), Table II).

Parity pins live in tests/test_oracle_*.py.  Parity is unpinned (no value from the
paper, no closed form) for truncating runs beyond agreement with themselves under chi
doubling; see the oracle tests for what each function is pinned to.
"""
