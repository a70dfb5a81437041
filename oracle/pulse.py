"""Plain FP64 reference of the pulse-level two-atom channel (Sec. II, Eqs. (LME_Hamiltonian),
(LME_Single_Site), (LME); Sec. III.A "MPO form of the noisy CZ gate").  Test infrastructure
only: nothing in the library imports it.

Levels per atom: 0, 1, r (index 2) and, for d = 4, the dark level (index 3).  Two atoms,
two-atom basis index x = x1 * d + x2.

Pulse Hamiltonian  H_p(t) = H_1(t) (x) I + I (x) H_2(t) + B |rr><rr|,
                   H_i(t) = Omega(t)/2 (|r><1| + |1><r|) + Delta(t) |r><r|   (same pulse on both).
Jump operators     L_j = sqrt(gamma_diss b_j) |j><r|  for j = 0, 1, dark (per atom),
                   L_deph = gamma_deph / sqrt(2) (|0><0| - |1><1|)           (per atom).

The pulse is cut into steps of length tau; each step channel is the product, applied to rho in
this order, of exp(tau D_L) for every jump operator (atom 1: L_0, L_1, L_dark, L_deph; then
atom 2), then the blockade phase exp(-i tau B|rr><rr|), then the single-atom drives
exp(-i tau H_i) of atom 2 and atom 1, with Omega and Delta taken at the middle of the step.
Every factor is the exact exponential of its own generator, by scipy.linalg.expm (no closed
forms): a jump operator's dissipator is exponentiated on its atom's vectorised d^2 space and
lifted to the pair by a tensor product with the identity; a drive is exponentiated on its
atom's d levels; the blockade phase is diagonal.  So the channel stays completely positive.
The pulse channel is the product of the step channels in time order.

Vectorisation: vec(rho)[x * D + y] = rho[x, y] (D = d*d), so rho -> A rho B is A (x) B^T.
`to_site_layout` reorders a channel to the per-atom vectorised index eta = sigma * d + sigma'
used for two-site gates: row eta_1 * d^2 + eta_2.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import expm

R = 2        # index of the Rydberg level
DARK = 3     # index of the dark level (d = 4)


def _e(d, i, j):
    m = np.zeros((d, d), dtype=np.complex128)
    m[i, j] = 1.0
    return m


def site_hamiltonian(omega: float, delta: float, d: int) -> np.ndarray:
    """H_i = Omega/2 (|r><1| + h.c.) + Delta |r><r| (Eq. (LME_Single_Site))."""
    return 0.5 * omega * (_e(d, R, 1) + _e(d, 1, R)) + delta * _e(d, R, R)


def jump_operators(d: int, gamma_diss: float, branch, gamma_deph: float):
    """Single-atom jump operators in the order the step applies them."""
    sinks = [0, 1] + ([DARK] if d == 4 else [])
    ops = [math.sqrt(gamma_diss * branch[k]) * _e(d, j, R) for k, j in enumerate(sinks)]
    ops.append(gamma_deph / math.sqrt(2.0) * (_e(d, 0, 0) - _e(d, 1, 1)))
    return ops


def _vec_left_right(A, B):
    """Superoperator of rho -> A rho B."""
    return np.kron(A, B.T)


def dissipator_generator(L: np.ndarray) -> np.ndarray:
    """D(rho) = L rho L^+ - 1/2 {L^+ L, rho}, vectorised (Eq. (LME))."""
    n = L.shape[0]
    I = np.eye(n)
    LdL = L.conj().T @ L
    return _vec_left_right(L, L.conj().T) - 0.5 * (_vec_left_right(LdL, I) + _vec_left_right(I, LdL))


def hamiltonian_generator(H: np.ndarray) -> np.ndarray:
    """-i [H, rho], vectorised."""
    n = H.shape[0]
    I = np.eye(n)
    return -1j * (_vec_left_right(H, I) - _vec_left_right(I, H))


def from_site_layout(S: np.ndarray, d: int) -> np.ndarray:
    """Inverse of to_site_layout: per-atom index (x1 d + y1) d^2 + (x2 d + y2) -> two-atom
    index (x1 d + x2) d^2 + (y1 d + y2), on rows and columns."""
    D = d * d
    T = S.reshape(d, d, d, d, d, d, d, d)          # x1 y1 x2 y2 | a1 b1 a2 b2
    T = T.transpose(0, 2, 1, 3, 4, 6, 5, 7)        # x1 x2 y1 y2 | a1 a2 b1 b2
    return T.reshape(D * D, D * D)


def _lift_site_channel(E: np.ndarray, atom: int, d: int) -> np.ndarray:
    """A single-atom channel (d^2 x d^2, vec index x d + y) acting on one atom of the pair."""
    I = np.eye(d * d)
    return from_site_layout(np.kron(E, I) if atom == 0 else np.kron(I, E), d)


def _conjugation(U: np.ndarray) -> np.ndarray:
    """Superoperator of rho -> U rho U^+."""
    return _vec_left_right(U, U.conj().T)


def step_channel(omega: float, delta: float, tau: float, d: int, blockade: float, gamma_diss: float,
                 branch, gamma_deph: float) -> np.ndarray:
    """One Trotter step of the two-atom LME (Sec. III.A), as a (d^4 x d^4) superoperator in the
    two-atom vectorisation."""
    I = np.eye(d)
    S = np.eye(d ** 4, dtype=np.complex128)
    for atom in (0, 1):
        for L in jump_operators(d, gamma_diss, branch, gamma_deph):
            S = _lift_site_channel(expm(tau * dissipator_generator(L)), atom, d) @ S
    rr = R * d + R
    PB = np.eye(d * d, dtype=np.complex128)
    PB[rr, rr] = np.exp(-1j * tau * blockade)
    S = _conjugation(PB) @ S
    u = expm(-1j * tau * site_hamiltonian(omega, delta, d))
    S = _conjugation(np.kron(I, u)) @ S
    S = _conjugation(np.kron(u, I)) @ S
    return S


def pulse_channel(omegas, deltas, tau: float, d: int, blockade: float, gamma_diss: float = 0.0,
                  branch=(0.0, 0.0, 0.0), gamma_deph: float = 0.0) -> np.ndarray:
    """Product of the step channels (time order), Omega/Delta given per step (midpoints)."""
    S = np.eye(d ** 4, dtype=np.complex128)
    for om, de in zip(omegas, deltas):
        S = step_channel(om, de, tau, d, blockade, gamma_diss, branch, gamma_deph) @ S
    return S


def trotter_unitary(omegas, deltas, tau: float, d: int, blockade: float) -> np.ndarray:
    """Noise-free limit: the product of the step unitaries (two-atom Hilbert space)."""
    I = np.eye(d)
    rr = R * d + R
    U = np.eye(d * d, dtype=np.complex128)
    for om, de in zip(omegas, deltas):
        h = site_hamiltonian(om, de, d)
        PB = np.eye(d * d, dtype=np.complex128)
        PB[rr, rr] = np.exp(-1j * tau * blockade)
        U = expm(-1j * tau * np.kron(h, I)) @ expm(-1j * tau * np.kron(I, h)) @ PB @ U
    return U


def to_site_layout(S: np.ndarray, d: int) -> np.ndarray:
    """Reorder a two-atom channel from vec index (x1 d + x2) * d^2 + (y1 d + y2) to the per-atom
    index (x1 d + y1) * d^2 + (x2 d + y2) on rows and columns."""
    D = d * d
    T = S.reshape(d, d, d, d, d, d, d, d)          # x1 x2 y1 y2 | a1 a2 b1 b2
    T = T.transpose(0, 2, 1, 3, 4, 6, 5, 7)        # x1 y1 x2 y2 | a1 b1 a2 b2
    return T.reshape(D * D, D * D)


# ------------------------------------------------------------------ pulse shapes (Fig. 1 caption)
def gaussian_samples(T: float, omega_max: float, delta: float, n_steps: int):
    """Gaussian pulse: Omega(t) = Omega_max [exp(-(t - t0)^2 / v^2) - a] / (1 - a), v = 0.1 T,
    t0 = T/2, a = exp(-(t0/v)^2); Delta constant.  Sampled at the step midpoints."""
    tau = T / n_steps
    t = (np.arange(n_steps) + 0.5) * tau
    v, t0 = 0.1 * T, 0.5 * T
    a = math.exp(-(t0 / v) ** 2)
    om = omega_max * (np.exp(-((t - t0) / v) ** 2) - a) / (1.0 - a)
    return om, np.full(n_steps, float(delta)), tau


def cz_infidelity(U4: np.ndarray):
    """Average gate infidelity of the qubit block U4 (basis 00, 01, 10, 11) against CZ up to a
    global phase and equal single-qubit Z phases: 1 - max_p (|tr(T_p^+ U)|^2 + tr(U^+ U)) / 20,
    T_p = diag(1, e^{ip}, e^{ip}, -e^{2ip})."""
    ps = np.linspace(0.0, 2.0 * math.pi, 4001)
    best = (np.inf, 0.0)
    norm = np.trace(U4.conj().T @ U4).real
    for p in ps:
        t = np.array([1.0, np.exp(1j * p), np.exp(1j * p), -np.exp(2j * p)])
        f = (abs(np.sum(t.conj() * np.diag(U4))) ** 2 + norm) / 20.0
        if 1.0 - f < best[0]:
            best = (1.0 - f, p)
    # refine around the best grid point
    lo, hi = best[1] - 2e-3, best[1] + 2e-3
    for _ in range(60):
        m1, m2 = lo + (hi - lo) / 3, hi - (hi - lo) / 3
        f1 = [(abs(np.sum(np.array([1, np.exp(1j * p), np.exp(1j * p), -np.exp(2j * p)]).conj() * np.diag(U4))) ** 2
               + norm) / 20.0 for p in (m1, m2)]
        if f1[0] > f1[1]:
            hi = m2
        else:
            lo = m1
    p = 0.5 * (lo + hi)
    t = np.array([1.0, np.exp(1j * p), np.exp(1j * p), -np.exp(2j * p)])
    return 1.0 - (abs(np.sum(t.conj() * np.diag(U4))) ** 2 + norm) / 20.0


def qubit_block(U: np.ndarray, d: int) -> np.ndarray:
    idx = [0 * d + 0, 0 * d + 1, 1 * d + 0, 1 * d + 1]
    return U[np.ix_(idx, idx)]
