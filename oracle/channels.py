"""Vectorised channels and the QAOA circuit model, written plainly in numpy (complex128).

Vectorisation (Sec. III.A, "MPO form of the noisy CZ gate"): the two Hilbert-space
indices of a site are fused into one, sigma sigma' -> eta.  Reading adopted here:
eta = sigma * d + sigma' (row-major), for which vec(A rho B) = (A kron B^T) vec(rho).
A Kraus map rho -> sum_k K rho K^dagger therefore has superoperator sum_k K kron conj(K).

Circuit model (Sec. IV, Eq. (tfim_model); noise of Sec. II): a layer is
    Ising phase blocks exp(-i gamma Z(x)Z) on even bonds (left to right), then on odd
    bonds (right to left), each block followed by a |1> -> |r> leak on both its atoms;
    then exp(-i beta X) on every atom;
    then qubit dephasing on every atom; then Rydberg decay on every atom.
(see ``circuit_ops`` for where the single-atom maps sit relative to later blocks).
Z and X act on the qubit levels {0,1} only and are zero on |r> (and on the lost level),
so the rotations are the identity there.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

# Branching of Rydberg decay into |0>, |1> and the dark ("lost") level (Fig. 1 caption).
DECAY_BRANCHING = (1.0 / 16.0, 1.0 / 16.0, 7.0 / 8.0)


def basis(d: int, a: int) -> np.ndarray:
    v = np.zeros(d, dtype=np.complex128)
    v[a] = 1.0
    return v


def ket_bra(d: int, a: int, b: int) -> np.ndarray:
    return np.outer(basis(d, a), basis(d, b).conj())


def vec(rho: np.ndarray) -> np.ndarray:
    """rho_{sigma sigma'} -> v[sigma*d + sigma'] (row-major flattening)."""
    return np.asarray(rho, dtype=np.complex128).reshape(-1).copy()


def unvec(v: np.ndarray, d: int) -> np.ndarray:
    return np.asarray(v).reshape(d, d)


def superop_1site(kraus) -> np.ndarray:
    """Superoperator (d^2 x d^2) of rho -> sum_k K rho K^dagger in the eta basis."""
    K0 = np.asarray(kraus[0])
    d = K0.shape[0]
    S = np.zeros((d * d, d * d), dtype=np.complex128)
    for K in kraus:
        K = np.asarray(K, dtype=np.complex128)
        # out[(a,a'),(s,s')] = K[a,s] conj(K[a',s'])
        S += np.einsum("as,bt->abst", K, K.conj()).reshape(d * d, d * d)
    return S


def superop_2site(kraus, d: int) -> np.ndarray:
    """Superoperator of a two-atom Kraus map in the (eta_i, eta_{i+1}) basis.

    Each K is (d^2 x d^2) on the two-atom Hilbert space with index sigma_i*d + sigma_{i+1}.
    Returns S[(eta_i*D2 + eta_{i+1}), (eta_i'*D2 + eta_{i+1}')] with D2 = d*d and
    eta = sigma*d + sigma' on each atom.
    """
    D2 = d * d
    S = np.zeros((D2, D2, D2, D2), dtype=np.complex128)
    for K in kraus:
        K4 = np.asarray(K, dtype=np.complex128).reshape(d, d, d, d)  # [a,b,s,t]
        # rho'[(a,b),(a',b')] = sum K[a,b,s,t] rho[(s,t),(s',t')] conj K[a',b',s',t']
        # eta_i = (a,a'), eta_{i+1} = (b,b'); inputs (s,s'), (t,t').
        S6 = np.einsum("abst,cduv->acbdsutv", K4, K4.conj())
        S += S6.reshape(D2, D2, D2, D2)
    return S.reshape(D2 * D2, D2 * D2)


def compose(*superops) -> np.ndarray:
    """compose(S1, S2, ...) applies S1 first, then S2, ... (returns ... S2 @ S1)."""
    out = superops[0]
    for S in superops[1:]:
        out = S @ out
    return out


def kron_superop(S_a: np.ndarray, S_b: np.ndarray) -> np.ndarray:
    """Two independent single-site superoperators as one on (eta_i, eta_{i+1})."""
    return np.kron(S_a, S_b)


# ---------------------------------------------------------------- operators on one atom
def z_ext(d: int) -> np.ndarray:
    Z = np.zeros((d, d), dtype=np.complex128)
    Z[0, 0], Z[1, 1] = 1.0, -1.0
    return Z


def x_ext(d: int) -> np.ndarray:
    X = np.zeros((d, d), dtype=np.complex128)
    X[0, 1] = X[1, 0] = 1.0
    return X


def proj(d: int, a: int) -> np.ndarray:
    return ket_bra(d, a, a)


def qubit_projector(d: int) -> np.ndarray:
    return proj(d, 0) + proj(d, 1)


# ---------------------------------------------------------------- gates and Kraus maps
def u_zz(gamma: float, d: int) -> np.ndarray:
    """exp(-i gamma Z(x)Z) on two atoms (Z acting on the qubit levels only)."""
    Z = z_ext(d)
    return scipy.linalg.expm(-1j * gamma * np.kron(Z, Z))


def u_x(beta: float, d: int) -> np.ndarray:
    """exp(-i beta X) on one atom (X acting on the qubit levels only)."""
    return scipy.linalg.expm(-1j * beta * x_ext(d))


def kraus_leak(p: float, d: int):
    """Blockade-induced leak |1> -> |r> with probability p."""
    K0 = np.eye(d, dtype=np.complex128) - (1.0 - np.sqrt(1.0 - p)) * proj(d, 1)
    K1 = np.sqrt(p) * ket_bra(d, 2, 1)
    return [K0, K1]


def kraus_dephasing(p: float, d: int):
    """Qubit dephasing: coherence rho_01 -> (1-2p) rho_01, populations untouched."""
    Pq = qubit_projector(d)
    rest = np.eye(d, dtype=np.complex128) - Pq
    return [np.sqrt(1.0 - p) * Pq + rest, np.sqrt(p) * z_ext(d)]


def kraus_decay(p: float, d: int):
    """Rydberg decay with probability p: r -> 1 for d=3; r -> {0,1,lost} for d=4."""
    K0 = np.eye(d, dtype=np.complex128) - (1.0 - np.sqrt(1.0 - p)) * proj(d, 2)
    out = [K0]
    if d == 3:
        out.append(np.sqrt(p) * ket_bra(d, 1, 2))
    elif d == 4:
        for j, b in zip((0, 1, 3), DECAY_BRANCHING):
            out.append(np.sqrt(p * b) * ket_bra(d, j, 2))
    else:
        raise ValueError("d must be 3 or 4")
    return out


def gate_kraus_2site(gamma: float, p_leak: float, d: int):
    """Ising block followed by the leak on both atoms, as two-atom Kraus operators."""
    U = u_zz(gamma, d)
    L = kraus_leak(p_leak, d)
    return [np.kron(La, Lb) @ U for La in L for Lb in L]


def plus_state(d: int) -> np.ndarray:
    v = np.zeros(d, dtype=np.complex128)
    v[0] = v[1] = 1.0 / np.sqrt(2.0)
    return np.outer(v, v.conj())


def circuit_ops(spec):
    """The circuit of a CircuitSpec as an ordered list of Kraus operations.

    Each item is ("k2", i, kraus) for a map on atoms (i, i+1), or ("k1", j, kraus).
    Layer k: Ising blocks on even bonds left to right, then on odd bonds right to left;
    then, on every atom, exp(-i beta_k X), dephasing and decay.  The single-atom maps of
    layer k commute with every operation of layer k+1 that does not touch their atom, so
    they are listed right before the first block of layer k+1 that acts on that atom (the
    ones of the last layer close the list).  As a channel this is exactly "noise after
    each layer"; the listed order fixes when each bond truncation sees that noise.
    """
    n, d = spec.n, spec.d
    ops = []
    pending = [[] for _ in range(n)]

    def flush(j):
        for kraus in pending[j]:
            ops.append(("k1", j, kraus))
        pending[j] = []

    for k in range(spec.p):
        g2 = gate_kraus_2site(spec.gamma[k], spec.p_leak, d)
        bonds = list(range(0, n - 1, 2)) + list(range(1, n - 1, 2))[::-1]
        for i in bonds:
            flush(i)
            flush(i + 1)
            ops.append(("k2", i, g2))
        ux = [u_x(spec.beta[k], d)]
        deph = kraus_dephasing(spec.p_deph, d)
        dec = kraus_decay(spec.p_decay, d)
        for j in range(n):
            pending[j] = [ux, deph, dec]
    for j in range(n):
        flush(j)
    return ops


def tfim_terms(n: int, d: int, g: float):
    """H = -sum Z_i Z_{i+1} - g sum X_i as (coefficient, {site: op}) product terms."""
    Z, X = z_ext(d), x_ext(d)
    terms = [(-1.0, {i: Z, i + 1: Z}) for i in range(n - 1)]
    terms += [(-g, {i: X}) for i in range(n)]
    return terms
