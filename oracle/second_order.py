"""Second-order observables: linear functions of rho (x) rho.  Test infrastructure only.

Plain definitions (dense rho, N <= 6), following Sec. III.E and Sec. III.F:
  purity                    tr(rho^2)
  collision probability     Z = sum_x p(x)^2 with p(x) = <x|rho|x> / tr rho over all d^N
                            basis states (the anticoncentration measure of Sec. III.F)
  second Renyi entropy      S2(X) = -log tr(rho_X^2), rho_X = tr_{not X}(rho) / tr rho
  Renyi-2 mutual info       I2(A:B) = S2(A) + S2(B) - S2(AB)

MPO route (Fig. 6c): with vec(rho)[eta_1 .. eta_N], eta_j = sigma_j d + sigma'_j, every such
quantity is
  E2 = sum_{eta, eta'} vec(rho)[eta] vec(rho)[eta'] prod_j M_j[eta_j, eta'_j]
for per-atom second-order operators M_j (D2 x D2):
  swap (purity of the atom's part)    M[(s,s'),(t,t')] = delta(s,t') delta(s',t)
  diagonal collision                  M[(s,s'),(t,t')] = delta(s,s') delta(t,t') delta(s,t)
  atom traced out in both copies      M[(s,s'),(t,t')] = delta(s,s') delta(t,t')
and E2 is contracted left to right with a doubled transfer matrix (one einsum per atom,
evaluated in the pairwise order numpy chooses).
"""
from __future__ import annotations

import math

import numpy as np


# ------------------------------------------------------------------ dense definitions
def dense_purity(rho: np.ndarray) -> float:
    """tr(rho^2) / (tr rho)^2."""
    tr = np.trace(rho)
    return float(np.real(np.trace(rho @ rho) / tr ** 2))


def dense_collision(rho: np.ndarray) -> float:
    """sum_x p(x)^2 with p(x) = rho_xx / tr rho."""
    p = np.real(np.diag(rho)) / np.real(np.trace(rho))
    return float(np.sum(p * p))


def dense_reduced(rho: np.ndarray, n: int, d: int, keep) -> np.ndarray:
    """Partial trace over the atoms not in `keep` (kept atoms in increasing order)."""
    keep = sorted(keep)
    T = rho.reshape((d,) * (2 * n))
    # trace out atoms from the highest index down so the remaining axis numbers stay valid
    cur_n = n
    for j in sorted(set(range(n)) - set(keep), reverse=True):
        T = np.trace(T, axis1=j, axis2=cur_n + j)
        cur_n -= 1
    k = len(keep)
    return T.reshape(d ** k, d ** k)


def dense_renyi2(rho: np.ndarray, n: int, d: int, sites) -> float:
    """S2 of the atoms in `sites` for rho / tr rho."""
    r = dense_reduced(rho, n, d, sites)
    r = r / np.trace(r)
    return float(-math.log(np.real(np.trace(r @ r))))


def dense_mutual_info(rho: np.ndarray, n: int, d: int, a, b) -> float:
    return dense_renyi2(rho, n, d, a) + dense_renyi2(rho, n, d, b) - dense_renyi2(rho, n, d, list(a) + list(b))


# ------------------------------------------------------------------ per-atom operators
def op_swap(d: int) -> np.ndarray:
    D2 = d * d
    M = np.zeros((D2, D2), dtype=np.complex128)
    for s in range(d):
        for sp in range(d):
            M[s * d + sp, sp * d + s] = 1.0
    return M


def op_collision(d: int) -> np.ndarray:
    D2 = d * d
    M = np.zeros((D2, D2), dtype=np.complex128)
    for s in range(d):
        M[s * d + s, s * d + s] = 1.0
    return M


def op_trace(d: int) -> np.ndarray:
    vI = np.eye(d, dtype=np.complex128).reshape(-1)
    return np.outer(vI, vI)


# ------------------------------------------------------------------ MPO contraction
def mpo_expect2(m, ops_by_site) -> complex:
    """E2 for the MPO oracle's site tensors A[l, eta, r]; atoms without an operator are traced
    out in both copies.  Unnormalised."""
    d = m.d
    tr_op = op_trace(d)
    E = np.ones((1, 1), dtype=np.complex128)
    for j, a in enumerate(m.A):
        M = np.asarray(ops_by_site.get(j, tr_op), dtype=np.complex128)
        E = np.einsum("ab,asc,st,btd->cd", E, a, M, a, optimize=True)
    return complex(E[0, 0])


def mpo_purity(m) -> float:
    tr = m.trace()
    return float(np.real(mpo_expect2(m, {j: op_swap(m.d) for j in range(m.n)}) / tr ** 2))


def mpo_collision(m) -> float:
    tr = m.trace()
    return float(np.real(mpo_expect2(m, {j: op_collision(m.d) for j in range(m.n)}) / tr ** 2))


def mpo_renyi2(m, sites) -> float:
    tr = m.trace()
    return float(-math.log(np.real(mpo_expect2(m, {j: op_swap(m.d) for j in sites}) / tr ** 2)))


def mpo_mutual_info(m, a, b) -> float:
    return mpo_renyi2(m, a) + mpo_renyi2(m, b) - mpo_renyi2(m, list(a) + list(b))
