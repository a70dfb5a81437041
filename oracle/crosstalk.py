"""Rydberg crosstalk gate of an atom pair with its two neighbours (test infrastructure).

Only tests/, __graft_entry__.smoke() and bench.py's CPU baseline use this module; the HIP
path shares nothing with it.

Sec. II, "MPO form of the noisy CZ gate with crosstalk": residual Rydberg population on the
neighbours i-1 and i+2 of a driven pair (i, i+1) shifts the pair's detunings through the
nearest-neighbour blockade B.  The neighbours are not driven, so their Rydberg projectors
commute with the whole pulse, and the gate is a sum of four pair gates selected by the
neighbours' Rydberg projectors:

    C = sum_{a,b in {0,1}} P^a_{i-1} (x) C_{i,i+1}(Delta_i + a B, Delta_{i+1} + b B) (x) P^b_{i+2}

with P^1 = |r><r| and P^0 = I - |r><r|.  As in the paper, the crosstalk gate is simulated
without noise, so each C_ab is a unitary U_ab and the four-site map is rho -> U rho U^+ with
U = sum_ab P^a (x) U_ab (x) P^b.  At an end of the chain the missing neighbour contributes
no shift (only a = 0, or only b = 0).
"""
from __future__ import annotations

import numpy as np


def rydberg_projectors(d: int, ryd: int):
    """(P^0, P^1): the projector off and onto the Rydberg level ryd of one atom."""
    p1 = np.zeros((d, d), dtype=np.complex128)
    p1[ryd, ryd] = 1.0
    return np.eye(d, dtype=np.complex128) - p1, p1


def crosstalk_operator(u, d: int, ryd: int, left: bool = True, right: bool = True) -> np.ndarray:
    """The gate's unitary on [i-1 if left] + [i, i+1] + [i+2 if right], in that kron order.

    u[a + 2 b] is the pair unitary (d^2 x d^2 on the index sigma_i d + sigma_{i+1}) with the
    detunings shifted by a B on atom i and b B on atom i+1.
    """
    P = rydberg_projectors(d, ryd)
    out = None
    for a in ((0, 1) if left else (0,)):
        for b in ((0, 1) if right else (0,)):
            term = np.asarray(u[a + 2 * b], dtype=np.complex128)
            if left:
                term = np.kron(P[a], term)
            if right:
                term = np.kron(term, P[b])
            out = term if out is None else out + term
    return out


def apply_crosstalk(dm, site: int, u, ryd: int) -> None:
    """Apply the crosstalk gate of pair (site, site+1) to a dense.DenseRho in place."""
    left = site >= 1
    right = site + 2 <= dm.n - 1
    U = crosstalk_operator(u, dm.d, ryd, left, right)
    sites = ([site - 1] if left else []) + [site, site + 1] + ([site + 2] if right else [])
    dm.apply_kraus([U], tuple(sites))


def _vec_superop(U: np.ndarray, d: int, k: int) -> np.ndarray:
    """rho -> U rho U^+ on k atoms as a matrix on the per-atom vectorised indices
    eta_j = sigma_j d + sigma'_j (atom-major), the layout of the MPO's physical legs."""
    S = np.einsum("ab,cd->acbd", U, U.conj())          # (sigma, sigma', s, s') as multi-indices
    S = S.reshape((d,) * (4 * k))
    sig = list(range(0, k))
    sigp = list(range(k, 2 * k))
    s_ = list(range(2 * k, 3 * k))
    sp = list(range(3 * k, 4 * k))
    order = [x for j in range(k) for x in (sig[j], sigp[j])] + [x for j in range(k) for x in (s_[j], sp[j])]
    D2 = d * d
    return np.transpose(S, order).reshape(D2 ** k, D2 ** k)


def apply_crosstalk_mpo(m, site: int, u, ryd: int, chi=None):
    """The crosstalk gate on the oracle MPO (oracle.mpo.MPO) with the paper's truncation.

    The region of the gate (the pair and its neighbours) is brought into canonical form, its
    sites are contracted, the gate's superoperator is applied, the bond between the two atoms
    of the pair is cut to chi with PPT (Eqs. (xiformula), (ppt); the same cut rule as the
    oracle's two-site update), and the two sides are split back into sites without a cut.
    """
    from . import ppt as ppt_mod
    from .mpo import _vI
    chi = m.chi if chi is None else chi
    d, D2, n = m.d, m.D2, m.n
    left, right = site >= 1, site + 2 <= n - 1
    lo, hi = (site - 1 if left else site), (site + 2 if right else site + 1)
    k = hi - lo + 1
    nl = site + 1 - lo                                   # atoms left of the pair's middle bond
    for j in range(m.lo, lo):
        m._move_right(j)
    for j in range(m.hi, hi, -1):
        m._move_left(j)
    T = m.A[lo]
    for j in range(lo + 1, hi + 1):
        T = np.tensordot(T, m.A[j], axes=(T.ndim - 1, 0))
    cl, cr = T.shape[0], T.shape[-1]
    T = T.reshape(cl, D2 ** k, cr)
    S = _vec_superop(crosstalk_operator(u, d, ryd, left, right), d, k)
    T = np.einsum("ab,lbr->lar", S, T)
    M = T.reshape(cl * D2 ** nl, D2 ** (k - nl) * cr)
    Uu, lam, Vh = np.linalg.svd(M, full_matrices=False)
    n_nz = int(np.sum(lam > m.eps_rel * lam[0])) if lam[0] > 0 else 0
    kk = max(1, min(chi, n_nz))
    vI = _vI(d)
    lv = m.left_trace(lo)
    for _ in range(nl):
        lv = np.kron(lv, vI)
    rv = m.right_trace(hi + 1)
    for _ in range(k - nl):
        rv = np.kron(vI, rv)
    Tv = np.real((lv @ Uu) * (Vh @ rv))
    lam_t = ppt_mod.ppt(lam, Tv, kk)[0] if m.use_ppt else lam[:kk].copy()
    L = Uu[:, :kk].reshape(cl, D2 ** nl, kk)
    R = (lam_t[:, None] * Vh[:kk]).reshape(kk, D2 ** (k - nl), cr)

    def split(X, sites):
        """X: (c_l, D2^len(sites), c_r) -> sites, exact (singular values above 1e-15 of the largest)"""
        cur = X
        for j in sites[:-1]:
            a, rest, b = cur.shape
            Mx = cur.reshape(a * D2, (rest // D2) * b)
            U2, s2, V2 = np.linalg.svd(Mx, full_matrices=False)
            r = max(1, int(np.sum(s2 > 1e-15 * s2[0])))
            m.A[j] = U2[:, :r].reshape(a, D2, r)
            cur = (s2[:r, None] * V2[:r]).reshape(r, rest // D2, b)
        m.A[sites[-1]] = cur

    split(L, list(range(lo, site + 1)))
    split(R, list(range(site + 1, hi + 1)))
    m.lo, m.hi = site, hi
