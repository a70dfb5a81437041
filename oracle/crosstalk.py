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
