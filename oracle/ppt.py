"""Purity-Preserving Truncation on vectors (Sec. III.D, Eqs. (xiformula) and (ppt); App. B).

With the MPO canonised at the cut bond, tr(rho) = sum_i T_i Lambda_i and
tr(rho^2) = |Lambda|^2 (the purity environment P is the identity).  PPT keeps
xi = tr(rho^2) / tr(rho)^2 fixed when Lambda is cut to its leading entries Lambda'
(T' is T cut the same way):

  phi   = angle(Lambda, T)
  theta = arccos(|T| cos(phi) / |T'|)                          Eq. (xiformula)
  sigma = angle(Lambda', T')
  Lambda~ = Lambda' + (tan(theta)/tan(sigma) - 1)
                      * (Lambda' - |Lambda'| cos(sigma) T' / |T'|)   Eq. (ppt)

When |T'| < |T| cos(phi) no angle theta exists; then theta = 0 (end of Sec. III.D).
Readings where the paper is silent:
  * sigma = 0 (Lambda' parallel to T'): there is no direction orthogonal to T' in the
    plane of Lambda' and T', so Lambda~ = Lambda' and the case is flagged.
  * cos(theta) is computed from the full-vector quantities exactly as in Eq. (xiformula).
"""
from __future__ import annotations

import math

import numpy as np

SIN_SIGMA_MIN = 1e-14


def ppt(lam_full, T_full, k: int):
    """Return (Lambda~, info) for the first k entries of descending `lam_full`."""
    lam = np.asarray(lam_full, dtype=np.float64)
    T = np.asarray(T_full, dtype=np.float64)
    lam_p = lam[:k].copy()
    T_p = T[:k].copy()
    nl, nT = np.linalg.norm(lam), np.linalg.norm(T)
    nlp, nTp = np.linalg.norm(lam_p), np.linalg.norm(T_p)
    info = {"feasible": True, "degenerate_sigma": False, "theta": float("nan"),
            "sigma": float("nan"), "x": 0.0}
    if nl == 0.0 or nT == 0.0 or nlp == 0.0 or nTp == 0.0:
        info["degenerate_sigma"] = True
        return lam_p, info
    cos_phi = float(T @ lam) / (nT * nl)
    cos_theta = nT * cos_phi / nTp
    if cos_theta > 1.0:
        info["feasible"] = False
        theta = 0.0
    else:
        theta = math.acos(max(-1.0, cos_theta))
    cos_sigma = float(T_p @ lam_p) / (nTp * nlp)
    cos_sigma = min(1.0, max(-1.0, cos_sigma))
    sigma = math.acos(cos_sigma)
    info["theta"], info["sigma"] = theta, sigma
    if math.sin(sigma) < SIN_SIGMA_MIN:
        info["degenerate_sigma"] = True
        return lam_p, info
    x = math.tan(theta) / math.tan(sigma) - 1.0
    info["x"] = x
    lam_t = lam_p + x * (lam_p - (nlp / nTp) * T_p * cos_sigma)
    return lam_t, info


def xi(lam, T) -> float:
    """tr(rho^2)/tr(rho)^2 for a canonised bond."""
    lam = np.asarray(lam, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    return float(lam @ lam) / float(T @ lam) ** 2
