"""Plain FP64 vectorised density-operator MPO (Sec. III.A and III.D), numpy + LAPACK.

State: site tensors A[j] of shape (chi_left, D2, chi_right), D2 = d*d, with the
vectorised physical index eta = sigma*d + sigma' in the middle.

Two-site update (Sec. III.A; Fig. (ansatzes)c; Fig. (mpo_mpdo_update_comparisons)a):
  1. bring the canonical centre onto the pair (i, i+1): every site left of i is a left
     isometry and every site right of i+1 a right isometry (the canonisation identities
     of Sec. III.A), by QR sweeps;
  2. merge: theta = S2 . (A[i] A[i+1]);
  3. split with the SVD theta = U diag(Lambda) V^dagger (LAPACK, no Gram matrix);
  4. cut to the k leading singular values (k <= chi), k = #{Lambda_j > eps_rel Lambda_0};
  5. PPT (Sec. III.D): trace environment T_j = (l . U_j)(V_j^dagger . r), where l, r are
     the trace vectors of the left and right parts of the chain (contractions with
     vec(I)); Lambda~ from ``ppt.ppt``;
  6. A[i] = U_k, A[i+1] = diag(Lambda~) V_k^dagger; the centre is now at i+1.
Single-atom channels multiply the physical index of one site.
Expectations of products of single-atom operators are transfer-matrix contractions
(Sec. III.E, linear observables): tr(rho O) = sum rho_{s s'} O_{s' s}.

Readings of the paper (silent points): T is taken real (its imaginary part is recorded);
cut ties are broken by index order; the trace is not renormalised unless asked.
"""
from __future__ import annotations

import numpy as np

from . import channels
from . import ppt as ppt_mod

EPS_REL = 1e-14


def _vI(d: int) -> np.ndarray:
    return channels.vec(np.eye(d))


class MPO:
    def __init__(self, site_rhos, chi: int, use_ppt: bool = True, eps_rel: float = EPS_REL,
                 renorm_trace: bool = False):
        self.d = site_rhos[0].shape[0]
        self.D2 = self.d * self.d
        self.n = len(site_rhos)
        self.chi = chi
        self.use_ppt = use_ppt
        self.eps_rel = eps_rel
        self.renorm_trace = renorm_trace
        self.A = [channels.vec(r).reshape(1, self.D2, 1) for r in site_rhos]
        # sites < lo are left isometries, sites > hi are right isometries
        self.lo, self.hi = 0, self.n - 1
        self.log = []

    # ---------------------------------------------------------------- canonical form
    def _move_right(self, j):
        """QR of site j as (chi_l*D2, chi_r); R goes into site j+1."""
        a = self.A[j]
        cl, D2, cr = a.shape
        Q, R = np.linalg.qr(a.reshape(cl * D2, cr))
        self.A[j] = Q.reshape(cl, D2, Q.shape[1])
        self.A[j + 1] = np.tensordot(R, self.A[j + 1], axes=(1, 0))

    def _move_left(self, j):
        """LQ of site j as (chi_l, D2*chi_r); L goes into site j-1."""
        a = self.A[j]
        cl, D2, cr = a.shape
        Q, R = np.linalg.qr(a.reshape(cl, D2 * cr).conj().T)
        # a = R^dagger Q^dagger
        self.A[j] = Q.conj().T.reshape(Q.shape[1], D2, cr)
        self.A[j - 1] = np.tensordot(self.A[j - 1], R.conj().T, axes=(2, 0))

    def canonicalize(self, i):
        """Make sites < i left isometries and sites > i+1 right isometries."""
        for j in range(self.lo, i):
            self._move_right(j)
        for j in range(self.hi, i + 1, -1):
            self._move_left(j)
        self.lo, self.hi = i, i + 1

    # ---------------------------------------------------------------- trace vectors
    def left_trace(self, i):
        """l[m] = contraction of sites 0..i-1 with vec(I) on every physical index."""
        vI = _vI(self.d)
        l = np.ones(1, dtype=np.complex128)
        for j in range(i):
            l = np.einsum("l,lsr,s->r", l, self.A[j], vI)
        return l

    def right_trace(self, j0):
        """r[m] = contraction of sites j0..n-1 with vec(I)."""
        vI = _vI(self.d)
        r = np.ones(1, dtype=np.complex128)
        for j in range(self.n - 1, j0 - 1, -1):
            r = np.einsum("lsr,s,r->l", self.A[j], vI, r)
        return r

    # ---------------------------------------------------------------- updates
    def apply_1site(self, j, S1):
        self.A[j] = np.einsum("ab,lbr->lar", S1, self.A[j])
        self.lo, self.hi = min(self.lo, j), max(self.hi, j)

    def apply_2site(self, i, S2, chi=None):
        chi = self.chi if chi is None else chi
        D2 = self.D2
        self.canonicalize(i)
        a, b = self.A[i], self.A[i + 1]
        cl, cr = a.shape[0], b.shape[2]
        merged = np.tensordot(a, b, axes=(2, 0))                  # (l, s1, s2, r)
        S4 = S2.reshape(D2, D2, D2, D2)
        theta = np.einsum("abst,lstr->labr", S4, merged)          # (l, s1', s2', r)
        M = theta.reshape(cl * D2, D2 * cr)
        U, lam, Vh = np.linalg.svd(M, full_matrices=False)
        n_nz = int(np.sum(lam > self.eps_rel * lam[0])) if lam[0] > 0 else 0
        k = max(1, min(chi, n_nz))
        # trace environment of every singular vector
        vI = _vI(self.d)
        lv = np.kron(self.left_trace(i), vI)                      # over (l, s1)
        rv = np.kron(vI, self.right_trace(i + 2))                 # over (s2, r)
        Tc = (lv @ U) * (Vh @ rv)
        T = np.real(Tc)
        info = {"bond": i, "chi_l": cl, "chi_r": cr, "kept": k,
                "n_sv": len(lam), "max_abs_imag_T": float(np.max(np.abs(np.imag(Tc)))),
                "trace_before": float(T @ lam), "xi_before": ppt_mod.xi(lam, T),
                "discarded_weight": float(np.sum(lam[k:] ** 2) / np.sum(lam ** 2)),
                "gap_at_cut": float(lam[k - 1] - lam[k]) if k < len(lam) else float("inf")}
        if self.use_ppt:
            lam_t, pinfo = ppt_mod.ppt(lam, T, k)
            info.update({"ppt_feasible": pinfo["feasible"], "ppt_theta": pinfo["theta"]})
        else:
            lam_t = lam[:k].copy()
        if self.renorm_trace:
            lam_t = lam_t * (T @ lam) / (T[:k] @ lam_t)
        info["trace_after"] = float(T[:k] @ lam_t)
        info["xi_after"] = ppt_mod.xi(lam_t, T[:k])
        self.A[i] = U[:, :k].reshape(cl, D2, k)
        self.A[i + 1] = (lam_t[:, None] * Vh[:k]).reshape(k, D2, cr)
        self.lo, self.hi = i + 1, i + 1
        self.log.append(info)
        return info

    def run(self, ops):
        for kind, site, kraus in ops:
            if kind == "k2":
                self.apply_2site(site, channels.superop_2site(kraus, self.d))
            else:
                self.apply_1site(site, channels.superop_1site(kraus))
        return self

    # ---------------------------------------------------------------- measurements
    def expect_product(self, ops_by_site) -> complex:
        """tr(rho prod_j O_j) by a left-to-right transfer-matrix sweep (unnormalised)."""
        vI = _vI(self.d)
        l = np.ones(1, dtype=np.complex128)
        for j in range(self.n):
            if j in ops_by_site:
                o = channels.vec(np.asarray(ops_by_site[j]).T)    # o[s d + s'] = O[s', s]
            else:
                o = vI
            l = np.einsum("l,lsr,s->r", l, self.A[j], o)
        return complex(l[0])

    def trace(self) -> complex:
        return self.expect_product({})

    def bond_dims(self):
        return [a.shape[2] for a in self.A[:-1]]

    def purity(self) -> float:
        """tr(rho^2) = <vec rho | vec rho> for Hermitian rho (vectorised 2-norm)."""
        E = np.ones((1, 1), dtype=np.complex128)
        for a in self.A:
            # two pairwise contractions (optimize=True); the plain three-operand loop would
            # cost chi^4 D2 per site
            E = np.einsum("ab,asc,bsd->cd", E, a.conj(), a, optimize=True)
        return float(np.real(E[0, 0]))

    def to_dense(self) -> np.ndarray:
        """Contract the chain into the dense d^N x d^N matrix (small N only)."""
        T = self.A[0]
        for a in self.A[1:]:
            T = np.tensordot(T, a, axes=(T.ndim - 1, 0))
        T = T.reshape((self.d, self.d) * self.n)
        rows = [2 * j for j in range(self.n)]
        cols = [2 * j + 1 for j in range(self.n)]
        M = np.transpose(T, rows + cols)
        dim = self.d ** self.n
        return M.reshape(dim, dim)


def run_spec(spec, chi=None, use_ppt=True, eps_rel=EPS_REL, renorm_trace=False) -> MPO:
    chi = spec.chi if chi is None else chi
    m = MPO([channels.plus_state(spec.d)] * spec.n, chi=chi, use_ppt=use_ppt,
            eps_rel=eps_rel, renorm_trace=renorm_trace)
    return m.run(channels.circuit_ops(spec))


def observables(m: MPO, g: float = 1.0) -> dict:
    n, d = m.n, m.d
    tr = m.trace()
    e = 0.0
    for c, term in channels.tfim_terms(n, d, g):
        e += c * m.expect_product(term)
    pops = np.zeros((n, d))
    for j in range(n):
        for a in range(d):
            pops[j, a] = np.real(m.expect_product({j: channels.proj(d, a)}) / tr)
    Pq = channels.qubit_projector(d)
    succ = m.expect_product({j: Pq for j in range(n)}) / tr
    return {
        "trace": tr,
        "energy_per_site": float(np.real(e / tr)) / n,
        "populations": pops,
        "p_success": float(np.real(succ)),
        "purity": m.purity() / float(np.real(tr)) ** 2,
    }
