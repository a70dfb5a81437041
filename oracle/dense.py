"""Exact dense density matrix: rho is a d^N x d^N complex128 array.

This is the plain definition of what the MPO method approximates (Sec. III.A): the
density matrix evolved by the same completely positive maps, with no truncation.  A map
on atoms S is applied as rho -> sum_k K rho K^dagger with K acting on the atoms of S.
Usable for N <= 6 (729 x 729 at d=3, 4096 x 4096 at d=4).
"""
from __future__ import annotations

import numpy as np

from . import channels


class DenseRho:
    def __init__(self, site_rhos):
        self.n = len(site_rhos)
        self.d = site_rhos[0].shape[0]
        rho = np.ones((1, 1), dtype=np.complex128)
        for r in site_rhos:
            rho = np.kron(rho, np.asarray(r, dtype=np.complex128))
        self.rho = rho

    # -------------------------------------------------------------- helpers
    def _tensor(self):
        return self.rho.reshape((self.d,) * (2 * self.n))

    def _apply_left(self, T, K, sites):
        """Multiply operator K (on `sites`, in that order) into the row indices of T."""
        k = len(sites)
        Kt = K.reshape((self.d,) * (2 * k))
        out = np.tensordot(Kt, T, axes=(list(range(k, 2 * k)), list(sites)))
        # the new row indices of `sites` are now the first k axes; move them back
        return np.moveaxis(out, list(range(k)), list(sites))

    def _apply_right_dagger(self, T, K, sites):
        """T -> T K^dagger on the column indices of `sites`."""
        cols = [self.n + s for s in sites]
        k = len(sites)
        Kt = K.conj().reshape((self.d,) * (2 * k))
        out = np.tensordot(Kt, T, axes=(list(range(k, 2 * k)), cols))
        return np.moveaxis(out, list(range(k)), cols)

    # -------------------------------------------------------------- evolution
    def apply_kraus(self, kraus, sites):
        T = self._tensor()
        acc = np.zeros_like(T)
        for K in kraus:
            K = np.asarray(K, dtype=np.complex128)
            acc += self._apply_right_dagger(self._apply_left(T, K, sites), K, sites)
        self.rho = acc.reshape(self.rho.shape)

    def run(self, ops):
        for kind, site, kraus in ops:
            if kind == "k2":
                self.apply_kraus(kraus, (site, site + 1))
            else:
                self.apply_kraus(kraus, (site,))
        return self

    # -------------------------------------------------------------- measurements
    def trace(self) -> complex:
        return complex(np.trace(self.rho))

    def expect_product(self, ops_by_site) -> complex:
        """tr(rho * prod_j O_j) for single-atom operators O_j (unnormalised)."""
        T = self._tensor()
        for j, O in ops_by_site.items():
            T = self._apply_left(T, np.asarray(O, dtype=np.complex128), (j,))
        M = T.reshape(self.rho.shape)
        return complex(np.trace(M))

    def purity(self) -> float:
        """tr(rho^2) (unnormalised)."""
        return float(np.real(np.vdot(self.rho.conj().T, self.rho)))

    def eigvalsh(self):
        return np.linalg.eigvalsh(0.5 * (self.rho + self.rho.conj().T))


def run_spec(spec) -> DenseRho:
    d = spec.d
    dm = DenseRho([channels.plus_state(d)] * spec.n)
    return dm.run(channels.circuit_ops(spec))


def observables(dm: DenseRho, g: float = 1.0) -> dict:
    """Energy per site, populations and purity, normalised by tr(rho) (raw form)."""
    n, d = dm.n, dm.d
    tr = dm.trace()
    e = 0.0
    for c, term in channels.tfim_terms(n, d, g):
        e += c * dm.expect_product(term)
    pops = np.zeros((n, d))
    for j in range(n):
        for a in range(d):
            pops[j, a] = np.real(dm.expect_product({j: channels.proj(d, a)}) / tr)
    Pq = channels.qubit_projector(d)
    succ = dm.expect_product({j: Pq for j in range(n)}) / tr
    return {
        "trace": tr,
        "energy_per_site": float(np.real(e / tr)) / n,
        "populations": pops,
        "p_success": float(np.real(succ)),
        "purity": dm.purity() / float(np.real(tr)) ** 2,
    }
