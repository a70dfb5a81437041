"""QAOA circuits on the GPU MPO: Kraus inputs and the driver loop.

Circuit (Sec. IV, Eq. (tfim_model); noise model of Sec. II as discrete maps):
layer k = exp(-i gamma_k Z(x)Z) blocks on even bonds left to right, then odd bonds right to
left, each followed by a |1> -> |r> leak on both atoms; then exp(-i beta_k X), qubit
dephasing and Rydberg decay on every atom.  The single-atom maps are queued in the library
and enter the next block that touches the atom (they commute with everything else), which
fixes the order of truncations; the last layer's maps act on the observables.
Measured: TFIM energy H = -sum Z_i Z_{i+1} - g sum X_i (Eq. (tfim_hamiltonian), b = 0),
per-atom level populations and the all-qubit probability (Sec. IV, qubit trace).
"""
from __future__ import annotations

import math
import time
from typing import Optional

import numpy as np

from .mpdo import MPDO, MPDO_FP32, MPDO_FP64

# decay branching into |0>, |1>, dark (Fig. 1 caption)
BRANCH = (1.0 / 16.0, 1.0 / 16.0, 7.0 / 8.0)


def _e(d, a, b):
    m = np.zeros((d, d), dtype=np.complex128)
    m[a, b] = 1.0
    return m


def zz_gate(gamma: float, d: int) -> np.ndarray:
    """exp(-i gamma Z(x)Z) with Z = |0><0| - |1><1| (zero on other levels): diagonal phases."""
    z = np.zeros(d)
    z[0], z[1] = 1.0, -1.0
    ph = np.exp(-1j * gamma * np.outer(z, z).reshape(-1))
    return np.diag(ph)


def x_rotation(beta: float, d: int) -> np.ndarray:
    """exp(-i beta X) with X = |0><1| + |1><0|: a rotation on {0,1}, identity elsewhere."""
    u = np.eye(d, dtype=np.complex128)
    u[0, 0] = u[1, 1] = math.cos(beta)
    u[0, 1] = u[1, 0] = -1j * math.sin(beta)
    return u


def leak_kraus(p: float, d: int):
    k0 = np.eye(d, dtype=np.complex128)
    k0[1, 1] = math.sqrt(1.0 - p)
    return [k0, math.sqrt(p) * _e(d, 2, 1)]


def dephasing_kraus(p: float, d: int):
    k0 = np.eye(d, dtype=np.complex128)
    k0[0, 0] = k0[1, 1] = math.sqrt(1.0 - p)
    k1 = np.zeros((d, d), dtype=np.complex128)
    k1[0, 0], k1[1, 1] = math.sqrt(p), -math.sqrt(p)
    return [k0, k1]


def decay_kraus(p: float, d: int):
    k0 = np.eye(d, dtype=np.complex128)
    k0[2, 2] = math.sqrt(1.0 - p)
    if d == 3:
        return [k0, math.sqrt(p) * _e(d, 1, 2)]
    return [k0] + [math.sqrt(p * b) * _e(d, j, 2) for j, b in zip((0, 1, 3), BRANCH)]


def block_kraus(gamma: float, p_leak: float, d: int):
    """Two-atom Kraus operators of one Ising block followed by the leak on both atoms."""
    u = zz_gate(gamma, d)
    lk = leak_kraus(p_leak, d)
    return [np.kron(a, b) @ u for a in lk for b in lk]


def plus_rho(d: int) -> np.ndarray:
    v = np.zeros(d, dtype=np.complex128)
    v[0] = v[1] = 1.0 / math.sqrt(2.0)
    return np.outer(v, v.conj())


def bond_order(n: int):
    return list(range(0, n - 1, 2)) + list(range(1, n - 1, 2))[::-1]


def run_circuit(spec, precision: int = MPDO_FP64, chi: Optional[int] = None, ppt: bool = True,
                infos: Optional[list] = None, m: Optional[MPDO] = None) -> MPDO:
    """Evolve |+><+|^N through the spec's circuit; returns the MPDO (state on the GPU)."""
    n, d = spec.n, spec.d
    chi = spec.chi if chi is None else chi
    if m is None:
        m = MPDO(n, d, chi, precision=precision, ppt=ppt)
    m.init_product_state([plus_rho(d)] * n)
    want_info = infos is not None
    for k in range(spec.p):
        kr = block_kraus(spec.gamma[k], spec.p_leak, d)
        for i in bond_order(n):
            inf = m.apply_gate_kraus(i, kr, info=want_info)
            if want_info:
                infos.append(inf)
        ux = [x_rotation(spec.beta[k], d)]
        dp = dephasing_kraus(spec.p_deph, d)
        dc = decay_kraus(spec.p_decay, d)
        for j in range(n):
            m.apply_channel(j, ux)
            m.apply_channel(j, dp)
            m.apply_channel(j, dc)
    return m


def observables(m: MPDO, g: float = 1.0) -> dict:
    n, d = m.n, m.d
    Z = np.zeros((d, d), dtype=np.complex128)
    Z[0, 0], Z[1, 1] = 1.0, -1.0
    X = np.zeros((d, d), dtype=np.complex128)
    X[0, 1] = X[1, 0] = 1.0
    terms = [(i, [Z, Z]) for i in range(n - 1)] + [(i, [X]) for i in range(n)]
    pops = [(j, [_e(d, a, a)]) for j in range(n) for a in range(d)]
    pq = _e(d, 0, 0) + _e(d, 1, 1)
    vals = m.expect(terms + pops + [(0, [pq] * n)], normalize=True)
    nzz = n - 1
    energy = -np.sum(vals[:nzz]).real - g * np.sum(vals[nzz:nzz + n]).real
    popv = vals[nzz + n:nzz + n + n * d].real.reshape(n, d)
    return {"trace": m.trace(), "energy_per_site": energy / n, "populations": popv,
            "p_success": float(vals[-1].real)}


def observable_terms(n: int, d: int):
    """Energy terms (ZZ bonds, X sites), per-atom populations and the all-qubit projector."""
    Z = np.zeros((d, d), dtype=np.complex128)
    Z[0, 0], Z[1, 1] = 1.0, -1.0
    X = np.zeros((d, d), dtype=np.complex128)
    X[0, 1] = X[1, 0] = 1.0
    terms = [(i, [Z, Z]) for i in range(n - 1)] + [(i, [X]) for i in range(n)]
    terms += [(j, [_e(d, a, a)]) for j in range(n) for a in range(d)]
    terms += [(0, [_e(d, 0, 0) + _e(d, 1, 1)] * n)]
    return terms


def summarize(values: np.ndarray, n: int, d: int, g: float = 1.0) -> dict:
    """Energy per site, populations and success probability from observable_terms values."""
    nzz = n - 1
    energy = -np.sum(values[:nzz]).real - g * np.sum(values[nzz:nzz + n]).real
    pops = values[nzz + n:nzz + n + n * d].real.reshape(n, d)
    return {"energy_per_site": energy / n, "populations": pops, "p_success": float(values[-1].real)}


def describe(spec, precision: int = MPDO_FP64, chi: Optional[int] = None, ppt: bool = True) -> dict:
    """The circuit of run_circuit as flat arrays for mpdo_run_batch."""
    n, d = spec.n, spec.d
    sets = []
    kind, site, which = [], [], []
    for k in range(spec.p):
        base = len(sets)
        sets += [block_kraus(spec.gamma[k], spec.p_leak, d), [x_rotation(spec.beta[k], d)],
                 dephasing_kraus(spec.p_deph, d), decay_kraus(spec.p_decay, d)]
        for i in bond_order(n):
            kind.append(0)
            site.append(i)
            which.append(base)
        for j in range(n):
            for q in (1, 2, 3):
                kind.append(1)
                site.append(j)
                which.append(base + q)
    counts = [len(s_) for s_ in sets]
    offs, flat, pos = [], [], 0
    for s_ in sets:
        offs.append(pos)
        for K in s_:
            flat.append(np.asarray(K, dtype=np.complex128).reshape(-1))
            pos += K.size
    terms = observable_terms(n, d)
    return {"n": n, "d": d, "chi": spec.chi if chi is None else chi, "precision": precision,
            "ppt": ppt, "op_kind": kind, "op_site": site, "op_set": which, "set_count": counts,
            "set_offset": offs, "kraus": np.concatenate(flat),
            "rho0": np.stack([plus_rho(d)] * n), "term_first": [t[0] for t in terms],
            "term_len": [len(t[1]) for t in terms],
            "term_ops": np.concatenate([np.stack(t[1]).reshape(-1) for t in terms])}


# ----------------------------------------------------------------- second-order observables
# Per-atom operators on the (eta, eta') pair of the two copies of vec(rho), eta = s d + s'
# (Fig. 6c): the swap pairs rho_{s s'} with rho_{s' s} (purity of the atom's part), the
# diagonal pairs rho_{ss} with rho_{ss} (collision probability), the trace pairs traces.
def swap_op(d: int) -> np.ndarray:
    M = np.zeros((d * d, d * d), dtype=np.complex128)
    for a in range(d):
        for b in range(d):
            M[a * d + b, b * d + a] = 1.0
    return M


def diagonal_op(d: int) -> np.ndarray:
    M = np.zeros((d * d, d * d), dtype=np.complex128)
    for a in range(d):
        M[a * d + a, a * d + a] = 1.0
    return M


def trace_op(d: int) -> np.ndarray:
    v = np.eye(d, dtype=np.complex128).reshape(-1)
    return np.outer(v, v)


def purity(m: MPDO) -> float:
    """tr(rho^2) / tr(rho)^2."""
    return float(m.expect2([(0, [swap_op(m.d)] * m.n)])[0].real)


def collision_probability(m: MPDO) -> float:
    """sum_x p(x)^2 over all d^N basis states, p(x) = rho_xx / tr rho (Sec. III.F)."""
    return float(m.expect2([(0, [diagonal_op(m.d)] * m.n)])[0].real)


def _block_term(m: MPDO, sites):
    lo, hi = min(sites), max(sites)
    ops = [swap_op(m.d) if j in sites else trace_op(m.d) for j in range(lo, hi + 1)]
    return (lo, ops)


def renyi2(m: MPDO, sites) -> float:
    """S2 = -log tr(rho_X^2) of the atoms in `sites`, rho normalised to unit trace."""
    return float(-math.log(m.expect2([_block_term(m, set(sites))])[0].real))


def renyi2_mutual_information(m: MPDO, a, b) -> float:
    """S2(A) + S2(B) - S2(AB) (Sec. III.F)."""
    a, b = set(a), set(b)
    v = m.expect2([_block_term(m, a), _block_term(m, b), _block_term(m, a | b)]).real
    return float(-math.log(v[0]) - math.log(v[1]) + math.log(v[2]))


# ------------------------------------------------------------ the pulse-level QAOA iteration
def _qubit_unitary(u2, d: int) -> np.ndarray:
    u = np.eye(d, dtype=np.complex128)
    u[:2, :2] = u2
    return u


def _site_superop(u: np.ndarray) -> np.ndarray:
    """vec(u rho u^+) with the per-atom vectorised index sigma d + sigma'."""
    return np.kron(u, u.conj())


def cz_phase(S: np.ndarray, d: int) -> float:
    """The single-qubit Z phase of a two-atom CZ channel S (mpdo_apply_gate's layout):
    arg(u_01 / u_00) read off S's action on |01><00| (a CZ pulse returns the qubit states to
    themselves up to these phases)."""
    D2 = d * d
    src = (0 * d + 0) * D2 + (1 * d + 0)     # |0><0| (x) |1><0|
    return float(np.angle(S[src, src]))


def pulse_qaoa_ops(cz: np.ndarray, alphas, betas, b: float, d: int, phase: float):
    """The QAOA iteration of Sec. IV from a two-atom CZ channel (Eqs. (HZ_block_representation),
    (HZ_representation)): per layer, on every bond exp(i alpha Z_i Z_j) = CNOT (I (x)
    exp(i alpha Z_j)) CNOT with CNOT = (I (x) Had) CZ (I (x) Had), the CZ's single-qubit Z
    phase `phase` (cz_phase of the noise-free pulse) undone on both atoms; then exp(i b alpha Z)
    and exp(i beta X) on every atom (single-atom gates on {0, 1}, noise free).  Returns
    [(block superoperator, [zfield, mixer])] per layer (superoperators in mpdo_apply_gate's
    layout; the mixer and field as unitaries)."""
    corr = _site_superop(_qubit_unitary(np.diag([1.0, np.exp(-1j * phase)]), d))
    czc = np.kron(corr, corr) @ cz
    had = _site_superop(_qubit_unitary(np.array([[1.0, 1.0], [1.0, -1.0]]) / math.sqrt(2.0), d))
    eye = np.eye(d * d, dtype=np.complex128)
    h2 = np.kron(eye, had)
    layers = []
    for a, bt in zip(alphas, betas):
        rz = np.kron(eye, _site_superop(_qubit_unitary(np.diag([np.exp(1j * a), np.exp(-1j * a)]), d)))
        blk = h2 @ czc @ h2 @ rz @ h2 @ czc @ h2
        zf = _qubit_unitary(np.diag([np.exp(1j * b * a), np.exp(-1j * b * a)]), d)
        mx = _qubit_unitary(np.array([[math.cos(bt), 1j * math.sin(bt)], [1j * math.sin(bt), math.cos(bt)]]), d)
        layers.append((blk, [zf, mx]))
    return layers


def run_pulse_qaoa(n: int, d: int, chi: int, layers, precision: int = MPDO_FP64) -> MPDO:
    """|+>^N through the layers of pulse_qaoa_ops: bonds left to right, then the single-atom
    gates on every atom (queued, they enter the next block)."""
    m = MPDO(n, d, chi, precision=precision)
    m.init_product_state([plus_rho(d)] * n)
    for blk, singles in layers:
        for i in range(n - 1):
            m.apply_gate(i, blk)
        for j in range(n):
            for u in singles:
                m.apply_channel(j, [u])
    return m
