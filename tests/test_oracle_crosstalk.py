"""Pins of the crosstalk oracle (Sec. II, "MPO form of the noisy CZ gate with crosstalk").

The four-term controlled form is checked against brute force: the exponential of the full
four-atom Hamiltonian, in which the neighbours' blockade terms B n_{i-1} n_i and
B n_{i+1} n_{i+2} appear explicitly, over a piecewise-constant two-segment pulse.  Special
cases: equal pair gates reduce to an ordinary two-site gate, the operator is unitary, the
chain ends drop the missing neighbour, and neighbours prepared in a definite Rydberg class
select one pair gate.
"""
import numpy as np
from scipy.linalg import expm

from oracle import crosstalk, dense


def _n(d, ryd):
    m = np.zeros((d, d), dtype=np.complex128)
    m[ryd, ryd] = 1.0
    return m


def _x(d):
    m = np.zeros((d, d), dtype=np.complex128)
    m[0, 1] = m[1, 0] = 1.0
    return m


def _embed(ops, n):
    """kron of per-atom operators (None = identity) over n atoms"""
    d = next(o.shape[0] for o in ops if o is not None)
    out = np.ones((1, 1), dtype=np.complex128)
    for j in range(n):
        out = np.kron(out, ops[j] if ops[j] is not None else np.eye(d))
    return out


def _pair_h(d, ryd, omega, d1, d2, bpair):
    n_, x_ = _n(d, ryd), _x(d)
    return (0.5 * omega * (_embed([x_, None], 2) + _embed([None, x_], 2)) + d1 * _embed([n_, None], 2)
            + d2 * _embed([None, n_], 2) + bpair * _embed([n_, n_], 2))


def _full_h(d, ryd, omega, d1, d2, bpair, B, left, right):
    """pair (atoms p, p+1) plus neighbours, with the neighbour blockade written out"""
    n_, x_ = _n(d, ryd), _x(d)
    atoms = int(left) + 2 + int(right)
    p = int(left)

    def at(**kw):
        ops = [None] * atoms
        for k, v in kw.items():
            ops[int(k[1:])] = v
        return _embed(ops, atoms)

    h = 0.5 * omega * (at(**{f"a{p}": x_}) + at(**{f"a{p + 1}": x_}))
    h = h + d1 * at(**{f"a{p}": n_}) + d2 * at(**{f"a{p + 1}": n_}) + bpair * at(**{f"a{p}": n_, f"a{p + 1}": n_})
    if left:
        h = h + B * at(a0=n_, **{f"a{p}": n_})
    if right:
        h = h + B * at(**{f"a{p + 1}": n_, f"a{p + 2}": n_})
    return h


def _pulse(d, ryd, B, left, right):
    """two constant segments; returns (u[4], full unitary)"""
    segs = [(1.3, 0.4, -0.7, 5.0, 0.37), (0.8, -0.9, 0.25, 5.0, 0.61)]   # omega, d1, d2, bpair, t
    u = []
    for q in range(4):
        a, b = q % 2, q // 2
        U = np.eye(d * d, dtype=np.complex128)
        for om, d1, d2, bp, t in segs:
            U = expm(-1j * t * _pair_h(d, ryd, om, d1 + a * B, d2 + b * B, bp)) @ U
        u.append(U)
    atoms = int(left) + 2 + int(right)
    Uf = np.eye(d ** atoms, dtype=np.complex128)
    for om, d1, d2, bp, t in segs:
        Uf = expm(-1j * t * _full_h(d, ryd, om, d1, d2, bp, B, left, right)) @ Uf
    return u, Uf


def test_four_term_form_equals_the_full_hamiltonian_evolution():
    for d, ryd in ((2, 1), (3, 2)):
        for left, right in ((True, True), (False, True), (True, False)):
            u, Uf = _pulse(d, ryd, B=2.3, left=left, right=right)
            U = crosstalk.crosstalk_operator(u, d, ryd, left, right)
            assert np.abs(U - Uf).max() <= 1e-12, (d, left, right)


def test_equal_pair_gates_reduce_to_a_two_site_gate_and_the_operator_is_unitary():
    rng = np.random.default_rng(3)
    d, ryd = 3, 2
    z = rng.normal(size=(d * d, d * d)) + 1j * rng.normal(size=(d * d, d * d))
    V, _ = np.linalg.qr(z)
    U = crosstalk.crosstalk_operator([V] * 4, d, ryd)
    assert np.abs(U - np.kron(np.kron(np.eye(d), V), np.eye(d))).max() <= 1e-13
    us = []
    for _ in range(4):
        z = rng.normal(size=(d * d, d * d)) + 1j * rng.normal(size=(d * d, d * d))
        us.append(np.linalg.qr(z)[0])
    U = crosstalk.crosstalk_operator(us, d, ryd)
    assert np.abs(U @ U.conj().T - np.eye(d ** 4)).max() <= 1e-12


def test_definite_neighbour_classes_select_one_pair_gate():
    rng = np.random.default_rng(5)
    d, ryd = 4, 2
    us = [np.linalg.qr(rng.normal(size=(16, 16)) + 1j * rng.normal(size=(16, 16)))[0] for _ in range(4)]
    z = rng.normal(size=(16, 16)) + 1j * rng.normal(size=(16, 16))
    rho_pair = z @ z.conj().T
    rho_pair /= np.trace(rho_pair)
    for a in (0, 1):
        for b in (0, 1):
            nl = np.zeros((d, d), dtype=np.complex128)
            nl[ryd if a else 0, ryd if a else 0] = 1.0
            nr = np.zeros((d, d), dtype=np.complex128)
            nr[ryd if b else 3, ryd if b else 3] = 1.0
            dm = dense.DenseRho([nl, np.eye(d) / d, np.eye(d) / d, nr])
            dm.rho = np.kron(np.kron(nl, rho_pair), nr)
            crosstalk.apply_crosstalk(dm, 1, us, ryd)
            expect = np.kron(np.kron(nl, us[a + 2 * b] @ rho_pair @ us[a + 2 * b].conj().T), nr)
            assert np.abs(dm.rho - expect).max() <= 1e-13, (a, b)


def _rand_state(rng, d, n):
    out = []
    for _ in range(n):
        z = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
        r = z @ z.conj().T + 0.5 * np.eye(d)
        out.append(r / np.trace(r))
    return out


def _unit(rng, k):
    return np.linalg.qr(rng.normal(size=(k, k)) + 1j * rng.normal(size=(k, k)))[0]


def test_mpo_form_equals_dense_when_nothing_is_cut():
    from oracle import channels, mpo
    rng = np.random.default_rng(0)
    d, n = 2, 5
    rhos = _rand_state(rng, d, n)
    dm, m = dense.DenseRho(rhos), mpo.MPO(rhos, chi=64)
    for s_ in (0, 2, 1, 3):
        V = _unit(rng, d * d)
        dm.apply_kraus([V], (s_, s_ + 1))
        m.apply_2site(s_, channels.superop_2site([V], d))
    for s_ in (0, 1, 2, 3):
        u = [_unit(rng, d * d) for _ in range(4)]
        crosstalk.apply_crosstalk(dm, s_, u, 1)
        crosstalk.apply_crosstalk_mpo(m, s_, u, 1)
        assert np.abs(m.to_dense() - dm.rho).max() <= 1e-13, s_


def test_mpo_form_cut_keeps_xi_with_ppt():
    """PPT keeps xi = tr(rho^2) / tr(rho)^2 through the cut (Eq. (ppt)); a plain cut does not"""
    from oracle import channels, mpo
    rng = np.random.default_rng(1)
    d, n = 2, 6
    rhos = _rand_state(rng, d, n)
    for use_ppt in (True, False):
        r2 = np.random.default_rng(2)
        m = mpo.MPO(rhos, chi=64, use_ppt=use_ppt)
        for s_ in (0, 2, 4, 1, 3):
            m.apply_2site(s_, channels.superop_2site([_unit(r2, d * d)], d))
        xi0 = m.purity() / abs(m.trace()) ** 2
        crosstalk.apply_crosstalk_mpo(m, 2, [_unit(r2, d * d) for _ in range(4)], 1, chi=4)
        assert m.bond_dims()[2] == 4
        xi1 = m.purity() / abs(m.trace()) ** 2
        if use_ppt:
            assert abs(xi1 - xi0) <= 1e-12 * xi0
        else:
            assert abs(xi1 - xi0) > 1e-6 * xi0
