"""Pins of the oracle's vectorisation and channel model against closed forms.

Vectorisation (Sec. III.A): checked against direct matrix products, not against the
Kronecker formula it is built from.  Single-atom maps: closed-form population and
coherence updates of each Kraus set (Sec. II noise, read as discrete maps).
"""
import math

import numpy as np
import pytest

from oracle import channels as ch


def _rand_rho(rng, dim):
    a = rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))
    r = a @ a.conj().T
    return r / np.trace(r)


def _apply_kraus(rho, kraus):
    return sum(K @ rho @ K.conj().T for K in kraus)


@pytest.mark.parametrize("d", [3, 4])
def test_superop_1site_matches_matrix_products(d):
    rng = np.random.default_rng(1)
    rho = _rand_rho(rng, d)
    for kraus in (ch.kraus_leak(0.3, d), ch.kraus_dephasing(0.2, d), ch.kraus_decay(0.4, d),
                  [ch.u_x(0.7, d)]):
        S = ch.superop_1site(kraus)
        got = ch.unvec(S @ ch.vec(rho), d)
        np.testing.assert_allclose(got, _apply_kraus(rho, kraus), atol=1e-14)


@pytest.mark.parametrize("d", [3, 4])
def test_superop_2site_matches_matrix_products(d):
    rng = np.random.default_rng(2)
    # a product of two single-atom states, written in the (eta_i, eta_{i+1}) basis
    r1, r2 = _rand_rho(rng, d), _rand_rho(rng, d)
    rho12 = np.kron(r1, r2)
    kraus = ch.gate_kraus_2site(0.9, 0.25, d)
    S = ch.superop_2site(kraus, d)
    v = np.kron(ch.vec(r1), ch.vec(r2))
    out = (S @ v).reshape(d, d, d, d)               # [a, a', b, b']
    want = _apply_kraus(rho12, kraus).reshape(d, d, d, d)   # [a, b, a', b']
    np.testing.assert_allclose(out, want.transpose(0, 2, 1, 3), atol=1e-14)
    # a correlated (entangled) two-atom input as well
    psi = rng.standard_normal(d * d) + 1j * rng.standard_normal(d * d)
    psi /= np.linalg.norm(psi)
    rho = np.outer(psi, psi.conj())
    v = rho.reshape(d, d, d, d).transpose(0, 2, 1, 3).reshape(-1)
    out = (S @ v).reshape(d, d, d, d).transpose(0, 2, 1, 3).reshape(d * d, d * d)
    np.testing.assert_allclose(out, _apply_kraus(rho, kraus), atol=1e-14)


@pytest.mark.parametrize("d", [3, 4])
def test_kraus_sets_are_trace_preserving(d):
    sets = [ch.kraus_leak(1e-3, d), ch.kraus_dephasing(0.3, d), ch.kraus_decay(0.2, d),
            ch.gate_kraus_2site(1.3, 0.01, d)]
    for ks in sets:
        dim = ks[0].shape[0]
        np.testing.assert_allclose(sum(K.conj().T @ K for K in ks), np.eye(dim), atol=1e-14)
    # trace preservation in the vectorised picture: vec(I)^T S = vec(I)^T
    vI = ch.vec(np.eye(d))
    S = ch.superop_1site(ch.kraus_decay(0.2, d))
    np.testing.assert_allclose(vI @ S, vI, atol=1e-14)


@pytest.mark.parametrize("d", [3, 4])
def test_single_atom_closed_forms(d):
    rng = np.random.default_rng(3)
    rho = _rand_rho(rng, d)
    p = 0.137
    # dephasing: rho_01 -> (1-2p) rho_01, populations unchanged, qubit/non-qubit
    # coherences scaled by sqrt(1-p)
    out = _apply_kraus(rho, ch.kraus_dephasing(p, d))
    assert abs(out[0, 1] - (1 - 2 * p) * rho[0, 1]) < 1e-14
    np.testing.assert_allclose(np.diag(out), np.diag(rho), atol=1e-14)
    assert abs(out[0, 2] - math.sqrt(1 - p) * rho[0, 2]) < 1e-14
    # decay: P_r -> (1-p) P_r, P_j += p b_j P_r
    out = _apply_kraus(rho, ch.kraus_decay(p, d))
    assert abs(out[2, 2] - (1 - p) * rho[2, 2]) < 1e-14
    if d == 3:
        assert abs(out[1, 1] - (rho[1, 1] + p * rho[2, 2])) < 1e-14
        assert abs(out[0, 0] - rho[0, 0]) < 1e-14
    else:
        for j, b in zip((0, 1, 3), (1 / 16, 1 / 16, 7 / 8)):
            assert abs(out[j, j] - (rho[j, j] + p * b * rho[2, 2])) < 1e-14
    # leak: P_1 -> (1-p) P_1, P_r += p P_1
    out = _apply_kraus(rho, ch.kraus_leak(p, d))
    assert abs(out[1, 1] - (1 - p) * rho[1, 1]) < 1e-14
    assert abs(out[2, 2] - (rho[2, 2] + p * rho[1, 1])) < 1e-14
    assert abs(out[0, 0] - rho[0, 0]) < 1e-14


@pytest.mark.parametrize("d", [3, 4])
def test_rotations_closed_forms(d):
    beta, gamma = 0.61, 1.17
    zero = np.zeros((d, d), complex)
    zero[0, 0] = 1
    out = _apply_kraus(zero, [ch.u_x(beta, d)])
    assert abs(out[1, 1] - math.sin(beta) ** 2) < 1e-14
    plus = ch.plus_state(d)
    np.testing.assert_allclose(_apply_kraus(plus, [ch.u_x(beta, d)]), plus, atol=1e-14)
    U = ch.u_zz(gamma, d)
    z = [1, -1] + [0] * (d - 2)
    want = np.diag([np.exp(-1j * gamma * z[a] * z[b]) for a in range(d) for b in range(d)])
    np.testing.assert_allclose(U, want, atol=1e-14)
