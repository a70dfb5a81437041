"""Pins of the dense and MPO oracles.

* dense rho vs the textbook checks: trace one, Hermitian, non-negative spectrum, and the
  pure-state limit against an independent qubit statevector;
* the MPO in the exact (non-truncating) regime against the dense rho (Sec. III.A);
* noiseless p=1 light-cone closed forms at N=100;
* gamma = beta = 0: every atom follows its own small Markov chain (closed form at N=100);
* Table II (Sec. IV) for the statevector conventions;
* truncating runs: PPT keeps xi at every feasible cut, and chi-doubling convergence.
"""
import math
import os

import numpy as np
import pytest

from oracle import channels as ch
from oracle import dense, mpo, statevector
from workloads import config_m0, noiseless_spec, random_spec

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#")


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dense_rho_is_a_state(seed):
    dm = dense.run_spec(config_m0(seed))
    rho = dm.rho
    assert abs(np.trace(rho) - 1.0) < 1e-13
    assert np.max(np.abs(rho - rho.conj().T)) < 1e-15
    ev = dm.eigvalsh()
    assert ev.min() > -1e-13
    # lambda_min >= -sqrt(tr rho^2 - lambda_max^2)  (Sec. III.E)
    assert ev.min() >= -math.sqrt(max(0.0, np.sum(ev ** 2) - ev.max() ** 2)) - 1e-15


def test_dense_pure_limit_matches_statevector():
    n, d = 5, 3
    gam, bet = (0.83, 0.4), (1.91, 0.2)
    dm = dense.run_spec(noiseless_spec(n, d, gam, bet, chi=1000))
    # statevector convention: exp(+i a H_zz) then exp(+i b sum X): a = -gamma, b = -beta
    psi = statevector.qaoa_state(n, [-g for g in gam], [-b for b in bet], b=0.0)
    # embed qubit amplitudes into d levels
    full = np.zeros((d,) * n, dtype=complex)
    idx = tuple([slice(0, 2)] * n)
    full[idx] = psi.reshape((2,) * n)
    full = full.reshape(-1)
    np.testing.assert_allclose(dm.rho, np.outer(full, full.conj()), atol=1e-13)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mpo_matches_dense_exact_regime_d3(seed):
    spec = config_m0(seed)
    dm = dense.run_spec(spec)
    m = mpo.run_spec(spec)
    np.testing.assert_allclose(m.to_dense(), dm.rho, atol=1e-13)
    od, om = dense.observables(dm), mpo.observables(m)
    assert abs(od["energy_per_site"] - om["energy_per_site"]) < 1e-13
    np.testing.assert_allclose(om["populations"], od["populations"], atol=1e-13)
    assert abs(od["purity"] - om["purity"]) < 1e-13
    assert abs(od["p_success"] - om["p_success"]) < 1e-13


def test_mpo_matches_dense_exact_regime_d4_two_layers():
    spec = random_spec(seed=11, n=5, d=4, p=2, chi=4096, rate_lo=1e-3, rate_hi=5e-2)
    dm = dense.run_spec(spec)
    m = mpo.run_spec(spec)
    assert max(x["discarded_weight"] for x in m.log) < 1e-24
    np.testing.assert_allclose(m.to_dense(), dm.rho, atol=1e-13)
    od, om = dense.observables(dm), mpo.observables(m)
    assert abs(od["energy_per_site"] - om["energy_per_site"]) < 1e-13
    np.testing.assert_allclose(om["populations"], od["populations"], atol=1e-13)


def test_mpo_centre_isometries_and_purity():
    spec = random_spec(seed=3, n=5, d=4, p=2, chi=4096)
    m = mpo.MPO([ch.plus_state(4)] * 5, chi=4096)
    m.run(ch.circuit_ops(spec))
    # bring the centre to bond (2,3): the left part is left-isometric, right part right-iso
    m.canonicalize(2)
    for j in range(2):
        a = m.A[j].reshape(-1, m.A[j].shape[2])
        np.testing.assert_allclose(a.conj().T @ a, np.eye(a.shape[1]), atol=1e-13)
    for j in range(4, 5):
        a = m.A[j].reshape(m.A[j].shape[0], -1)
        np.testing.assert_allclose(a @ a.conj().T, np.eye(a.shape[0]), atol=1e-13)
    # |Lambda|^2 = tr rho^2 at the centre (Sec. III.D): contract theta directly
    theta = np.tensordot(m.A[2], m.A[3], axes=(2, 0))
    assert abs(np.vdot(theta, theta).real - m.purity()) < 1e-13
    dm = dense.run_spec(spec)
    assert abs(m.purity() - dm.purity()) < 1e-13


def test_noiseless_p1_light_cone_n100():
    gamma, beta = 0.83, 1.91
    n = 100
    m = mpo.run_spec(noiseless_spec(n, 4, (gamma,), (beta,), chi=64))
    assert max(m.bond_dims()) <= 9
    X, Z = ch.x_ext(4), ch.z_ext(4)
    tr = m.trace().real
    assert abs(tr - 1.0) < 1e-12
    c2, s2 = math.cos(2 * gamma), math.sin(2 * gamma)
    for j in (0, 1, 50, 98, 99):
        want = c2 if j in (0, n - 1) else c2 * c2
        assert abs(m.expect_product({j: X}).real - want) < 1e-12
    s4b = math.sin(4 * beta)
    for j in (0, 1, 49, 98):
        got = m.expect_product({j: Z, j + 1: Z}).real
        if j in (0, n - 2):
            want = 0.5 * s4b * s2 * (1 + c2)
        else:
            want = s4b * s2 * c2
        assert abs(got - want) < 1e-12


def test_light_cone_formula_against_statevector():
    """The ZZ closed form used above, checked against an independent qubit statevector."""
    gamma, beta, n = 0.83, 1.91, 8
    psi = statevector.qaoa_state(n, [-gamma], [-beta], b=0.0)
    zz, xs = statevector.expect_zz_x(psi, n)
    c2, s2, s4b = math.cos(2 * gamma), math.sin(2 * gamma), math.sin(4 * beta)
    assert abs(zz[0] - 0.5 * s4b * s2 * (1 + c2)) < 1e-12
    assert abs(zz[3] - s4b * s2 * c2) < 1e-12
    assert abs(xs[0] - c2) < 1e-12 and abs(xs[4] - c2 * c2) < 1e-12


def _site_markov(n_gates, p_leak, p_deph, p_dec, layers):
    """Populations (0,1,r,lost) of one atom with gamma = beta = 0 (d = 4)."""
    P = np.array([0.5, 0.5, 0.0, 0.0])
    b0, b1, bd = 1 / 16, 1 / 16, 7 / 8
    for _ in range(layers):
        for _ in range(n_gates):
            P = np.array([P[0], (1 - p_leak) * P[1], P[2] + p_leak * P[1], P[3]])
        # dephasing leaves populations unchanged
        pr = P[2]
        P = np.array([P[0] + p_dec * b0 * pr, P[1] + p_dec * b1 * pr, (1 - p_dec) * pr,
                      P[3] + p_dec * bd * pr])
    return P


def test_markov_populations_n100():
    n, p = 100, 3
    spec = random_spec(seed=5, n=n, d=4, p=p, chi=16, rate_lo=1e-3, rate_hi=3e-2)
    spec = spec.__class__(**{**spec.as_dict(), "gamma": (0.0,) * p, "beta": (0.0,) * p})
    m = mpo.run_spec(spec)
    assert max(m.bond_dims()) == 1
    obs = mpo.observables(m)
    want_succ = 1.0
    for j in range(n):
        gates = 1 if j in (0, n - 1) else 2
        P = _site_markov(gates, spec.p_leak, spec.p_deph, spec.p_decay, p)
        np.testing.assert_allclose(obs["populations"][j], P, atol=1e-14)
        want_succ *= P[0] + P[1]
    assert abs(obs["p_success"] - want_succ) < 1e-13 * want_succ + 1e-300
    assert abs(obs["trace"] - 1.0) < 1e-13


def test_table2_energy_density_n20():
    params = _load("table1_qaoa_params.txt")
    table = _load("table2_qaoa_energy.txt")
    alphas, betas = params[:, 1], params[:, 2]
    psi = statevector.qaoa_state(20, alphas, betas, b=0.2)
    eps = statevector.tfim_energy(psi, 20, b=0.2, g=1.2) / 20
    row = table[table[:, 0] == 20][0]
    # printed to 5 decimals; unexplained residual ~1.2e-4 (parameter rounding)
    assert abs(eps - row[1]) < 2e-4
    # the QAOA state lies above the DMRG ground state
    assert eps > row[2]


def test_truncating_ppt_keeps_xi_and_converges():
    spec = random_spec(seed=8, n=8, d=4, p=3, chi=1000, rate_lo=1e-3, rate_hi=1e-2)
    ref = mpo.observables(mpo.run_spec(spec, chi=1000))
    errs = []
    for chi in (16, 32, 64):
        m = mpo.run_spec(spec, chi=chi)
        cut = [x for x in m.log if x["discarded_weight"] > 0]
        assert cut, "expected truncation at this chi"
        for x in cut:
            if x.get("ppt_feasible", True):
                assert abs(x["xi_after"] - x["xi_before"]) <= 1e-10 * abs(x["xi_before"])
        errs.append(abs(mpo.observables(m)["energy_per_site"] - ref["energy_per_site"]))
    assert errs[2] < errs[0]


def test_stored_full_size_oracle_values_are_consistent():
    """The cached oracle output for the N=100 chi=512 p=3 workload obeys what the maps fix:
    trace 1 (no value above the cut is dropped at these bonds, so tr rho is kept), populations of
    every atom sum to 1 and lie in [0, 1], and the all-qubit probability is at most the
    smallest single-atom qubit probability."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "m3_seed0_oracle.json")
    with open(path) as f:
        o = json.load(f)
    pops = np.array(o["populations"])
    assert pops.shape == (100, 4)
    assert abs(complex(*o["trace"]) - 1.0) < 1e-12
    np.testing.assert_allclose(pops.sum(axis=1), 1.0, atol=1e-12)
    assert pops.min() > -1e-12 and pops.max() < 1 + 1e-12
    assert o["p_success"] <= float(np.min(pops[:, 0] + pops[:, 1])) + 1e-12
    assert max(o["bond_dims"]) <= 512
