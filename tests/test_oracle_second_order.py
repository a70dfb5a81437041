"""Pins of the second-order oracle (oracle/second_order.py) against what fixes it independently:
the dense definitions, closed forms for product states, identities of pure states, the
vectorised-norm purity of the MPO oracle, and the inequality between collision probability
and purity."""
import math

import numpy as np
import pytest

from oracle import channels as ch
from oracle import dense, mpo, second_order as so
from workloads import config_m0, random_spec, noiseless_spec


def _rand_rho(rng, d):
    g = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    r = g @ g.conj().T
    return r / np.trace(r)


def test_product_state_closed_forms():
    rng = np.random.default_rng(3)
    d, n = 3, 4
    rhos = [_rand_rho(rng, d) for _ in range(n)]
    m = mpo.MPO(rhos, chi=8)
    pur = np.prod([np.real(np.trace(r @ r)) for r in rhos])
    col = np.prod([np.sum(np.real(np.diag(r)) ** 2) for r in rhos])
    assert abs(so.mpo_purity(m) - pur) < 1e-13
    assert abs(so.mpo_collision(m) - col) < 1e-13
    # single-atom Renyi-2 entropy and zero mutual information for a product state
    assert abs(so.mpo_renyi2(m, [2]) + math.log(np.real(np.trace(rhos[2] @ rhos[2])))) < 1e-12
    assert abs(so.mpo_mutual_info(m, [0], [3])) < 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_mpo_route_equals_dense_definitions(seed):
    spec = config_m0(seed)
    dm = dense.run_spec(spec)
    m = mpo.run_spec(spec)
    n, d = spec.n, spec.d
    assert abs(so.mpo_purity(m) - so.dense_purity(dm.rho)) < 1e-12
    assert abs(so.mpo_collision(m) - so.dense_collision(dm.rho)) < 1e-12
    for sites in ([1], [1, 4], [0, 2, 3]):
        assert abs(so.mpo_renyi2(m, sites) - so.dense_renyi2(dm.rho, n, d, sites)) < 1e-10
    assert abs(so.mpo_mutual_info(m, [1], [4]) - so.dense_mutual_info(dm.rho, n, d, [1], [4])) < 1e-10


def test_swap_purity_equals_vectorised_norm():
    """tr(rho^2) by the swap operator equals ||vec rho||^2 (rho Hermitian), two different formulas."""
    spec = random_spec(seed=4, n=7, d=4, p=2, chi=200, rate_lo=1e-3, rate_hi=1e-2)
    m = mpo.run_spec(spec)
    tr = m.trace()
    assert abs(so.mpo_purity(m) - m.purity() / np.real(tr) ** 2) < 1e-12


def test_pure_state_identities():
    """Noiseless circuit: purity 1, S2 of a block equals S2 of its complement, and for
    complementary A, B the mutual information is 2 S2(A)."""
    spec = noiseless_spec(n=6, d=3, gamma=[0.83, 0.41], beta=[1.91, 0.57], chi=729)
    m = mpo.run_spec(spec)
    assert abs(so.mpo_purity(m) - 1.0) < 1e-12
    a, b = [0, 1], [2, 3, 4, 5]
    assert abs(so.mpo_renyi2(m, a) - so.mpo_renyi2(m, b)) < 1e-10
    assert abs(so.mpo_mutual_info(m, a, b) - 2 * so.mpo_renyi2(m, a)) < 1e-10
    assert so.mpo_renyi2(m, a) > 1e-3   # the circuit does entangle


def test_collision_at_most_purity_and_planted_error_caught():
    spec = random_spec(seed=6, n=5, d=3, p=2, chi=100, rate_lo=1e-3, rate_hi=1e-2)
    dm = dense.run_spec(spec)
    m = mpo.run_spec(spec)
    assert so.mpo_collision(m) <= so.mpo_purity(m) + 1e-14
    # planted slip: pairing (s, s') with (s, s') instead of (s', s) gives tr(rho rho^T), which
    # differs from the purity once rho has complex coherences; the dense check must see it
    D2 = spec.d * spec.d
    bad = {j: np.eye(D2, dtype=np.complex128) for j in range(spec.n)}
    val = np.real(so.mpo_expect2(m, bad) / m.trace() ** 2)
    assert abs(val - so.dense_purity(dm.rho)) > 1e-6
