"""GPU parity of the second-order observables (mpdo_expect2, through the C ABI): purity,
collision probability, second Renyi entropies and Renyi-2 mutual information against the
dense oracle (exact regime) and the MPO oracle (truncating regime), and closed forms for a
product state with queued channels.

Tolerances: FP64 1e-10 relative on purity and collision probability, 1e-9 absolute on S2
and I2 (logarithms of quantities held to 1e-10 relative).
"""
import math

import numpy as np
import pytest

from workloads import config_m0, random_spec

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08572_amd import circuits, mpdo
    mpdo.load_library()
    return circuits, mpdo


@pytest.mark.parametrize("seed", [0, 1])
def test_second_order_exact_regime_against_dense(seed):
    circuits, mpdo = _gpu()
    from oracle import dense, second_order as so
    spec = config_m0(seed)
    print(f"[gpu] second order m0 seed={seed}", flush=True)
    rho = dense.run_spec(spec).rho
    m = circuits.run_circuit(spec)   # the last layer's single-atom maps stay queued
    n, d = spec.n, spec.d
    p_ref = so.dense_purity(rho)
    assert abs(circuits.purity(m) - p_ref) <= 1e-10 * p_ref
    z_ref = so.dense_collision(rho)
    assert abs(circuits.collision_probability(m) - z_ref) <= 1e-10 * z_ref
    for sites in ([1], [1, 4], [0, 2, 3], [5]):
        assert abs(circuits.renyi2(m, sites) - so.dense_renyi2(rho, n, d, sites)) <= 1e-9, sites
    i_ref = so.dense_mutual_info(rho, n, d, [1], [4])
    assert abs(circuits.renyi2_mutual_information(m, [1], [4]) - i_ref) <= 1e-9


@pytest.mark.parametrize("seed", [8, 9])
def test_second_order_truncating_against_mpo_oracle(seed):
    circuits, mpdo = _gpu()
    from oracle import mpo, second_order as so
    spec = random_spec(seed=seed, n=8, d=4, p=3, chi=64, rate_lo=1e-3, rate_hi=1e-2)
    print(f"[gpu] second order truncating seed={seed}", flush=True)
    ref = mpo.run_spec(spec)
    m = circuits.run_circuit(spec)
    p_ref = so.mpo_purity(ref)
    assert abs(circuits.purity(m) - p_ref) <= 1e-10 * p_ref
    z_ref = so.mpo_collision(ref)
    assert abs(circuits.collision_probability(m) - z_ref) <= 1e-10 * z_ref
    assert abs(circuits.renyi2(m, [2, 3]) - so.mpo_renyi2(ref, [2, 3])) <= 1e-9
    assert abs(circuits.renyi2_mutual_information(m, [1], [4]) - so.mpo_mutual_info(ref, [1], [4])) <= 1e-9


def test_product_state_with_queued_channels_closed_form():
    """|psi> product state, a queued dephasing on atom 1 and decay on atom 2: purity and
    collision probability factorise over atoms, and I2 vanishes."""
    circuits, mpdo = _gpu()
    d, n = 4, 5
    rng = np.random.default_rng(11)
    rhos = []
    for _ in range(n):
        g = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        r = g @ g.conj().T
        rhos.append(r / np.trace(r))
    m = mpdo.MPDO(n, d, 16)
    m.init_product_state(rhos)
    deph = circuits.dephasing_kraus(0.2, d)
    dec = circuits.decay_kraus(0.3, d)
    m.apply_channel(1, deph)
    m.apply_channel(2, dec)
    after = list(rhos)
    after[1] = sum(K @ rhos[1] @ K.conj().T for K in deph)
    after[2] = sum(K @ rhos[2] @ K.conj().T for K in dec)
    pur = float(np.prod([np.real(np.trace(r @ r)) for r in after]))
    col = float(np.prod([np.sum(np.real(np.diag(r)) ** 2) for r in after]))
    assert abs(circuits.purity(m) - pur) <= 1e-12
    assert abs(circuits.collision_probability(m) - col) <= 1e-12
    assert abs(circuits.renyi2(m, [2]) + math.log(np.real(np.trace(after[2] @ after[2])))) <= 1e-12
    assert abs(circuits.renyi2_mutual_information(m, [1], [2])) <= 1e-12


def test_expect2_rejects_bad_terms():
    circuits, mpdo = _gpu()
    m = mpdo.MPDO(4, 3, 9)
    m.init_product_state([circuits.plus_rho(3)] * 4)
    with pytest.raises(mpdo.MpdoError):
        m.expect2([(3, [circuits.swap_op(3)] * 2)])
    bad = circuits.swap_op(3).copy()
    bad[0, 0] = np.nan
    with pytest.raises(mpdo.MpdoError):
        m.expect2([(0, [bad])])
