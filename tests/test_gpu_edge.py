"""Degenerate shapes through the C ABI.

* The two-atom chain: one bond, both chain ends at the pair.  Noisy gate sequences (two-atom
  Kraus maps and queued single-atom channels) against the dense oracle, d = 2, 3, 4, with
  chi_max = d^2 so nothing is cut: the contracted density matrix must equal the exact one to
  1e-10 of max|rho|.
* The crosstalk gate on the two-atom chain: no neighbour exists, so the four-term form
  (Sec. II, crosstalk) reduces to its first pair gate (the chain-end reading); checked against
  the dense oracle.
* chi_max = 1: every cut keeps one Schmidt value and PPT acts on a single value (its
  parallel case, Lambda' parallel to T', where the rescaling is the identity).  Against the
  MPO oracle with the same chi on a four-atom chain, entrywise on the contracted density
  matrix to 1e-10.
"""
import numpy as np
import pytest

from oracle import channels, crosstalk, dense, mpo

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08572_amd import mpdo
    mpdo.load_library()
    return mpdo


def _unitary(rng, n):
    z = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _kraus2(rng, d):
    """a random two-atom channel: a unitary mixed with a dephased copy"""
    V = _unitary(rng, d * d)
    p = 0.2
    Z = np.diag(np.exp(2j * np.pi * np.arange(d) / d))
    return [np.sqrt(1 - p) * V, np.sqrt(p) * np.kron(Z, np.eye(d)) @ V]


def _kraus1(rng, d):
    """a random unitary followed by amplitude damping 1 -> 0"""
    V = _unitary(rng, d)
    g = 0.1
    K1 = np.zeros((d, d), dtype=np.complex128)
    K1[0, 1] = np.sqrt(g)
    K0 = np.eye(d, dtype=np.complex128)
    K0[1, 1] = np.sqrt(1 - g)
    return [K0 @ V, K1 @ V]


def _rho0(rng, d):
    z = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    r = z @ z.conj().T + 0.5 * np.eye(d)
    return r / np.trace(r)


def _dense_from_sites(m, n, d):
    v = np.ones((1, 1), dtype=np.complex128)
    for j in range(n):
        A = m.get_site(j)                      # cl x D2 x cr
        cl, D2, cr = A.shape
        v = (v @ A.reshape(cl, D2 * cr)).reshape(-1, cr)
    t = v.reshape((d, d) * n)                  # (sigma_0, sigma'_0, sigma_1, sigma'_1, ...)
    t = np.transpose(t, list(range(0, 2 * n, 2)) + list(range(1, 2 * n, 2)))
    return t.reshape(d ** n, d ** n)


@pytest.mark.parametrize("d", [2, 3, 4])
def test_two_atom_chain_matches_dense(d):
    mpdo = _gpu()
    rng = np.random.default_rng(30 + d)
    rhos = [_rho0(rng, d) for _ in range(2)]
    dm = dense.DenseRho(rhos)
    m = mpdo.MPDO(2, d, d * d, precision=mpdo.MPDO_FP64)
    m.init_product_state(rhos)
    print(f"[gpu] two-atom chain d={d} chi={d * d}", flush=True)
    for step in range(4):
        K = _kraus2(rng, d)
        dm.apply_kraus(K, (0, 1))
        m.apply_gate_kraus(0, K)
        K1 = _kraus1(rng, d)
        dm.apply_kraus(K1, (step % 2,))
        m.apply_channel(step % 2, K1)
    K = _kraus2(rng, d)
    dm.apply_kraus(K, (0, 1))
    m.apply_gate_kraus(0, K)
    got = _dense_from_sites(m, 2, d)
    err = np.abs(got - dm.rho).max() / np.abs(dm.rho).max()
    tr = m.trace()
    print(f"[gpu] max |rho - rho_oracle| / max|rho| = {err:.2e}, trace {tr:.15f}", flush=True)
    m.close()
    assert err <= 1e-10
    assert abs(tr - 1.0) <= 1e-10


def test_crosstalk_on_a_two_atom_chain_is_its_first_pair_gate():
    mpdo = _gpu()
    rng = np.random.default_rng(41)
    d, ryd = 3, 2
    rhos = [_rho0(rng, d) for _ in range(2)]
    dm = dense.DenseRho(rhos)
    m = mpdo.MPDO(2, d, d * d, precision=mpdo.MPDO_FP64)
    m.init_product_state(rhos)
    K = _kraus2(rng, d)
    dm.apply_kraus(K, (0, 1))
    m.apply_gate_kraus(0, K)
    u4 = [_unitary(rng, d * d) for _ in range(4)]
    print("[gpu] crosstalk gate on N=2 d=3", flush=True)
    plain = dense.DenseRho(rhos)
    plain.rho = dm.rho.copy()
    crosstalk.apply_crosstalk(dm, 0, u4, ryd)
    plain.apply_kraus([u4[0]], (0, 1))             # the pair gate with no detuning shift
    m.apply_gate_crosstalk(0, ryd, u4)
    got = _dense_from_sites(m, 2, d)
    err = np.abs(got - dm.rho).max() / np.abs(dm.rho).max()
    err_plain = np.abs(got - plain.rho).max() / np.abs(plain.rho).max()
    print(f"[gpu] max |rho - rho_oracle| / max|rho| = {err:.2e}, against u[0] alone {err_plain:.2e}", flush=True)
    m.close()
    assert err <= 1e-10 and err_plain <= 1e-10


def test_chi_one_matches_the_mpo_oracle():
    mpdo = _gpu()
    rng = np.random.default_rng(52)
    d, n, chi = 2, 4, 1
    rhos = [_rho0(rng, d) for _ in range(n)]
    om = mpo.MPO(rhos, chi=chi)
    m = mpdo.MPDO(n, d, chi, precision=mpdo.MPDO_FP64)
    m.init_product_state(rhos)
    print(f"[gpu] chi_max=1 N={n} d={d}", flush=True)
    infos = []
    for s_ in (0, 2, 1, 0, 2):
        K = _kraus2(rng, d)
        om.apply_2site(s_, channels.superop_2site(K, d))
        infos.append(m.apply_gate_kraus(s_, K, info=True))
    assert m.bond_dims() == [1, 1, 1] and om.bond_dims() == [1, 1, 1]
    assert all(i["kept"] == 1 for i in infos)
    assert max(i["discarded_weight"] for i in infos) > 1e-3   # the cuts are real
    got, ref = _dense_from_sites(m, n, d), om.to_dense()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"[gpu] max |rho - rho_oracle| / max|rho| = {err:.2e}, "
          f"discarded {[round(i['discarded_weight'], 4) for i in infos]}", flush=True)
    m.close()
    assert err <= 1e-10


def test_empty_expectation_lists_and_a_cut_that_removes_nothing():
    """No terms: empty results, no error.  mpdo_truncate to the bond's own dimension cuts only
    Schmidt values at the 1e-14 cutoff, and PPT is the identity when nothing is discarded, so
    the density matrix is unchanged to rounding."""
    mpdo = _gpu()
    rng = np.random.default_rng(61)
    d, n = 3, 5
    rhos = [_rho0(rng, d) for _ in range(n)]
    m = mpdo.MPDO(n, d, 81, precision=mpdo.MPDO_FP64)
    m.init_product_state(rhos)
    for s_ in (0, 2, 1, 3):
        m.apply_gate_kraus(s_, _kraus2(rng, d))
    print("[gpu] empty expect lists, no-op truncate N=5 d=3", flush=True)
    before = _dense_from_sites(m, n, d)
    assert m.expect([]).shape == (0,)
    assert m.expect2([]).shape == (0,)
    b = m.bond_dims()
    info = m.truncate(1, b[1])
    after = _dense_from_sites(m, n, d)
    err = np.abs(after - before).max() / np.abs(before).max()
    print(f"[gpu] bonds {b} -> {m.bond_dims()}, discarded {info['discarded_weight']:.1e}, change {err:.1e}",
          flush=True)
    bonds_after = m.bond_dims()
    m.close()
    assert bonds_after[1] <= b[1]
    # 1 - sum_kept Lambda^2 / |Lambda|^2: zero up to the rounding of the two sums
    assert info["discarded_weight"] <= 1e-14
    assert err <= 1e-12
