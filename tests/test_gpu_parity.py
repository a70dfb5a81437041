"""GPU parity: libmpdo (through its C ABI) against the CPU oracle on the same seeded inputs.

Tolerances (stated with each test): FP64 mode 1e-10 relative on the per-site energy,
populations, success probability and trace (the bar for the double-precision path); the
FP32-MFMA mode 1e-5 absolute on the per-site energy and populations.
"""
import math

import numpy as np
import pytest

from workloads import config_m0, config_m1, noiseless_spec, random_spec

pytestmark = pytest.mark.gpu

FP64_REL = 1e-10
FP32_ABS = 1e-5


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08572_amd import circuits, mpdo
    mpdo.load_library()
    return circuits, mpdo


def _oracle_obs(spec, chi=None):
    from oracle import mpo
    m = mpo.run_spec(spec, chi=chi)
    return mpo.observables(m), m


def _check_fp64(o, g, label):
    scale = max(1.0, abs(o["energy_per_site"]))
    assert abs(g["energy_per_site"] - o["energy_per_site"]) <= FP64_REL * scale, label
    np.testing.assert_allclose(g["populations"], o["populations"], rtol=0, atol=FP64_REL, err_msg=label)
    assert abs(g["p_success"] - o["p_success"]) <= FP64_REL * max(1.0, o["p_success"]), label
    assert abs(g["trace"] - o["trace"]) <= FP64_REL * abs(o["trace"]), label


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_m0_exact_against_dense_and_mpo(seed):
    circuits, mpdo = _gpu()
    from oracle import dense
    spec = config_m0(seed)
    print(f"[gpu] m0 seed={seed}", flush=True)
    od = dense.observables(dense.run_spec(spec))
    m = circuits.run_circuit(spec)
    g = circuits.observables(m)
    _check_fp64(od, g, f"m0 seed {seed} vs dense")
    om, _ = _oracle_obs(spec)
    _check_fp64(om, g, f"m0 seed {seed} vs mpo")


@pytest.mark.parametrize("seed", [0, 1])
def test_m1_shape_fp64(seed):
    circuits, mpdo = _gpu()
    spec = config_m1(seed, n=16)
    print(f"[gpu] m1(n=16) seed={seed}", flush=True)
    o, ref = _oracle_obs(spec)
    infos = []
    m = circuits.run_circuit(spec, infos=infos)
    g = circuits.observables(m)
    _check_fp64(o, g, f"m1 seed {seed}")
    # counts may differ by a Schmidt value sitting at the 1e-14 relative cutoff
    assert all(abs(a - b) <= 1 for a, b in zip(m.bond_dims(), ref.bond_dims()))
    assert sum(abs(a - b) for a, b in zip(m.bond_dims(), ref.bond_dims())) <= 2


@pytest.mark.parametrize("seed", [8, 9])
def test_truncating_fp64(seed):
    circuits, mpdo = _gpu()
    spec = random_spec(seed=seed, n=8, d=4, p=3, chi=64, rate_lo=1e-3, rate_hi=1e-2)
    print(f"[gpu] truncating seed={seed}", flush=True)
    o, ref = _oracle_obs(spec)
    infos = []
    m = circuits.run_circuit(spec, infos=infos)
    g = circuits.observables(m)
    # the cut is well separated in these cases (gap >= 4e-6 sigma_1); see the oracle log
    _check_fp64(o, g, f"truncating seed {seed}")
    for x in infos:
        if x["kept"] < x["chi_l"] * 16 and x["ppt_feasible"] and x["discarded_weight"] > 0:
            assert abs(x["xi_after"] - x["xi_before"]) <= 1e-9 * abs(x["xi_before"])


@pytest.mark.parametrize("seed", [0, 1])
def test_m1_shape_fp32(seed):
    circuits, mpdo = _gpu()
    spec = config_m1(seed, n=16)
    print(f"[gpu] m1(n=16) fp32 seed={seed}", flush=True)
    o, _ = _oracle_obs(spec)
    m = circuits.run_circuit(spec, precision=mpdo.MPDO_FP32)
    g = circuits.observables(m)
    de = abs(g["energy_per_site"] - o["energy_per_site"])
    dp = float(np.max(np.abs(g["populations"] - o["populations"])))
    print(f"[gpu] fp32 energy err {de:.2e} population err {dp:.2e}", flush=True)
    assert de <= FP32_ABS
    assert dp <= FP32_ABS


def test_single_atom_closed_forms():
    circuits, mpdo = _gpu()
    d, p = 4, 0.137
    m = mpdo.MPDO(3, d, 8)
    rho = np.zeros((d, d), complex)
    rho[1, 1] = 0.6
    rho[2, 2] = 0.3
    rho[0, 0] = 0.1
    rho[0, 1] = rho[1, 0] = 0.2
    m.init_product_state([rho] * 3)
    m.apply_channel(0, circuits.dephasing_kraus(p, d))
    m.apply_channel(1, circuits.decay_kraus(p, d))
    m.apply_channel(2, circuits.leak_kraus(p, d))
    P = [np.diag(np.eye(d)[a]).astype(complex) for a in range(d)]
    coh = np.zeros((d, d), complex)
    coh[1, 0] = 1.0   # tr(rho |1><0|) = rho_01
    vals = m.expect([(0, [coh])] + [(j, [P[a]]) for j in range(3) for a in range(d)])
    assert abs(vals[0] - (1 - 2 * p) * 0.2) < 1e-14
    pops = vals[1:].real.reshape(3, d)
    np.testing.assert_allclose(pops[0], [0.1, 0.6, 0.3, 0.0], atol=1e-14)
    b = (1 / 16, 1 / 16, 7 / 8)
    np.testing.assert_allclose(pops[1], [0.1 + p * b[0] * 0.3, 0.6 + p * b[1] * 0.3, (1 - p) * 0.3,
                                         p * b[2] * 0.3], atol=1e-14)
    np.testing.assert_allclose(pops[2], [0.1, (1 - p) * 0.6, 0.3 + p * 0.6, 0.0], atol=1e-14)


def test_noiseless_light_cone_n100():
    circuits, mpdo = _gpu()
    gamma, beta, n = 0.83, 1.91, 100
    spec = noiseless_spec(n, 4, (gamma,), (beta,), chi=64)
    print("[gpu] light cone n=100", flush=True)
    m = circuits.run_circuit(spec)
    assert max(m.bond_dims()) <= 9
    X = np.zeros((4, 4), complex)
    X[0, 1] = X[1, 0] = 1
    Z = np.diag([1, -1, 0, 0]).astype(complex)
    sites = [0, 1, 50, 98, 99]
    vx = m.expect([(j, [X]) for j in sites]).real
    c2, s2, s4b = math.cos(2 * gamma), math.sin(2 * gamma), math.sin(4 * beta)
    for j, v in zip(sites, vx):
        assert abs(v - (c2 if j in (0, n - 1) else c2 * c2)) < 1e-12
    bonds = [0, 1, 49, 98]
    vzz = m.expect([(j, [Z, Z]) for j in bonds]).real
    for j, v in zip(bonds, vzz):
        want = 0.5 * s4b * s2 * (1 + c2) if j in (0, n - 2) else s4b * s2 * c2
        assert abs(v - want) < 1e-12


def test_truncate_entry_point_against_oracle():
    circuits, mpdo = _gpu()
    from oracle import channels as ch
    from oracle import mpo
    n = 6
    spec = random_spec(seed=21, n=n, d=4, p=2, chi=256, rate_lo=1e-3, rate_hi=1e-2)
    print("[gpu] truncate entry point", flush=True)
    ops = ch.circuit_ops(spec)
    main, tail = ops[:-3 * n], ops[-3 * n:]
    ref = mpo.MPO([ch.plus_state(4)] * n, chi=256)
    ref.run(main)
    assert max(ref.bond_dims()) > 6
    # on the GPU the last layer's single-atom maps are queued; the cut of bond (2,3) folds
    # in those of atoms 2 and 3 only, so the oracle applies exactly those before its cut
    ref.run([op for op in tail if op[1] in (2, 3)])
    ref.apply_2site(2, np.eye(256, dtype=complex), chi=6)
    ref.run([op for op in tail if op[1] not in (2, 3)])
    m = circuits.run_circuit(spec)
    info = m.truncate(2, 6)
    assert info["kept"] == 6
    _check_fp64(mpo.observables(ref), circuits.observables(m), "truncate")
    assert abs(info["xi_after"] - info["xi_before"]) <= 1e-9 * abs(info["xi_before"])


def test_bad_arguments_raise():
    circuits, mpdo = _gpu()
    m = mpdo.MPDO(4, 4, 16)
    m.init_product_state([circuits.plus_rho(4)] * 4)
    with pytest.raises(mpdo.MpdoError):
        m.apply_gate_kraus(3, circuits.block_kraus(0.3, 0.0, 4))   # bond out of range
    with pytest.raises(mpdo.MpdoError):
        m.apply_channel(0, [2.0 * np.eye(4)])                       # not trace preserving
    with pytest.raises(mpdo.MpdoError):
        m.truncate(0, 17)                                           # chi above chi_max
    # the context is still usable
    m.apply_gate_kraus(0, circuits.block_kraus(0.3, 0.01, 4))
    assert abs(m.trace() - 1.0) < 1e-13


def test_gemm_autotuner_gives_the_same_circuit(monkeypatch):
    """With the k-split autotuner on (MPDO_GEMM_AUTOTUNE=1) every product is still computed by
    the same kernel, only split differently over k: the N=16 circuit must agree with the
    untuned run to the FP64 bar (rounding of the split sums only)."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08572_amd import circuits
    from workloads.qaoa import config_m1
    spec = config_m1(0, n=16)
    print("[gpu] M1-shaped N=16, GEMM autotuner off / on", flush=True)
    ref = circuits.observables(circuits.run_circuit(spec))
    monkeypatch.setenv("MPDO_GEMM_AUTOTUNE", "1")
    got = circuits.observables(circuits.run_circuit(spec))
    assert abs(got["energy_per_site"] - ref["energy_per_site"]) <= 1e-10 * max(1.0, abs(ref["energy_per_site"]))
    np.testing.assert_allclose(got["populations"], ref["populations"], rtol=0, atol=1e-10)


def test_repeated_runs_agree_to_rounding():
    """Products whose k range is split add their partial tiles in a fixed order (no atomics), so
    run-to-run differences come only from the tridiagonal reduction's on-chip accumulation (LDS
    atomics of the matrix-vector products, whose order varies): the same truncating circuit,
    run three times and four more times as a batch on four streams, must agree to 1e-13."""
    circuits, mpdo = _gpu()
    spec = random_spec(seed=8, n=8, d=4, p=3, chi=64, rate_lo=1e-3, rate_hi=1e-2)
    print("[gpu] truncating N=8 p=3 chi=64, three runs and a batch of four", flush=True)
    runs = []
    for _ in range(3):
        m = circuits.run_circuit(spec)
        runs.append((circuits.observables(m), m.bond_dims()))
        m.close()
    for r in mpdo.run_batch([circuits.describe(spec)] * 4, n_workers=4):
        runs.append((circuits.summarize(r["values"], spec.n, spec.d), r["bonds"]))
    ref, bonds = runs[0]
    for g, b in runs[1:]:
        assert b == bonds
        assert abs(g["energy_per_site"] - ref["energy_per_site"]) <= 1e-13
        assert float(np.max(np.abs(g["populations"] - ref["populations"]))) <= 1e-13
