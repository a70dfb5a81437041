"""GPU tests of the subspace-iteration range basis, the split used where the exact range basis
would need an eigenproblem above the tridiagonal solver's limit (the saturated chi = 512 regime).

The environment variable MPDO_SUBSPACE_MIN_ORDER lowers the order at which the library switches
to it, so it can be checked where the exact path also works:

* where theta's rank bound (r chi_mid <= 756 in this circuit) is within the subspace width
  chi + 256, one pass from a random block spans range(theta), so the circuit must match the
  stored FP64 oracle values to the usual 1e-10;
* on a truncating circuit (chi = 64, width 320 below rank bounds up to 576) the block is
  iterated until the captured weight changes by less than 1e-12 of itself; observables must
  agree with the exact split to 1e-8, far below the truncation error of that circuit.
"""
import json
import os

import numpy as np
import pytest

from workloads import config_m3

pytestmark = pytest.mark.gpu

GOLDEN_DEEP = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "qaoa_n8_p4_chi512_seed0_oracle.json")


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08572_amd import circuits, mpdo
    mpdo.load_library()
    return circuits, mpdo


def test_forced_subspace_path_matches_stored_oracle(monkeypatch):
    circuits, mpdo = _gpu()
    with open(GOLDEN_DEEP) as f:
        o = json.load(f)
    monkeypatch.setenv("MPDO_SUBSPACE_MIN_ORDER", "200")
    print("[gpu] N=8 chi=512 p=4 fp64, subspace path above order 200", flush=True)
    m = circuits.run_circuit(config_m3(0, n=8, p=4))
    g = circuits.observables(m)
    print(f"[gpu] |dE/N| = {abs(g['energy_per_site'] - o['energy_per_site']):.2e}", flush=True)
    assert abs(g["energy_per_site"] - o["energy_per_site"]) <= 1e-10 * max(1.0, abs(o["energy_per_site"]))
    np.testing.assert_allclose(g["populations"], np.array(o["populations"]), rtol=0, atol=1e-10)
    assert abs(g["p_success"] - o["p_success"]) <= 1e-10
    assert abs(circuits.purity(m) - o["purity"]) <= 1e-10 * o["purity"]
    diff = [a - b for a, b in zip(m.bond_dims(), o["bond_dims"])]
    assert max(abs(x) for x in diff) <= 1, (m.bond_dims(), o["bond_dims"])
    m.close()


def test_subspace_path_on_a_truncating_circuit_agrees_with_exact_split(monkeypatch):
    circuits, mpdo = _gpu()
    spec = config_m3(0, n=8, p=4, chi=64)
    print("[gpu] N=8 chi=64 p=4 fp64, exact split", flush=True)
    m = circuits.run_circuit(spec)
    ref = circuits.observables(m)
    ref_purity = circuits.purity(m)
    m.close()
    monkeypatch.setenv("MPDO_SUBSPACE_MIN_ORDER", "100")
    print("[gpu] N=8 chi=64 p=4 fp64, subspace path above order 100", flush=True)
    m = circuits.run_circuit(spec)
    g = circuits.observables(m)
    de = abs(g["energy_per_site"] - ref["energy_per_site"])
    dp = float(np.max(np.abs(g["populations"] - ref["populations"])))
    dpur = abs(circuits.purity(m) - ref_purity)
    print(f"[gpu] subspace vs exact: |dE/N| {de:.2e}, max |d pop| {dp:.2e}, |d purity| {dpur:.2e}", flush=True)
    assert de <= 1e-8 and dp <= 1e-8 and dpur <= 1e-8
    assert max(m.bond_dims()) == 64
    m.close()


def _compare_cut_logs(gpu_infos, oracle_log, chi, rel=1e-10):
    """Per-update, gauge-invariant quantities of the cut against the oracle's log: tr(rho) and
    xi = tr(rho^2)/tr(rho)^2 of the whole merged tensor before the cut (what PPT reads,
    Eq. (xiformula)), the kept count (equal where chi makes the cut; elsewhere it may differ by
    a value sitting at the 1e-14 relative cutoff), the discarded weight, the trace after PPT."""
    assert len(gpu_infos) == len(oracle_log)
    worst = 0.0
    for g, o in zip(gpu_infos, oracle_log):
        assert g["bond"] == o["bond"]
        assert abs(g["kept"] - o["kept"]) <= (0 if o["kept"] == chi else 1), (g["bond"], g["kept"], o["kept"])
        for k in ("trace_before", "xi_before", "trace_after"):
            err = abs(g[k] - o[k]) / abs(o[k])
            worst = max(worst, err)
            assert err <= rel, (k, g["bond"], g[k], o[k])
        assert abs(g["discarded_weight"] - o["discarded_weight"]) <= rel
    return worst


def test_forced_subspace_truncating_circuit_matches_oracle(monkeypatch):
    """The subspace split, forced on (above order 100), on a circuit that cuts at chi = 64 while
    the subspace block (64 + 256 = 320) stays below theta's rank (up to 576), so the block is
    iterated: every update's trace, xi and discarded weight (which PPT computes from the whole
    theta, not from the part the block captured) and the final observables must match the CPU
    oracle (LAPACK SVD) to 1e-10."""
    circuits, mpdo = _gpu()
    from oracle import mpo
    spec = config_m3(0, n=8, p=4, chi=64)
    print("[gpu] N=8 chi=64 p=4 fp64, subspace path above order 100, against the oracle", flush=True)
    ref = mpo.run_spec(spec)
    o = mpo.observables(ref)
    monkeypatch.setenv("MPDO_SUBSPACE_MIN_ORDER", "100")
    infos = []
    m = circuits.run_circuit(spec, infos=infos)
    g = circuits.observables(m)
    worst = _compare_cut_logs(infos, ref.log, spec.chi)
    cut = [x for x in ref.log if x["discarded_weight"] > 0]
    de = abs(g["energy_per_site"] - o["energy_per_site"])
    print(f"[gpu] {len(cut)} cuts; worst per-update rel err {worst:.2e}; |dE/N| {de:.2e}", flush=True)
    assert len(cut) >= 5
    assert de <= 1e-10 * max(1.0, abs(o["energy_per_site"]))
    np.testing.assert_allclose(g["populations"], o["populations"], rtol=0, atol=1e-10)
    assert abs(g["p_success"] - o["p_success"]) <= 1e-10
    assert abs(circuits.purity(m) - o["purity"]) <= 1e-10 * o["purity"]
    assert max(abs(a - b) for a, b in zip(m.bond_dims(), ref.bond_dims())) <= 1
    m.close()
