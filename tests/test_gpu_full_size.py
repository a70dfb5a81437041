"""GPU parity at the full-size workload of the benchmark: noisy QAOA, N=100 atoms, d=4,
chi_max=512, p=3, rates 1e-3, seed 0, through the C ABI, against the CPU oracle's values
stored in tests/golden/m3_seed0_oracle.json (written by tests/golden/make_m3_oracle.py,
which calls only oracle/; the oracle needs ~4 min for this circuit).

Tolerances: FP64 1e-10 relative on per-site energy, success probability and trace, 1e-10
absolute on every population; FP32-MFMA 1e-5 absolute on per-site energy and populations.
"""
import json
import os

import numpy as np
import pytest

from workloads import config_m3

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "m3_seed0_oracle.json")


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08572_amd import circuits, mpdo
    mpdo.load_library()
    return circuits, mpdo


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_m3_fp64_matches_stored_oracle():
    circuits, mpdo = _gpu()
    o = _golden()
    spec = config_m3(0)
    print("[gpu] M3 N=100 chi=512 p=3 fp64", flush=True)
    m = circuits.run_circuit(spec)
    g = circuits.observables(m)
    e_ref = o["energy_per_site"]
    assert abs(g["energy_per_site"] - e_ref) <= 1e-10 * max(1.0, abs(e_ref))
    np.testing.assert_allclose(g["populations"], np.array(o["populations"]), rtol=0, atol=1e-10)
    assert abs(g["p_success"] - o["p_success"]) <= 1e-10
    tr_ref = complex(*o["trace"])
    assert abs(g["trace"] - tr_ref) <= 1e-10 * abs(tr_ref)
    diff = [a - b for a, b in zip(m.bond_dims(), o["bond_dims"])]
    assert max(abs(x) for x in diff) <= 1 and sum(abs(x) for x in diff) <= 4, (m.bond_dims(), o["bond_dims"])


def test_m3_fp32_within_1e5_of_stored_oracle():
    circuits, mpdo = _gpu()
    o = _golden()
    spec = config_m3(0)
    print("[gpu] M3 N=100 chi=512 p=3 fp32", flush=True)
    m = circuits.run_circuit(spec, precision=mpdo.MPDO_FP32)
    g = circuits.observables(m)
    de = abs(g["energy_per_site"] - o["energy_per_site"])
    dp = float(np.max(np.abs(g["populations"] - np.array(o["populations"]))))
    print(f"[gpu] fp32 energy err {de:.2e} population err {dp:.2e}", flush=True)
    assert de <= 1e-5
    assert dp <= 1e-5


def test_m3_purity_by_swap_transfer_matches_oracle_norm():
    """Purity at the full-size workload: the GPU's doubled transfer matrix with the swap
    operator against the oracle's vectorised 2-norm ||vec rho||^2 / tr(rho)^2 (two different
    formulas of tr(rho^2) for Hermitian rho), FP64 1e-10 relative."""
    circuits, mpdo = _gpu()
    o = _golden()
    spec = config_m3(0)
    print("[gpu] M3 purity", flush=True)
    m = circuits.run_circuit(spec)
    p = circuits.purity(m)
    assert abs(p - o["purity"]) <= 1e-10 * o["purity"]


# Deeper circuit: N=8, p=4, chi_max=512, rates 1e-3, seed 0.  Its centre bond grows to 311 and
# the split's Gram matrices reach orders 512..1024, where the tridiagonal solver takes over from
# the small-order paths; values stored by `make_m3_oracle.py deep` (oracle only, ~4 min).
GOLDEN_DEEP = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "qaoa_n8_p4_chi512_seed0_oracle.json")


def test_deep_fp64_and_fp32_match_stored_oracle():
    circuits, mpdo = _gpu()
    with open(GOLDEN_DEEP) as f:
        o = json.load(f)
    spec = config_m3(0, n=8, p=4)
    print("[gpu] N=8 chi=512 p=4 fp64", flush=True)
    m = circuits.run_circuit(spec)
    g = circuits.observables(m)
    assert abs(g["energy_per_site"] - o["energy_per_site"]) <= 1e-10 * max(1.0, abs(o["energy_per_site"]))
    np.testing.assert_allclose(g["populations"], np.array(o["populations"]), rtol=0, atol=1e-10)
    assert abs(g["p_success"] - o["p_success"]) <= 1e-10
    tr_ref = complex(*o["trace"])
    assert abs(g["trace"] - tr_ref) <= 1e-10 * abs(tr_ref)
    assert abs(circuits.purity(m) - o["purity"]) <= 1e-10 * o["purity"]
    diff = [a - b for a, b in zip(m.bond_dims(), o["bond_dims"])]
    assert max(abs(x) for x in diff) <= 1, (m.bond_dims(), o["bond_dims"])
    m.close()
    print("[gpu] N=8 chi=512 p=4 fp32", flush=True)
    m = circuits.run_circuit(spec, precision=mpdo.MPDO_FP32)
    g = circuits.observables(m)
    de = abs(g["energy_per_site"] - o["energy_per_site"])
    dp = float(np.max(np.abs(g["populations"] - np.array(o["populations"]))))
    print(f"[gpu] fp32 |dE/N| = {de:.2e}, max |d pop| = {dp:.2e}", flush=True)
    assert de <= 1e-5 and dp <= 1e-5
    m.close()
