"""GPU property test of the saturated chi = 512 regime, where the oracle cannot follow (an
8192 x 8192 complex SVD per update) and the split runs by subspace iteration: a 16-atom chain
with the benchmark's gate set is run until its centre bonds are at 512, and properties that
hold at any size are checked on every update and on the final state:

* every update succeeds (the orthonormality check would fail one that lost accuracy);
* wherever the cut is feasible PPT keeps xi = tr(rho^2)/tr(rho)^2 to 1e-9 (Eq. (ppt));
* the trace stays near 1: PPT keeps the trace of the kept Schmidt pairs, so each cut moves it
  by the trace carried by the discarded pairs, at most about sqrt(discarded weight) by
  Cauchy-Schwarz (linear in the discarded singular values); the purity lies in (0, 1];
* the centre bond reaches chi = 512.
"""
import numpy as np
import pytest

from workloads import config_m3

pytestmark = pytest.mark.gpu


def test_saturated_chain_keeps_the_ppt_invariants():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08572_amd import circuits
    spec = config_m3(0, n=16, p=6)
    print("[gpu] N=16 chi=512 p=6 fp64 (saturating)", flush=True)
    infos = []
    m = circuits.run_circuit(spec, infos=infos)
    bonds = m.bond_dims()
    print(f"[gpu] bonds {bonds}", flush=True)
    assert max(bonds) == 512
    sat = [x for x in infos if x["chi_l"] >= 512 and x["chi_mid"] >= 512 and x["chi_r"] >= 512]
    print(f"[gpu] {len(sat)} updates with all three bonds at 512", flush=True)
    assert len(sat) >= 3
    sqrt_discarded = 0.0
    for x in infos:
        sqrt_discarded += np.sqrt(x["discarded_weight"])
        if x["ppt_feasible"] and x["discarded_weight"] > 0:
            assert abs(x["xi_after"] - x["xi_before"]) <= 1e-9 * abs(x["xi_before"])
    g = circuits.observables(m)
    tr = g["trace"]
    assert abs(tr.imag) <= 1e-10
    print(f"[gpu] |tr - 1| = {abs(tr.real - 1.0):.2e}, sum sqrt(discarded weight) = {sqrt_discarded:.2e}",
          flush=True)
    assert abs(tr.real - 1.0) <= 1e-10 + 10.0 * sqrt_discarded
    p = circuits.purity(m)
    assert 0.0 < p <= 1.0 + 1e-10
    assert np.all(np.isfinite(g["populations"]))
    assert abs(np.sum(g["populations"], axis=1) - 1.0).max() <= 1e-10   # normalised by the trace
    m.close()
