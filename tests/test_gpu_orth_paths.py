"""GPU parity of the two ways the split builds its range bases, each against the CPU oracle.

The two-site update first builds every range basis of order <= 256 from a pivoted Cholesky
factorisation of the level's Gram matrix (kernel family "pchol"); when a basis fails its
orthonormality check the update is recomputed with bases from Gram eigenvectors (the
tridiagonal and Jacobi eigensolvers).  MPDO_ORTH_EIG=1 forces the second path everywhere, so
both are checked here on the same circuits, with the bars of the other parity tests: FP64
1e-10 relative on the per-site energy, populations, success probability and trace; FP32 1e-5
absolute on the per-site energy and populations.  The kernel profile shows which path ran."""
import numpy as np
import pytest

from workloads import config_m1, random_spec

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08572_amd import circuits, mpdo
    mpdo.load_library()
    return circuits, mpdo


def _run(circuits, mpdo, spec, prec):
    m = mpdo.MPDO(spec.n, spec.d, spec.chi, precision=prec)
    m.profile(True)
    infos = []
    circuits.run_circuit(spec, m=m, infos=infos)
    g = circuits.observables(m)
    prof = m.profile_read()
    m.close()
    return g, prof, infos


CASES = {
    "m1_n16": lambda: config_m1(1, n=16),
    "truncating_n8_chi64": lambda: random_spec(seed=9, n=8, d=4, p=3, chi=64, rate_lo=1e-3, rate_hi=1e-2),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("prec_name", ["fp64", "fp32"])
def test_pivoted_cholesky_and_eigen_bases_match_the_oracle(case, prec_name, monkeypatch):
    circuits, mpdo = _gpu()
    from oracle import mpo
    spec = CASES[case]()
    prec = mpdo.MPDO_FP64 if prec_name == "fp64" else mpdo.MPDO_FP32
    o = mpo.observables(mpo.run_spec(spec))
    res = {}
    for path in ("pchol", "eigen"):
        if path == "eigen":
            monkeypatch.setenv("MPDO_ORTH_EIG", "1")
        else:
            monkeypatch.delenv("MPDO_ORTH_EIG", raising=False)
        print(f"[gpu] {case} {prec_name} range bases by {path}", flush=True)
        g, prof, infos = _run(circuits, mpdo, spec, prec)
        eig_launches = prof["tri_reduce"]["launches"] + prof["eig_small"]["launches"]
        print(f"[gpu]   pchol launches {prof['pchol']['launches']}, eigensolver launches {eig_launches}, "
              f"recomputed {sum(x['retried'] for x in infos)}", flush=True)
        if path == "pchol":
            assert prof["pchol"]["launches"] > 0
        else:
            assert prof["pchol"]["launches"] == 0
        de = abs(g["energy_per_site"] - o["energy_per_site"])
        dp = float(np.max(np.abs(g["populations"] - o["populations"])))
        print(f"[gpu]   |dE/N| {de:.2e}, max |d pop| {dp:.2e}", flush=True)
        if prec_name == "fp64":
            scale = max(1.0, abs(o["energy_per_site"]))
            assert de <= 1e-10 * scale
            assert dp <= 1e-10
            assert abs(g["p_success"] - o["p_success"]) <= 1e-10 * max(1.0, o["p_success"])
            assert abs(g["trace"] - o["trace"]) <= 1e-10 * abs(o["trace"])
        else:
            assert de <= 1e-5 and dp <= 1e-5
        res[path] = g
    if prec_name == "fp64":
        # the same state up to rounding, whichever basis the split used
        assert abs(res["pchol"]["energy_per_site"] - res["eigen"]["energy_per_site"]) <= 1e-11
