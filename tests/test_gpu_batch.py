"""GPU parity of the batched runtime (mpdo_run_batch): independent circuits of uneven N,
chi, d and depth run concurrently on worker streams; each must match the CPU oracle as in
the single-circuit path (FP64: 1e-10 relative)."""
import numpy as np
import pytest

from workloads import config_m0, config_m1, random_spec

pytestmark = pytest.mark.gpu


def test_batch_matches_oracle():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import mpo
    from paper_2309_08572_amd import circuits, mpdo
    specs = [config_m0(0), config_m0(1), config_m1(0, n=12),
             random_spec(seed=8, n=8, d=4, p=3, chi=64, rate_lo=1e-3, rate_hi=1e-2),
             random_spec(seed=3, n=10, d=4, p=2, chi=32), random_spec(seed=4, n=5, d=3, p=2, chi=16)]
    print("[gpu] batch of", len(specs), flush=True)
    res = mpdo.run_batch([circuits.describe(s) for s in specs], n_workers=4)
    for spec, r in zip(specs, res):
        assert r["status"] == 0
        ref = mpo.run_spec(spec)
        o = mpo.observables(ref)
        g = circuits.summarize(r["values"], spec.n, spec.d)
        scale = max(1.0, abs(o["energy_per_site"]))
        assert abs(g["energy_per_site"] - o["energy_per_site"]) <= 1e-10 * scale, spec
        np.testing.assert_allclose(g["populations"], o["populations"], rtol=0, atol=1e-10)
        assert abs(g["p_success"] - o["p_success"]) <= 1e-10
        assert abs(r["trace"] - o["trace"]) <= 1e-10 * abs(o["trace"])
        # counts may differ where a Schmidt value sits at the 1e-14 relative cutoff
        diff = [a - b for a, b in zip(r["bonds"], ref.bond_dims())]
        assert sum(abs(x) for x in diff) <= 2, (spec, r["bonds"], ref.bond_dims())


def test_batch_rejects_bad_circuit():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08572_amd import circuits, mpdo
    d = circuits.describe(config_m0(0))
    d["chi"] = 0
    with pytest.raises(mpdo.MpdoError):
        mpdo.run_batch([d], n_workers=1)


def test_batch_reports_the_first_failure_message():
    """A circuit that fails while it runs (a gate on a site past the chain) reports its own
    status, the others still run, and the batch's error names the failing circuit with the
    context's message."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08572_amd import circuits, mpdo
    d0, d1 = circuits.describe(config_m0(0)), circuits.describe(config_m0(1))
    sites = np.array(d1["op_site"]).copy()
    sites[0] = 99
    d1["op_site"] = sites
    with pytest.raises(mpdo.MpdoError) as err:
        mpdo.run_batch([d0, d1], n_workers=2)
    print(f"[gpu] {err.value}", flush=True)
    assert "circuit 1:" in str(err.value)


def test_batch_of_m2_circuits_matches_oracle_and_single_runs():
    """The first 8 circuits of the 256-circuit batch workload (N 23..91, chi 64/128/256, p 1..3,
    rates log-uniform in [1e-4, 1e-2]) through mpdo_run_batch on 4 worker streams: each must
    match the stored CPU oracle values (tests/golden/make_m3_oracle.py m2) to the FP64 bar and
    the same circuit run alone through the single-circuit entry points."""
    import json
    import os
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08572_amd import circuits, mpdo
    from workloads import config_m2_batch
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "m2_seed0_first8_oracle.json")) as f:
        gold = json.load(f)["circuits"]
    specs = config_m2_batch(0)[:8]
    print("[gpu] batch of the first 8 M2 circuits", [(s.n, s.chi, s.p) for s in specs], flush=True)
    res = mpdo.run_batch([circuits.describe(s) for s in specs], n_workers=4)
    for c, (spec, r, o) in enumerate(zip(specs, res, gold)):
        assert r["status"] == 0
        g = circuits.summarize(r["values"], spec.n, spec.d)
        scale = max(1.0, abs(o["energy_per_site"]))
        assert abs(g["energy_per_site"] - o["energy_per_site"]) <= 1e-10 * scale, c
        np.testing.assert_allclose(g["populations"], np.array(o["populations"]), rtol=0, atol=1e-10)
        assert abs(g["p_success"] - o["p_success"]) <= 1e-10, c
        assert abs(r["trace"] - complex(*o["trace"])) <= 1e-10, c
        diff = [a - b for a, b in zip(r["bonds"], o["bond_dims"])]
        assert sum(abs(x) for x in diff) <= 2, (c, r["bonds"], o["bond_dims"])
        if c in (0, 3, 5):   # one circuit per depth, alone on the stream of the caller
            m = circuits.run_circuit(spec)
            s = circuits.observables(m)
            assert abs(s["energy_per_site"] - g["energy_per_site"]) <= 1e-10 * scale, c
            np.testing.assert_allclose(s["populations"], g["populations"], rtol=0, atol=1e-10)
            assert m.bond_dims() == r["bonds"], c
            m.close()


def test_batch_on_sixteen_streams_reproduces_single_runs():
    """96 truncating circuits (N=16, d=4, chi=64, p=3, rates log-uniform in [1e-4, 1e-2]) on 16
    worker streams, whose kernels share compute units, against the same circuits run one at a
    time.  The tridiagonal reduction once cleared an entry of p that other waves of its
    workgroup still had to read; alone on a compute unit the waves read it in time, next to
    other streams' kernels some did not, and the batch returned wrong bases (caught by the
    basis check, then recomputed) or failed circuits.  Every circuit must succeed and match
    its single run to 1e-10 on the per-site energy and the populations (the eigensolver's LDS
    sums are not bitwise reproducible, so equality is to rounding)."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08572_amd import circuits, mpdo
    specs = [random_spec(seed=100 + s, n=16, d=4, p=3, chi=64) for s in range(96)]
    print("[gpu] batch of 96 truncating circuits on 16 streams", flush=True)
    res = mpdo.run_batch([circuits.describe(s) for s in specs], n_workers=16)
    worst = 0.0
    for spec, r in zip(specs, res):
        assert r["status"] == 0, spec
        g = circuits.summarize(r["values"], spec.n, spec.d)
        m = circuits.run_circuit(spec)
        o = circuits.observables(m)
        m.close()
        de = abs(g["energy_per_site"] - o["energy_per_site"])
        dp = float(np.max(np.abs(g["populations"] - o["populations"])))
        worst = max(worst, de, dp)
        assert de <= 1e-10 and dp <= 1e-10, (spec.seed, de, dp)
    print(f"[gpu] largest difference batch vs single {worst:.2e}", flush=True)
