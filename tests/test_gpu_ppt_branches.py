"""GPU parity of the two PPT branches that ordinary circuits rarely reach, through the C ABI,
against the CPU oracle (oracle/mpo.py, LAPACK SVD) on the same seeded inputs:

* the infeasible cut (end of Sec. III.D): when the kept trace vector is too short for any
  angle theta to keep xi (|T'| < |T| cos(phi)), theta = 0 is used, which makes the kept
  spectrum parallel to T'.  A heavy cut (chi 1 or 3) of a noisy chain reaches it; both sides
  must report the cut infeasible and give the same state (observables to 1e-10, with the
  gauge-invariant cut quantities: trace before and after, xi before, kept count, gap);
* the optional trace renormalisation (reading: the paper leaves the trace after PPT as it
  is; with renorm_trace each cut spectrum is rescaled so tr(rho) is unchanged): the GPU must
  match the oracle's renormalised run to 1e-10 and keep the trace at 1.
"""
import numpy as np
import pytest

from workloads import random_spec

pytestmark = pytest.mark.gpu

REL = 1e-10


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08572_amd import circuits, mpdo
    mpdo.load_library()
    return circuits, mpdo


def _check(o, g, label):
    scale = max(1.0, abs(o["energy_per_site"]))
    assert abs(g["energy_per_site"] - o["energy_per_site"]) <= REL * scale, label
    np.testing.assert_allclose(g["populations"], o["populations"], rtol=0, atol=REL, err_msg=label)
    assert abs(g["p_success"] - o["p_success"]) <= REL * max(1.0, o["p_success"]), label
    assert abs(g["trace"] - o["trace"]) <= REL * abs(o["trace"]), label


# (seed, atoms, levels, depth, bond, chi): cuts the oracle finds infeasible, with the gap at the
# cut far above rounding (0.77 and 0.18 of a spectrum of order 1)
INFEASIBLE = [(0, 6, 4, 2, 3, 1), (0, 4, 3, 3, 0, 3)]


@pytest.mark.parametrize("seed,n,d,p,bond,chi", INFEASIBLE)
def test_infeasible_cut_falls_back_to_theta_zero(seed, n, d, p, bond, chi):
    circuits, mpdo = _gpu()
    from oracle import channels as ch
    from oracle import mpo
    spec = random_spec(seed=seed, n=n, d=d, p=p, chi=256, rate_lo=1e-3, rate_hi=1e-2)
    print(f"[gpu] infeasible PPT cut: seed {seed} N={n} d={d} p={p} bond {bond} chi {chi}", flush=True)
    ops = ch.circuit_ops(spec)
    main, tail = ops[:-3 * n], ops[-3 * n:]
    ref = mpo.MPO([ch.plus_state(d)] * n, chi=256)
    ref.run(main)
    # the GPU queues the last layer's single-atom maps; the cut folds in those of its two atoms
    ref.run([op for op in tail if op[1] in (bond, bond + 1)])
    oi = ref.apply_2site(bond, np.eye(d ** 4, dtype=complex), chi=chi)
    ref.run([op for op in tail if op[1] not in (bond, bond + 1)])
    assert not oi["ppt_feasible"]
    m = circuits.run_circuit(spec)
    gi = m.truncate(bond, chi)
    print(f"[gpu] feasible {gi['ppt_feasible']} theta {gi['ppt_theta']:.3e} kept {gi['kept']} "
          f"tr {gi['trace_before']:.6f} -> {gi['trace_after']:.6f} (oracle {oi['trace_after']:.6f}) "
          f"gap {gi['sigma_gap_at_cut']:.4f} (oracle {oi['gap_at_cut']:.4f})", flush=True)
    assert gi["ppt_feasible"] == 0
    assert gi["ppt_theta"] == 0.0
    assert gi["kept"] == oi["kept"]
    assert abs(gi["trace_before"] - oi["trace_before"]) <= REL * abs(oi["trace_before"])
    assert abs(gi["trace_after"] - oi["trace_after"]) <= REL * abs(oi["trace_after"])
    assert abs(gi["xi_before"] - oi["xi_before"]) <= REL * abs(oi["xi_before"])
    assert abs(gi["discarded_weight"] - oi["discarded_weight"]) <= REL
    # the gap of a chi cut is resolved to the Gram's accuracy (~sqrt(eps) sigma_max)
    assert gi["sigma_next_exact"] == 1
    assert abs(gi["sigma_gap_at_cut"] - oi["gap_at_cut"]) <= 1e-7 * max(1.0, gi["sigma_max"])
    _check(mpo.observables(ref), circuits.observables(m), "infeasible cut")
    m.close()


def test_renorm_trace_matches_oracle():
    circuits, mpdo = _gpu()
    from oracle import mpo
    spec = random_spec(seed=8, n=8, d=4, p=3, chi=16, rate_lo=1e-3, rate_hi=1e-2)
    print("[gpu] renorm_trace: N=8 d=4 p=3 chi=16", flush=True)
    ref = mpo.run_spec(spec, renorm_trace=True)
    o = mpo.observables(ref)
    m = mpdo.MPDO(spec.n, spec.d, spec.chi, renorm_trace=True)
    infos = []
    circuits.run_circuit(spec, infos=infos, m=m)
    g = circuits.observables(m)
    cut = [x for x in infos if x["discarded_weight"] > 1e-12]
    print(f"[gpu] {len(cut)} cuts, |tr - 1| = {abs(g['trace'] - 1):.2e}", flush=True)
    assert len(cut) >= 5
    for x in infos:
        assert abs(x["trace_after"] - x["trace_before"]) <= 1e-12 * abs(x["trace_before"])
    assert abs(g["trace"] - 1.0) <= 1e-12
    _check(o, g, "renorm_trace")
    # normalised observables do not depend on the renormalisation (every later step is linear
    # or scale-equivariant); the trace itself does
    plain = circuits.run_circuit(spec)
    gp = circuits.observables(plain)
    assert abs(gp["energy_per_site"] - g["energy_per_site"]) <= REL
    assert abs(gp["trace"] - 1.0) > 1e-8
    plain.close()
    m.close()
