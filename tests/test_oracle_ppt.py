"""Pins of the oracle's PPT (Sec. III.D, Eqs. (xiformula), (ppt); App. B).

Checked against: the invariant PPT exists for (xi kept), the algebra of App. B, a brute
force search along the ray Lambda' + y Delta' on small vectors, the no-truncation limit,
scale behaviour and the infeasible fallback.
"""
import math

import numpy as np
import pytest

from oracle import ppt as P


def _case(seed, n, k):
    rng = np.random.default_rng(seed)
    lam = np.sort(np.abs(rng.standard_normal(n)))[::-1] * rng.uniform(0.5, 2.0)
    T = rng.standard_normal(n) + 0.8
    return lam, T, k


def _feasible_cases():
    out = []
    for seed in range(200):
        lam, T, k = _case(seed, 3 + seed % 6, 1 + seed % 4)
        if k >= len(lam):
            continue
        lt, info = P.ppt(lam, T, k)
        if info["feasible"] and not info["degenerate_sigma"]:
            out.append((lam, T, k, lt, info))
    return out


def test_xi_is_preserved():
    cases = _feasible_cases()
    assert len(cases) > 30
    for lam, T, k, lt, _ in cases:
        assert abs(P.xi(lt, T[:k]) - P.xi(lam, T)) <= 1e-12 * abs(P.xi(lam, T))


def test_trace_component_and_plane():
    for lam, T, k, lt, _ in _feasible_cases():
        Tp, lp = T[:k], lam[:k]
        # T' . Lambda~ = T' . Lambda'
        assert abs(Tp @ lt - Tp @ lp) < 1e-12 * (abs(Tp @ lp) + 1)
        # Lambda~ lies in span{Lambda', T'}
        B = np.stack([lp, Tp], axis=1)
        coef, *_ = np.linalg.lstsq(B, lt, rcond=None)
        assert np.linalg.norm(B @ coef - lt) < 1e-12 * np.linalg.norm(lt)


def test_appendix_b_algebra():
    for lam, T, k, lt, info in _feasible_cases():
        Tp, lp = T[:k], lam[:k]
        s = info["sigma"]
        delta = lp - np.linalg.norm(lp) * math.cos(s) * Tp / np.linalg.norm(Tp)
        assert abs(delta @ delta - (lp @ lp) * math.sin(s) ** 2) < 1e-12 * (lp @ lp)
        assert abs(lp @ delta - (lp @ lp) * math.sin(s) ** 2) < 1e-12 * (lp @ lp)
        x = math.tan(info["theta"]) / math.tan(s) - 1.0
        np.testing.assert_allclose(lt, lp + x * delta, rtol=1e-12, atol=1e-14)


def test_brute_force_ray_search():
    """Scan y on Lambda' + y Delta' for the angle theta with T' (positive branch)."""
    n_checked = 0
    for lam, T, k, lt, info in _feasible_cases()[:20]:
        Tp, lp = T[:k], lam[:k]
        s = info["sigma"]
        delta = lp - np.linalg.norm(lp) * math.cos(s) * Tp / np.linalg.norm(Tp)
        ys = np.linspace(-1.0, 6.0, 700001)
        v = lp[None, :] + ys[:, None] * delta[None, :]
        ang = np.arccos(np.clip(v @ Tp / (np.linalg.norm(v, axis=1) * np.linalg.norm(Tp)),
                                -1, 1))
        want = info["theta"]
        j = int(np.argmin(np.abs(ang - want)))
        if abs(ang[j] - want) > 1e-4:
            continue        # target outside the scanned window
        y = ys[j]
        np.testing.assert_allclose(lp + y * delta, lt, rtol=2e-4, atol=2e-5)
        n_checked += 1
    assert n_checked >= 10


def test_no_truncation_is_identity():
    for seed in range(20):
        lam, T, _ = _case(seed, 6, 6)
        lt, info = P.ppt(lam, T, 6)
        np.testing.assert_allclose(lt, lam, rtol=1e-9, atol=1e-12)


def test_scale_behaviour():
    lam, T, k = _case(7, 6, 3)
    lt, _ = P.ppt(lam, T, k)
    lt2, _ = P.ppt(3.7 * lam, T, k)
    np.testing.assert_allclose(lt2, 3.7 * lt, rtol=1e-12)
    lt3, _ = P.ppt(lam, 0.4 * T, k)
    np.testing.assert_allclose(lt3, lt, rtol=1e-12)


def test_infeasible_falls_back_to_theta_zero():
    # |T'| < |T| cos(phi): almost all of the trace sits in the discarded entries
    lam = np.array([1.0, 0.9, 0.8])
    T = np.array([0.05, 0.02, 3.0])
    lt, info = P.ppt(lam, T, 2)
    assert not info["feasible"]
    Tp = T[:2]
    cosang = lt @ Tp / (np.linalg.norm(lt) * np.linalg.norm(Tp))
    assert abs(cosang - 1.0) < 1e-12
    # the trace of the cut state is still T'.Lambda'
    assert abs(Tp @ lt - Tp @ lam[:2]) < 1e-12


@pytest.mark.parametrize("k", [1, 2])
def test_parallel_lambda_and_t(k):
    lam = np.array([2.0, 1.0, 0.5])
    T = 0.3 * lam
    lt, info = P.ppt(lam, T, k)
    assert info["degenerate_sigma"]
    np.testing.assert_allclose(lt, lam[:k])


def test_renorm_trace_option_keeps_the_trace_and_the_normalised_observables():
    """The oracle's optional trace renormalisation (a reading: the paper leaves the trace after
    PPT as the cut leaves it): on a heavily truncating circuit (chi 16) the plain run's trace
    drifts, the renormalised run's final trace is 1 to rounding (every channel is trace
    preserving, so only the cuts could change it), and the normalised observables of the two
    runs agree (every later step is linear in rho or, like PPT and the relative cutoff,
    equivariant under rho -> c rho)."""
    from oracle import mpo
    from workloads import random_spec
    spec = random_spec(seed=8, n=8, d=4, p=3, chi=16, rate_lo=1e-3, rate_hi=1e-2)
    a = mpo.run_spec(spec)
    b = mpo.run_spec(spec, renorm_trace=True)
    assert abs(a.trace() - 1.0) > 1e-3
    assert abs(b.trace() - 1.0) < 1e-12
    cuts = [x for x in b.log if x["discarded_weight"] > 1e-12]
    assert len(cuts) >= 5
    oa, ob = mpo.observables(a), mpo.observables(b)
    assert abs(oa["energy_per_site"] - ob["energy_per_site"]) < 1e-12
    np.testing.assert_allclose(oa["populations"], ob["populations"], rtol=0, atol=1e-12)
    assert abs(oa["p_success"] - ob["p_success"]) < 1e-12
