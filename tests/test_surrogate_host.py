"""Host-side pins of the surrogate's input map: the observables are periodic with period pi in
every QAOA angle (checked on the dense oracle, full four-level noisy model), and the analytic
chain rule of the harmonic features agrees with finite differences."""
import dataclasses
import math

import numpy as np

from oracle import dense
from workloads.qaoa import CircuitSpec


def test_observables_are_pi_periodic_in_every_angle():
    base = CircuitSpec(n=3, d=4, p=2, gamma=(0.7, 2.1), beta=(0.4, 1.3), p_leak=3e-3, p_deph=2e-3,
                       p_decay=4e-3, chi=256)
    o0 = dense.observables(dense.run_spec(base))
    for k in range(4):
        g, b = list(base.gamma), list(base.beta)
        if k < 2:
            g[k] += math.pi
        else:
            b[k - 2] -= math.pi
        o = dense.observables(dense.run_spec(dataclasses.replace(base, gamma=tuple(g), beta=tuple(b))))
        assert abs(o["energy_per_site"] - o0["energy_per_site"]) < 1e-13
        assert abs(o["p_success"] - o0["p_success"]) < 1e-13
    # and not with half the period (the features must not assume more symmetry than there is)
    o = dense.observables(dense.run_spec(dataclasses.replace(base, gamma=(0.7 + 0.5 * math.pi, 2.1))))
    assert abs(o["energy_per_site"] - o0["energy_per_site"]) > 1e-3


def test_feature_chain_rule_matches_finite_differences():
    from paper_2309_08572_amd import surrogate as sur
    task = sur.Task(n=6, p=2)
    rng = np.random.default_rng(0)
    a = rng.uniform(0, math.pi, size=(3, 4))
    r = np.full((3, 3), 1e-3)
    w = rng.standard_normal(task.n_in)
    g = sur.angle_grad(a, np.tile(w, (3, 1)))
    h = 1e-6
    for i in range(4):
        e = np.zeros(4)
        e[i] = h
        fd = (sur.features(task, a + e, r) @ w - sur.features(task, a - e, r) @ w) / (2 * h)
        np.testing.assert_allclose(g[:, i], fd, rtol=0, atol=1e-8)
    assert sur.features(task, a, r).shape == (3, task.n_in)
    np.testing.assert_allclose(sur.features(task, a + math.pi, r), sur.features(task, a, r), atol=1e-12)


def test_wrap_distance_is_periodic():
    from paper_2309_08572_amd import surrogate as sur
    assert sur.wrap_distance([0.01, 1.0], [math.pi - 0.01, 1.0]) < 0.0201
    assert abs(sur.wrap_distance([0.0, 0.0], [0.5 * math.pi, 0.2]) - 0.5 * math.pi) < 1e-12
