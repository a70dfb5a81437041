"""Pins of the pulse-level channel oracle (oracle/pulse.py, Sec. II and Sec. III.A):

* every step channel is trace preserving and completely positive (Choi matrix >= 0);
* the step product converges to an independent integration of the Lindblad equation (a
  Runge-Kutta solve of drho/dt written out on 9 x 9 matrices), at first order in the step;
* the noise-free, blockade-free channel is Ad(u (x) u) with u the single-atom propagator of an
  independent ODE solve, at second order in the step (midpoint samples);
* dissipation alone follows the closed form of the split step: the r population survives as
  exp(-gamma T), the sinks fill with the per-step fractions, which tend to b_j (1 - exp(-gamma T));
  qubit dephasing multiplies rho_01 by exp(-gamma_deph^2 T);
* the Gaussian CZ pulse of the paper (T = 2.165 us, Omega_max/2pi = 17 MHz, Delta/2pi = -14.7 MHz,
  B/2pi = 60 MHz) returns the qubit populations and is a CZ up to single-qubit Z phases with an
  average gate infidelity below 1e-6 (the paper quotes 6e-8 for its combined fidelity measure);
  read with MHz as angular units the same numbers give no CZ at all;
* the reordering to the per-atom layout agrees with a direct vectorisation.
"""
import math

import numpy as np
from scipy.integrate import solve_ivp

from oracle import pulse

TWO_PI = 2.0 * math.pi


def _choi_min_eig(S, d):
    D = d * d
    T = S.reshape(D, D, D, D)               # x y | a b
    C = T.transpose(0, 2, 1, 3).reshape(D * D, D * D)   # (x a), (y b)
    return np.linalg.eigvalsh(0.5 * (C + C.conj().T)).min()


def test_step_channel_is_trace_preserving_and_completely_positive():
    for d in (3, 4):
        br = (0.25, 0.6, 0.15) if d == 4 else (0.4, 0.6, 0.0)
        S = pulse.step_channel(3.1, -1.7, 0.05, d, blockade=40.0, gamma_diss=0.8, branch=br, gamma_deph=0.5)
        D = d * d
        vecI = np.eye(D).reshape(-1)
        np.testing.assert_allclose(vecI @ S, vecI, atol=1e-13)
        assert _choi_min_eig(S, d) > -1e-12


def _lindblad_ode_channel(om_fn, de_fn, T, d, B, gd, br, gp):
    """Independent reference: integrate drho/dt for all d^4 basis inputs at once."""
    D = d * d
    h_r1 = np.zeros((d, d), complex)
    h_r1[2, 1] = h_r1[1, 2] = 1.0
    h_rr = np.zeros((d, d), complex)
    h_rr[2, 2] = 1.0
    I = np.eye(d)
    Hb = np.zeros((D, D), complex)
    Hb[2 * d + 2, 2 * d + 2] = B
    sinks = [0, 1] + ([3] if d == 4 else [])
    Ls = []
    for atom in (0, 1):
        single = []
        for k, j in enumerate(sinks):
            m = np.zeros((d, d), complex)
            m[j, 2] = math.sqrt(gd * br[k])
            single.append(m)
        z = np.zeros((d, d), complex)
        z[0, 0], z[1, 1] = gp / math.sqrt(2), -gp / math.sqrt(2)
        single.append(z)
        Ls += [np.kron(m, I) if atom == 0 else np.kron(I, m) for m in single]

    def rhs(t, y):
        rho = y.reshape(D * D, D, D)
        h = 0.5 * om_fn(t) * h_r1 + de_fn(t) * h_rr
        H = np.kron(h, I) + np.kron(I, h) + Hb
        out = -1j * (H @ rho - rho @ H)
        for L in Ls:
            LdL = L.conj().T @ L
            out += L @ rho @ L.conj().T - 0.5 * (LdL @ rho + rho @ LdL)
        return out.reshape(-1)

    y0 = np.zeros((D * D, D, D), complex)
    for a in range(D):
        for b in range(D):
            y0[a * D + b, a, b] = 1.0
    sol = solve_ivp(rhs, (0, T), y0.reshape(-1), method="DOP853", rtol=1e-9, atol=1e-10)
    out = sol.y[:, -1].reshape(D * D, D * D)     # [input (a b), output (x y)]
    return out.T


def test_step_product_converges_to_the_lindblad_equation():
    d, T, B, gd, br, gp = 3, 0.4, 25.0, 1.5, (0.35, 0.65, 0.0), 0.9
    om_fn = lambda t: 30.0 * math.sin(math.pi * t / T) ** 2
    de_fn = lambda t: -6.0 + 20.0 * t
    ref = _lindblad_ode_channel(om_fn, de_fn, T, d, B, gd, br, gp)
    errs = []
    for n in (50, 100, 200):
        tau = T / n
        t = (np.arange(n) + 0.5) * tau
        S = pulse.pulse_channel([om_fn(x) for x in t], [de_fn(x) for x in t], tau, d, B, gd, br, gp)
        errs.append(np.abs(S - ref).max())
    assert errs[2] < 2e-2
    # first-order splitting: the error halves with the step
    assert 1.6 < errs[0] / errs[1] < 2.5 and 1.6 < errs[1] / errs[2] < 2.5, errs


def test_noise_free_product_is_the_single_atom_propagator():
    d, T = 3, 0.5
    om_fn = lambda t: 40.0 * math.exp(-((t - 0.25) / 0.1) ** 2)
    de_fn = lambda t: 8.0 * math.cos(7.0 * t)

    def f(t, y):
        h = pulse.site_hamiltonian(om_fn(t), de_fn(t), d)
        return (-1j * h @ y.reshape(d, d)).reshape(-1)

    u = solve_ivp(f, (0, T), np.eye(d, dtype=complex).reshape(-1), method="DOP853", rtol=1e-12,
                  atol=1e-13).y[:, -1].reshape(d, d)
    U = np.kron(u, u)
    ref = np.kron(U, U.conj())
    errs = []
    for n in (100, 200):
        tau = T / n
        t = (np.arange(n) + 0.5) * tau
        S = pulse.pulse_channel([om_fn(x) for x in t], [de_fn(x) for x in t], tau, d, blockade=0.0)
        errs.append(np.abs(S - ref).max())
    assert errs[1] < 1e-3
    assert 3.3 < errs[0] / errs[1] < 4.7, errs       # midpoint samples: second order


def test_dissipation_closed_form_of_the_split_step():
    d, n, tau, gd, br, gp = 4, 16, 0.05, 3.0, (0.25, 0.15, 0.6), 1.3
    S = pulse.pulse_channel(np.zeros(n), np.zeros(n), tau, d, blockade=17.0, gamma_diss=gd, branch=br,
                            gamma_deph=gp)
    D = d * d
    rho = np.zeros((D, D), complex)
    rho[2 * d + 0, 2 * d + 0] = 1.0                 # atom 1 in r, atom 2 in 0
    out = (S @ rho.reshape(-1)).reshape(D, D)
    p1 = np.array([sum(out[a * d + b, a * d + b].real for b in range(d)) for a in range(d)])
    e = [math.exp(-gd * b * tau) for b in br]
    surv = e[0] * e[1] * e[2]
    per_step = [1 - e[0], e[0] * (1 - e[1]), e[0] * e[1] * (1 - e[2])]
    T = n * tau
    assert abs(p1[2] - math.exp(-gd * T)) < 1e-13
    geo = (1 - surv ** n) / (1 - surv)
    for k, j in enumerate((0, 1, 3)):
        assert abs(p1[j] - per_step[k] * geo) < 1e-13
        assert abs(p1[j] - br[k] * (1 - math.exp(-gd * T))) < gd * tau * br[k]   # first-order split error
    # dephasing of the qubit coherence
    rho = np.zeros((D, D), complex)
    rho[0 * d + 0, 1 * d + 0] = 1.0
    out = (S @ rho.reshape(-1)).reshape(D, D)
    assert abs(out[0, d] - math.exp(-gp * gp * T)) < 1e-13


def test_gaussian_cz_pulse_of_the_paper():
    om, de, tau = pulse.gaussian_samples(2.165, TWO_PI * 17.0, TWO_PI * -14.7, 12000)
    U = pulse.trotter_unitary(om, de, tau, 4, TWO_PI * 60.0)
    Uq = pulse.qubit_block(U, 4)
    assert np.all(np.abs(np.abs(np.diag(Uq)) - 1.0) < 1e-6)
    assert pulse.cz_infidelity(Uq) < 1e-6
    # the entangling phase is pi
    ph = np.angle(np.diag(Uq))
    ent = (ph[3] - ph[1] - ph[2] + ph[0]) % (2 * math.pi)
    assert abs(ent - math.pi) < 5e-3      # B = 2pi x 60 MHz is the paper's rounded value
    # MHz taken as angular units: no CZ
    om2, de2, tau2 = pulse.gaussian_samples(2.165, 17.0, -14.7, 2000)
    U2 = pulse.qubit_block(pulse.trotter_unitary(om2, de2, tau2, 4, TWO_PI * 60.0), 4)
    assert pulse.cz_infidelity(U2) > 0.1


def test_site_layout_matches_direct_vectorisation():
    d = 3
    rng = np.random.default_rng(0)
    K = rng.standard_normal((d * d, d * d)) + 1j * rng.standard_normal((d * d, d * d))
    S = np.kron(K, K.conj())                       # rho -> K rho K^+
    L = pulse.to_site_layout(S, d)
    rho = rng.standard_normal((d * d, d * d)) + 1j * rng.standard_normal((d * d, d * d))
    out = K @ rho @ K.conj().T

    def site_vec(r):
        t = r.reshape(d, d, d, d)                  # x1 x2 y1 y2
        return t.transpose(0, 2, 1, 3).reshape(-1)  # (x1 y1) (x2 y2)
    np.testing.assert_allclose(L @ site_vec(rho), site_vec(out), atol=1e-12)
