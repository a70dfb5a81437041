"""Write the CPU oracle's qubit trace of the paper's pulse-level QAOA iteration (Sec. IV):
tests/golden/qtrace_gaussian_cz_oracle.json.  Only oracle/ is used.

    python tests/golden/make_qtrace_oracle.py       # ~10 min (the pulse channel dominates)

Circuit (Sec. IV, Eqs. (HZ_block_representation), (HZ_representation)): |+>^N on d = 4 levels
{0, 1, r, dark}; layer k = 1..8 with Table I's (alpha_k, beta_k): on every bond, left to right,
exp(i alpha_k Z_i Z_j) = CNOT_ij (I (x) exp(i alpha_k Z_j)) CNOT_ij with CNOT_ij = (I (x) Had_j)
CZ_ij (I (x) Had_j), each CZ the Gaussian pulse's channel (Fig. 1 caption; Sec. II) with its
single-qubit Z phases undone on both atoms (the pulse is a CZ up to those phases); then
exp(i b alpha_k Z_l) (b = 0.2) and exp(i beta_k X_l) on every atom.  The single-atom gates act on
{0, 1} and are the identity on r and the dark state; they are noise free, as in the paper.
Rydberg dissipation gamma (in units of 1/T, T the pulse length) with branching (1/16, 1/16,
7/8) to (0, 1, dark); no dephasing.  The qubit trace tr(rho prod_j Pi_q) is recorded for N = 4,
6, 8 at gamma = 0.02 (MPO oracle, LAPACK SVD with PPT, chi 64), and the slope
c = -d ln tr_q / (gamma dN) between them, which the paper states as 0.1556.
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import channels, mpo, pulse  # noqa: E402

D = 4
T = 2.165
N_STEPS = 1000
GAMMA = 0.02
CHI = 64
ALPHAS = [0.11076513, 0.2771272, 0.36282021, 0.40618171, 0.43256044, 0.44492256, 0.42887337, 0.3225842]
BETAS = [0.75428624, 0.73016842, 0.7096901, 0.68739375, 0.65733871, 0.60978220, 0.51570246, 0.19145101]
BFIELD = 0.2


def _qubit_op(u2):
    u = np.eye(D, dtype=np.complex128)
    u[:2, :2] = u2
    return u


def _site_superop(u):
    return np.kron(u, u.conj())   # vec(u rho u^+), eta = sigma d + sigma'


def main():
    t0 = time.time()
    two_pi = 2.0 * math.pi
    om, de, tau = pulse.gaussian_samples(T, two_pi * 17.0, two_pi * -14.7, N_STEPS)
    blockade = two_pi * 60.0
    u0 = pulse.trotter_unitary(om, de, tau, D, blockade)
    ub = pulse.qubit_block(u0, D)
    phase = float(np.angle(ub[1, 1] / ub[0, 0]))            # the pulse's single-qubit Z phase
    corr = _qubit_op(np.diag([1.0, np.exp(-1j * phase)]))
    S = pulse.to_site_layout(pulse.pulse_channel(om, de, tau, D, blockade, gamma_diss=GAMMA / T,
                                                 branch=(1.0 / 16, 1.0 / 16, 7.0 / 8)), D)
    cz = np.kron(_site_superop(corr), _site_superop(corr)) @ S
    had = _qubit_op(np.array([[1.0, 1.0], [1.0, -1.0]]) / math.sqrt(2.0))
    i16 = np.eye(D * D, dtype=np.complex128)
    h2 = np.kron(i16, _site_superop(had))
    pq = channels.qubit_projector(D)
    out = {"workload": "Sec. IV QAOA iteration (Table I, 8 layers, b = 0.2) with the Gaussian CZ pulse channel "
                       "(%d steps, B/2pi = 60 MHz, Z phases undone), Rydberg dissipation %.3g/T, chi %d" %
                       (N_STEPS, GAMMA, CHI),
           "gamma_per_T": GAMMA, "n_steps": N_STEPS, "chi": CHI, "cz_phase": phase, "qubit_trace": {}}
    for n in (4, 6, 8):
        m = mpo.MPO([channels.plus_state(D)] * n, chi=CHI)
        for a, b in zip(ALPHAS, BETAS):
            rz = _qubit_op(np.diag([np.exp(1j * a), np.exp(-1j * a)]))
            blk = h2 @ cz @ h2 @ np.kron(i16, _site_superop(rz)) @ h2 @ cz @ h2
            for i in range(n - 1):
                m.apply_2site(i, blk)
            zb = _site_superop(_qubit_op(np.diag([np.exp(1j * BFIELD * a), np.exp(-1j * BFIELD * a)])))
            xb = _site_superop(_qubit_op(np.array([[math.cos(b), 1j * math.sin(b)],
                                                   [1j * math.sin(b), math.cos(b)]])))
            for j in range(n):
                m.apply_1site(j, zb)
                m.apply_1site(j, xb)
        tr = complex(m.trace())
        tq = complex(m.expect_product({j: pq for j in range(n)}))
        out["qubit_trace"][str(n)] = {"tr_q": tq.real / tr.real, "trace": [tr.real, tr.imag]}
        print("N=%d tr_q %.12f trace %.12f (%.0f s)" % (n, tq.real / tr.real, tr.real, time.time() - t0), flush=True)
    q = out["qubit_trace"]
    out["slope_4_8"] = -(math.log(q["8"]["tr_q"]) - math.log(q["4"]["tr_q"])) / (GAMMA * 4)
    out["seconds"] = time.time() - t0
    with open(os.path.join(HERE, "qtrace_gaussian_cz_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("slope %.4f; wrote qtrace_gaussian_cz_oracle.json" % out["slope_4_8"], flush=True)


if __name__ == "__main__":
    main()
