"""Write stored oracle values for the chi_max=512 noisy QAOA circuits (workloads.config_m3,
rates 1e-3, seed 0), computed by the CPU oracle (oracle/mpo.py, LAPACK SVD):

    python tests/golden/make_m3_oracle.py          # N=100, p=3 -> m3_seed0_oracle.json (~4 min)
    python tests/golden/make_m3_oracle.py deep     # N=8, p=4 -> qaoa_n8_p4_chi512_seed0_oracle.json
                                                   # (bonds of a few hundred; tens of minutes)

Stores the per-site energy, all per-atom populations, the all-qubit probability, the purity
tr(rho^2)/tr(rho)^2 (as the vectorised 2-norm), the trace and the bond dimensions.  Only oracle/ and workloads/ are used.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import mpo  # noqa: E402
from workloads import config_m3  # noqa: E402


CASES = {
    "m3": (dict(n=100, p=3), "m3_seed0_oracle.json", "noisy QAOA N=100 d=4 chi_max=512 p=3 rates 1e-3 seed 0"),
    "deep": (dict(n=8, p=4), "qaoa_n8_p4_chi512_seed0_oracle.json",
             "noisy QAOA N=8 d=4 chi_max=512 p=4 rates 1e-3 seed 0"),
}


def main():
    case = sys.argv[1] if len(sys.argv) > 1 else "m3"
    kw, fname, label = CASES[case]
    spec = config_m3(0, **kw)
    t0 = time.time()
    m = mpo.run_spec(spec)
    o = mpo.observables(m)
    out = {
        "workload": label,
        "energy_per_site": float(o["energy_per_site"]),
        "p_success": float(o["p_success"]),
        "purity": float(o["purity"]),
        "trace": [float(complex(o["trace"]).real), float(complex(o["trace"]).imag)],
        "populations": [[float(x) for x in row] for row in o["populations"]],
        "bond_dims": [int(b) for b in m.bond_dims()],
        "seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, fname), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote %s in %.0f s" % (fname, out["seconds"]))


if __name__ == "__main__":
    main()
