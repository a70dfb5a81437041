"""Write m3_seed0_oracle.json: the CPU oracle (oracle/mpo.py, LAPACK SVD) on the full-size
noisy QAOA workload N=100, d=4, chi_max=512, p=3, rates 1e-3, seed 0 (workloads.config_m3).

    python tests/golden/make_m3_oracle.py      # ~4 min on 8 cores

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


def main():
    spec = config_m3(0)
    t0 = time.time()
    m = mpo.run_spec(spec)
    o = mpo.observables(m)
    out = {
        "workload": "noisy QAOA N=100 d=4 chi_max=512 p=3 rates 1e-3 seed 0",
        "energy_per_site": float(o["energy_per_site"]),
        "p_success": float(o["p_success"]),
        "purity": float(o["purity"]),
        "trace": [float(complex(o["trace"]).real), float(complex(o["trace"]).imag)],
        "populations": [[float(x) for x in row] for row in o["populations"]],
        "bond_dims": [int(b) for b in m.bond_dims()],
        "seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, "m3_seed0_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote m3_seed0_oracle.json in %.0f s" % out["seconds"])


if __name__ == "__main__":
    main()
