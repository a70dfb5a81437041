"""Write stored oracle values for circuits too slow for the CPU oracle to rerun inside a GPU test,
computed by the CPU oracle (oracle/mpo.py: LAPACK SVD, FP64) on the seeded workloads:

    python tests/golden/make_m3_oracle.py          # N=100, p=3, chi 512 -> m3_seed0_oracle.json (~4 min)
    python tests/golden/make_m3_oracle.py deep     # N=8, p=4, chi 512 -> qaoa_n8_p4_chi512_seed0_oracle.json
    python tests/golden/make_m3_oracle.py m1       # N=40, p=2, chi 128, seeds 0 and 1 -> m1_n40_seed{0,1}_oracle.json
    python tests/golden/make_m3_oracle.py m2       # the first 8 circuits of the 256-circuit batch -> m2_seed0_first8_oracle.json
    python tests/golden/make_m3_oracle.py sat      # N=12, p=6, chi 512 (centre saturated) -> qaoa_n12_p6_chi512_seed0_oracle.json

Each record holds the per-site energy, all per-atom populations, the all-qubit probability,
the purity tr(rho^2)/tr(rho)^2 (as the vectorised 2-norm), the trace, the bond dimensions and,
for the truncating cases, the per-update log of the cut (trace and xi before the cut, kept
count, discarded weight, gap at the cut, PPT feasibility).  Only oracle/ and workloads/ are
used.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import channels, mpo  # noqa: E402
from workloads import config_m1, config_m2_batch, config_m3  # noqa: E402


def _record(spec, label, with_log=False):
    t0 = time.time()
    if with_log:
        # the steps of mpo.run_spec, with a progress line per two-site update
        m = mpo.MPO([channels.plus_state(spec.d)] * spec.n, chi=spec.chi)
        for kind, site, kraus in channels.circuit_ops(spec):
            if kind == "k2":
                x = m.apply_2site(site, channels.superop_2site(kraus, spec.d))
                print("  %6.0f s  bond %d  chi_l %d chi_r %d kept %d" % (time.time() - t0, site, x["chi_l"],
                                                                      x["chi_r"], x["kept"]), flush=True)
            else:
                m.apply_1site(site, channels.superop_1site(kraus))
    else:
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
    if with_log:
        keys = ("bond", "chi_l", "chi_r", "kept", "trace_before", "xi_before", "trace_after", "xi_after",
                "discarded_weight", "gap_at_cut", "ppt_feasible", "n_sv")
        out["log"] = [{k: (float(x[k]) if isinstance(x[k], float) else int(x[k])) for k in keys if k in x}
                      for x in m.log]
    return out


def _write(fname, rec):
    with open(os.path.join(HERE, fname), "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote %s in %.0f s" % (fname, rec["seconds"] if "seconds" in rec else 0.0), flush=True)


def main():
    case = sys.argv[1] if len(sys.argv) > 1 else "m3"
    if case == "m3":
        _write("m3_seed0_oracle.json",
               _record(config_m3(0), "noisy QAOA N=100 d=4 chi_max=512 p=3 rates 1e-3 seed 0"))
    elif case == "deep":
        _write("qaoa_n8_p4_chi512_seed0_oracle.json",
               _record(config_m3(0, n=8, p=4), "noisy QAOA N=8 d=4 chi_max=512 p=4 rates 1e-3 seed 0"))
    elif case == "m1":
        for seed in (0, 1):
            _write("m1_n40_seed%d_oracle.json" % seed,
                   _record(config_m1(seed), "noisy QAOA N=40 d=4 chi_max=128 p=2, rates log-U[1e-4,1e-2], "
                                            "seed %d" % seed))
    elif case == "m2":
        t0 = time.time()
        recs = []
        for c, spec in enumerate(config_m2_batch(0)[:8]):
            r = _record(spec, "batch circuit %d: N=%d chi=%d p=%d" % (c, spec.n, spec.chi, spec.p))
            print("  circuit %d (N=%d chi=%d p=%d) %.0f s" % (c, spec.n, spec.chi, spec.p, r["seconds"]), flush=True)
            recs.append(r)
        _write("m2_seed0_first8_oracle.json", {"circuits": recs, "seconds": time.time() - t0})
    elif case == "sat":
        _write("qaoa_n12_p6_chi512_seed0_oracle.json",
               _record(config_m3(0, n=12, p=6), "noisy QAOA N=12 d=4 chi_max=512 p=6 rates 1e-3 seed 0 "
                                                 "(centre bonds saturate at 512)", with_log=True))
    else:
        raise SystemExit("unknown case " + case)


if __name__ == "__main__":
    main()
