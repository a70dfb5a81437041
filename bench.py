#!/usr/bin/env python3
"""Throughput of the two-site density-operator MPO update with PPT on one MI355X.

Workload (one "step"): the noisy QAOA circuit on an open chain of N=100 atoms with d=4
levels ({0,1,r,lost}, vectorised site dimension 16), bond cap chi_max=512, depth p=3,
seeded angles and noise probabilities 1e-3 (leak per block, dephasing and decay per
layer), from |+>^N: 3 * 99 = 297 two-site updates (merge, split, cut, PPT), the
single-atom maps, then the TFIM energy, all per-atom populations and the all-qubit
probability by transfer matrices.  Inputs are synthetic and generated on the host before
the timed region; the device state is initialised inside each step.

Prints one JSON line: value = whole-job two-site updates/s of the FP64 path (the one
that matches the oracle to 1e-10); the FP32-MFMA path is reported beside it with its
error against the FP64 result.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _oracle_sample(spec, budget_s: float):
    """The oracle on the circuit's two-site updates in order until budget_s has passed:
    (per-layer update times, updates done, seconds)."""
    from oracle import channels as ch
    from oracle import mpo
    ops = ch.circuit_ops(spec)
    m = mpo.MPO([ch.plus_state(spec.d)] * spec.n, chi=spec.chi)
    per_layer = {}
    layer = 0
    seen = 0
    t0 = time.time()
    for kind, site, kraus in ops:
        if kind == "k2":
            ts = time.time()
            m.apply_2site(site, ch.superop_2site(kraus, spec.d))
            per_layer.setdefault(layer, []).append(time.time() - ts)
            seen += 1
            if seen % (spec.n - 1) == 0:
                layer += 1
        else:
            m.apply_1site(site, ch.superop_1site(kraus))
        if time.time() - t0 > budget_s:
            break
    return per_layer, sum(len(v) for v in per_layer.values()), time.time() - t0


def _extrapolate(spec, per_layer) -> float:
    """Circuit seconds from each reached layer's mean update time (later layers as the last)."""
    import numpy as np
    reached = sorted(per_layer)
    total = 0.0
    for k in range(spec.p):
        total += float(np.mean(per_layer.get(k, per_layer[reached[-1]]))) * (spec.n - 1)
    return total


def _blas():
    try:
        from threadpoolctl import threadpool_info
        info = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if info:
            return (f"{info[0].get('internal_api')} {info[0].get('version')}",
                    max(int(i.get("num_threads", 1)) for i in info))
    except Exception:
        pass
    return "unknown", os.cpu_count() or 1


def _cpu_baseline(spec, budget_s: float, small_specs=()) -> dict:
    """The CPU oracle (numpy + LAPACK SVD, FP64; the oracle as it stands) on the host: a bounded
    sample of the benchmark circuit on all BLAS threads, the circuit time extrapolated per
    layer (the headline record), the same sample on one thread (a third of the budget), and
    the small circuits in small_specs timed in full."""
    vendor, threads = _blas()
    per_layer, done, secs = _oracle_sample(spec, budget_s)
    rec = {
        "value": (spec.p * (spec.n - 1)) / _extrapolate(spec, per_layer),
        "unit": "two-site updates/s",
        "cores": int(threads),
        "kind": "oracle",
        "blas": vendor,
        "sample": (f"CPU oracle (numpy/LAPACK SVD, FP64) on the first {done} two-site updates "
                   f"of the same circuit ({secs:.1f} s), circuit time extrapolated "
                   f"from each layer's mean update time (layers reached: {len(per_layer)})"),
    }
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1, user_api="blas"):
            pl1, done1, secs1 = _oracle_sample(spec, budget_s / 3.0)
        rec["single_thread"] = {"value": (spec.p * (spec.n - 1)) / _extrapolate(spec, pl1),
                                "unit": "two-site updates/s", "cores": 1,
                                "sample": f"first {done1} two-site updates ({secs1:.1f} s), extrapolated per layer"}
    except Exception as e:   # threadpoolctl missing: the record says so
        rec["single_thread"] = {"error": str(e)}
    full = {}
    for name, sp in small_specs:
        t0 = time.time()
        from oracle import mpo
        mpo.run_spec(sp)
        dt = time.time() - t0
        full[name] = {"seconds": dt, "two_site_updates": sp.n_two_site_updates(),
                      "updates_per_s": sp.n_two_site_updates() / dt}
    if full:
        rec["full_circuits"] = full
    return rec


def _batch(count: int, workers: int) -> dict:
    """Circuits of the batch workload (N in [20,100], chi in {64,128,256}, p in {1,2,3},
    d=4, log-uniform noise): all at once on worker streams vs one at a time."""
    from paper_2309_08572_amd import circuits, mpdo
    from workloads import config_m2_batch
    specs = config_m2_batch(0)[:count]
    descs = [circuits.describe(s) for s in specs]
    updates = sum(s.n_two_site_updates() for s in specs)
    t0 = time.perf_counter()
    mpdo.run_batch(descs, n_workers=1)
    t_seq = time.perf_counter() - t0
    t0 = time.perf_counter()
    res = mpdo.run_batch(descs, n_workers=workers)
    t_par = time.perf_counter() - t0
    return {"circuits": count, "workers": workers, "two_site_updates": updates,
            "updates_per_s_batched": updates / t_par, "updates_per_s_one_at_a_time": updates / t_seq,
            "speedup": t_seq / t_par,
            "max_bond": max(max(r["bonds"]) for r in res)}


def _second_order(spec, reps: int) -> dict:
    """Second-order observables (linear functions of rho (x) rho by the doubled transfer step)
    on the benchmark circuit's final FP64 state, built untimed: purity, collision probability,
    the Renyi-2 entropy of the left half of the chain and the Renyi-2 mutual information of two
    10-atom blocks 20 atoms apart; each timed over `reps` calls after one untimed call."""
    import torch
    from paper_2309_08572_amd import circuits, mpdo
    n = spec.n
    m = mpdo.MPDO(n, spec.d, spec.chi, precision=mpdo.MPDO_FP64)
    circuits.run_circuit(spec, m=m)
    a, b = list(range(20, 30)), list(range(50, 60))
    tasks = {"purity": lambda: circuits.purity(m),
             "collision_probability": lambda: circuits.collision_probability(m),
             "renyi2_left_half": lambda: circuits.renyi2(m, range(n // 2)),
             "renyi2_mutual_information_20_29_50_59": lambda: circuits.renyi2_mutual_information(m, a, b)}
    out = {"workload": f"final state of the noisy QAOA circuit, N={n} atoms, d={spec.d}, "
                       f"chi_max={spec.chi}, p={spec.p}, FP64", "max_bond": max(m.bond_dims()), "reps": reps}
    for name, f in tasks.items():
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            v = f()
        torch.cuda.synchronize()
        out[name] = {"value": v, "ms_per_call": 1e3 * (time.perf_counter() - t0) / reps}
    m.close()
    return out


def _oracle_on_state(bonds, sites, centre, bond, kraus, d, chi):
    """The CPU oracle's two-site update of `bond` on the given chain (FP64 site tensors, canonical
    about `centre`, no queued maps): (seconds, the oracle's cut record)."""
    from oracle import channels as ch
    from oracle import mpo
    m = mpo.MPO([ch.plus_state(d)] * len(sites), chi=chi)
    m.A = [a.copy() for a in sites]
    m.lo = m.hi = centre
    S2 = ch.superop_2site(kraus, d)
    t0 = time.time()
    info = m.apply_2site(bond, S2)
    return time.time() - t0, info


def _saturated(max_warm: int, precisions, cpu_updates: int = 0) -> dict:
    """The saturated steady state at chi = 512, FP32 and split-BF16 matrix cores against FP64 on
    the same updates.

    The benchmark circuit's gate set (seed-0 angles, rates 1e-3) runs on a 20-atom chain in FP64,
    untimed, layer by layer until the three centre bonds are at 512 (at most `max_warm` layers),
    then through the even bonds of one more layer.  After the even bonds every atom has taken
    its queued single-atom maps, so the state is the chain alone.  Each update of the odd bonds
    whose three bonds are all 512 (theta of 8192 x 8192, rank <= 4608) is then run twice from
    the same state, the canonical centre already on the pair (moved there untimed in FP64): by
    the FP64 context, and by an FP32 and a split-BF16 context loaded with that state
    (mpdo_set_state with the FP64 context's canonical centre).  All are timed, bracketed by
    synchronisations, with HIP events on the theta contraction (merge and gate products), the
    other products and the eigensolver families; after each, the per-site energy and the
    populations of each result are compared with the FP64 one.  The per-update cost does not depend on N
    (only on the three bond dimensions and d), so the 20-atom chain stands for the saturated
    bulk of the N=100 chain."""
    import numpy as np
    import torch
    from paper_2309_08572_amd import circuits, mpdo
    from workloads import config_m3
    n, chi = 20, 512
    spec = config_m3(0, n=n, p=10, chi=chi)          # one fixed angle set for up to 10 layers
    max_warm = min(max_warm, spec.p - 1)
    d = spec.d

    def maps(m, k):
        for j in range(n):
            m.apply_channel(j, [circuits.x_rotation(spec.beta[k], d)])
            m.apply_channel(j, circuits.dephasing_kraus(spec.p_deph, d))
            m.apply_channel(j, circuits.decay_kraus(spec.p_decay, d))

    a = mpdo.MPDO(n, d, chi, precision=mpdo.MPDO_FP64)
    a.init_product_state([circuits.plus_rho(d)] * n)
    warm = 0
    while warm < max_warm and min(a.bond_dims()[n // 2 - 2:n // 2 + 1]) < chi:
        kr = circuits.block_kraus(spec.gamma[warm], spec.p_leak, d)
        for i in circuits.bond_order(n):
            a.apply_gate_kraus(i, kr)
        maps(a, warm)
        warm += 1
    kr = circuits.block_kraus(spec.gamma[warm], spec.p_leak, d)
    for i in range(0, n - 1, 2):
        a.apply_gate_kraus(i, kr)
    # the other precisions, each loaded with the FP64 state before every timed update
    others = {k: mpdo.MPDO(n, d, chi, precision=v) for k, v in
              (("fp32", mpdo.MPDO_FP32), ("bf16x3", mpdo.MPDO_BF16X3)) if k in precisions}
    fams = ("theta", "gemm", "tri_reduce", "tri_solve", "tri_back", "eig_small", "pchol", "phys", "other")
    cpu = []   # the CPU oracle on the same saturated updates (cpu_updates of them)
    from oracle import channels as och
    okraus = och.gate_kraus_2site(spec.gamma[warm], spec.p_leak, d)
    acc = {k: {"t": [], "prof": None, "kept": []} for k in ["fp64"] + list(others)}
    errs_e = {k: [] for k in others}
    errs_p = {k: [] for k in others}

    def timed(m, i, key):
        m.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        inf = m.apply_gate_kraus(i, kr, info=True)
        m.synchronize()
        acc[key]["t"].append(time.perf_counter() - t0)
        p = m.profile_read()
        m.profile(False)
        pr = acc[key]["prof"]
        acc[key]["prof"] = p if pr is None else {f: {q: pr[f][q] + p[f][q] for q in p[f]} for f in p}
        acc[key]["kept"].append(inf["kept"])
        return inf

    for i in list(range(1, n - 1, 2))[::-1]:
        bd = a.bond_dims()
        sat = 0 < i < n - 2 and bd[i - 1] >= chi and bd[i] >= chi and bd[i + 1] >= chi
        if not sat:
            a.apply_gate_kraus(i, kr)
            continue
        # the centre moves onto the pair first (untimed, in FP64), so that both precisions time
        # the update alone and the FP32 context starts from exactly the FP64 chain (an FP32
        # canonical move would itself compress the bonds it crosses to what FP32 resolves)
        a.move_centre(i + 1)
        ocase = None
        if others or len(cpu) < cpu_updates:
            bonds, sites, centre = a.get_state()
            for key, b in others.items():
                b.set_state(bonds, sites, centre)
                timed(b, i, key)
            if len(cpu) < cpu_updates:
                ocase = _oracle_on_state(bonds, sites, centre, i, okraus, d, chi)
            del sites
        ginf = timed(a, i, "fp64")
        if ocase is not None:
            osec, oinf = ocase
            cpu.append({"bond": i, "seconds": osec, "kept": oinf["kept"], "gpu_kept": ginf["kept"],
                        "rel_err_trace_before": abs(ginf["trace_before"] - oinf["trace_before"]) / abs(oinf["trace_before"]),
                        "rel_err_xi_before": abs(ginf["xi_before"] - oinf["xi_before"]) / abs(oinf["xi_before"]),
                        "rel_err_trace_after": abs(ginf["trace_after"] - oinf["trace_after"]) / abs(oinf["trace_after"]),
                        "abs_err_discarded_weight": abs(ginf["discarded_weight"] - oinf["discarded_weight"]),
                        "oracle_gap_at_cut": oinf["gap_at_cut"], "gpu_sigma_gap_at_cut": ginf["sigma_gap_at_cut"]})
        if others:
            oa = circuits.observables(a)
            for key, b in others.items():
                ob = circuits.observables(b)
                errs_e[key].append(abs(oa["energy_per_site"] - ob["energy_per_site"]))
                errs_p[key].append(float(np.max(np.abs(oa["populations"] - ob["populations"]))))
    res = {}
    for key in acc:
        t, prof = acc[key]["t"], acc[key]["prof"]
        if not t:
            continue
        tot = float(np.sum(t))
        # split-BF16: three BF16 products per real product, judged against a third of the BF16 peak
        peak = {"fp64": PEAK["fp64_mfma"], "fp32": PEAK["fp32_mfma"], "bf16x3": PEAK["bf16_mfma"] / 3}[key]
        fam_rec = {}
        for f in fams:
            v = prof[f]
            if not v["launches"]:
                continue
            r = {"launches": v["launches"], "ms": v["ms"], "share_of_update_time": 1e-3 * v["ms"] / tot}
            if f in ("theta", "gemm"):
                r["flop"] = v["flops"]
                r["tflops"] = v["flops"] / (1e-3 * v["ms"]) / 1e12 if v["ms"] else 0.0
                # the gemm family mixes split-BF16 products with plain FP32 ones in bf16x3 mode
                r["frac_of_peak"] = r["tflops"] / (peak if f == "theta" or key != "bf16x3" else PEAK["fp32_mfma"])
            fam_rec[f] = r
        th = prof["theta"]
        res[key] = {
            "saturated_updates": len(t),
            "updates_per_s": len(t) / tot,
            "ms_per_update": 1e3 * tot / len(t),
            "kept": acc[key]["kept"],
            "families": fam_rec,
            # algorithmic a2 work per update at chi = 512, d = 4: merge 2.75e11 + gate 1.37e11 flop
            "theta_contraction": {"flop_per_update_algorithmic": 4.12e11,
                                  "ms_per_update": th["ms"] / len(t),
                                  "tflops": th["flops"] / (1e-3 * th["ms"]) / 1e12 if th["ms"] else 0.0,
                                  "peak_tflops": peak,
                                  "frac": (th["flops"] / (1e-3 * th["ms"]) / 1e12 / peak) if th["ms"] else 0.0},
            # every executed product (theta, subspace passes, Grams, rebuild) over the update time
            "gemm_executed_tflops_per_update_time": (prof["gemm"]["flops"] + th["flops"]) / tot / 1e12,
            "mfma_algorithmic_tflops_per_update_time": 2.9e12 * len(t) / tot / 1e12,
        }
    a.close()
    for b in others.values():
        b.close()
    if cpu:
        vendor, threads = _blas()
        res["cpu_oracle"] = {"updates": cpu, "seconds_per_update": float(np.mean([c["seconds"] for c in cpu])),
                             "cores": threads, "blas": vendor,
                             "note": "the CPU oracle (numpy/LAPACK SVD of the 8192 x 8192 theta) on the same "
                                     "saturated updates, from the FP64 GPU chain; its cut record beside the GPU's"}
    out = {"workload": f"noisy QAOA gate set, N={n} atoms, d=4, chi_max={chi}, seed 0, rates 1e-3: FP64 layers "
                       f"until the centre bonds reach {chi} ({warm} layers), the even bonds of the next; then each "
                       f"odd-bond update with chi_l = chi_m = chi_r = {chi} run from the same state in FP64, "
                       f"FP32 and split-BF16 (state loaded with mpdo_set_state)",
           "untimed_layers": warm, **res}
    for key in others:
        if "fp64" in res and key in res:
            out[f"{key}_speedup_vs_fp64"] = res["fp64"]["ms_per_update"] / res[key]["ms_per_update"]
            out[f"{key}_theta_speedup_vs_fp64"] = (res["fp64"]["theta_contraction"]["ms_per_update"] /
                                                   res[key]["theta_contraction"]["ms_per_update"])
            out[f"{key}_abs_err_energy_per_site_vs_fp64_max"] = max(errs_e[key])
            out[f"{key}_abs_err_populations_vs_fp64_max"] = max(errs_p[key])
    return out


def _pulse_gate(n_steps: int) -> dict:
    """The pulse-level gate builder on the paper's Gaussian CZ pulse (d=4, dissipation 0.001/T,
    branching 1/16, 1/16, 7/8): wall time of one call, host in and host out."""
    from paper_2309_08572_amd import pulse
    gd = 0.001 / 2.165
    pulse.gaussian_cz(n_steps=64, gamma_diss=gd)            # load and warm up
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        pulse.gaussian_cz(n_steps=n_steps, gamma_diss=gd)
        times.append(time.perf_counter() - t0)
    t = sorted(times)[1]
    return {"workload": "Gaussian CZ pulse T=2.165 us, d=4, 256 basis inputs, gamma_diss=0.001/T",
            "steps": n_steps, "ms_per_channel": 1e3 * t, "us_per_step": 1e6 * t / n_steps}


def _crosstalk(layers: int) -> dict:
    """The crosstalk gate on the benchmark chain (N=100, d=4, chi_max=512, FP64): every Ising
    block of the first `layers` QAOA layers is applied as a crosstalk gate whose four pair
    unitaries add a phase phi (a n_i + b n_{i+1}) on the Rydberg level 2 (n = |2><2|) of the
    driven atoms when the left (a) or right (b) neighbour is in level 2, the blockade's detuning
    shift over the block; the block's leak is queued on its two atoms, the mixer and the
    single-atom noise follow as in the benchmark.  The first layer is untimed (it also
    allocates the gate's block buffers); the others are timed."""
    import numpy as np
    from paper_2309_08572_amd import circuits
    from paper_2309_08572_amd.mpdo import MPDO, MPDO_FP64
    from workloads import config_m3
    spec = config_m3(0)
    n, d, phi = spec.n, spec.d, 0.3
    nr = np.zeros(d)
    nr[2] = 1.0
    m = MPDO(n, d, spec.chi, precision=MPDO_FP64)
    m.init_product_state([circuits.plus_rho(d)] * n)
    timed_s, timed_gates = 0.0, 0
    for k in range(min(layers, spec.p)):
        zz = circuits.zz_gate(spec.gamma[k], d)
        u4 = [np.diag(np.exp(-1j * phi * (a * np.kron(nr, np.ones(d)) + b * np.kron(np.ones(d), nr)))) @ zz
              for b in (0, 1) for a in (0, 1)]
        lk = circuits.leak_kraus(spec.p_leak, d)
        t0 = time.perf_counter()
        for i in circuits.bond_order(n):
            m.apply_gate_crosstalk(i, 2, u4)
            m.apply_channel(i, lk)
            m.apply_channel(i + 1, lk)
        for j in range(n):
            m.apply_channel(j, [circuits.x_rotation(spec.beta[k], d)])
            m.apply_channel(j, circuits.dephasing_kraus(spec.p_deph, d))
            m.apply_channel(j, circuits.decay_kraus(spec.p_decay, d))
        tr = m.trace()
        if k > 0:
            timed_s += time.perf_counter() - t0
            timed_gates += n - 1
    bonds = m.bond_dims()
    m.close()
    return {"workload": "noisy QAOA chain N=100, d=4, chi_max=512, Ising blocks as crosstalk gates "
                        "(Rydberg level 2, phase 0.3 per neighbour class), FP64",
            "timed_layers": max(0, min(layers, spec.p) - 1), "crosstalk_updates": timed_gates,
            "updates_per_s": timed_gates / timed_s if timed_s > 0 else 0.0,
            "ms_per_update": 1e3 * timed_s / timed_gates if timed_gates else 0.0,
            "max_bond": max(bonds), "trace": [tr.real, tr.imag]}


PEAK = {"fp64_mfma": 78.6, "fp32_mfma": 157.3, "bf16_mfma": 2500.0, "fp64_vector": 78.6, "hbm_gbs": 8000.0}


# The GEMM families' kernels carry their own event stamps (hipExtLaunchKernelGGL), so their
# per-launch average is kernel execution time at any length.  For the other families an event
# pair around a launch also times its dispatch (~10 us here), so their average is a kernel
# duration only for launches well above that.  The roofline kernel is the family with the most
# event time among the stamped families and those averaging >= MIN_LAUNCH_US per launch.
STAMPED_FAMILIES = ("gemm", "theta", "split_sum")
MIN_LAUNCH_US = 50.0


# HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE on the FP64 run of
# this workload, each counter scaled by what it reads for a plain 256 MiB device copy (fetch
# x 2.00, write x 1.00).  Valid only for the kernel source it was taken on: the entry names the
# file and the first 16 hex digits of its SHA-256, and traffic is null when the file differs.
TRAFFIC = {
    # the complex GEMM kernels of the FP64 command (36562 dispatches, 32 x 32 tiles; plain and
    # with operand transforms): FETCH_SIZE 396.89 KiB, WRITE_SIZE 308.29 KiB per dispatch.  The
    # writes hold the k-split partial tiles, the fetches the A and B panels read once per XCD
    "gemm": {"source": "paper_2309_08572_amd/csrc/gemm.hip", "sha256_16": "75cf86fb53f0c4b7",
             "bytes_per_launch": 1128412.0},
    # the timed family is the on-chip reduction of the core splits (orders 33..192; the range
    # bases take the pivoted Cholesky, the gate factorisations are cached after the warm-up):
    # 486 dispatches, FETCH_SIZE 73.96 KiB, WRITE_SIZE 54.04 KiB
    "tri_reduce": {"source": "paper_2309_08572_amd/csrc/tri.hip", "sha256_16": "72a41ec2d3e706d8",
                   "bytes_per_launch": 206784.0},
    # all pivoted-Cholesky launches of the FP64 command (2486 dispatches over the three order
    # classes): FETCH_SIZE 29.47 KiB, WRITE_SIZE 41.72 KiB per dispatch
    "pchol": {"source": "paper_2309_08572_amd/csrc/pchol.hip", "sha256_16": "fb8cff16ca15d597",
              "bytes_per_launch": 103064.0},
}


def _traffic(fam: str):
    import hashlib
    t = TRAFFIC.get(fam)
    if t is None:
        return None
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), t["source"])
    try:
        h = hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    return t["bytes_per_launch"] if h == t["sha256_16"] else None


def roofline_family(prof: dict) -> str:
    """The dominant long-launch kernel family of a profiled step."""
    long_fams = [k for k, v in prof.items() if v["launches"] and
                 (k in STAMPED_FAMILIES or 1e3 * v["ms"] / v["launches"] >= MIN_LAUNCH_US)]
    return max(long_fams or list(prof), key=lambda k: prof[k]["ms"])


def roofline_of(prof: dict, fam: str, fp64: bool) -> dict:
    """Roofline entry for kernel family `fam` from HIP events recorded over the timed steps."""
    d = prof[fam]
    n = max(1, d["launches"])
    avg_s = d["ms"] * 1e-3 / n
    flop, byts = d["flops"] / n, d["bytes"] / n
    if fam in ("gemm", "theta", "eig_rotate"):
        peak = PEAK["fp64_mfma"] if (fp64 or fam == "eig_rotate") else PEAK["fp32_mfma"]
        ach = flop / avg_s / 1e12 if avg_s > 0 else 0.0
        rf = {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s"}
    elif fam in ("transfer", "phys"):
        ach = byts / avg_s / 1e9 if avg_s > 0 else 0.0
        rf = {"bound": "hbm", "achieved": ach, "peak": PEAK["hbm_gbs"], "unit": "GB/s"}
    else:
        ach = flop / avg_s / 1e12 if avg_s > 0 else 0.0
        rf = {"bound": "alu", "achieved": ach, "peak": PEAK["fp64_vector"], "unit": "TFLOP/s"}
    rf["frac"] = rf["achieved"] / rf["peak"]
    if fam in ("tri_reduce", "eig_small", "pchol"):
        # one workgroup on one of the 256 compute units: its own FP64 ceiling is peak / 256
        rf["workgroups"] = 1
        rf["frac_of_one_cu"] = rf["achieved"] / (rf["peak"] / 256.0)
    rf["traffic"] = _traffic(fam)
    rf["kernel_family"] = fam
    rf["launches"] = d["launches"]
    rf["avg_launch_us"] = avg_s * 1e6
    rf["per_launch"] = {"flop": flop, "bytes": byts}
    return rf


def _truncation_summary(infos, obs) -> dict:
    """Per-update truncation records of one circuit (mpdo_trunc_info), summarised: discarded
    weight (1 - sum of the kept Lambda^2 over |Lambda|^2, per update), the trace drift of each
    cut (PPT keeps xi = tr rho^2 / (tr rho)^2, not the trace) and how well xi was kept."""
    dw = [i["discarded_weight"] for i in infos]
    tdrift = [abs(i["trace_after"] - i["trace_before"]) / abs(i["trace_before"])
              for i in infos if i["trace_before"] != 0.0]
    xdrift = [abs(i["xi_after"] - i["xi_before"]) / abs(i["xi_before"])
              for i in infos if i["xi_before"] != 0.0]
    tr = obs["trace"]
    return {"updates": len(infos), "updates_truncated": int(sum(1 for x in dw if x > 0.0)),
            "discarded_weight_sum": float(sum(dw)), "discarded_weight_max": float(max(dw) if dw else 0.0),
            "trace_drift_per_update_max": float(max(tdrift) if tdrift else 0.0),
            "trace_drift_circuit": float(abs(complex(tr) - 1.0)),
            "xi_rel_change_per_update_max": float(max(xdrift) if xdrift else 0.0),
            "ppt_infeasible": int(sum(1 for i in infos if not i["ppt_feasible"])),
            "updates_recomputed": int(sum(i.get("retried", 0) for i in infos))}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--n", type=int, default=100)
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16x3", "both"], default="both")
    ap.add_argument("--cpu-baseline-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-circuits", type=int, default=256,
                    help="also time this many circuits of the 256-circuit batch workload "
                         "(on worker streams vs one at a time; all 256 take about a minute)")
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--saturated-layers", type=int, default=8,
                    help="at most this many untimed layers before the saturated chi=512 updates are timed "
                         "(0: skip that leg)")
    ap.add_argument("--saturated-only", action="store_true",
                    help="run only the saturated chi=512 leg and print its record (for profiling)")
    ap.add_argument("--cpu-saturated", type=int, default=0,
                    help="also run the CPU oracle on this many of the saturated chi=512 updates (minutes each)")
    ap.add_argument("--crosstalk-layers", type=int, default=3,
                    help="layers of the crosstalk-gate leg (the first is untimed); 0 skips it")
    ap.add_argument("--second-order-reps", type=int, default=3,
                    help="time the second-order observables this many times each on the final state (0: skip)")
    ap.add_argument("--pulse-steps", type=int, default=20000,
                    help="also time the pulse-level CZ gate builder with this many steps (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (this build runs "
              f"the update on a single MI355X)", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2309_08572_amd import circuits, mpdo
    from workloads import config_m3

    spec = config_m3(args.seed, n=args.n)
    updates = spec.n_two_site_updates()
    modes = {"fp64": mpdo.MPDO_FP64, "fp32": mpdo.MPDO_FP32, "bf16x3": mpdo.MPDO_BF16X3}
    run = ["fp64", "fp32"] if args.precision == "both" else [args.precision]
    # the saturated leg also times the split-BF16 mode (it differs from FP32 only in the products
    # with theta, which the circuit's factored updates never form)
    sat_run = run + ["bf16x3"] if args.precision == "both" else run
    if args.saturated_only:
        print(json.dumps({"saturated": _saturated(max(1, args.saturated_layers), sat_run, args.cpu_saturated)}))
        return 0
    results = {}
    for name in run:
        m = mpdo.MPDO(spec.n, spec.d, spec.chi, precision=modes[name])
        for _ in range(args.warmup):
            circuits.run_circuit(spec, m=m)
            circuits.observables(m)
        # One untimed step with an event pair around every launch gives the per-family breakdown
        # and picks the roofline family.  Event pairs cost host time at every launch they bracket
        # (a quarter of the step when all ~170 launches of an update carry them), so the timed
        # steps record events only around the roofline family's launches.
        # The same untimed step collects each update's truncation record (a host read per update).
        m.profile(True)
        infos = []
        torch.cuda.synchronize()
        tp = time.perf_counter()
        circuits.run_circuit(spec, m=m, infos=infos)
        obs_p = circuits.observables(m)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp
        prof = m.profile_read()
        fam = roofline_family(prof)
        m.profile_families([fam])
        # a stamped family has many short launches: stamp about two per update (every
        # stride-th launch), so the timed steps run almost as without any events
        stride = max(1, round(prof[fam]["launches"] / (2.0 * updates))) if fam in STAMPED_FAMILIES else 1
        m.profile_stride(stride)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            circuits.run_circuit(spec, m=m)
            obs = circuits.observables(m)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof_timed = m.profile_read()
        m.profile(False)
        results[name] = {"seconds": dt, "obs": obs, "prof": prof, "profiled_seconds": tp, "fam": fam, "stride": stride,
                         "truncation": _truncation_summary(infos, obs_p),
                         "prof_timed": prof_timed, "bonds": max(m.bond_dims())}
        m.close()

    main_mode = "fp64" if "fp64" in results else run[0]
    r = results[main_mode]
    ms = 1e3 * r["seconds"] / args.steps
    value = updates * args.steps / r["seconds"]
    out = {
        "metric": "MPDO 2-site updates/s + TFLOP/s at N=100 chi=512, FP32-MFMA vs FP64, same error",
        "value": value,
        "unit": "two-site updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_mode == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"noisy QAOA circuit, N={spec.n} atoms, d=4, chi_max={spec.chi}, "
                               f"p={spec.p}, noise 1e-3, seed {args.seed}",
                   "n": spec.n, "d": spec.d, "chi_max": spec.chi, "p": spec.p,
                   "updates_per_step": updates, "max_bond_reached": r["bonds"]},
    }
    # executed product flop (every GEMM the update ran, theta included) over their event time
    gf = r["prof"]["gemm"]["flops"] + r["prof"]["theta"]["flops"]
    gms = r["prof"]["gemm"]["ms"] + r["prof"]["theta"]["ms"]
    out["tflops_gemm_executed"] = (gf / (1e-3 * gms) / 1e12) if gms else 0.0
    out["roofline"] = roofline_of(r["prof_timed"], r["fam"], main_mode == "fp64")
    out["roofline"]["sampled_one_launch_in"] = r["stride"]
    # the breakdown below comes from the untimed profiled step (events around every launch)
    out["kernel_time_share"] = {k: v["ms"] / (1e3 * r["profiled_seconds"]) for k, v in r["prof"].items()
                                if isinstance(v, dict) and "ms" in v}
    out["kernel_families"] = {k: {"launches": v["launches"], "ms": v["ms"],
                                  "avg_launch_us": 1e3 * v["ms"] / v["launches"] if v["launches"] else 0.0,
                                  "flop": v["flops"], "bytes": v["bytes"]}
                              for k, v in r["prof"].items() if v["launches"]}
    if "fp32" in results and "fp64" in results:
        a, b = results["fp64"]["obs"], results["fp32"]["obs"]
        out["fp32"] = {
            "updates_per_s": updates * args.steps / results["fp32"]["seconds"],
            "speedup_vs_fp64": results["fp64"]["seconds"] / results["fp32"]["seconds"],
            "abs_err_energy_per_site_vs_fp64": abs(a["energy_per_site"] - b["energy_per_site"]),
            "abs_err_populations_vs_fp64": float(np.max(np.abs(a["populations"] - b["populations"]))),
        }
    out["truncation"] = r["truncation"]
    if "fp32" in results and "fp64" in results:
        out["fp32"]["truncation"] = results["fp32"]["truncation"]
    out["observables"] = {"energy_per_site": r["obs"]["energy_per_site"],
                          "p_success": r["obs"]["p_success"],
                          "trace": [r["obs"]["trace"].real, r["obs"]["trace"].imag]}
    if args.batch_circuits > 0:
        out["batch"] = _batch(args.batch_circuits, args.workers)
    if args.pulse_steps > 0:
        out["pulse_gate"] = _pulse_gate(args.pulse_steps)
    if args.saturated_layers > 0:
        out["saturated"] = _saturated(args.saturated_layers, sat_run, args.cpu_saturated)
    if args.second_order_reps > 0:
        try:
            out["second_order"] = _second_order(spec, args.second_order_reps)
        except Exception as e:   # reported in the record; the headline measurement stands
            out["second_order"] = {"error": str(e)}
    if args.crosstalk_layers > 0:
        try:
            out["crosstalk"] = _crosstalk(args.crosstalk_layers)
        except Exception as e:   # a rejected gate (bond too large for chi_max) is reported, not fatal
            out["crosstalk"] = {"error": str(e)}
    if not args.no_cpu_baseline:
        from workloads import config_m0, config_m1
        out["cpu_baseline"] = _cpu_baseline(spec, args.cpu_baseline_seconds,
                                            small_specs=(("m0_n6_d3_p1", config_m0(0)),
                                                         ("m1_n40_d4_p2_chi128", config_m1(0))))
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
