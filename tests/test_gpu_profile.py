"""The context's kernel timing (instrumentation): the GEMM families carry event stamps attached
to the kernels themselves, and mpdo_profile_stride samples one launch in N of them.  On an
M1-shaped N=16 circuit (after a warm-up run of the same circuit on the same context): every
family's launches are counted, a stamped GEMM launch averages a kernel-like duration
(1 us .. 1 ms), and with stride 8 the GEMM family counts about an eighth of the launches of
the fully stamped run while the unrecorded families count none."""
import pytest

from workloads import config_m1

pytestmark = pytest.mark.gpu


def test_gemm_stamps_and_sampling():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08572_amd import circuits, mpdo
    spec = config_m1(0, n=16)
    print("[gpu] profile stamps on M1-shaped N=16", flush=True)
    m = mpdo.MPDO(spec.n, spec.d, spec.chi)
    circuits.run_circuit(spec, m=m)
    m.profile(True)
    circuits.run_circuit(spec, m=m)
    full = m.profile_read()
    n_g = full["gemm"]["launches"]
    assert n_g > 100
    avg_us = 1e3 * full["gemm"]["ms"] / n_g
    assert 1.0 < avg_us < 1000.0, avg_us
    assert full["gemm"]["flops"] > 0 and full["gemm"]["bytes"] > 0
    m.profile_families(["gemm"])
    m.profile_stride(8)
    circuits.run_circuit(spec, m=m)
    samp = m.profile_read()
    m.profile(False)
    print(f"[gpu] gemm launches {n_g} stamped, {samp['gemm']['launches']} sampled (1 in 8), "
          f"{avg_us:.2f} us per launch", flush=True)
    assert abs(samp["gemm"]["launches"] - n_g / 8.0) <= 0.05 * n_g / 8.0 + 2
    assert samp["pchol"]["launches"] == 0 and samp["tri_reduce"]["launches"] == 0
    assert 1.0 < 1e3 * samp["gemm"]["ms"] / samp["gemm"]["launches"] < 1000.0
    m.close()
