"""GPU test of the allocation-free pulse-channel entry point (mpdo_pulse_channel_noalloc, through
the C ABI): its buffers come from a fixed per-device scratch block instead of hipMalloc, and it
must give the same channel as mpdo_pulse_channel (FP64, the same kernels: 1e-12 of the largest
entry), on two calls in a row, the second with a smaller input, and reject a step count beyond
the block with E_ARG before any device work."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08572_amd import mpdo, pulse
    return mpdo, pulse


def _noisy_pulse(n_steps, d):
    from paper_2309_08572_amd import pulse
    two_pi = 2.0 * np.pi
    om, de, tau = pulse.gaussian(2.165, two_pi * 17.0, two_pi * -14.7, n_steps)
    branch = (1.0 / 16, 1.0 / 16, 7.0 / 8) if d == 4 else (0.5, 0.5, 0.0)
    return dict(omega=om, delta=de, tau=tau, d=d, blockade=two_pi * 60.0, gamma_diss=0.01,
                branch=branch, gamma_deph=0.02)


@pytest.mark.parametrize("first,second", [((9000, 4), (1500, 4)), ((6000, 4), (700, 3))])
def test_noalloc_channel_matches_the_allocating_entry_point(first, second):
    mpdo, pulse = _gpu()
    for n_steps, d in (first, second):
        print(f"[gpu] pulse channel no-alloc vs alloc: {n_steps} steps, d={d}", flush=True)
        kw = _noisy_pulse(n_steps, d)
        ref = pulse.channel(**kw)
        got = pulse.channel(**kw, noalloc=True)
        err = float(np.max(np.abs(got - ref)))
        print(f"[gpu] max |diff| = {err:.2e} (max |entry| {np.max(np.abs(ref)):.3f})", flush=True)
        assert np.all(np.isfinite(got))
        assert err <= 1e-12 * np.max(np.abs(ref))


def test_noalloc_rejects_a_step_count_beyond_its_scratch():
    mpdo, pulse = _gpu()
    kw = _noisy_pulse(131073, 4)
    print("[gpu] pulse channel no-alloc: 131073 steps must be rejected", flush=True)
    with pytest.raises(mpdo.MpdoError, match="too large"):
        pulse.channel(**kw, noalloc=True)
    # the limit itself is accepted and agrees with the allocating call
    kw = _noisy_pulse(131072, 4)
    got = pulse.channel(**kw, noalloc=True)
    ref = pulse.channel(**kw)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
