"""CPU checks of the C-ABI boundary: the library loads and exports every declared symbol,
config validation rejects bad input without touching a GPU, and the product-side circuit
inputs are valid channels in the serpentine order.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpdo.h")
MLP_HEADER = os.path.join(ROOT, "include", "mpdo_mlp.h")
PULSE_HEADER = os.path.join(ROOT, "include", "mpdo_pulse.h")


def _declared_symbols(path=HEADER):
    text = open(path).read()
    return sorted(set(re.findall(r"\b(mpdo_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2309_08572_amd import mpdo
    if not os.path.exists(mpdo.library_path()):
        pytest.skip("libmpdo.so not built (run __graft_entry__.build())")
    return mpdo.load_library()


def test_header_declares_the_paper_calls():
    names = _declared_symbols()
    for want in ("mpdo_init_product_state", "mpdo_apply_gate", "mpdo_apply_channel",
                 "mpdo_truncate", "mpdo_expect"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for path in (HEADER, MLP_HEADER, PULSE_HEADER):
        for name in _declared_symbols(path):
            assert hasattr(lib, name), name


def test_surrogate_binding_covers_its_header(lib):
    from paper_2309_08572_amd import surrogate
    assert sorted(surrogate.EXPORTS) == _declared_symbols(MLP_HEADER)


def test_pulse_binding_covers_its_header(lib):
    from paper_2309_08572_amd import pulse
    assert sorted(pulse.EXPORTS) == _declared_symbols(PULSE_HEADER)


def test_pulse_argument_checks_without_gpu(lib):
    """Parameter checks happen before any device call."""
    from paper_2309_08572_amd import pulse
    lib = pulse._lib()
    om = np.zeros(4)
    out = np.zeros(2 * 256 * 256)
    dp = C.POINTER(C.c_double)

    def call(**kw):
        base = dict(d=4, n_steps=4, tau=0.1, blockade=1.0, gamma_diss=0.0, branch=(0.0, 0.0, 0.0), gamma_deph=0.0)
        base.update(kw)
        p = pulse.PulseParams(base["d"], base["n_steps"], base["tau"], base["blockade"], base["gamma_diss"],
                              (C.c_double * 3)(*base["branch"]), base["gamma_deph"])
        return lib.mpdo_pulse_channel(C.byref(p), om.ctypes.data_as(dp), om.ctypes.data_as(dp),
                                      out.ctypes.data_as(dp), None)
    assert call(d=5) == 1
    assert call(n_steps=0) == 1
    assert call(tau=0.0) == 1
    assert call(tau=float("nan")) == 1
    assert call(gamma_diss=-1.0) == 1
    assert call(d=3, branch=(0.5, 0.4, 0.1)) == 1
    assert b"d = 4" in lib.mpdo_pulse_last_error()


def test_mlp_argument_checks_without_gpu(lib):
    """Size checks happen before any device call."""
    ip = C.POINTER(C.c_int)
    h = C.c_void_p()
    lib.mpdo_mlp_create.argtypes = [C.c_int, ip, C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]
    bad_widths = (C.c_int * 3)(4, 0, 2)
    assert lib.mpdo_mlp_create(2, bad_widths, 8, None, C.byref(h)) == 1
    ok_widths = (C.c_int * 3)(4, 8, 2)
    assert lib.mpdo_mlp_create(2, ok_widths, 0, None, C.byref(h)) == 1
    lib.mpdo_mlp_param_count.argtypes = [C.c_int, ip]
    lib.mpdo_mlp_param_count.restype = C.c_size_t
    assert lib.mpdo_mlp_param_count(2, ok_widths) == 8 * 4 + 8 + 2 * 8 + 2


def test_binding_covers_header(lib):
    from paper_2309_08572_amd import mpdo
    assert sorted(mpdo.EXPORTS) == _declared_symbols()


def test_config_validation_without_gpu(lib):
    from paper_2309_08572_amd.mpdo import Config
    ctx = C.c_void_p()
    bad = [Config(1, 4, 8, 0, 0.0, 1, 0, None), Config(4, 5, 8, 0, 0.0, 1, 0, None),
           Config(4, 4, 0, 0, 0.0, 1, 0, None), Config(4, 4, 8, 7, 0.0, 1, 0, None),
           Config(4, 4, 8, 0, 2.0, 1, 0, None)]
    for cfg in bad:
        assert lib.mpdo_create(C.byref(cfg), C.byref(ctx)) == 1
        assert lib.mpdo_last_error(None)
    good = Config(6, 3, 81, 0, 0.0, 1, 0, None)
    assert lib.mpdo_create(C.byref(good), C.byref(ctx)) == 0
    assert lib.mpdo_workspace_bytes(C.byref(good)) > 0
    # calls that need a state refuse cleanly before init (no device work)
    rho = np.zeros((6, 3, 3), dtype=np.complex128)
    out = np.zeros(2)
    assert lib.mpdo_trace(ctx, out.ctypes.data_as(C.POINTER(C.c_double))) == 2
    assert lib.mpdo_destroy(ctx) == 0


def test_product_kraus_inputs_are_channels():
    from paper_2309_08572_amd import circuits as pc
    for d in (3, 4):
        for ks in (pc.leak_kraus(0.01, d), pc.dephasing_kraus(0.2, d), pc.decay_kraus(0.3, d),
                   [pc.x_rotation(0.7, d)], pc.block_kraus(1.1, 0.02, d)):
            dim = ks[0].shape[0]
            np.testing.assert_allclose(sum(k.conj().T @ k for k in ks), np.eye(dim), atol=1e-14)
    assert pc.bond_order(6) == [0, 2, 4, 3, 1]
    assert pc.bond_order(7) == [0, 2, 4, 5, 3, 1]


def test_eigh_and_profile_stride_argument_checks_without_gpu(lib):
    """mpdo_eigh and mpdo_profile_stride refuse bad arguments before any device work."""
    from paper_2309_08572_amd.mpdo import Config
    dp = C.POINTER(C.c_double)
    H = np.eye(2, dtype=np.complex128)
    ev = np.zeros(2)
    V = np.zeros((2, 2), dtype=np.complex128)
    m = C.c_int(-1)

    def eigh(n, tau, cap):
        return lib.mpdo_eigh(n, H.ctypes.data_as(dp), tau, cap, C.byref(m), ev.ctypes.data_as(dp),
                             V.ctypes.data_as(dp))
    for n, tau, cap in [(0, 0.0, 0), (1025, 0.0, 1), (2, -1.0, 2), (2, float("nan"), 2), (2, 0.0, 3),
                        (2, 0.0, -1)]:
        assert eigh(n, tau, cap) == 1, (n, tau, cap)
        assert lib.mpdo_last_error(None)
    assert eigh(2, 0.0, 0) == 0 and m.value == 0          # nothing asked for: no device work
    ctx = C.c_void_p()
    good = Config(6, 3, 81, 0, 0.0, 1, 0, None)
    assert lib.mpdo_create(C.byref(good), C.byref(ctx)) == 0
    assert lib.mpdo_profile_stride(ctx, 0) == 1
    assert lib.mpdo_profile_stride(ctx, 4) == 0             # not recording: no effect
    assert lib.mpdo_profile_enable_mask(ctx, 1) == 0
    assert lib.mpdo_profile_stride(ctx, 4) == 0
    assert lib.mpdo_profile_enable_mask(ctx, 0) == 0
    assert lib.mpdo_destroy(ctx) == 0
