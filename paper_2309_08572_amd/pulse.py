"""Binding of the pulse-level two-atom gate builder (include/mpdo_pulse.h): the channel of one
laser pulse on a pair of atoms, integrated on the GPU from the Lindblad master equation by
Trotterised steps (Sec. II; Sec. III.A), in the layout mpdo_apply_gate takes.

Pulse shapes (Fig. 1 caption) are sampled here at the step midpoints; the time integration is
the library's kernel.  Frequencies and rates are angular (radians per time unit): the paper's
values in MHz are Omega/2pi, so they enter multiplied by 2 pi, with time in microseconds.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import mpdo

EXPORTS = ("mpdo_pulse_channel", "mpdo_pulse_channel_noalloc", "mpdo_pulse_last_error")


class PulseParams(C.Structure):
    _fields_ = [("d", C.c_int), ("n_steps", C.c_int), ("tau", C.c_double), ("blockade", C.c_double),
                ("gamma_diss", C.c_double), ("branch", C.c_double * 3), ("gamma_deph", C.c_double)]


def _lib():
    lib = mpdo.load_library()
    if not getattr(lib, "_pulse_bound", False):
        dp = C.POINTER(C.c_double)
        lib.mpdo_pulse_channel.argtypes = [C.POINTER(PulseParams), dp, dp, dp, C.c_void_p]
        lib.mpdo_pulse_channel.restype = C.c_int
        lib.mpdo_pulse_channel_noalloc.argtypes = [C.POINTER(PulseParams), dp, dp, dp, C.c_void_p]
        lib.mpdo_pulse_channel_noalloc.restype = C.c_int
        lib.mpdo_pulse_last_error.argtypes = []
        lib.mpdo_pulse_last_error.restype = C.c_char_p
        lib._pulse_bound = True
    return lib


def channel(omega, delta, tau: float, d: int = 4, blockade: float = 0.0, gamma_diss: float = 0.0,
            branch=(1.0 / 16, 1.0 / 16, 7.0 / 8), gamma_deph: float = 0.0, noalloc: bool = False) -> np.ndarray:
    """The pulse's two-atom channel: (d^4 x d^4) complex, rows eta_1 d^2 + eta_2 (per-atom
    vectorised index eta = sigma d + sigma'), ready for MPDO.apply_gate.  omega/delta: values at
    the middle of each of the len(omega) steps of length tau.  The default branching ratios are
    the paper's (1/16, 1/16, 7/8); with d = 3 the dark branch must be 0.  noalloc: use the entry
    point that allocates no device memory (fixed per-device scratch; see mpdo_pulse.h)."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the pulse channel is integrated on the GPU; no CPU fallback exists")
    om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
    de = np.ascontiguousarray(np.asarray(delta, dtype=np.float64))
    if om.shape != de.shape or om.ndim != 1:
        raise ValueError("omega and delta must be 1-D arrays of equal length")
    br = tuple(float(b) for b in branch)
    p = PulseParams(int(d), int(om.size), float(tau), float(blockade), float(gamma_diss),
                    (C.c_double * 3)(*br), float(gamma_deph))
    m2 = d ** 4
    out = np.zeros((m2, m2), dtype=np.complex128)
    lib = _lib()
    dp = C.POINTER(C.c_double)
    fn = lib.mpdo_pulse_channel_noalloc if noalloc else lib.mpdo_pulse_channel
    st = fn(C.byref(p), om.ctypes.data_as(dp), de.ctypes.data_as(dp), out.ctypes.data_as(dp), None)
    if st != 0:
        msg = lib.mpdo_pulse_last_error()
        raise mpdo.MpdoError(st, msg.decode() if msg else "")
    return out


def gaussian(T: float, omega_max: float, delta: float, n_steps: int):
    """Gaussian pulse (Fig. 1 caption): Omega(t) = Omega_max [exp(-(t - t0)^2 / v^2) - a] / (1 - a)
    with v = 0.1 T, t0 = T/2, a = exp(-(t0/v)^2), Delta constant.  Returns (omega, delta, tau)
    sampled at the step midpoints."""
    tau = T / n_steps
    t = (np.arange(n_steps) + 0.5) * tau
    v, t0 = 0.1 * T, 0.5 * T
    a = math.exp(-(t0 / v) ** 2)
    om = omega_max * (np.exp(-((t - t0) / v) ** 2) - a) / (1.0 - a)
    return om, np.full(n_steps, float(delta)), tau


def gaussian_cz(n_steps: int = 20000, gamma_diss: float = 0.0, gamma_deph: float = 0.0, d: int = 4) -> np.ndarray:
    """The paper's Gaussian CZ pulse: T = 2.165 us, Omega_max/2pi = 17 MHz, Delta/2pi = -14.7 MHz,
    B/2pi = 60 MHz, branching (1/16, 1/16, 7/8); rates in 1/us."""
    two_pi = 2.0 * math.pi
    om, de, tau = gaussian(2.165, two_pi * 17.0, two_pi * -14.7, n_steps)
    branch = (1.0 / 16, 1.0 / 16, 7.0 / 8) if d == 4 else (0.5, 0.5, 0.0)
    return channel(om, de, tau, d=d, blockade=two_pi * 60.0, gamma_diss=gamma_diss, branch=branch,
                   gamma_deph=gamma_deph)
