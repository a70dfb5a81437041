"""Pure-state QAOA on qubits (the noiseless limit), plain numpy statevector.

Eq. (tfim_model): |psi> -> prod_k exp(i alpha_k H_z) exp(i beta_k H_t) |psi_0>, with
H_z = sum_<ij> S^z_i S^z_j + b sum_i S^z_i, H_t = sum_i S^x_i, |psi_0> = |+>^N
(Sec. IV), open chain.  Reading adopted (pinned by Table II): S are Pauli matrices and,
in time order, layer k applies exp(i alpha_k H_z) first and exp(i beta_k H_t) second.
The energy is that of Eq. (tfim_hamiltonian), H = -J (H_z) - g H_t with J = 1.
"""
from __future__ import annotations

import numpy as np


def _z_diag(n: int):
    """z[i][x] = +1 if bit i of basis state x is 0 else -1 (site 0 is the slowest index)."""
    x = np.arange(2 ** n)
    return [1.0 - 2.0 * ((x >> (n - 1 - i)) & 1) for i in range(n)]


def _apply_rx_all(psi: np.ndarray, n: int, beta: float) -> np.ndarray:
    """exp(i beta sum_i X_i) = prod_i (cos beta + i sin beta X_i)."""
    c, s = np.cos(beta), np.sin(beta)
    t = psi.reshape((2,) * n)
    for i in range(n):
        flipped = np.flip(t, axis=i)
        t = c * t + 1j * s * flipped
    return t.reshape(-1)


def qaoa_state(n: int, alphas, betas, b: float = 0.0, sign: float = +1.0) -> np.ndarray:
    z = _z_diag(n)
    hz = np.zeros(2 ** n)
    for i in range(n - 1):
        hz += z[i] * z[i + 1]
    for i in range(n):
        hz += b * z[i]
    psi = np.full(2 ** n, 2.0 ** (-n / 2), dtype=np.complex128)
    for a, bt in zip(alphas, betas):
        psi = np.exp(sign * 1j * a * hz) * psi
        psi = _apply_rx_all(psi, n, sign * bt)
    return psi


def tfim_energy(psi: np.ndarray, n: int, b: float, g: float) -> float:
    z = _z_diag(n)
    p = np.abs(psi) ** 2
    ezz = sum(float(p @ (z[i] * z[i + 1])) for i in range(n - 1))
    ez = sum(float(p @ z[i]) for i in range(n))
    t = psi.reshape((2,) * n)
    ex = 0.0
    for i in range(n):
        ex += float(np.real(np.vdot(t, np.flip(t, axis=i))))
    return -(ezz + b * ez) - g * ex


def expect_zz_x(psi: np.ndarray, n: int):
    """Per-bond <Z_i Z_{i+1}> and per-site <X_i>."""
    z = _z_diag(n)
    p = np.abs(psi) ** 2
    zz = np.array([float(p @ (z[i] * z[i + 1])) for i in range(n - 1)])
    t = psi.reshape((2,) * n)
    xs = np.array([float(np.real(np.vdot(t, np.flip(t, axis=i)))) for i in range(n)])
    return zz, xs
