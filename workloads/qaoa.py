"""Seeded QAOA circuit descriptions shaped like the paper's workloads.

The paper's circuits (Sec. IV, Eq. (tfim_model)) alternate a layer of nearest-neighbour
Ising phase blocks with a layer of single-atom transverse-field rotations, starting from
the product of |+> states, on open chains of tens to about a hundred atoms, at shallow
depth.  Noise enters as Rydberg decay, qubit dephasing (Sec. II) and population leaked
into |r> by the blockade gate.

A CircuitSpec is pure data: the number of atoms ``n``, levels per atom ``d`` (3 means
{0,1,r}; 4 means {0,1,r,lost}), depth ``p``, angles ``gamma[k]`` (cost layer) and
``beta[k]`` (mixer layer), per-layer noise probabilities and the bond-dimension cap
``chi``.  How these numbers become channels is left to whoever consumes the spec.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np


@dataclasses.dataclass(frozen=True)
class CircuitSpec:
    n: int                 # atoms in the open chain
    d: int                 # levels per atom (3 or 4)
    p: int                 # QAOA depth (number of cost+mixer layers)
    gamma: tuple           # cost angles, one per layer: gate exp(-i gamma Z(x)Z)
    beta: tuple            # mixer angles, one per layer: exp(-i beta X) per atom
    p_leak: float          # probability |1> -> |r> on each atom of each two-atom gate
    p_deph: float          # qubit dephasing probability per atom per layer
    p_decay: float         # Rydberg decay probability per atom per layer
    chi: int               # bond-dimension cap of the density-operator MPO
    g: float = 1.0         # transverse field of the measured TFIM Hamiltonian
    seed: int = -1
    name: str = ""

    def as_dict(self) -> dict:
        return dataclasses.asdict(self)

    def n_two_site_updates(self) -> int:
        return self.p * (self.n - 1)


def _angles(rng: np.random.Generator, p: int):
    gamma = tuple(float(x) for x in rng.uniform(0.0, math.pi, size=p))
    beta = tuple(float(x) for x in rng.uniform(0.0, math.pi, size=p))
    return gamma, beta


def _log_uniform(rng: np.random.Generator, lo: float, hi: float) -> float:
    return float(math.exp(rng.uniform(math.log(lo), math.log(hi))))


def config_m0(seed: int = 0) -> CircuitSpec:
    """N=6 atoms, d=3, p=1, all rates 1e-3, chi=81 (no truncation can occur)."""
    rng = np.random.default_rng(seed)
    gamma, beta = _angles(rng, 1)
    return CircuitSpec(n=6, d=3, p=1, gamma=gamma, beta=beta, p_leak=1e-3,
                       p_deph=1e-3, p_decay=1e-3, chi=81, seed=seed, name="m0")


def config_m1(seed: int = 0, n: int = 40) -> CircuitSpec:
    """N=40, d=4, p=2, rates log-uniform in [1e-4, 1e-2], chi=128."""
    rng = np.random.default_rng(1000 + seed)
    gamma, beta = _angles(rng, 2)
    rates = [_log_uniform(rng, 1e-4, 1e-2) for _ in range(3)]
    return CircuitSpec(n=n, d=4, p=2, gamma=gamma, beta=beta, p_leak=rates[0],
                       p_deph=rates[1], p_decay=rates[2], chi=128, seed=seed, name="m1")


def config_m2_batch(seed: int = 0, count: int = 256) -> List[CircuitSpec]:
    """Batch of independent circuits: N in [20,100], chi in {64,128,256}, p in {1,2,3}."""
    rng = np.random.default_rng(2000 + seed)
    out = []
    for c in range(count):
        n = int(rng.integers(20, 101))
        chi = int(rng.choice([64, 128, 256]))
        p = int(rng.integers(1, 4))
        gamma, beta = _angles(rng, p)
        rates = [_log_uniform(rng, 1e-4, 1e-2) for _ in range(3)]
        out.append(CircuitSpec(n=n, d=4, p=p, gamma=gamma, beta=beta, p_leak=rates[0],
                               p_deph=rates[1], p_decay=rates[2], chi=chi,
                               seed=seed * 100000 + c, name="m2"))
    return out


def config_m3(seed: int = 0, n: int = 100, p: int = 3, chi: int = 512) -> CircuitSpec:
    """N=100, d=4, chi=512, p=3, all rates 1e-3."""
    rng = np.random.default_rng(3000 + seed)
    gamma, beta = _angles(rng, p)
    return CircuitSpec(n=n, d=4, p=p, gamma=gamma, beta=beta, p_leak=1e-3,
                       p_deph=1e-3, p_decay=1e-3, chi=chi, seed=seed, name="m3")


def random_spec(seed: int, n: int, d: int, p: int, chi: int,
                rate_lo: float = 1e-4, rate_hi: float = 1e-2) -> CircuitSpec:
    """Generic seeded spec, used for parity cases of intermediate size."""
    rng = np.random.default_rng(4000 + seed)
    gamma, beta = _angles(rng, p)
    rates = [_log_uniform(rng, rate_lo, rate_hi) for _ in range(3)]
    return CircuitSpec(n=n, d=d, p=p, gamma=gamma, beta=beta, p_leak=rates[0],
                       p_deph=rates[1], p_decay=rates[2], chi=chi, seed=seed, name="rand")


def noiseless_spec(n: int, d: int, gamma, beta, chi: int) -> CircuitSpec:
    """All noise probabilities zero (the pure-state limit)."""
    gamma = tuple(float(x) for x in gamma)
    beta = tuple(float(x) for x in beta)
    return CircuitSpec(n=n, d=d, p=len(gamma), gamma=gamma, beta=beta, p_leak=0.0,
                       p_deph=0.0, p_decay=0.0, chi=chi, name="noiseless")


def random_unit_vectors(seed: int, count: int, dim: int) -> np.ndarray:
    """Real random draws used by property tests (e.g. spectra and trace environments)."""
    rng = np.random.default_rng(5000 + seed)
    return rng.standard_normal((count, dim))
