"""Density matrices and noise channels (oracle; test infrastructure only).

Sec. 2.4.3: besides state vectors the simulator evolves density matrices, so
that circuits may contain noise channels.  Plain definitions, dense
2^n x 2^n matrices (small n):

* a gate U (with controls) acts as rho -> U rho U^dagger, U the full
  Kronecker matrix of the gate (statevec.full_unitary);
* a channel with Kraus operators K_i acts as rho -> sum_i K_i rho K_i^dagger;
* expectation values are Tr(H rho).

The named channels are the textbook ones (Nielsen & Chuang, Sec. 8.3):
depolarising rho -> (1 - p) rho + p I/2, amplitude damping with decay gamma,
phase damping with lambda, bit and phase flips with probability p.
"""
from __future__ import annotations

import numpy as np

from . import gates, observables, statevec


def pure(psi) -> np.ndarray:
    psi = np.asarray(psi, dtype=np.complex128)
    return np.outer(psi, psi.conj())


def apply_gate(rho, U, targets, controls=()):
    n = int(np.log2(rho.shape[0]))
    F = statevec.full_unitary(n, np.asarray(U, dtype=np.complex128), targets, controls)
    return F @ rho @ F.conj().T


def apply_channel(rho, kraus, targets):
    n = int(np.log2(rho.shape[0]))
    out = np.zeros_like(rho)
    for K in kraus:
        F = statevec.full_unitary(n, np.asarray(K, dtype=np.complex128), targets)
        out += F @ rho @ F.conj().T
    return out


def expectation(rho, terms) -> float:
    n = int(np.log2(rho.shape[0]))
    return float(np.trace(observables.dense_pauli_sum(n, terms) @ rho).real)


def kraus(name: str, p: float):
    I2 = np.eye(2, dtype=np.complex128)
    X, Y, Z = gates.PAULI["X"], gates.PAULI["Y"], gates.PAULI["Z"]
    if name == "depolarizing":
        return [np.sqrt(1 - 3 * p / 4) * I2, np.sqrt(p / 4) * X, np.sqrt(p / 4) * Y, np.sqrt(p / 4) * Z]
    if name == "amplitude_damping":
        return [np.array([[1, 0], [0, np.sqrt(1 - p)]], dtype=np.complex128),
                np.array([[0, np.sqrt(p)], [0, 0]], dtype=np.complex128)]
    if name == "phase_damping":
        return [np.array([[1, 0], [0, np.sqrt(1 - p)]], dtype=np.complex128),
                np.array([[0, 0], [0, np.sqrt(p)]], dtype=np.complex128)]
    if name == "bit_flip":
        return [np.sqrt(1 - p) * I2, np.sqrt(p) * X]
    if name == "phase_flip":
        return [np.sqrt(1 - p) * I2, np.sqrt(p) * Z]
    raise ValueError(name)


def run(n: int, spec, rho0=None, params=None) -> np.ndarray:
    """Apply a ``qsynth`` gate list to rho0 (default |0..0><0..0|); records
    named ``CH:<channel>`` are channels with parameter theta."""
    rho = pure(statevec.zeros(n)) if rho0 is None else np.asarray(rho0, dtype=np.complex128).copy()
    for g in spec:
        if g.name.startswith("CH:"):
            rho = apply_channel(rho, kraus(g.name[3:], g.theta), g.targets)
        else:
            rho = apply_gate(rho, gates.gate_matrix(g, params), g.targets, g.controls)
    return rho


def as_vector(rho) -> np.ndarray:
    """rho[r][c] at index r 2^n + c: the 2n-qubit vector the GPU path stores."""
    return np.asarray(rho, dtype=np.complex128).reshape(-1)
