"""Hamiltonian expectation values (oracle; test infrastructure only).

The energy of a state is <psi|H|psi> (Sec. 2.4.4, the Energy callback).  A
Pauli-sum H = sum_t c_t P_t is applied term by term through the gate
contraction of Eq. (1) with the 2x2 Pauli matrices; the Ising Hamiltonian of
the adiabatic problem is diagonal in the computational basis, with
Z|0> = +|0>, so z_q = 1 - 2 sigma_q.  The real part is returned and not divided
by the norm.
"""
from __future__ import annotations

import numpy as np

from . import gates, statevec


def apply_pauli_string(psi: np.ndarray, s: str) -> np.ndarray:
    out = psi
    for q, p in enumerate(s):
        if p != "I":
            out = statevec.apply(out, gates.PAULI[p], (q,))
    return out


def apply_pauli_sum(psi: np.ndarray, terms) -> np.ndarray:
    """H psi for H = sum_t c_t P_t."""
    out = np.zeros_like(psi, dtype=np.complex128)
    for c, s in terms:
        out += c * apply_pauli_string(psi, s)
    return out


def expectation(psi: np.ndarray, terms) -> complex:
    """<psi|H|psi> as a complex number (its imaginary part is rounding)."""
    return np.vdot(psi, apply_pauli_sum(psi, terms))


def dense_pauli_sum(n: int, terms) -> np.ndarray:
    """2^n x 2^n matrix of sum_t c_t P_t built with Kronecker products (n <= 12)."""
    H = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for c, s in terms:
        M = np.array([[1.0 + 0j]])
        for p in s:
            M = np.kron(M, gates.PAULI[p])
        H += c * M
    return H


def spins(n: int, xs=None) -> np.ndarray:
    """z_q(x) = 1 - 2 sigma_q(x), shape (len(xs), n)."""
    if xs is None:
        xs = np.arange(1 << n, dtype=np.int64)
    xs = np.asarray(xs, dtype=np.int64)
    bits = (xs[:, None] >> (n - 1 - np.arange(n)[None, :])) & 1
    return 1.0 - 2.0 * bits


def ising_energies(J: np.ndarray, h: np.ndarray, xs=None) -> np.ndarray:
    """E(z) = sum_{i<j} J_ij z_i z_j + sum_i h_i z_i for every basis index."""
    n = len(h)
    z = spins(n, xs)
    E = z @ h
    for i in range(n):
        for j in range(i + 1, n):
            if J[i, j] != 0.0:
                E = E + J[i, j] * z[:, i] * z[:, j]
    return E


def ising_terms(J: np.ndarray, h: np.ndarray):
    """The same Hamiltonian as a Pauli sum."""
    n = len(h)
    out = []
    for i in range(n):
        for j in range(i + 1, n):
            if J[i, j] != 0.0:
                s = ["I"] * n
                s[i] = s[j] = "Z"
                out.append((float(J[i, j]), "".join(s)))
    for i in range(n):
        s = ["I"] * n
        s[i] = "Z"
        out.append((float(h[i]), "".join(s)))
    return out


def norm2(psi: np.ndarray) -> float:
    return float(np.vdot(psi, psi).real)
