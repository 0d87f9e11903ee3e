"""Adiabatic evolution (oracle; test infrastructure only).

Sec. 2.6: i d/dt psi = H(t) psi (Eq. (2)) with H(t) = (1 - s) H0 + s H1
(Eq. (3)), H0 = -sum_i X_i (Eq. (4)), whose ground state -- the uniform
superposition -- is the initial condition; s = t/T (linear schedule).  The
Trotter method maps each time step to a circuit of few-qubit gates (the
decomposition cited in Sec. 2.6); the observed delta-t^4 convergence of the
overlap (Sec. 3.5) implies a second-order split.  Reading used here, per step
k with s_k = (k + 1/2) dt / T (the step midpoint):

    exp(-i H(s_k) dt) ~ exp(-i (1-s_k) H0 dt/2) exp(-i s_k H1 dt) exp(-i (1-s_k) H0 dt/2)

where exp(+i a X dt/2) = RX(-a dt) on every qubit and, for a diagonal H1 with
energies E(x), exp(-i s dt H1) multiplies amplitude x by exp(-i s dt E(x)).

The general form below also covers a transverse field inside H1 (the TFIM of
Eq. (5)): H(s) = -cx(s) sum_i X_i + s * diag(E).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import gates, statevec


def rx_layer(psi: np.ndarray, n: int, angle: float) -> np.ndarray:
    R = gates.matrix("RX", angle)
    for q in range(n):
        psi = statevec.apply(psi, R, (q,))
    return psi


def trotter(n: int, E: np.ndarray, T: float, dt: float, cx=None, psi0=None, steps=None) -> np.ndarray:
    """Second-order Trotter evolution from the plus state (or psi0).
    E: diagonal energies of H1 over all 2^n indices; cx(s): transverse-field
    coefficient (default 1 - s, i.e. H0 = -sum X and H1 = diag(E)).  steps:
    stop after that many steps of the T-schedule (default: all T/dt)."""
    if cx is None:
        cx = lambda s: 1.0 - s  # noqa: E731
    K = int(round(T / dt)) if steps is None else int(steps)
    psi = statevec.plus(n) if psi0 is None else np.asarray(psi0, dtype=np.complex128).copy()
    for k in range(K):
        s = (k + 0.5) * dt / T
        a = cx(s)
        psi = rx_layer(psi, n, -a * dt)
        psi = psi * np.exp(-1j * s * dt * E)
        psi = rx_layer(psi, n, -a * dt)
    return psi


def sum_x_sparse(n: int) -> sp.csr_matrix:
    """sum_i X_i as a sparse matrix: X_q flips bit n-1-q."""
    N = 1 << n
    rows, cols = [], []
    idx = np.arange(N)
    for q in range(n):
        rows.append(idx)
        cols.append(idx ^ (1 << (n - 1 - q)))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    return sp.csr_matrix((np.ones(r.size), (r, c)), shape=(N, N))


def exact_piecewise(n: int, E: np.ndarray, T: float, dt: float, cx=None, psi0=None) -> np.ndarray:
    """Same time grid, each step propagated exactly: psi <- exp(-i H(s_k) dt) psi
    with H(s) = -cx(s) sum X + s diag(E) (the 'exp' solver, Eq. (6))."""
    if cx is None:
        cx = lambda s: 1.0 - s  # noqa: E731
    K = int(round(T / dt))
    SX = sum_x_sparse(n)
    D = sp.diags(E)
    psi = statevec.plus(n) if psi0 is None else np.asarray(psi0, dtype=np.complex128).copy()
    for k in range(K):
        s = (k + 0.5) * dt / T
        H = (-cx(s)) * SX + s * D
        psi = spla.expm_multiply(-1j * dt * H.tocsc(), psi)
    return psi


def single_qubit_trotter(h_q: float, T: float, dt: float) -> np.ndarray:
    """J = 0 factorisation: with no couplings H(s) is a sum of commuting
    one-qubit terms -(1-s) X + s h Z, so the n-qubit Trotter state is the
    tensor product of these 2-component Trotter evolutions."""
    K = int(round(T / dt))
    v = np.array([1.0, 1.0], dtype=np.complex128) / np.sqrt(2)
    Zd = np.array([1.0, -1.0])
    for k in range(K):
        s = (k + 0.5) * dt / T
        R = gates.matrix("RX", -(1.0 - s) * dt)
        v = R @ v
        v = v * np.exp(-1j * s * dt * h_q * Zd)
        v = R @ v
    return v


def energy(psi: np.ndarray, E: np.ndarray) -> float:
    return float(np.sum(np.abs(psi) ** 2 * E))
