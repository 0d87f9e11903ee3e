"""Circuit execution and QFT closed forms (oracle; test infrastructure only).

A circuit is a queue of gates applied in order (Sec. 2.3); executing it gives
the final state.  The QFT closed forms pin the QFT workload (Sec. 3.1).
"""
from __future__ import annotations

import numpy as np

from . import gates, statevec


def run(n: int, spec, psi0=None, params=None) -> np.ndarray:
    psi = statevec.zeros(n) if psi0 is None else np.asarray(psi0, dtype=np.complex128).copy()
    for g in spec:
        psi = statevec.apply(psi, gates.gate_matrix(g, params), g.targets, g.controls)
    return psi


def inverse(spec, params=None):
    """The adjoint circuit: reversed order, conjugate-transposed matrices."""
    from qsynth import gate
    out = []
    for g in reversed(spec):
        U = gates.gate_matrix(g, params).conj().T
        out.append(gate("MAT", g.targets, g.controls, mat=U))
    return out


def circuit_unitary(n: int, spec, params=None) -> np.ndarray:
    """Product of the brute-force Kronecker matrices (O4); n <= 10."""
    U = np.eye(1 << n, dtype=np.complex128)
    for g in spec:
        U = statevec.full_unitary(n, gates.gate_matrix(g, params), g.targets, g.controls) @ U
    return U


def qft_basis_amplitudes(n: int, x: int, ys) -> np.ndarray:
    """QFT|x> = 2^(-n/2) sum_y exp(2 pi i x y / 2^n) |y>; the phase is taken from
    the exact integer (x*y) mod 2^n so that it is exact for any n <= 62."""
    ys = np.asarray(ys, dtype=np.uint64)
    N = np.uint64(1) << np.uint64(n)
    prod = (np.uint64(x) * ys) & (N - np.uint64(1))   # exact modular product (wraps in u64)
    ang = 2 * np.pi * (prod.astype(np.float64) / float(1 << n))
    return np.exp(1j * ang) * 2.0 ** (-n / 2)


def qft_via_fft(psi: np.ndarray) -> np.ndarray:
    """QFT of an arbitrary state with the big-endian index: sqrt(N) * ifft(psi)."""
    return np.sqrt(psi.size) * np.fft.ifft(psi)


def product_state_amplitudes(n: int, theta, phi, xs) -> np.ndarray:
    """Closed form for |0..0> -> RY(theta_q) RZ(phi_q) on every qubit -> CZ(q, q+1):
    psi(x) = prod_q a_q(sigma_q) * (-1)^(sum_q sigma_q sigma_{q+1}),
    a_q(0) = cos(theta_q/2) e^{-i phi_q/2}, a_q(1) = sin(theta_q/2) e^{i phi_q/2}."""
    xs = np.asarray(xs, dtype=np.int64)
    out = np.ones(xs.shape, dtype=np.complex128)
    prev = None
    sign = np.zeros(xs.shape, dtype=np.int64)
    for q in range(n):
        b = (xs >> (n - 1 - q)) & 1
        a0 = np.cos(theta[q] / 2) * np.exp(-0.5j * phi[q])
        a1 = np.sin(theta[q] / 2) * np.exp(0.5j * phi[q])
        out *= np.where(b == 1, a1, a0)
        if prev is not None:
            sign += prev * b
        prev = b
    return out * np.where(sign % 2 == 1, -1.0, 1.0)
