"""Gate matrices (oracle; test infrastructure only).

The paper names its gates (H, X, RX, CZPow, SWAP ... Sec. 2.3 listing, Sec. 3.1)
but prints no matrices; these are the standard textbook forms.  Rotations are
R_P(theta) = exp(-i theta P / 2) for a Pauli P; U1(lam) = diag(1, e^{i lam}),
so the paper's CZPow(t) is U1(pi t) with one control.
"""
from __future__ import annotations

import numpy as np

_S2 = 1.0 / np.sqrt(2.0)

PAULI = {
    "I": np.eye(2, dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def matrix(name: str, theta: float = 0.0, mat=None) -> np.ndarray:
    """2^k x 2^k complex128 matrix of a named gate; row index = output."""
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    if name == "H":
        return np.array([[_S2, _S2], [_S2, -_S2]], dtype=np.complex128)
    if name in ("X", "Y", "Z"):
        return PAULI[name].copy()
    if name == "S":
        return np.diag([1, 1j]).astype(np.complex128)
    if name == "T":
        return np.diag([1, np.exp(1j * np.pi / 4)]).astype(np.complex128)
    if name == "RX":
        return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)
    if name == "RY":
        return np.array([[c, -s], [s, c]], dtype=np.complex128)
    if name == "RZ":
        return np.diag([np.exp(-0.5j * theta), np.exp(0.5j * theta)]).astype(np.complex128)
    if name == "U1":
        return np.diag([1, np.exp(1j * theta)]).astype(np.complex128)
    if name == "SWAP":
        m = np.zeros((4, 4), dtype=np.complex128)
        m[0, 0] = m[1, 2] = m[2, 1] = m[3, 3] = 1
        return m
    if name == "MAT":
        return np.asarray(mat, dtype=np.complex128)
    raise ValueError(f"unknown gate {name}")


def generator(name: str) -> np.ndarray:
    """Pauli P with U(theta) = exp(-i theta P/2) for the rotation gates."""
    if name in ("RX", "RY", "RZ"):
        return PAULI[name[1]].copy()
    raise ValueError(f"{name} is not a Pauli rotation")


def gate_matrix(g, params=None) -> np.ndarray:
    """Matrix of a ``qsynth.G`` record; trainable angles come from params."""
    theta = g.theta if (g.pidx < 0 or params is None) else float(params[g.pidx])
    return matrix(g.name, theta, g.mat)
