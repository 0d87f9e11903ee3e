"""State tensors and gate application (oracle; test infrastructure only).

O1: the state is a numpy array of shape (2,)*n; axis q is qubit q; the flat
    C-order index is x = sum_q sigma_q 2^(n-1-q) (Sec. 2.3: psi(sigma_1..sigma_N)
    stored as a rank-N tensor or a 2^N vector).
O3: a k-qubit gate G(tau, tau') acts by Eq. (1): contract its column indices
    with the target axes of the state.  With controls (Sec. 2.4.1) only the
    sub-tensor where every control qubit is 1 is transformed.
O4: brute force -- the same gate as an explicit 2^n x 2^n matrix built from
    Kronecker products and a qubit-reordering permutation.
"""
from __future__ import annotations

import numpy as np


def zeros(n: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def basis(n: int, x: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[x] = 1.0
    return psi


def plus(n: int) -> np.ndarray:
    return np.full(1 << n, 2.0 ** (-n / 2), dtype=np.complex128)


def apply(psi: np.ndarray, U: np.ndarray, targets, controls=()) -> np.ndarray:
    """Eq. (1): psi'(..tau..) = sum_tau' G(tau, tau') psi(..tau'..), restricted to
    the sub-tensor where all controls are 1.  targets[0] is the most
    significant index of G.  Returns a new flat array."""
    n = int(np.log2(psi.size))
    k = len(targets)
    assert U.shape == (1 << k, 1 << k)
    assert len(set(targets) | set(controls)) == k + len(controls)
    t = psi.astype(np.complex128).reshape((2,) * n).copy()
    Gt = U.reshape((2,) * (2 * k))
    sel = [slice(None)] * n
    for c in controls:
        sel[c] = 1
    sel = tuple(sel)
    sub = t[sel]
    remaining = [q for q in range(n) if q not in controls]
    axes = [remaining.index(q) for q in targets]
    out = np.tensordot(Gt, sub, axes=(list(range(k, 2 * k)), axes))
    out = np.moveaxis(out, list(range(k)), axes)
    t[sel] = out
    return t.reshape(-1)


def project_controls(psi: np.ndarray, controls) -> np.ndarray:
    """Zero every component whose control qubits are not all 1."""
    n = int(np.log2(psi.size))
    t = psi.reshape((2,) * n)
    out = np.zeros_like(t)
    sel = [slice(None)] * n
    for c in controls:
        sel[c] = 1
    out[tuple(sel)] = t[tuple(sel)]
    return out.reshape(-1)


# ----------------------------------------------------------------------------
# O4: brute-force Kronecker construction
# ----------------------------------------------------------------------------

def reorder_matrix(n: int, order) -> np.ndarray:
    """Permutation P with (P psi)[x'] = psi[x], where qubit j of x' holds the
    value of qubit order[j] of x."""
    N = 1 << n
    P = np.zeros((N, N))
    for x in range(N):
        bits = [(x >> (n - 1 - q)) & 1 for q in range(n)]
        xp = 0
        for j in range(n):
            xp = (xp << 1) | bits[order[j]]
        P[xp, x] = 1.0
    return P


def full_unitary(n: int, U: np.ndarray, targets, controls=()) -> np.ndarray:
    """2^n x 2^n matrix of a (controlled) gate:  move controls then targets to
    the front, build (I - Pc) (x) I + Pc (x) G with Pc = |1..1><1..1| on the
    controls, extend with the identity, move the qubits back."""
    k, c = len(targets), len(controls)
    rest = [q for q in range(n) if q not in targets and q not in controls]
    order = list(controls) + list(targets) + rest
    dc = 1 << c
    Pc = np.zeros((dc, dc))
    Pc[-1, -1] = 1.0
    CG = np.kron(np.eye(dc) - Pc, np.eye(1 << k)) + np.kron(Pc, U)
    M = np.kron(CG, np.eye(1 << (n - c - k)))
    P = reorder_matrix(n, order)
    return P.T @ M @ P
