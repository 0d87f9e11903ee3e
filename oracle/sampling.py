"""Measurement sampling (oracle; test infrastructure only).

Sec. 2.4.2: measurement samples the final state vector; the outcome
distribution of the measured qubits is the trace-out of |psi|^2 over the
unmeasured ones.  A sample is drawn by inverse-CDF:

    x_j = min { x : CDF(x) > u_j * CDF(last) }           (natural index order)

and the outcome is the measured qubits' bits of x_j, the first listed qubit
being the most significant bit of the outcome.  Drawing x from |psi|^2 and
reading off the measured bits samples exactly the traced-out marginal.

Uniforms are either given, or drawn with Philox4x32-10 (Salmon, Moraes, Dror,
Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11): shot j uses
counter (j mod 2^32, j div 2^32, 0, 0) and key (seed mod 2^32, seed div 2^32);
u_j = ((w0 << 32 | w1) >> 11) * 2^-53 from the first two output words.
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57     # Philox4x32 multipliers (SC'11)
W0, W1 = 0x9E3779B9, 0xBB67AE85     # Weyl key increments (SC'11)
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Ten Philox rounds on a 4x32-bit counter with a 2x32-bit key (pure Python)."""
    x0, x1, x2, x3 = (int(c) & MASK for c in ctr)
    k0, k1 = (int(k) & MASK for k in key)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * x0
        p1 = M1 * x2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


def philox_uniforms(seed: int, shots: int, first: int = 0) -> np.ndarray:
    out = np.empty(shots)
    key = (seed & MASK, (seed >> 32) & MASK)
    for i in range(shots):
        j = first + i
        w0, w1, _, _ = philox4x32_10((j & MASK, (j >> 32) & MASK, 0, 0), key)
        out[i] = (((w0 << 32) | w1) >> 11) * 2.0 ** -53
    return out


def marginal(psi: np.ndarray, qubits) -> np.ndarray:
    """Trace-out: p(y) = sum over unmeasured qubits of |psi|^2, listed order,
    first listed qubit = most significant bit of y."""
    n = int(np.log2(psi.size))
    p = (np.abs(psi) ** 2).reshape((2,) * n)
    others = tuple(q for q in range(n) if q not in qubits)
    p = p.sum(axis=others) if others else p
    kept = [q for q in range(n) if q in qubits]          # axes left, ascending
    p = np.transpose(p, [kept.index(q) for q in qubits])
    return p.reshape(-1)


def extract_bits(n: int, xs, qubits) -> np.ndarray:
    xs = np.asarray(xs, dtype=np.int64)
    y = np.zeros_like(xs)
    for q in qubits:
        y = (y << 1) | ((xs >> (n - 1 - q)) & 1)
    return y


def sample_indices(psi: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Inverse-CDF over the full index in natural order (float64 CDF)."""
    cdf = np.cumsum(np.abs(psi.astype(np.complex128)) ** 2)
    return np.searchsorted(cdf, np.asarray(u) * cdf[-1], side="right")


def sample(psi: np.ndarray, qubits, u: np.ndarray) -> np.ndarray:
    n = int(np.log2(psi.size))
    return extract_bits(n, sample_indices(psi, u), qubits)


def boundary_distance(psi: np.ndarray, u: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """How far u_j*total lies from the nearest edge of the CDF interval of
    index idx_j (relative to the total); tiny values mark shots where any
    summation order may legitimately pick a neighbouring index."""
    cdf = np.cumsum(np.abs(psi.astype(np.complex128)) ** 2)
    t = np.asarray(u) * cdf[-1]
    idx = np.asarray(idx, dtype=np.int64)
    lo = np.where(idx > 0, cdf[np.maximum(idx - 1, 0)], 0.0)
    hi = cdf[np.minimum(idx, cdf.size - 1)]
    return np.minimum(np.abs(t - lo), np.abs(hi - t)) / cdf[-1]
