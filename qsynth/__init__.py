"""Seeded synthetic workloads for the state-vector simulator.

This module is shared by the tests, the benchmark and the oracle.  It holds
random draws and circuit *layouts* only: which named gate acts on which qubits
with which angle.  It contains none of the simulation arithmetic -- no gate
matrices, no state updates, no expectation values -- so a mistake in either the
oracle or the HIP path cannot hide behind a shared helper.

Conventions (paper, Sec. 2.3: a state is psi(sigma_1..sigma_N), a circuit is a
queue of gates acting by Eq. (1)):

* qubit q is the most significant index bit of its sub-tensor, i.e. flat index
  x = sum_q sigma_q * 2**(n-1-q);
* a gate record is ``G(name, targets, controls, theta, pidx, mat)``.  ``name``
  is one of H X Y Z S T RX RY RZ U1 SWAP MAT; ``controls`` are qubits that must
  all be 1 (controlled gates, Sec. 2.4.1); ``theta`` is the angle of RX/RY/RZ/U1;
  ``pidx`` >= 0 marks a trainable rotation whose angle is ``params[pidx]``;
  ``mat`` carries an explicit matrix for ``MAT`` gates (Haar draws).
* a Pauli-sum Hamiltonian is a list of ``(coeff, string)`` with one character
  of ``IXYZ`` per qubit, character j acting on qubit j.
"""
from __future__ import annotations

from collections import namedtuple
from math import pi

import numpy as np

G = namedtuple("G", "name targets controls theta pidx mat")


def gate(name, targets, controls=(), theta=0.0, pidx=-1, mat=None):
    return G(name, tuple(int(t) for t in targets), tuple(int(c) for c in controls),
             float(theta), int(pidx), mat)


# ----------------------------------------------------------------------------
# states
# ----------------------------------------------------------------------------

def random_state(n: int, seed: int) -> np.ndarray:
    """Real and imaginary parts ~ N(0,1), then normalised in float64."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((2, 1 << n))
    psi = v[0] + 1j * v[1]
    psi /= np.sqrt(np.vdot(psi, psi).real)
    return psi


def random_basis_index(n: int, seed: int) -> int:
    return int(np.random.default_rng(seed).integers(0, 1 << n))


def haar_unitary(dim: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed unitary: QR of a complex Gaussian matrix with the
    phases of R's diagonal folded back (Mezzadri's recipe)."""
    z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))


# ----------------------------------------------------------------------------
# circuit layouts
# ----------------------------------------------------------------------------

def qft(n: int, swaps: bool = True):
    """Quantum Fourier transform (Sec. 3.1: H, controlled phase, SWAP).

    Textbook order: for qubit j, H(j), then the phase 2*pi/2**(k-j+1)
    controlled by each later qubit k; finally the qubit order is reversed
    with SWAPs.  n(n+1)/2 H + CU1 gates and floor(n/2) SWAPs."""
    out = []
    for j in range(n):
        out.append(gate("H", (j,)))
        for k in range(j + 1, n):
            out.append(gate("U1", (j,), (k,), theta=2 * pi / 2 ** (k - j + 1)))
    if swaps:
        for j in range(n // 2):
            out.append(gate("SWAP", (j, n - 1 - j)))
    return out


def ghz(n: int):
    return [gate("H", (0,))] + [gate("X", (j,), (0,)) for j in range(1, n)]


def ry_rz_cz_layers(n: int, params: np.ndarray):
    """Layers of RY on every qubit, RZ on every qubit, CZ on (i, i+1).
    ``params`` has shape (depth, n, 2) = [layer, qubit, (theta_RY, phi_RZ)];
    parameter index = params' flat C-order index."""
    depth = params.shape[0]
    out = []
    for l in range(depth):
        for q in range(n):
            out.append(gate("RY", (q,), theta=params[l, q, 0], pidx=(l * n + q) * 2))
        for q in range(n):
            out.append(gate("RZ", (q,), theta=params[l, q, 1], pidx=(l * n + q) * 2 + 1))
        for q in range(n - 1):
            out.append(gate("Z", (q + 1,), (q,)))
    return out


def ry_layers(n: int, params: np.ndarray):
    """Layers of RY on every qubit, no entangling gate (a product state).
    ``params`` has shape (layers, n); parameter index = l*n + q."""
    params = np.atleast_2d(params)
    return [gate("RY", (q,), theta=params[l, q], pidx=l * n + q)
            for l in range(params.shape[0]) for q in range(n)]


def ry_rz_layers(n: int, theta: np.ndarray, phi: np.ndarray):
    """Layers of RY on every qubit then RZ on every qubit, no entangling gate.
    theta, phi: (layers, n); per layer the n RY parameters come first, then
    the n RZ parameters: index l*2n + q (RY) and l*2n + n + q (RZ)."""
    out = []
    for l in range(theta.shape[0]):
        out += [gate("RY", (q,), theta=theta[l, q], pidx=2 * l * n + q) for q in range(n)]
        out += [gate("RZ", (q,), theta=phi[l, q], pidx=2 * l * n + n + q) for q in range(n)]
    return out


def ry_czring_layers(n: int, params: np.ndarray):
    """Layers of RY on every qubit then CZ on the ring (i, (i+1) mod n).
    ``params`` has shape (layers, n); parameter index = l*n + q."""
    out = []
    for l in range(params.shape[0]):
        for q in range(n):
            out.append(gate("RY", (q,), theta=params[l, q], pidx=l * n + q))
        for q in range(n):
            a, b = q, (q + 1) % n
            if a != b:
                out.append(gate("Z", (max(a, b),), (min(a, b),)))
    return out


def ry_then_phases(n: int, theta: np.ndarray, seed: int):
    """RY(theta_q) on every qubit (parameter index q), then controlled phase
    gates U1(phi) on the ring (q, q+1 mod n) and on the pairs (q, q + n/2),
    phi ~ U[0.1, 3.0] from ``seed`` (never a multiple of pi)."""
    rng = np.random.default_rng(seed)
    out = [gate("RY", (q,), theta=theta[q], pidx=q) for q in range(n)]
    pairs = [(q, (q + 1) % n) for q in range(n)] + [(q, q + n // 2) for q in range(n // 2)]
    for a, b in pairs:
        if a != b:
            out.append(gate("U1", (max(a, b),), (min(a, b),), theta=float(rng.uniform(0.1, 3.0))))
    return out


def random_layers(n: int, depth: int, seed: int):
    """Depth x (Haar 1-qubit gate on every qubit, then CZ on a seeded random
    perfect matching of the qubits)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(depth):
        for q in range(n):
            out.append(gate("MAT", (q,), mat=haar_unitary(2, rng)))
        perm = rng.permutation(n)
        for i in range(0, n - 1, 2):
            a, b = int(perm[i]), int(perm[i + 1])
            out.append(gate("Z", (b,), (a,)))
    return out


CHANNELS = ("depolarizing", "amplitude_damping", "phase_damping", "bit_flip", "phase_flip")


def noisy_layers(n: int, depth: int, seed: int, with_rot: bool = True):
    """Depth x (Haar 1-qubit gate or trainable RX/RY/RZ on every qubit, CZ on
    a seeded random matching, then a random named channel with p ~ U[0, 0.3)
    on two random qubits).  Channel records are named ``CH:<channel>`` with
    the parameter in theta (density-matrix circuits only)."""
    rng = np.random.default_rng(seed)
    out, k = [], 0
    for _ in range(depth):
        for q in range(n):
            if with_rot and rng.random() < 0.5:
                out.append(gate("R" + "XYZ"[int(rng.integers(3))], (q,), pidx=k))
                k += 1
            else:
                out.append(gate("MAT", (q,), mat=haar_unitary(2, rng)))
        perm = rng.permutation(n)
        for i in range(0, n - 1, 2):
            out.append(gate("Z", (int(perm[i + 1]),), (int(perm[i]),)))
        for q in rng.choice(n, min(2, n), replace=False):
            out.append(gate("CH:" + CHANNELS[int(rng.integers(len(CHANNELS)))], (int(q),),
                            theta=float(rng.uniform(0, 0.3))))
    params = rng.uniform(0, 2 * pi, k)
    return out, params


def random_mixed(n: int, count: int, seed: int, max_k: int = 2, max_ctrl: int = 2):
    """A random list mixing every gate kind: named gates, rotations, Haar
    matrices on 1..max_k targets, with 0..max_ctrl controls."""
    rng = np.random.default_rng(seed)
    names = ["H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "U1", "SWAP", "MAT"]
    out = []
    for _ in range(count):
        name = names[int(rng.integers(0, len(names)))]
        if name == "SWAP" and n < 2:
            name = "H"
        if name == "SWAP":
            k = 2
        elif name == "MAT":
            k = int(rng.integers(1, max_k + 1))
        else:
            k = 1
        k = min(k, n)
        nc = int(rng.integers(0, max_ctrl + 1))
        nc = min(nc, n - k)
        qs = rng.permutation(n)[: k + nc]
        tg, ct = qs[:k], qs[k:]
        th = float(rng.uniform(0, 2 * pi))
        mat = haar_unitary(1 << k, rng) if name == "MAT" else None
        out.append(gate(name, tg, ct, theta=th, mat=mat))
    return out


# ----------------------------------------------------------------------------
# Hamiltonians (Pauli sums, Ising couplings)
# ----------------------------------------------------------------------------

def pauli_string(n: int, ops: dict) -> str:
    s = ["I"] * n
    for q, p in ops.items():
        s[q] = p
    return "".join(s)


def zz_chain(n: int, periodic: bool):
    m = n if periodic else n - 1
    return [(1.0, pauli_string(n, {i: "Z", (i + 1) % n: "Z"})) for i in range(m)]


def zz_ring_plus_x(n: int, hx: float = 0.5):
    return zz_chain(n, periodic=True) + [(hx, pauli_string(n, {i: "X"})) for i in range(n)]


def z_sum(n: int):
    return [(1.0, pauli_string(n, {i: "Z"})) for i in range(n)]


def random_pauli_sum(n: int, terms: int, seed: int):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(terms):
        s = "".join("IXYZ"[int(i)] for i in rng.integers(0, 4, n))
        out.append((float(rng.standard_normal()), s))
    return out


def ising_couplings(n: int, seed: int):
    """J_ij for i<j drawn in lexicographic order, then h_i; all ~ N(0,1).
    Returned as an n x n array with only the strict upper triangle set."""
    rng = np.random.default_rng(seed)
    iu = np.triu_indices(n, 1)
    J = np.zeros((n, n))
    J[iu] = rng.standard_normal(len(iu[0]))
    h = rng.standard_normal(n)
    return J, h


# ----------------------------------------------------------------------------
# the named workloads
# ----------------------------------------------------------------------------

def variational_10q(seed: int = 0):
    """10 qubits, depth 20 of RY/RZ on all qubits + CZ(i,i+1); observable
    sum_{i=0}^{8} Z_i Z_{i+1}."""
    n, depth = 10, 20
    params = np.random.default_rng(seed).uniform(0, 2 * pi, (depth, n, 2))
    return n, ry_rz_cz_layers(n, params), params.reshape(-1), zz_chain(n, periodic=False)


def gradient_20q(seed: int = 0, n: int = 20, layers: int = 10):
    """RY layer + CZ ring, ``layers`` times; H = sum Z_i Z_{i+1 mod n} + 0.5 sum X_i."""
    params = np.random.default_rng(seed).uniform(0, 2 * pi, (layers, n))
    return n, ry_czring_layers(n, params), params.reshape(-1), zz_ring_plus_x(n)


def batch_instances(seed: int = 0, count: int = 512, nmin: int = 8, nmax: int = 18,
                    dmin: int = 4, dmax: int = 12):
    """Per instance, in order: n ~ U{nmin..nmax}, depth ~ U{dmin..dmax}, then the
    RY/RZ parameters (depth, n, 2); layer = RY all, RZ all, CZ chain; H = sum Z_i."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        d = int(rng.integers(dmin, dmax + 1))
        p = rng.uniform(0, 2 * pi, (d, n, 2))
        out.append((n, ry_rz_cz_layers(n, p), p.reshape(-1), z_sum(n)))
    return out


def adiabatic_24q(seed: int = 0, n: int = 24):
    J, h = ising_couplings(n, seed)
    return n, J, h, 10.0, 0.01
