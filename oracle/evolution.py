"""Time evolution by integrating the Schroedinger equation, and entanglement
entropy (oracle; test infrastructure only).

Sec. 2.6: besides the Trotter circuit, the paper integrates
i dpsi/dt = H(t) psi with an ODE solver: the default "exp" solver multiplies
the state by exp(-i H dt) every step (Eq. (6)); "rk4" and "rk45" are fourth-
and fifth-order Runge-Kutta integrators.  With H(t) = (1 - s) H0 + s H1 and
s = t / T (the linear schedule of Eq. (3)).  Readings used here:

* "exp": piecewise-constant H at the step midpoint s_k = (k + 1/2) dt / T
  (the same time grid as the Trotter reading), propagated by the dense matrix
  exponential for small n;
* "rk4": the classical four-stage tableau on the continuous schedule;
* "rk45": the Dormand-Prince 5(4) tableau with a fixed step, advancing the
  fifth-order solution.

H psi is applied term by term from the Pauli sums (Sec. 3.5 notes that the
Runge-Kutta route with a Trotter Hamiltonian takes these products term by
term instead of building the 2^N x 2^N matrix).

Entanglement entropy (Sec. 2.4.4 lists it among the callbacks): for the
bipartition into the first a qubits and the rest, the reduced density
matrix rho_A = M M^dagger with M = psi reshaped to 2^a x 2^(n-a); the entropy
is -sum lambda log lambda over its eigenvalues (natural logarithm).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import observables

# Dormand-Prince 5(4): nodes, stage coefficients and fifth-order weights
DP_C = [0.0, 1 / 5, 3 / 10, 4 / 5, 8 / 9, 1.0]
DP_A = [
    [],
    [1 / 5],
    [3 / 40, 9 / 40],
    [44 / 45, -56 / 15, 32 / 9],
    [19372 / 6561, -25360 / 2187, 64448 / 6561, -212 / 729],
    [9017 / 3168, -355 / 33, 46732 / 5247, 49 / 176, -5103 / 18656],
]
DP_B = [35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84]

RK4_C = [0.0, 0.5, 0.5, 1.0]
RK4_A = [[], [0.5], [0.0, 0.5], [0.0, 0.0, 1.0]]
RK4_B = [1 / 6, 1 / 3, 1 / 3, 1 / 6]


def h_apply(psi, h0, h1, s):
    """H(s) psi = (1 - s) H0 psi + s H1 psi, each Pauli sum term by term."""
    return (1.0 - s) * observables.apply_pauli_sum(psi, h0) + s * observables.apply_pauli_sum(psi, h1)


def rk_step(psi, h0, h1, t, dt, T, A, B, Cn):
    """One explicit Runge-Kutta step of dpsi/dt = -i H(t/T) psi."""
    ks = []
    for j in range(len(B)):
        y = psi.copy()
        for l, a in enumerate(A[j]):
            if a != 0.0:
                y = y + dt * a * ks[l]
        ks.append(-1j * h_apply(y, h0, h1, (t + Cn[j] * dt) / T))
    out = psi.copy()
    for l, b in enumerate(B):
        if b != 0.0:
            out = out + dt * b * ks[l]
    return out


def dense_h(n, h0, h1, s):
    return (1.0 - s) * observables.dense_pauli_sum(n, h0) + s * observables.dense_pauli_sum(n, h1)


def evolve(n, h0, h1, T, dt, solver, psi0, every=0, energy_terms=None, entropy_qubits=0):
    """Integrate from psi0 over [0, T] in K = T/dt steps.  Returns the final
    state and, when every > 0, the energies <energy_terms> and entropies of
    the first entropy_qubits qubits after steps every, 2 every, ..."""
    K = int(round(T / dt))
    psi = np.asarray(psi0, dtype=np.complex128).copy()
    energies, entropies = [], []
    for k in range(K):
        t = k * dt
        if solver == "exp":
            H = dense_h(n, h0, h1, (k + 0.5) * dt / T)
            psi = sla.expm(-1j * dt * H) @ psi
        elif solver == "rk4":
            psi = rk_step(psi, h0, h1, t, dt, T, RK4_A, RK4_B, RK4_C)
        elif solver == "rk45":
            psi = rk_step(psi, h0, h1, t, dt, T, DP_A, DP_B, DP_C)
        else:
            raise ValueError(solver)
        if every and (k + 1) % every == 0:
            if energy_terms is not None:
                energies.append(float(observables.expectation(psi, energy_terms).real))
            if entropy_qubits:
                entropies.append(entanglement_entropy(psi, entropy_qubits))
    return psi, np.array(energies), np.array(entropies)


def entanglement_entropy(psi, a):
    """-tr(rho_A log rho_A) for the first a qubits; eigenvalues below 1e-15
    (rounding of zero) contribute nothing."""
    n = int(np.log2(psi.size))
    M = np.asarray(psi, dtype=np.complex128).reshape(1 << a, 1 << (n - a))
    rho = M @ M.conj().T
    w = np.linalg.eigvalsh(rho)
    w = w[w > 1e-15]
    return float(-np.sum(w * np.log(w)))
