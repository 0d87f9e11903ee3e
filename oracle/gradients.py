"""Gradients of an energy with respect to circuit angles (oracle; test
infrastructure only).

E(theta) = <psi_L|H|psi_L>, psi_L = U_L .. U_1 psi_0, with trainable gates
U_l = exp(-i theta_l P_l / 2) (Sec. 2.3 rotations; the energy is the Energy
callback of Sec. 2.4.4).  Three independent routes:

* adjoint recurrence (Jones & Gacon 2020): lambda = H psi_L; walking l = L..1,
  dE/dtheta_l += Im <lambda | Pc P_l psi>, then psi <- U_l^dag psi and
  lambda <- U_l^dag lambda (Pc projects on the controls being 1);
* parameter shift: dE/dtheta = [E(theta + pi/2) - E(theta - pi/2)] / 2, exact
  for exp(-i theta P/2) with P^2 = I and no controls;
* central finite differences.

For product states (no entangling gate) a fourth, closed-form route:
every qubit evolves on its own 2-component vector, so <Z_i Z_j> =
<Z_i><Z_j> and each single-qubit expectation and its derivative come from a
2x2 evolution (the derivative by the two-term shift rule, which is exact for
a single exp(-i theta P / 2) acting on one qubit).
"""
from __future__ import annotations

import numpy as np

from . import circuits, gates, observables, statevec


def energy(n, spec, params, terms, psi0=None) -> float:
    psi = circuits.run(n, spec, psi0, params)
    return float(observables.expectation(psi, terms).real)


def adjoint(n, spec, params, terms, psi0=None):
    params = np.asarray(params, dtype=np.float64)
    psi = circuits.run(n, spec, psi0, params)
    lam = observables.apply_pauli_sum(psi, terms)
    E = float(np.vdot(psi, lam).real)
    grad = np.zeros(params.size)
    for g in reversed(spec):
        U = gates.gate_matrix(g, params)
        if g.pidx >= 0:
            P = gates.generator(g.name)
            Ppsi = statevec.apply(statevec.project_controls(psi, g.controls), P, g.targets)
            grad[g.pidx] += float(np.vdot(lam, Ppsi).imag)
        Ud = U.conj().T
        psi = statevec.apply(psi, Ud, g.targets, g.controls)
        lam = statevec.apply(lam, Ud, g.targets, g.controls)
    return E, grad


def parameter_shift(n, spec, params, terms, psi0=None) -> np.ndarray:
    params = np.asarray(params, dtype=np.float64)
    for g in spec:
        if g.pidx >= 0 and g.controls:
            raise ValueError("two-term shift rule needs uncontrolled rotations")
    grad = np.zeros(params.size)
    for i in range(params.size):
        p = params.copy()
        p[i] += np.pi / 2
        ep = energy(n, spec, p, terms, psi0)
        p[i] -= np.pi
        em = energy(n, spec, p, terms, psi0)
        grad[i] = 0.5 * (ep - em)
    return grad


def finite_difference(n, spec, params, terms, h=1e-6, psi0=None, which=None) -> np.ndarray:
    params = np.asarray(params, dtype=np.float64)
    idx = range(params.size) if which is None else which
    grad = np.zeros(params.size)
    for i in idx:
        p = params.copy()
        p[i] += h
        ep = energy(n, spec, p, terms, psi0)
        p[i] -= 2 * h
        em = energy(n, spec, p, terms, psi0)
        grad[i] = (ep - em) / (2 * h)
    return grad


def _single_qubit_expectations(layers):
    """<Z> and <X> of RZ(phi_L) RY(theta_L) ... RZ(phi_1) RY(theta_1) |0>
    for one qubit; layers = [(theta_l, phi_l), ...] (phi may be None)."""
    v = np.array([1.0, 0.0], dtype=np.complex128)
    for th, ph in layers:
        v = gates.matrix("RY", th) @ v
        if ph is not None:
            v = gates.matrix("RZ", ph) @ v
    z = float(np.vdot(v, gates.PAULI["Z"] @ v).real)
    x = float(np.vdot(v, gates.PAULI["X"] @ v).real)
    return z, x


def product_ring_energy(theta, phi=None, hx=0.5):
    """Energy and gradient of H = sum_i Z_i Z_{(i+1) mod n} + hx sum_i X_i
    for the product state prod_q [prod_l RZ(phi[l, q]) RY(theta[l, q])] |0>.

    theta, phi: arrays (layers, n) (phi may be None: RY layers only).  The
    gradient is returned with the same layout as the parameters of
    ``qsynth.ry_rz_layers`` (per layer: theta of every qubit, then phi of
    every qubit) or, without phi, of ``qsynth.ry_layers`` (layer-major)."""
    theta = np.atleast_2d(np.asarray(theta, dtype=np.float64))
    Lyr, n = theta.shape
    ph = None if phi is None else np.atleast_2d(np.asarray(phi, dtype=np.float64))

    def layers_of(q, th_over=None, ph_over=None):
        out = []
        for l in range(Lyr):
            t = theta[l, q] if th_over is None or th_over[0] != l else th_over[1]
            p = None
            if ph is not None:
                p = ph[l, q] if ph_over is None or ph_over[0] != l else ph_over[1]
            out.append((t, p))
        return out

    zx = [_single_qubit_expectations(layers_of(q)) for q in range(n)]
    z = np.array([a for a, _ in zx])
    x = np.array([b for _, b in zx])
    if n < 3:
        raise ValueError("the ring needs at least three qubits")
    ring = [(i, (i + 1) % n) for i in range(n)]
    E = sum(z[i] * z[j] for i, j in ring) + hx * float(np.sum(x))

    def dE(q, dz, dx):
        nb = sum(z[j] for i, j in ring if i == q) + sum(z[i] for i, j in ring if j == q)
        return dz * nb + hx * dx

    per_layer = 2 if ph is not None else 1
    grad = np.zeros(Lyr * n * per_layer)
    for l in range(Lyr):
        for q in range(n):
            zp, xp = _single_qubit_expectations(layers_of(q, th_over=(l, theta[l, q] + np.pi / 2)))
            zm, xm = _single_qubit_expectations(layers_of(q, th_over=(l, theta[l, q] - np.pi / 2)))
            grad[l * n * per_layer + q] = dE(q, 0.5 * (zp - zm), 0.5 * (xp - xm))
            if ph is not None:
                zp, xp = _single_qubit_expectations(layers_of(q, ph_over=(l, ph[l, q] + np.pi / 2)))
                zm, xm = _single_qubit_expectations(layers_of(q, ph_over=(l, ph[l, q] - np.pi / 2)))
                grad[l * n * 2 + n + q] = dE(q, 0.5 * (zp - zm), 0.5 * (xp - xm))
    return float(E), grad
