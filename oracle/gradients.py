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
