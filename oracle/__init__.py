"""CPU oracle for the dense state-vector simulator -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct complex128 implementation of what the GPU
path computes, written from the paper (Qibo, arXiv:2009.01845): the state is a
rank-N tensor psi(sigma_1..sigma_N) and a gate acts by the contraction of
Eq. (1) (Sec. 2.3), controls select the sub-tensor where every control qubit is
1 (Sec. 2.4.1), measurements sample the traced-out outcome distribution
(Sec. 2.4.2), adiabatic evolution follows Eq. (3) with a Trotter split
(Sec. 2.6).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
and never imports it; the only common module is ``qsynth`` (seeded inputs,
which holds no simulation arithmetic).

Module map
  gates       O2   named gate matrices and Pauli generators
  statevec    O1/O3/O4  tensor-contraction apply, Kronecker brute force
  circuits    circuit runner, QFT closed forms
  observables O5   Pauli sums, Ising energies, dense Hamiltonians
  sampling    O6   trace-out marginals, inverse-CDF sampling, Philox4x32-10
  adiabatic   O8   second-order Trotter steps and the exact piecewise reference
  gradients   O9   adjoint recurrence, parameter shift, finite differences
  evolution        Runge-Kutta and exponential integration of the Schroedinger
                   equation (Sec. 2.6), entanglement entropy (Sec. 2.4.4)
  density          density matrices, gates and Kraus channels (Sec. 2.4.3)
"""
from . import gates, statevec, circuits, observables, sampling, adiabatic, gradients, evolution, density  # noqa: F401
