"""Pins of the CPU oracle against facts it does not compute itself: textbook
matrix identities, a Kronecker brute force, closed forms (GHZ, QFT of a basis
state, product states), a library FFT, exact exponentials, published
known-answer vectors, and the delta-t^4 Trotter law of Sec. 3.5.

Each pin is chosen so that a plausible mistake (a transposed operand, a wrong
bit order, a dropped term, a wrong sign) fails at least one of them.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import qsynth
from oracle import adiabatic, circuits, gates, gradients, observables, sampling, statevec

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------- gates
@pytest.mark.parametrize("p", ["X", "Y", "Z"])
def test_rotations_are_pauli_exponentials(p):
    # R_P(theta) = exp(-i theta P / 2), by scipy's matrix exponential
    for th in (0.3, 1.7, -2.9):
        assert np.allclose(gates.matrix("R" + p, th), sla.expm(-0.5j * th * gates.PAULI[p]), atol=1e-14)


def test_named_gate_identities():
    H, X, Y, Z = (gates.matrix(k) for k in "HXYZ")
    assert np.allclose(H @ H, np.eye(2))
    assert np.allclose(H @ Z @ H, X)
    assert np.allclose(X @ Y, 1j * Z)
    S, T = gates.matrix("S"), gates.matrix("T")
    assert np.allclose(T @ T, S) and np.allclose(S @ S, Z)
    assert np.allclose(gates.matrix("U1", np.pi), Z)
    # RZ is U1 up to a global phase
    th = 0.77
    assert np.allclose(gates.matrix("RZ", th), np.exp(-0.5j * th) * gates.matrix("U1", th))
    sw = gates.matrix("SWAP")
    assert np.allclose(sw @ sw, np.eye(4))


# --------------------------------------------------------------- bit convention
def test_big_endian_bit_convention():
    n = 4
    # X on qubit 0 of |0000> lands on the most significant bit
    psi = statevec.apply(statevec.zeros(n), gates.matrix("X"), (0,))
    assert np.argmax(np.abs(psi)) == 8
    # CNOT control 0 -> target 3 maps |1000> to |1001>
    psi = statevec.apply(statevec.basis(n, 8), gates.matrix("X"), (3,), (0,))
    assert np.argmax(np.abs(psi)) == 9
    # control not satisfied: unchanged
    psi = statevec.apply(statevec.basis(n, 1), gates.matrix("X"), (2,), (0,))
    assert np.argmax(np.abs(psi)) == 1
    # two-qubit matrix: targets[0] is the MSB of the matrix index.
    # |01> on (q1=0, q3=1) with M = |10><01| gives |10>
    M = np.zeros((4, 4), dtype=complex)
    M[2, 1] = 1
    M[1, 2] = M[0, 0] = M[3, 3] = 1
    psi = statevec.apply(statevec.basis(n, 0b0001), M, (1, 3))
    assert np.argmax(np.abs(psi)) == 0b0100


# ------------------------------------------------------------ P1: brute force
@pytest.mark.parametrize("seed", range(6))
def test_apply_matches_kronecker_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = 5 + seed % 2
    psi = qsynth.random_state(n, seed)
    for g in qsynth.random_mixed(n, 12, seed + 100, max_k=3, max_ctrl=2):
        U = gates.gate_matrix(g)
        a = statevec.apply(psi, U, g.targets, g.controls)
        b = statevec.full_unitary(n, U, g.targets, g.controls) @ psi
        assert np.allclose(a, b, atol=1e-13), g
        psi = a
    del rng


def test_circuit_unitary_is_unitary_and_matches_run():
    n = 5
    spec = qsynth.random_mixed(n, 25, 7, max_k=3, max_ctrl=2)
    U = circuits.circuit_unitary(n, spec)
    assert np.allclose(U.conj().T @ U, np.eye(1 << n), atol=1e-12)
    psi0 = qsynth.random_state(n, 3)
    assert np.allclose(U @ psi0, circuits.run(n, spec, psi0), atol=1e-12)


# ------------------------------------------------------------- P2: GHZ closed form
@pytest.mark.parametrize("n", [2, 5, 9, 14])
def test_ghz_closed_form(n):
    psi = circuits.run(n, qsynth.ghz(n))
    exp = np.zeros(1 << n, dtype=complex)
    exp[0] = exp[-1] = 2 ** -0.5
    assert np.max(np.abs(psi - exp)) < 1e-14


# ------------------------------------------------------------- P3 / P4: QFT
@pytest.mark.parametrize("n", [1, 3, 6, 10])
def test_qft_basis_closed_form(n):
    spec = qsynth.qft(n)
    assert sum(g.name in ("H", "U1") for g in spec) == n * (n + 1) // 2
    assert sum(g.name == "SWAP" for g in spec) == n // 2
    x = qsynth.random_basis_index(n, 11)
    psi = circuits.run(n, spec, statevec.basis(n, x))
    exp = circuits.qft_basis_amplitudes(n, x, np.arange(1 << n))
    assert np.max(np.abs(psi - exp)) < 1e-13


@pytest.mark.parametrize("n", [4, 8, 11])
def test_qft_random_state_matches_fft(n):
    psi0 = qsynth.random_state(n, n)
    psi = circuits.run(n, qsynth.qft(n), psi0)
    assert np.max(np.abs(psi - circuits.qft_via_fft(psi0))) < 1e-13


def test_qft_closed_form_exact_at_large_n():
    # the closed form uses exact modular integer arithmetic: compare with a direct
    # big-integer evaluation at n = 30 for a few indices
    n, x = 30, 0x2F0F1234
    ys = np.array([0, 1, 12345, (1 << 30) - 1, 0x15555555])
    got = circuits.qft_basis_amplitudes(n, x, ys)
    for y, g in zip(ys, got):
        ang = 2 * np.pi * ((int(x) * int(y)) % (1 << n)) / (1 << n)
        assert abs(g - np.exp(1j * ang) * 2 ** (-n / 2)) < 1e-18


# ------------------------------------------------------------- P5: product state
def test_product_state_closed_form():
    n = 8
    rng = np.random.default_rng(5)
    th, ph = rng.uniform(0, 2 * np.pi, n), rng.uniform(0, 2 * np.pi, n)
    params = np.stack([th, ph], axis=1)[None]
    psi = circuits.run(n, qsynth.ry_rz_cz_layers(n, params), params=params.reshape(-1))
    exp = circuits.product_state_amplitudes(n, th, ph, np.arange(1 << n))
    assert np.max(np.abs(psi - exp)) < 1e-14


# ------------------------------------------------------------- P6 / P7 invariants
def test_norm_and_inverse():
    n = 7
    spec = qsynth.random_mixed(n, 40, 9, max_k=3, max_ctrl=2)
    psi0 = qsynth.random_state(n, 9)
    psi = circuits.run(n, spec, psi0)
    assert abs(observables.norm2(psi) - 1) < 1e-13
    back = circuits.run(n, circuits.inverse(spec), psi)
    assert np.max(np.abs(back - psi0)) < 1e-13


# ------------------------------------------------------------- P8 expectation
def test_expectation_closed_forms():
    n = 6
    zz = qsynth.zz_chain(n, periodic=False)
    assert abs(observables.expectation(statevec.zeros(n), zz) - (n - 1)) < 1e-14
    xs = [(1.0, qsynth.pauli_string(n, {i: "X"})) for i in range(n)]
    assert abs(observables.expectation(statevec.plus(n), xs) - n) < 1e-13
    rng = np.random.default_rng(1)
    th = rng.uniform(0, 2 * np.pi, n)
    psi = statevec.zeros(n)
    for q in range(n):
        psi = statevec.apply(psi, gates.matrix("RY", th[q]), (q,))
    for q in range(n):
        ez = observables.expectation(psi, [(1.0, qsynth.pauli_string(n, {q: "Z"}))])
        ex = observables.expectation(psi, [(1.0, qsynth.pauli_string(n, {q: "X"}))])
        ey = observables.expectation(psi, [(1.0, qsynth.pauli_string(n, {q: "Y"}))])
        assert abs(ez - np.cos(th[q])) < 1e-14
        assert abs(ex - np.sin(th[q])) < 1e-14
        assert abs(ey) < 1e-14
    e = observables.expectation(psi, [(1.0, qsynth.pauli_string(n, {1: "Z", 4: "Z"}))])
    assert abs(e - np.cos(th[1]) * np.cos(th[4])) < 1e-14


def test_expectation_matches_dense_matrix():
    n = 6
    terms = qsynth.random_pauli_sum(n, 15, 4)
    psi = qsynth.random_state(n, 4)
    H = observables.dense_pauli_sum(n, terms)
    assert np.allclose(H, H.conj().T)
    assert abs(observables.expectation(psi, terms) - np.vdot(psi, H @ psi)) < 1e-13
    assert abs(observables.expectation(psi, terms).imag) < 1e-13


def test_ising_energy_matches_pauli_sum():
    n = 6
    J, h = qsynth.ising_couplings(n, 2)
    E = observables.ising_energies(J, h)
    Hd = observables.dense_pauli_sum(n, observables.ising_terms(J, h))
    assert np.allclose(np.diag(Hd).real, E, atol=1e-13)
    assert np.allclose(Hd - np.diag(np.diag(Hd)), 0)


# ------------------------------------------------------------- P9 sampling
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        assert sampling.philox4x32_10(v[0:4], v[4:6]) == tuple(v[6:10])


def test_philox_uniforms_are_uniform():
    u = sampling.philox_uniforms(12345, 20000)
    assert np.all((u >= 0) & (u < 1))
    hist, _ = np.histogram(u, bins=20, range=(0, 1))
    chi2 = np.sum((hist - 1000.0) ** 2 / 1000.0)
    assert chi2 < 45  # 19 dof, p ~ 1e-3


def test_sampling_prefix_equals_marginal_inverse_cdf():
    n = 8
    psi = qsynth.random_state(n, 21)
    u = np.random.default_rng(3).random(5000)
    got = sampling.sample(psi, [0, 1, 2], u)
    pm = sampling.marginal(psi, [0, 1, 2])
    ref = np.searchsorted(np.cumsum(pm), u * pm.sum(), side="right")
    assert np.array_equal(got, ref)


def test_sampling_matches_traced_out_marginal_statistically():
    n = 7
    psi = qsynth.random_state(n, 22)
    q = [5, 1, 3]
    u = sampling.philox_uniforms(99, 40000)
    y = sampling.sample(psi, q, u)
    p = sampling.marginal(psi, q)
    cnt = np.bincount(y, minlength=p.size)
    assert 0.5 * np.sum(np.abs(cnt / cnt.sum() - p)) < 0.02
    # marginal of a product of |0>/|1> on those qubits is a single outcome
    psi_b = statevec.basis(n, 0b0100010)  # qubits 1 and 5 set
    assert np.allclose(sampling.marginal(psi_b, q), np.eye(8)[0b110])


def test_sampling_ghz_and_uniform():
    n = 10
    psi = circuits.run(n, qsynth.ghz(n))
    y = sampling.sample(psi, list(range(n)), sampling.philox_uniforms(5, 2000))
    assert set(np.unique(y)) == {0, (1 << n) - 1}
    hplus = statevec.plus(n)
    u = np.random.default_rng(0).random(1000)
    assert np.array_equal(sampling.sample(hplus, list(range(n)), u), np.floor(u * (1 << n)).astype(int))


# ------------------------------------------------------------- P11 Trotter
def tfim_setup(n):
    z = observables.spins(n)
    E = -sum(z[:, i] * z[:, (i + 1) % n] for i in range(n))
    return E


def test_trotter_error_scales_as_dt4():
    n, T, hx = 10, 1.0, 1.0
    E = tfim_setup(n)
    cx = lambda s: (1 - s) + s * hx  # noqa: E731   H1 = -sum(ZZ + h X)
    infid = []
    dts = [0.1, 0.05, 0.025, 0.0125]
    for dt in dts:
        a = adiabatic.trotter(n, E, T, dt, cx)
        b = adiabatic.exact_piecewise(n, E, T, dt, cx)
        infid.append(1 - abs(np.vdot(a, b)) ** 2)
    slope = np.polyfit(np.log(dts), np.log(infid), 1)[0]
    assert 3.6 < slope < 4.4, (slope, infid)


def test_trotter_j0_factorises():
    n = 6
    _, h = qsynth.ising_couplings(n, 3)
    E = observables.ising_energies(np.zeros((n, n)), h)
    psi = adiabatic.trotter(n, E, 1.0, 0.05)
    prod = np.array([1.0 + 0j])
    for q in range(n):
        prod = np.kron(prod, adiabatic.single_qubit_trotter(h[q], 1.0, 0.05))
    assert np.max(np.abs(psi - prod)) < 1e-13


def test_trotter_exact_for_commuting_parts():
    # with E = 0 the plus state is an eigenstate of every RX: only a global phase
    n = 5
    psi = adiabatic.trotter(n, np.zeros(1 << n), 1.0, 0.1)
    assert np.max(np.abs(np.abs(psi) - 2 ** (-n / 2))) < 1e-14
    phase = psi / statevec.plus(n)
    assert np.max(np.abs(phase - phase[0])) < 1e-14
    # total phase: sum over steps of n * (1 - s_k) * dt
    exp_phase = np.exp(1j * n * sum((1 - (k + 0.5) * 0.1) * 0.1 for k in range(10)))
    assert abs(phase[0] - exp_phase) < 1e-13


def test_adiabatic_energy_bounds_and_ground_state():
    n = 8
    J, h = qsynth.ising_couplings(n, 1)
    E = observables.ising_energies(J, h)
    psi = adiabatic.trotter(n, E, 10.0, 0.05)
    e = adiabatic.energy(psi, E)
    assert E.min() - 1e-12 <= e <= E.max()
    # a slow sweep ends close to the ground state (adiabatic theorem, Sec. 2.6)
    assert np.abs(psi[np.argmin(E)]) ** 2 > 0.5
    # eigh of the dense H1 finds the same ground state
    w, v = np.linalg.eigh(np.diag(E))
    assert abs(w[0] - E.min()) < 1e-12 and np.argmax(np.abs(v[:, 0])) == np.argmin(E)


# ------------------------------------------------------------- P10 gradients
def test_gradients_three_routes_agree():
    n, spec, params, terms = qsynth.gradient_20q(seed=3, n=5, layers=3)
    E, g_adj = gradients.adjoint(n, spec, params, terms)
    assert abs(E - gradients.energy(n, spec, params, terms)) < 1e-13
    g_ps = gradients.parameter_shift(n, spec, params, terms)
    g_fd = gradients.finite_difference(n, spec, params, terms, h=1e-6)
    assert np.max(np.abs(g_adj - g_ps)) < 1e-12
    assert np.max(np.abs(g_adj - g_fd)) < 1e-6


def test_adjoint_handles_controlled_rotations():
    n = 4
    spec = [qsynth.gate("RY", (0,), theta=0.4, pidx=0), qsynth.gate("H", (1,)),
            qsynth.gate("RX", (2,), (1,), theta=0.9, pidx=1),
            qsynth.gate("RZ", (3,), (0, 2), theta=1.3, pidx=2), qsynth.gate("X", (3,), (2,))]
    params = np.array([0.4, 0.9, 1.3])
    terms = qsynth.random_pauli_sum(n, 6, 8)
    _, g_adj = gradients.adjoint(n, spec, params, terms)
    g_fd = gradients.finite_difference(n, spec, params, terms, h=1e-6)
    assert np.max(np.abs(g_adj - g_fd)) < 1e-7


# ------------------------------------------------------- gate signs (S, T)
def test_s_and_t_signs_from_rz_exponentials():
    # S and T are Z rotations by pi/2 and pi/4 up to a global phase:
    # S = e^{i pi/4} exp(-i (pi/2) Z/2), T = e^{i pi/8} exp(-i (pi/4) Z/2);
    # the conjugate matrices (which also satisfy T T = S, S S = Z) fail this
    Z = np.diag([1.0, -1.0]).astype(complex)
    S_ref = np.exp(0.25j * np.pi) * sla.expm(-0.5j * (np.pi / 2) * Z)
    T_ref = np.exp(0.125j * np.pi) * sla.expm(-0.5j * (np.pi / 4) * Z)
    assert np.allclose(gates.matrix("S"), S_ref, atol=1e-15)
    assert np.allclose(gates.matrix("T"), T_ref, atol=1e-15)
    assert not np.allclose(gates.matrix("S").conj(), S_ref)


# ----------------------------------------------- sampling boundary distances
def test_boundary_distance_on_a_dyadic_cdf():
    # four amplitudes 1/2: probabilities 1/4 each, CDF 1/4, 1/2, 3/4, 1 (exact
    # in binary).  A target on an edge has distance 0, one inside an interval
    # the smaller gap to its edges
    psi = np.full(4, 0.5, dtype=complex)
    u = np.array([0.5, 0.6, 0.1, 0.25, 0.875, 0.0])
    idx = sampling.sample_indices(psi, u)
    assert list(idx) == [2, 2, 0, 1, 3, 0]
    d = sampling.boundary_distance(psi, u, idx)
    assert np.allclose(d, [0.0, 0.1, 0.1, 0.0, 0.125, 0.0], atol=1e-15)
    # an index that is not the sampled one: distance to that interval's edges
    d2 = sampling.boundary_distance(psi, np.array([0.6]), np.array([0]))
    assert np.isclose(d2[0], 0.35)


# ------------------------- diagonal gates after the rotations: sum Z unchanged
@pytest.mark.parametrize("n", [4, 6])
def test_phases_after_ry_layer_leave_z_sum_closed_form(n):
    # controlled phases are diagonal: they commute with every Z_i, so after
    # RY(t_q)|0> they change neither <sum Z_i> = sum cos t_q nor its gradient
    # -sin t_q, whatever their angles
    th = np.random.default_rng(n + 7).uniform(0, 2 * np.pi, n)
    spec = qsynth.ry_then_phases(n, th, seed=n)
    assert sum(g.name == "U1" for g in spec) >= n
    E, g = gradients.adjoint(n, spec, th, qsynth.z_sum(n))
    assert abs(E - float(np.sum(np.cos(th)))) < 1e-13
    assert np.max(np.abs(g + np.sin(th))) < 1e-13
    # the phases do act on the state
    psi = circuits.run(n, spec, None, th)
    psi_ry = circuits.run(n, qsynth.ry_layers(n, th), None, th)
    assert np.max(np.abs(psi - psi_ry)) > 1e-3


# ------------------------------------------- product-state energy closed form
@pytest.mark.parametrize("n", [3, 6])
def test_ry_layer_ring_energy_closed_form(n):
    # RY(theta_q)|0> has <Z> = cos theta, <X> = sin theta, so for
    # H = sum Z_i Z_{i+1 mod n} + 0.5 sum X_i the energy of one RY layer is
    # E = sum cos t_i cos t_{i+1} + 0.5 sum sin t_i and
    # dE/dt_k = -sin t_k (cos t_{k-1} + cos t_{k+1}) + 0.5 cos t_k
    th = np.random.default_rng(n).uniform(0, 2 * np.pi, n)
    c, s = np.cos(th), np.sin(th)
    E_formula = float(np.sum(c * np.roll(c, -1)) + 0.5 * np.sum(s))
    g_formula = -s * (np.roll(c, 1) + np.roll(c, -1)) + 0.5 * c
    E_cf, g_cf = gradients.product_ring_energy(th[None, :])
    assert abs(E_cf - E_formula) < 1e-13 and np.max(np.abs(g_cf - g_formula)) < 1e-13
    spec = qsynth.ry_layers(n, th)
    E_adj, g_adj = gradients.adjoint(n, spec, th, qsynth.zz_ring_plus_x(n))
    assert abs(E_adj - E_formula) < 1e-13 and np.max(np.abs(g_adj - g_formula)) < 1e-13


def test_product_state_energy_multi_layer_matches_adjoint():
    n, L = 5, 3
    rng = np.random.default_rng(11)
    th, ph = rng.uniform(0, 2 * np.pi, (L, n)), rng.uniform(0, 2 * np.pi, (L, n))
    spec = qsynth.ry_rz_layers(n, th, ph)
    params = np.concatenate([np.concatenate([th[l], ph[l]]) for l in range(L)])
    E_cf, g_cf = gradients.product_ring_energy(th, ph, hx=0.5)
    E_adj, g_adj = gradients.adjoint(n, spec, params, qsynth.zz_ring_plus_x(n))
    assert abs(E_cf - E_adj) < 1e-13
    assert np.max(np.abs(g_cf - g_adj)) < 1e-13


# ------------------------------------------------------ ODE evolution, entropy
def _tfim_terms(n):
    h0 = [(-1.0, qsynth.pauli_string(n, {q: "X"})) for q in range(n)]
    J, h = qsynth.ising_couplings(n, 3)
    return h0, observables.ising_terms(J, h), J, h


def test_rk4_step_is_the_fourth_order_taylor_polynomial():
    # for a constant H the classical Runge-Kutta step is exactly
    # sum_{j<=4} (-i H dt)^j / j! applied to psi
    from oracle import evolution as ev
    n = 4
    h0, h1, _, _ = _tfim_terms(n)
    psi = qsynth.random_state(n, 5)
    H = observables.dense_pauli_sum(n, h1)
    dt = 0.37
    got = ev.rk_step(psi, h1, h1, 0.0, dt, 1.0, ev.RK4_A, ev.RK4_B, ev.RK4_C)
    Z = -1j * dt * H
    term, exp = psi.copy(), psi.copy()
    for j in range(1, 5):
        term = Z @ term / j
        exp = exp + term
    assert np.max(np.abs(got - exp)) < 1e-13


def test_dormand_prince_weights_satisfy_the_order_conditions():
    # quadrature conditions sum b_i c_i^(k-1) = 1/k for k = 1..5 and the row
    # sums of A equal c: a wrong coefficient breaks one of them
    from oracle import evolution as ev
    b, c = np.array(ev.DP_B), np.array(ev.DP_C)
    for k in range(1, 6):
        assert abs(np.sum(b * c ** (k - 1)) - 1.0 / k) < 1e-14, k
    for j in range(1, 6):
        assert abs(sum(ev.DP_A[j]) - c[j]) < 1e-14, j
    A = np.zeros((6, 6))
    for j in range(6):
        A[j, :len(ev.DP_A[j])] = ev.DP_A[j]
    assert abs(b @ A @ c - 1 / 6) < 1e-14 and abs(b @ A @ c ** 2 - 1 / 12) < 1e-14
    assert abs(b @ A @ A @ c - 1 / 24) < 1e-14


@pytest.mark.parametrize("solver,order", [("rk4", 4), ("rk45", 5)])
def test_runge_kutta_global_error_order(solver, order):
    # the final state against the exact piecewise-exponential one on a fine
    # grid: halving dt divides the error by about 2^order
    from oracle import evolution as ev
    n = 4
    h0, h1, _, _ = _tfim_terms(n)
    psi0 = np.full(1 << n, 2.0 ** (-n / 2), dtype=complex)
    T = 1.0
    ref, _, _ = ev.evolve(n, h0, h1, T, 1 / 2048, "exp", psi0)
    errs = []
    for dt in (0.1, 0.05, 0.025):
        psi, _, _ = ev.evolve(n, h0, h1, T, dt, solver, psi0)
        errs.append(np.linalg.norm(psi - ref))
    slope = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
    assert all(order - 0.5 < s < order + 0.7 for s in slope), (errs, slope)


def test_exp_solver_matches_expm_multiply_route():
    # the dense-exponential steps against the oracle's sparse expm_multiply
    # route over the same midpoint grid (H0 = -sum X, H1 = Ising)
    from oracle import evolution as ev
    n = 6
    h0, h1, J, h = _tfim_terms(n)
    E = observables.ising_energies(J, h)
    psi0 = statevec.plus(n)
    a, _, _ = ev.evolve(n, h0, h1, 0.5, 0.05, "exp", psi0)
    b = adiabatic.exact_piecewise(n, E, 0.5, 0.05)
    assert np.max(np.abs(a - b)) < 1e-12


def test_entanglement_entropy_closed_forms():
    from oracle import evolution as ev
    n = 6
    # product state: 0; GHZ: log 2 for every cut; Bell pairs (0,3), (1,4):
    # the cut after qubit 2 crosses two of them
    prod = circuits.run(n, [qsynth.gate("RY", (q,), theta=0.3 + q) for q in range(n)])
    ghz = circuits.run(n, qsynth.ghz(n))
    bell = circuits.run(n, [qsynth.gate("H", (0,)), qsynth.gate("X", (3,), (0,)),
                            qsynth.gate("H", (1,)), qsynth.gate("X", (4,), (1,))])
    for a in range(1, n):
        assert abs(ev.entanglement_entropy(prod, a)) < 1e-12
        assert abs(ev.entanglement_entropy(ghz, a) - np.log(2)) < 1e-12
    assert abs(ev.entanglement_entropy(bell, 3) - 2 * np.log(2)) < 1e-12
    assert abs(ev.entanglement_entropy(bell, 1) - np.log(2)) < 1e-12
    r = qsynth.random_state(n, 8)
    for a in range(1, n):  # S(A) = S(B), bounded by min(a, n - a) log 2
        assert abs(ev.entanglement_entropy(r, a) - ev.entanglement_entropy(
            r.reshape((2,) * n).transpose(list(range(a, n)) + list(range(a))).reshape(-1), n - a)) < 1e-12
        assert ev.entanglement_entropy(r, a) <= min(a, n - a) * np.log(2) + 1e-12


# ------------------------------------------------ density matrices, channels
@pytest.mark.parametrize("name", ["depolarizing", "amplitude_damping", "phase_damping", "bit_flip", "phase_flip"])
def test_named_channels_are_trace_preserving(name):
    from oracle import density
    for p in (0.0, 0.13, 0.7, 1.0):
        K = density.kraus(name, p)
        S = sum(k.conj().T @ k for k in K)
        assert np.allclose(S, np.eye(2), atol=1e-14), (name, p)


def test_named_channels_fixed_points_and_limits():
    from oracle import density
    rng = np.random.default_rng(2)
    psi = qsynth.random_state(1, 4)
    rho = density.pure(psi)
    # depolarising with p = 1 gives the maximally mixed state; with p, the
    # Bloch vector shrinks by 1 - p
    assert np.allclose(density.apply_channel(rho, density.kraus("depolarizing", 1.0), (0,)), np.eye(2) / 2, atol=1e-14)
    r = density.apply_channel(rho, density.kraus("depolarizing", 0.3), (0,))
    assert np.allclose(r, 0.7 * rho + 0.3 * np.eye(2) / 2, atol=1e-14)
    # amplitude damping with gamma = 1 ends in |0><0|; gamma scales the excited
    # population and sqrt(1 - gamma) the coherence
    assert np.allclose(density.apply_channel(rho, density.kraus("amplitude_damping", 1.0), (0,)), np.diag([1, 0]),
                       atol=1e-14)
    g = 0.4
    r = density.apply_channel(rho, density.kraus("amplitude_damping", g), (0,))
    assert np.isclose(r[1, 1], (1 - g) * rho[1, 1]) and np.isclose(r[0, 1], np.sqrt(1 - g) * rho[0, 1])
    # phase damping keeps populations and scales coherences by sqrt(1 - lambda)
    r = density.apply_channel(rho, density.kraus("phase_damping", 0.64), (0,))
    assert np.allclose(np.diag(r), np.diag(rho)) and np.isclose(r[0, 1], 0.6 * rho[0, 1])
    # bit flip: (1 - p) rho + p X rho X
    X = gates.PAULI["X"]
    r = density.apply_channel(rho, density.kraus("bit_flip", 0.2), (0,))
    assert np.allclose(r, 0.8 * rho + 0.2 * X @ rho @ X)
    del rng


def test_density_matrix_of_a_unitary_circuit_is_the_pure_state():
    from oracle import density
    n = 4
    spec = qsynth.random_mixed(n, 20, 3, max_k=2, max_ctrl=1)
    psi = circuits.run(n, spec)
    rho = density.pure(statevec.zeros(n))
    for g in spec:
        rho = density.apply_gate(rho, gates.gate_matrix(g), g.targets, g.controls)
    assert np.allclose(rho, density.pure(psi), atol=1e-13)
    terms = qsynth.random_pauli_sum(n, 8, 1)
    assert abs(density.expectation(rho, terms) - observables.expectation(psi, terms).real) < 1e-12
    # a channel on two qubits (Kraus operators K x K) keeps the trace
    K = density.kraus("amplitude_damping", 0.3)
    K2 = [np.kron(a, b) for a in K for b in K]
    rho2 = density.apply_channel(rho, K2, (1, 3))
    assert abs(np.trace(rho2) - 1) < 1e-13


def test_density_run_of_noisy_layers_keeps_trace_and_hermiticity():
    from oracle import density
    n = 4
    spec, params = qsynth.noisy_layers(n, 3, 7)
    rho = density.run(n, spec, params=params)
    assert abs(np.trace(rho) - 1) < 1e-13
    assert np.allclose(rho, rho.conj().T, atol=1e-14)
    assert np.min(np.linalg.eigvalsh(rho)) > -1e-13
    # without channels: the pure state of the same gates
    clean = [g for g in spec if not g.name.startswith("CH:")]
    assert np.allclose(density.run(n, clean, params=params),
                       density.pure(circuits.run(n, clean, params=params)), atol=1e-13)
