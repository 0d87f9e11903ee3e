"""Parity of the HIP path with the CPU oracle, element by element, on seeded
inputs.  Tolerances: max-abs amplitude error 1e-12 (complex128) and 1e-5
(complex64); complex64 runs are compared with the oracle applied to the
complex64-rounded input."""
import numpy as np
import pytest

import qsynth
from oracle import adiabatic as oad
from oracle import circuits as ocirc
from oracle import gates as ogates
from oracle import gradients as ograd
from oracle import observables as oobs
from oracle import sampling as osamp
from oracle import statevec as osv

from gpu_util import TOL, assert_samples_match, banner, gpu_state, maxabs, oracle_input

pytestmark = pytest.mark.gpu
DTS = ["c64", "c128"]


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2009_01845_amd import api as a
    return a


# ---------------------------------------------------------------- single gates
@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("n", [1, 2, 3, 6, 11, 14])
def test_single_gates(api, dt, n):
    banner("single gates", dt, n)
    psi0 = qsynth.random_state(n, 100 + n)
    st = gpu_state(api, n, dt, psi0)
    ref = oracle_input(psi0, dt)
    spec = qsynth.random_mixed(n, 30, 7 + n, max_k=min(n, 5), max_ctrl=min(2, n - 1))
    worst = 0.0
    for g in spec:
        U = ogates.gate_matrix(g)
        api.apply(st.h, U, g.targets, g.controls)
        ref = osv.apply(ref, U, g.targets, g.controls)
        if n <= 6:
            worst = max(worst, maxabs(st.download(), ref))
            assert worst < TOL[dt], (g, worst)
    assert maxabs(st.download(), ref) < TOL[dt]


@pytest.mark.parametrize("dt", DTS)
def test_every_bit_position_1q_and_controlled(api, dt):
    n = 13
    banner("every bit", dt, n)
    psi0 = qsynth.random_state(n, 5)
    st = gpu_state(api, n, dt, psi0)
    ref = oracle_input(psi0, dt)
    rng = np.random.default_rng(1)
    for q in range(n):
        U = qsynth.haar_unitary(2, rng)
        api.apply(st.h, U, (q,))
        ref = osv.apply(ref, U, (q,))
        c = (q + 5) % n
        api.apply(st.h, ogates.matrix("RY", 0.3 + q), (q,), (c,))
        ref = osv.apply(ref, ogates.matrix("RY", 0.3 + q), (q,), (c,))
    assert maxabs(st.download(), ref) < TOL[dt]


# ---------------------------------------------------------------- circuits
TILES = [dict(), dict(tile_bits=6, low_bits=1), dict(tile_bits=8, low_bits=3), dict(tile_bits=10, low_bits=4),
         dict(tile_bits=12, low_bits=6), dict(tile_bits=13, low_bits=8), dict(lane_ops=1),
         dict(tile_bits=13, low_bits=8, lane_ops=1)]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("ti", range(len(TILES)))
def test_random_circuit_tilings(api, dt, ti):
    opts = dict(TILES[ti])
    if dt == "c128" and opts.get("tile_bits", 0) > 12:
        opts["tile_bits"] = 12
    n = 15
    banner("random circuit", dt, opts)
    spec = qsynth.random_mixed(n, 160, 42, max_k=3, max_ctrl=2)
    psi0 = qsynth.random_state(n, 9)
    c = api.Circuit.from_spec(n, spec, **opts)
    st = gpu_state(api, n, dt, psi0)
    c.run(st)
    ref = ocirc.run(n, spec, oracle_input(psi0, dt))
    assert maxabs(st.download(), ref) < TOL[dt]


@pytest.mark.parametrize("dt", DTS)
def test_rollout_schedule_plans_vs_oracle(api, dt):
    # plans whose high tile bits the one-step rollout chose: a 2-qubit
    # brickwork on 8-bit tiles (one LDS sweep per op) and twelve RY + CZ-ring
    # layers at 20 qubits on 12-bit register-staged tiles (forward and adjoint)
    banner("rollout plans", dt)
    n = 16
    rng = np.random.default_rng(5)
    brick = [qsynth.gate("MAT", (q, q + 1), mat=qsynth.haar_unitary(4, rng))
             for d in range(8) for q in range(d % 2, n - 1, 2)]
    c = api.Circuit.from_spec(n, brick, tile_bits=8, low_bits=3)
    assert c.schedule() == 2
    psi0 = qsynth.random_state(n, 61)
    st = gpu_state(api, n, dt, psi0)
    c.run(st)
    assert maxabs(st.download(), ocirc.run(n, brick, oracle_input(psi0, dt))) < TOL[dt]
    n, spec, params, terms = qsynth.gradient_20q(seed=0, n=20, layers=12)
    # rows of 2^6 amplitudes: with rows left open the planner takes the
    # shorter-row plan here, which has fewer passes
    c = api.Circuit.from_spec(n, spec, low_bits=6)
    assert c.schedule() == 2
    psi, lam = api.State(n, dt), api.State(n, dt)
    c.run(psi, params)
    assert maxabs(psi.download(), ocirc.run(n, spec, None, params)) < TOL[dt]
    if dt == "c128":
        H = api.Observable.pauli_sum(n, terms)
        e, g = api.adjoint(c.h, params, H.h, psi.h, lam.h, c.nparams)
        e_ref, g_ref = ograd.adjoint(n, spec, params, terms)
        assert abs(e - e_ref) < 1e-10 and np.max(np.abs(g - g_ref)) < 1e-10


@pytest.mark.parametrize("dt", DTS)
def test_variational_10q_depth20(api, dt):
    banner("variational 10q", dt)
    n, spec, params, terms = qsynth.variational_10q(0)
    c = api.Circuit.from_spec(n, spec)
    st = gpu_state(api, n, dt)
    c.run(st, params)
    ref = ocirc.run(n, spec, None, params)
    assert maxabs(st.download(), ref) < TOL[dt]
    H = api.Observable.pauli_sum(n, terms)
    e = H.expectation(st)
    assert abs(e - oobs.expectation(ref, terms).real) < (1e-12 if dt == "c128" else 1e-5)


@pytest.mark.parametrize("dt", DTS)
def test_rotation_angles_across_periods(api, dt):
    # X and Y rotation angles on multiples of pi/2 and between them, tiny,
    # negative and beyond 4 pi; forward state and adjoint gradient against
    # the oracle
    n = 14
    banner("rotation angles", dt)
    k = np.arange(-8, 9)
    angles = np.concatenate([k * np.pi / 2, k * np.pi + 0.3, [1e-9, -1e-9, 13.7, -21.2]])
    spec, params = [], []
    for layer in range(3):
        for q in range(n):
            spec.append(qsynth.gate("RY" if (q + layer) % 2 else "RX", (q,), pidx=len(params)))
            params.append(angles[(layer * n + q) % len(angles)])
        spec += [qsynth.gate("Z", (q + 1,), (q,)) for q in range(n - 1)]
    params = np.array(params)
    c = api.Circuit.from_spec(n, spec)
    psi0 = qsynth.random_state(n, 31)
    st = gpu_state(api, n, dt, psi0)
    c.run(st, params)
    ref = ocirc.run(n, spec, oracle_input(psi0, dt), params)
    assert maxabs(st.download(), ref) < TOL[dt]
    terms = qsynth.zz_ring_plus_x(n)
    E_ref, g_ref = ograd.adjoint(n, spec, params, terms)
    psi, lam = api.State(n, dt), api.State(n, dt)
    c.run(psi, params)
    H = api.Observable.pauli_sum(n, terms)
    E, g = api.adjoint(c.h, params, H.h, psi.h, lam.h, c.nparams)
    tol = 1e-10 if dt == "c128" else 1e-4
    assert abs(E - E_ref) < tol
    assert np.max(np.abs(g - g_ref)) < tol


@pytest.mark.parametrize("dt", DTS)
def test_qft_random_state_vs_fft(api, dt):
    n = 18
    banner("qft fft", dt, n)
    psi0 = qsynth.random_state(n, 3)
    c = api.Circuit.from_spec(n, qsynth.qft(n))
    st = gpu_state(api, n, dt, psi0)
    c.run(st)
    assert maxabs(st.download(), ocirc.qft_via_fft(oracle_input(psi0, dt))) < TOL[dt]


@pytest.mark.parametrize("dt,low_bits", [("c64", 7), ("c128", 6), ("c128", 7)])
def test_qft_long_rows_vs_fft(api, dt, low_bits):
    # rows longer than the default: the closing bit reversal still fits the
    # permutation kernel's tile
    n = 16
    banner("qft long rows", dt, n, low_bits)
    psi0 = qsynth.random_state(n, 4)
    c = api.Circuit.from_spec(n, qsynth.qft(n), low_bits=low_bits)
    st = gpu_state(api, n, dt, psi0)
    c.run(st)
    assert maxabs(st.download(), ocirc.qft_via_fft(oracle_input(psi0, dt))) < TOL[dt]


@pytest.mark.parametrize("dt,n", [("c64", 28), ("c128", 28), ("c64", 30)])
def test_qft_basis_closed_form_large(api, dt, n):
    banner("qft basis large", dt, n)
    import torch
    x = qsynth.random_basis_index(n, 2024 + n)
    c = api.Circuit.from_spec(n, qsynth.qft(n))
    st = api.State(n, dt)
    st.set_basis(x)
    c.run(st)
    rng = np.random.default_rng(0)
    ys = np.concatenate([[0, 1, (1 << n) - 1, 1 << (n - 1)], rng.integers(0, 1 << n, 200000)]).astype(np.int64)
    got = st.tensor[torch.from_numpy(ys).cuda()].cpu().numpy()
    exp = ocirc.qft_basis_amplitudes(n, x, ys.astype(np.uint64))
    assert maxabs(got, exp) < TOL[dt]
    assert abs(st.norm2() - 1) < (1e-12 if dt == "c128" else 1e-5)
    del st
    torch.cuda.empty_cache()


def test_ghz_and_product_state_at_30_qubits(api):
    import torch
    n = 30
    banner("ghz / product 30")
    st = api.State(n, "c64")
    api.Circuit.from_spec(n, qsynth.ghz(n)).run(st)
    rng = np.random.default_rng(1)
    ys = np.concatenate([[0, (1 << n) - 1], rng.integers(1, (1 << n) - 1, 100000)]).astype(np.int64)
    got = st.tensor[torch.from_numpy(ys).cuda()].cpu().numpy()
    exp = np.zeros(ys.size, dtype=complex)
    exp[0] = exp[1] = 2 ** -0.5
    assert maxabs(got, exp) < 1e-6
    # one RY/RZ/CZ layer from |0..0>: closed-form product state
    th, ph = rng.uniform(0, 2 * np.pi, n), rng.uniform(0, 2 * np.pi, n)
    params = np.stack([th, ph], axis=1)[None]
    st.set_basis(0)
    api.Circuit.from_spec(n, qsynth.ry_rz_cz_layers(n, params)).run(st, params.reshape(-1))
    got = st.tensor[torch.from_numpy(ys).cuda()].cpu().numpy()
    exp = ocirc.product_state_amplitudes(n, th, ph, ys)
    assert maxabs(got, exp) < 1e-5
    del st
    torch.cuda.empty_cache()


# ---------------------------------------------------------------- observables
@pytest.mark.parametrize("dt", DTS)
def test_expectation_and_norm(api, dt):
    n = 12
    banner("expectation", dt)
    psi0 = qsynth.random_state(n, 77)
    st = gpu_state(api, n, dt, psi0)
    ref = oracle_input(psi0, dt)
    terms = qsynth.random_pauli_sum(n, 40, 3)
    H = api.Observable.pauli_sum(n, terms)
    tol = 1e-12 if dt == "c128" else 1e-6
    assert abs(H.expectation(st) - oobs.expectation(ref, terms).real) < tol
    assert abs(st.norm2() - oobs.norm2(ref)) < tol
    J, h = qsynth.ising_couplings(n, 4)
    I = api.Observable.ising(n, J, h)
    assert abs(I.expectation(st) - float(np.sum(np.abs(ref) ** 2 * oobs.ising_energies(J, h)))) < tol * 10


@pytest.mark.parametrize("dt", DTS)
def test_sign_only_phases_ry_cz_ring(api, dt):
    # CZ rings, CZ pairs and Z gates only flip signs: the planner marks such
    # phase ops and the kernel applies them as parity masks
    n = 16
    banner("sign phases", dt)
    rng = np.random.default_rng(21)
    _, spec, params, terms = qsynth.gradient_20q(seed=5, n=n, layers=4)
    extra = [qsynth.gate("Z", (int(q),)) for q in rng.integers(0, n, 5)]
    extra += [qsynth.gate("Z", (int(a),), (int(b),)) for a, b in rng.permutation(n).reshape(-1, 2)[:4]]
    spec = spec[: len(spec) // 2] + extra + spec[len(spec) // 2:]
    c = api.Circuit.from_spec(n, spec)
    st = gpu_state(api, n, dt)
    c.run(st, params)
    ref = ocirc.run(n, spec, None, params)
    assert maxabs(st.download(), ref) < TOL[dt]
    from oracle import gradients as ograd
    gtol = 1e-10 if dt == "c128" else 1e-4
    psi, lam = api.State(n, dt), api.State(n, dt)
    c.run(psi, params)
    H = api.Observable.pauli_sum(n, terms)
    e, g = api.adjoint(c.h, params, H.h, psi.h, lam.h, c.nparams)
    e_ref, g_ref = ograd.adjoint(n, spec, params, terms)
    assert abs(e - e_ref) < gtol and np.max(np.abs(g - g_ref)) < gtol


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("n", [5, 15, 20])
def test_diagonal_polynomial_expectation(api, dt, n):
    # diagonal groups with at most two Z factors per term take the polynomial
    # path (rows of 2^12 amplitudes, high-bit and cross terms per row); a
    # group with a three-Z term takes the generic term loop
    banner("diagonal expectation", dt, n)
    psi0 = qsynth.random_state(n, 300 + n)
    st = gpu_state(api, n, dt, psi0)
    ref = oracle_input(psi0, dt)
    tol = 1e-11 if dt == "c128" else 2e-6
    J, h = qsynth.ising_couplings(n, n)
    I = api.Observable.ising(n, J, h)
    e_ref = float(np.sum(np.abs(ref) ** 2 * oobs.ising_energies(J, h)))
    assert abs(I.expectation(st) - e_ref) < tol * max(1.0, abs(e_ref))
    for terms in (qsynth.zz_ring_plus_x(n),
                  qsynth.zz_chain(n, periodic=False) + [(0.7, qsynth.pauli_string(n, {0: "Z", 1: "Z", n - 1: "Z"}))]):
        H = api.Observable.pauli_sum(n, terms)
        assert abs(H.expectation(st) - oobs.expectation(ref, terms).real) < tol * n


@pytest.mark.parametrize("dt", DTS)
def test_pauli_tile_sets_expectation_and_adjoint(api, dt):
    # flip masks spread over every bit (several tile sets), Y factors, a
    # diagonal group with a three-Z term (no polynomial form), and an
    # observable with only off-diagonal groups (the first set writes lambda)
    n = 16
    banner("pauli sets", dt)
    rng = np.random.default_rng(17)
    psi0 = qsynth.random_state(n, 23)
    st = gpu_state(api, n, dt, psi0)
    ref = oracle_input(psi0, dt)
    tol = 1e-11 if dt == "c128" else 2e-6
    mixed = [(float(rng.normal()), qsynth.pauli_string(n, {int(q): "XYZ"[int(rng.integers(3))]
                                                          for q in rng.choice(n, int(rng.integers(1, 4)), replace=False)}))
             for _ in range(40)]
    mixed.append((0.3, qsynth.pauli_string(n, {1: "Z", 5: "Z", 12: "Z"})))
    # flips on more high bits than a tile holds: the direct per-group path
    mixed.append((0.45, qsynth.pauli_string(n, {q: "XY"[q % 2] for q in range(9)})))
    mixed.append((-0.2, qsynth.pauli_string(n, {q: "X" for q in range(0, 16, 2)})))
    only_x = [(0.5 + 0.1 * q, qsynth.pauli_string(n, {q: "X"})) for q in range(n)]
    for terms in (mixed, only_x):
        H = api.Observable.pauli_sum(n, terms)
        assert abs(H.expectation(st) - oobs.expectation(ref, terms).real) < tol * 10
    gtol = 1e-10 if dt == "c128" else 2e-4
    _, spec, params, _ = qsynth.gradient_20q(seed=3, n=n, layers=2)
    c = api.Circuit.from_spec(n, spec)
    for terms in (mixed, only_x):
        psi, lam = api.State(n, dt), api.State(n, dt)
        c.run(psi, params)
        H = api.Observable.pauli_sum(n, terms)
        e, g = api.adjoint(c.h, params, H.h, psi.h, lam.h, c.nparams)
        e_ref, g_ref = ograd.adjoint(n, spec, params, terms)
        assert abs(e - e_ref) < gtol and np.max(np.abs(g - g_ref)) < gtol


# ---------------------------------------------------------------- sampling
@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("shots", [1, 7, 4099])
def test_sampling_shared_uniforms(api, dt, shots):
    n = 13
    banner("sampling", dt, shots)
    psi0 = qsynth.random_state(n, 8)
    st = gpu_state(api, n, dt, psi0)
    ref = oracle_input(psi0, dt)
    u = np.random.default_rng(shots).random(shots)
    for qubits in (list(range(n)), [4, 0, 9], [12]):
        got = api.sample(st.h, qubits, shots, uniforms=u)
        # a mismatch is only acceptable at a CDF boundary (summation order)
        assert_samples_match(got, ref, qubits, u)


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("n", [7, 22])
def test_sampling_block_and_chunk_edges(api, dt, n):
    # n = 7: one block shorter than a block (128 of 1024 amplitudes); n = 22:
    # 4096 block sums, a prefix over four chunks of 1024
    banner("sampling edges", dt, n)
    psi0 = qsynth.random_state(n, 40 + n)
    st = gpu_state(api, n, dt, psi0)
    ref = oracle_input(psi0, dt)
    u = np.random.default_rng(n).random(2000)
    for qubits in (list(range(n)), [n - 1, 0]):
        got = api.sample(st.h, qubits, len(u), uniforms=u)
        assert_samples_match(got, ref, qubits, u)


def test_sampling_philox_seed_mode_matches_oracle_generator(api):
    n = 12
    banner("sampling philox")
    psi0 = qsynth.random_state(n, 2)
    st = gpu_state(api, n, "c128", psi0)
    got = api.sample(st.h, list(range(n)), 3000, seed=0xDEADBEEF12345)
    # the oracle's own Philox4x32-10 stream (pinned by the published
    # known-answer vectors) drives the oracle's inverse-CDF draw
    u = osamp.philox_uniforms(0xDEADBEEF12345, 3000)
    assert_samples_match(got, psi0, list(range(n)), u)
    got = api.sample(st.h, [3, 11, 0], 3000, seed=7)
    assert_samples_match(got, psi0, [3, 11, 0], osamp.philox_uniforms(7, 3000))


@pytest.mark.parametrize("dt", DTS)
def test_sampling_sparse_state_never_draws_zero_probability(api, dt):
    # mass on a few indices of very different size (several in one block,
    # whole lanes and blocks empty), uniforms on and next to every CDF edge:
    # wherever rounding moves a draw, it must still land on a nonzero amplitude
    n = 14
    banner("sampling sparse", dt)
    psi = np.zeros(1 << n, dtype=np.complex128)
    support = [0, 3, 17, 1000, 1023, 1024, 5000, 9000, 16383]
    mags = [1.0, 1e-9, 0.5, 1e-12, 0.25, 1e-7, 2.0, 1e-15, 0.75]
    for x, a in zip(support, mags):
        psi[x] = a * (1 + 0.5j)
    psi /= np.linalg.norm(psi)
    st = gpu_state(api, n, dt, psi)
    ref = oracle_input(psi, dt)
    p = np.abs(ref) ** 2
    cdf = np.cumsum(p) / np.sum(p)
    edges = cdf[np.array(support)]
    u = np.concatenate([edges, np.nextafter(edges, 0), np.nextafter(np.nextafter(edges, 0), 0),
                        np.random.default_rng(3).random(20000)])
    u = u[(u >= 0) & (u < 1)]
    got = api.sample(st.h, list(range(n)), len(u), uniforms=u)
    assert np.all(p[got] > 0), np.unique(got[p[got] == 0])
    assert_samples_match(got, ref, list(range(n)), u)


def test_sampling_ghz_and_uniform(api):
    n = 20
    banner("sampling ghz")
    st = api.State(n, "c64")
    api.Circuit.from_spec(n, qsynth.ghz(n)).run(st)
    y = api.sample(st.h, list(range(n)), 10000, seed=3)
    assert set(np.unique(y)) <= {0, (1 << n) - 1}
    assert 0.45 < np.mean(y == 0) < 0.55


# ---------------------------------------------------------------- adiabatic
@pytest.mark.parametrize("dt", DTS)
def test_adiabatic_trotter_vs_oracle(api, dt):
    n = 9
    banner("adiabatic", dt)
    J, h = qsynth.ising_couplings(n, 5)
    E = oobs.ising_energies(J, h)
    ref = oad.trotter(n, E, 2.0, 0.05)
    st = api.State(n, dt)
    st.set_plus()
    I = api.Observable.ising(n, J, h)
    e = api.adiabatic_run(st.h, I.h, 2.0, 0.05)
    assert maxabs(st.download(), ref) < (1e-11 if dt == "c128" else 2e-5)
    assert abs(e - oad.energy(ref, E)) < (1e-10 if dt == "c128" else 1e-4)


def test_adiabatic_plans_kept_on_the_observable(api):
    # later runs with the same H1 reuse the Trotter plans kept on it: the same
    # amplitudes bit for bit as with a fresh observable, in both precisions and
    # across block lengths (12 steps: one block; 40 steps: blocks of 8)
    n = 9
    banner("adiabatic plan reuse")
    J, h = qsynth.ising_couplings(n, 6)
    E = oobs.ising_energies(J, h)
    kept = api.Observable.ising(n, J, h)
    for dt in ("c64", "c128", "c64"):
        for steps in (12, 40, 12):
            a = api.State(n, dt)
            a.set_plus()
            ea = api.adiabatic_run(a.h, kept.h, steps * 0.05, 0.05)
            fresh = api.Observable.ising(n, J, h)
            b = api.State(n, dt)
            b.set_plus()
            eb = api.adiabatic_run(b.h, fresh.h, steps * 0.05, 0.05)
            assert np.array_equal(a.download(), b.download()) and ea == eb
            ref = oad.trotter(n, E, steps * 0.05, 0.05)
            assert maxabs(a.download(), ref) < (1e-11 if dt == "c128" else 2e-5)


@pytest.mark.parametrize("dt", DTS)
def test_adiabatic_trotter_staged_blocks(api, dt):
    # register-staged passes, 37 steps = four blocks of 8 shared-pass steps
    # plus a block of 5, full random couplings
    n = 13
    banner("adiabatic staged", dt)
    J, h = qsynth.ising_couplings(n, 8)
    E = oobs.ising_energies(J, h)
    ref = oad.trotter(n, E, 0.37, 0.01)
    st = api.State(n, dt)
    st.set_plus()
    I = api.Observable.ising(n, J, h)
    e = api.adiabatic_run(st.h, I.h, 0.37, 0.01)
    assert maxabs(st.download(), ref) < (1e-11 if dt == "c128" else 2e-5)
    assert abs(e - oad.energy(ref, E)) < (1e-10 if dt == "c128" else 1e-4)


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("steps", [10, 16, 32])
def test_adiabatic_block_boundaries(api, dt, steps):
    # up to 16 steps run as one block; 32 = four blocks of 8 with no remainder.
    # Either way the last segment carries the closing half rotation layer
    n = 13
    banner("adiabatic blocks", dt, steps)
    J, h = qsynth.ising_couplings(n, 9)
    E = oobs.ising_energies(J, h)
    T = steps * 0.01
    ref = oad.trotter(n, E, T, 0.01)
    st = api.State(n, dt)
    st.set_plus()
    I = api.Observable.ising(n, J, h)
    e = api.adiabatic_run(st.h, I.h, T, 0.01)
    assert maxabs(st.download(), ref) < (1e-11 if dt == "c128" else 2e-5)
    assert abs(e - oad.energy(ref, E)) < (1e-10 if dt == "c128" else 1e-4)


def test_adiabatic_j0_factorised_20q(api):
    n = 20
    banner("adiabatic J=0", n)
    _, h = qsynth.ising_couplings(n, 6)
    T, dt = 1.0, 0.01
    st = api.State(n, "c128")
    st.set_plus()
    I = api.Observable.ising(n, np.zeros((n, n)), h)
    api.adiabatic_run(st.h, I.h, T, dt)
    got = st.download()
    prod = np.array([1.0 + 0j])
    for q in range(n):
        prod = np.kron(prod, oad.single_qubit_trotter(h[q], T, dt))
    assert maxabs(got, prod) < 1e-12


# ---------------------------------------------------------------- adjoint
@pytest.mark.parametrize("dt", DTS)
def test_adjoint_gradient_small(api, dt):
    n = 8
    banner("adjoint small", dt)
    spec = [qsynth.gate("RY", (q,), theta=0.0, pidx=q) for q in range(n)]
    spec += [qsynth.gate("H", (2,)), qsynth.gate("RX", (3,), (1,), pidx=n), qsynth.gate("X", (5,), (0,))]
    spec += [qsynth.gate("RZ", (6,), (2, 4), pidx=n + 1), qsynth.gate("U1", (7,), (3,), theta=0.8)]
    spec += [qsynth.gate("RX", (q,), pidx=n + 2 + q) for q in range(n)]
    spec += [qsynth.gate("SWAP", (0, 7)), qsynth.gate("RY", (0,), pidx=2 * n + 2)]
    params = np.random.default_rng(4).uniform(0, 2 * np.pi, 2 * n + 3)
    terms = qsynth.random_pauli_sum(n, 12, 6)
    E_ref, g_ref = ograd.adjoint(n, spec, params, terms)
    c = api.Circuit.from_spec(n, spec)
    psi = api.State(n, dt)
    c.run(psi, params)
    lam = api.State(n, dt)
    H = api.Observable.pauli_sum(n, terms)
    E, g = api.adjoint(c.h, params, H.h, psi.h, lam.h, c.nparams)
    tol = 1e-10 if dt == "c128" else 1e-4
    assert abs(E - E_ref) < tol
    assert np.max(np.abs(g - g_ref)) < tol
    # psi was walked back to the input |0..0>
    back = psi.download()
    assert abs(back[0] - 1) < (1e-10 if dt == "c128" else 1e-4)


def test_adjoint_variational_12q_vs_parameter_shift(api):
    n, spec, params, terms = qsynth.gradient_20q(seed=1, n=12, layers=4)
    banner("adjoint 12q")
    g_ps = ograd.parameter_shift(n, spec, params, terms)
    c = api.Circuit.from_spec(n, spec)
    for dt, tol in (("c128", 1e-10), ("c64", 1e-4)):
        psi = api.State(n, dt)
        c.run(psi, params)
        lam = api.State(n, dt)
        H = api.Observable.pauli_sum(n, terms)
        _, g = api.adjoint(c.h, params, H.h, psi.h, lam.h, c.nparams)
        assert np.max(np.abs(g - g_ps)) < tol, dt


def test_autograd_energy(api):
    import torch
    from paper_2009_01845_amd.autograd import energy
    n, spec, params, terms = qsynth.gradient_20q(seed=2, n=6, layers=2)
    banner("autograd")
    c = api.Circuit.from_spec(n, spec)
    H = api.Observable.pauli_sum(n, terms)
    p = torch.tensor(params, requires_grad=True)
    E = energy(p, c, H, "c128")
    E.backward()
    E_ref, g_ref = ograd.adjoint(n, spec, params, terms)
    assert abs(E.item() - E_ref) < 1e-12
    assert np.max(np.abs(p.grad.numpy() - g_ref)) < 1e-10
    # a second backward through the same graph gives the same gradient
    p2 = torch.tensor(params, requires_grad=True)
    E2 = energy(p2, c, H, "c128")
    g1, = torch.autograd.grad(E2, p2, retain_graph=True)
    g2, = torch.autograd.grad(E2, p2)
    assert np.max(np.abs(g1.numpy() - g_ref)) < 1e-10
    assert np.max(np.abs(g2.numpy() - g_ref)) < 1e-10


# ---------------------------------------------------------------- determinism
def test_bitwise_determinism(api):
    n = 16
    banner("determinism")
    spec = qsynth.random_mixed(n, 100, 5, max_k=2, max_ctrl=1)
    c = api.Circuit.from_spec(n, spec)
    psi0 = qsynth.random_state(n, 1)
    H = api.Observable.pauli_sum(n, qsynth.random_pauli_sum(n, 10, 1))
    outs = []
    for _ in range(2):
        st = gpu_state(api, n, "c64", psi0)
        c.run(st)
        outs.append((st.download(), H.expectation(st), st.norm2()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1] and outs[0][2] == outs[1][2]


@pytest.mark.parametrize("dt", DTS)
def test_lane_op_plans_forward_and_adjoint(api, dt):
    # register stages that also take one-qubit gates across lanes (DPP):
    # the forward passes hold lane ops, the adjoint runs their lane-free form
    n = 16
    banner("lane ops", dt)
    rng = np.random.default_rng(11)
    params = rng.uniform(0, 2 * np.pi, (6, n))
    spec = qsynth.ry_czring_layers(n, params)
    terms = qsynth.zz_ring_plus_x(n)
    flat = params.reshape(-1)
    c = api.Circuit.from_spec(n, spec, lane_ops=1)
    st = api.State(n, dt)
    c.run(st, flat)
    ref = ocirc.run(n, spec, None, flat)
    assert maxabs(st.download(), ref) < TOL[dt]
    H = api.Observable.pauli_sum(n, terms)
    lam = api.State(n, dt)
    E, g = api.adjoint(c.h, flat, H.h, st.h, lam.h, c.nparams)
    E_ref, g_ref = ograd.adjoint(n, spec, flat, terms)
    gtol = 1e-10 if dt == "c128" else 2e-4
    assert abs(E - E_ref) < gtol and np.max(np.abs(g - g_ref)) < gtol
