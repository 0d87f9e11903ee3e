"""Parity at the sizes of the benchmarked workloads, through the C ABI.

Every case compares the HIP path with something it does not compute itself:
the CPU oracle (run at the workload's own size where it finishes in seconds),
a library FFT, or a closed form pinned against the oracle in
``test_oracle_pins.py``.  Tolerances are the ones stated for the path:
max-abs amplitude error 1e-12 (complex128) and 1e-5 (complex64); gradients
1e-10 (complex128) and 2e-4 (complex64 with float64 accumulation);
finite differences (h = 1e-6, complex128) within 1e-6.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import qsynth
from oracle import adiabatic as oad
from oracle import circuits as ocirc
from oracle import gradients as ograd
from oracle import observables as oobs

from gpu_util import TOL, banner, gpu_state, maxabs, oracle_input

pytestmark = pytest.mark.gpu
GTOL = {"c64": 2e-4, "c128": 1e-10}


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2009_01845_amd import api as a
    return a


def _free():
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _oracle_pool(fn, items):
    """Run independent oracle evaluations on host threads (numpy releases the
    interpreter lock inside its array loops); BLAS is held to one thread each."""
    from threadpoolctl import threadpool_limits
    workers = max(1, min(16, (os.cpu_count() or 2)))
    with threadpool_limits(1), ThreadPoolExecutor(workers) as ex:
        return list(ex.map(fn, items))


# ---------------------------------------------------------------------------
# QFT-28 on a random state (Sec. 3.1): the QFT of an arbitrary state is
# sqrt(N) * inverse FFT with the big-endian index
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def qft28_input():
    n = 28
    banner("qft28 input")
    return n, qsynth.random_state(n, 2028)


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_qft28_random_state_vs_fft(api, qft28_input, dt):
    import torch
    n, psi0 = qft28_input
    banner("qft28 random state", dt)
    c = api.Circuit.from_spec(n, qsynth.qft(n))
    st = gpu_state(api, n, dt, psi0)
    c.run(st)
    st.sync()
    ref = ocirc.qft_via_fft(oracle_input(psi0, dt))
    rng = np.random.default_rng(28)
    ys = np.concatenate([[0, 1, (1 << n) - 1, 1 << (n - 1)], rng.integers(0, 1 << n, 1_000_000)]).astype(np.int64)
    got = st.tensor[torch.from_numpy(ys).cuda()].cpu().numpy()
    err = maxabs(got, ref[ys])
    banner("qft28", dt, "max-abs", err)
    assert err < TOL[dt]
    del st, ref
    _free()


# ---------------------------------------------------------------------------
# gradient workload: 20 qubits, 10 x (RY all + CZ ring), 200 parameters,
# H = sum Z_i Z_{i+1 mod 20} + 0.5 sum X_i
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def grad20():
    n, spec, params, terms = qsynth.gradient_20q(0)
    banner("gradient 20q oracle adjoint")
    E_ref, g_ref = ograd.adjoint(n, spec, params, terms)
    return n, spec, params, terms, E_ref, g_ref


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_gradient_20q_all_200_vs_oracle_adjoint(api, grad20, dt):
    n, spec, params, terms, E_ref, g_ref = grad20
    banner("gradient 20q", dt)
    assert params.size == 200
    c = api.Circuit.from_spec(n, spec)
    H = api.Observable.pauli_sum(n, terms)
    psi, lam = api.State(n, dt), api.State(n, dt)
    c.run(psi, params)
    E, g = api.adjoint(c.h, params, H.h, psi.h, lam.h, c.nparams)
    err = float(np.max(np.abs(g - g_ref)))
    banner("gradient 20q", dt, "|dE|", abs(E - E_ref), "max|dgrad|", err)
    assert abs(E - E_ref) < GTOL[dt]
    assert err < GTOL[dt]


def test_gradient_20q_finite_differences_of_gpu_energies(api, grad20):
    # central differences, h = 1e-6, of complex128 energies computed by the
    # library: truncation ~h^2, rounding ~eps |E| / h, well inside 1e-6
    n, spec, params, terms, E_ref, g_ref = grad20
    banner("gradient 20q finite differences")
    c = api.Circuit.from_spec(n, spec)
    H = api.Observable.pauli_sum(n, terms)
    st = api.State(n, "c128")
    h = 1e-6
    for k in np.random.default_rng(20).choice(params.size, 10, replace=False):
        e = []
        for sgn in (1.0, -1.0):
            p = params.copy()
            p[k] += sgn * h
            st.set_basis(0)
            c.run(st, p)
            e.append(H.expectation(st))
        fd = (e[0] - e[1]) / (2 * h)
        assert abs(fd - g_ref[k]) < 1e-6, (k, fd, g_ref[k])


# ---------------------------------------------------------------------------
# adjoint at 24 and 30 qubits against a closed form: a product state (no
# entangling gate) has <Z_i Z_j> = <Z_i><Z_j>, each factor from a 2x2
# evolution (pinned against the oracle adjoint in test_oracle_pins.py)
# ---------------------------------------------------------------------------
def test_adjoint_30q_one_ry_layer_closed_form(api):
    n = 30
    banner("adjoint 30q closed form, one RY layer")
    th = np.random.default_rng(30).uniform(0, 2 * np.pi, n)
    c, s = np.cos(th), np.sin(th)
    E_cf = float(np.sum(c * np.roll(c, -1)) + 0.5 * np.sum(s))
    g_cf = -s * (np.roll(c, 1) + np.roll(c, -1)) + 0.5 * c
    circ = api.Circuit.from_spec(n, qsynth.ry_layers(n, th))
    H = api.Observable.pauli_sum(n, qsynth.zz_ring_plus_x(n))
    psi, lam = api.State(n, "c64"), api.State(n, "c64")
    circ.run(psi, th)
    E, g = api.adjoint(circ.h, th, H.h, psi.h, lam.h, circ.nparams)
    err = float(np.max(np.abs(g - g_cf)))
    banner("adjoint 30q closed form", "|dE|", abs(E - E_cf), "max|dgrad|", err)
    assert abs(E - E_cf) < GTOL["c64"] and err < GTOL["c64"]
    # the sweep walked psi back to |0..0>
    assert abs(psi.tensor[0].item() - 1) < 1e-5
    del psi, lam
    _free()


@pytest.mark.parametrize("n,dt", [(24, "c128"), (30, "c64")])
def test_adjoint_full_size_product_layers_closed_form(api, n, dt):
    # three layers of RY then RZ on every qubit: 6n parameters spread over
    # passes that hold many rotations; every gradient against the closed form
    banner("adjoint closed form, RY/RZ layers", n, dt)
    rng = np.random.default_rng(n + 1)
    L = 3
    th, ph = rng.uniform(0, 2 * np.pi, (L, n)), rng.uniform(0, 2 * np.pi, (L, n))
    spec = qsynth.ry_rz_layers(n, th, ph)
    params = np.concatenate([np.concatenate([th[l], ph[l]]) for l in range(L)])
    E_cf, g_cf = ograd.product_ring_energy(th, ph, hx=0.5)
    circ = api.Circuit.from_spec(n, spec)
    H = api.Observable.pauli_sum(n, qsynth.zz_ring_plus_x(n))
    psi, lam = api.State(n, dt), api.State(n, dt)
    circ.run(psi, params)
    E, g = api.adjoint(circ.h, params, H.h, psi.h, lam.h, circ.nparams)
    err = float(np.max(np.abs(g - g_cf)))
    banner("adjoint closed form", n, dt, "|dE|", abs(E - E_cf), "max|dgrad|", err)
    assert abs(E - E_cf) < GTOL[dt] and err < GTOL[dt]
    del psi, lam
    _free()


@pytest.mark.parametrize("n,dt", [(24, "c128"), (24, "c64"), (27, "c64")])
def test_adjoint_general_phases_with_tile_index_k_bits_closed_form(api, n, dt):
    # RY on every qubit, then controlled phases (angles not multiples of pi)
    # on the ring and on pairs n/2 apart, H = sum Z_i: the phases commute with
    # H, so E = sum cos t_q and dE/dt_q = -sin t_q (pinned through the oracle
    # in test_oracle_pins.py).  At 24 and more qubits the two-state passes
    # walk tiles whose index has bits above the grid, so this checks the
    # general-phase tables of the adjoint at those sizes; a phase misplaced on
    # a rotation's target bit would show in its gradient
    banner("adjoint closed form, general phases", n, dt)
    th = np.random.default_rng(n + 7).uniform(0, 2 * np.pi, n)
    spec = qsynth.ry_then_phases(n, th, seed=n)
    circ = api.Circuit.from_spec(n, spec)
    H = api.Observable.pauli_sum(n, qsynth.z_sum(n))
    psi, lam = api.State(n, dt), api.State(n, dt)
    circ.run(psi, th)
    E, g = api.adjoint(circ.h, th, H.h, psi.h, lam.h, circ.nparams)
    err = float(np.max(np.abs(g + np.sin(th))))
    banner("general phases", n, dt, "|dE|", abs(E - float(np.sum(np.cos(th)))), "max|dgrad|", err)
    assert abs(E - float(np.sum(np.cos(th)))) < GTOL[dt] and err < GTOL[dt]
    del psi, lam
    _free()


# ---------------------------------------------------------------------------
# batch workload: 512 instances (n ~ U{8..18}, depth ~ U{4..12}); every
# instance with n >= 16 against its oracle adjoint
# ---------------------------------------------------------------------------
NCHUNK = 8


@pytest.fixture(scope="module")
def batch512(api):
    banner("batch 512 on the GPU")
    insts = qsynth.batch_instances(seed=0)
    circs = [api.Circuit.from_spec(n, spec) for n, spec, _, _ in insts]
    obs = [api.Observable.pauli_sum(n, terms) for n, _, _, terms in insts]
    b = api.Batch(circs, obs, "c64")
    params = np.concatenate([p for _, _, p, _ in insts])
    E, G = b.run(params)
    offs = np.cumsum([0] + [p.size for _, _, p, _ in insts])
    big = [i for i, it in enumerate(insts) if it[0] >= 16]
    return insts, E, G, offs, big


@pytest.mark.parametrize("chunk", range(NCHUNK))
def test_batch512_large_instances_vs_oracle(batch512, chunk):
    insts, E, G, offs, big = batch512
    mine = big[chunk::NCHUNK]
    banner("batch 512 n>=16 chunk", chunk, len(mine), "of", len(big))
    refs = _oracle_pool(lambda i: ograd.adjoint(*insts[i]), mine)
    for i, (e_ref, g_ref) in zip(mine, refs):
        n = insts[i][0]
        assert abs(E[i] - e_ref) < GTOL["c64"], (i, n, E[i], e_ref)
        assert np.max(np.abs(G[offs[i]:offs[i + 1]] - g_ref)) < GTOL["c64"], (i, n)


def test_batch_18q_complex128_vs_oracle(api):
    insts = [it for it in qsynth.batch_instances(seed=0) if it[0] == 18][:6]
    banner("batch c128 n=18", len(insts))
    circs = [api.Circuit.from_spec(n, spec) for n, spec, _, _ in insts]
    obs = [api.Observable.pauli_sum(n, terms) for n, _, _, terms in insts]
    b = api.Batch(circs, obs, "c128")
    params = np.concatenate([p for _, _, p, _ in insts])
    E, G = b.run(params)
    refs = _oracle_pool(lambda it: ograd.adjoint(*it), insts)
    off = 0
    for i, (it, (e_ref, g_ref)) in enumerate(zip(insts, refs)):
        p = it[2]
        assert abs(E[i] - e_ref) < GTOL["c128"], i
        assert np.max(np.abs(G[off:off + p.size] - g_ref)) < GTOL["c128"], i
        off += p.size


# ---------------------------------------------------------------------------
# adiabatic workload (Sec. 2.6): T = 10, dt = 0.01, 1000 second-order steps
# ---------------------------------------------------------------------------
def test_adiabatic_24q_j0_factorised_1000_steps(api):
    # with J = 0 the Hamiltonian is a sum of commuting one-qubit terms, so the
    # Trotter state is the tensor product of 24 one-qubit Trotter evolutions
    n = 24
    banner("adiabatic 24q J=0, 1000 steps")
    _, h = qsynth.ising_couplings(n, 24)
    T, dt = 10.0, 0.01
    st = api.State(n, "c128")
    st.set_plus()
    I = api.Observable.ising(n, np.zeros((n, n)), h)
    e = api.adiabatic_run(st.h, I.h, T, dt)
    prod = np.array([1.0 + 0j])
    for q in range(n):
        prod = np.kron(prod, oad.single_qubit_trotter(h[q], T, dt))
    got = st.download()
    err = maxabs(got, prod)
    banner("adiabatic 24q J=0 max-abs", err)
    assert err < 1e-12
    E = oobs.ising_energies(np.zeros((n, n)), h)
    assert abs(e - oad.energy(prod, E)) < 1e-10
    del st
    _free()


@pytest.mark.parametrize("n", [8, 10, 12])
def test_adiabatic_full_couplings_1000_steps_and_ground_overlap(api, n):
    banner("adiabatic full J, 1000 steps", n)
    J, h = qsynth.ising_couplings(n, 0)
    T, dt = 10.0, 0.01
    E = oobs.ising_energies(J, h)
    ref = oad.trotter(n, E, T, dt)
    st = api.State(n, "c128")
    st.set_plus()
    I = api.Observable.ising(n, J, h)
    e = api.adiabatic_run(st.h, I.h, T, dt)
    got = st.download()
    assert maxabs(got, ref) < TOL["c128"]
    assert abs(e - oad.energy(ref, E)) < 1e-10
    # overlap with the ground state of H1 found by dense diagonalisation
    w, V = np.linalg.eigh(np.diag(E))
    gs = V[:, 0]
    ov_gpu = abs(np.vdot(gs, got)) ** 2
    ov_ref = abs(np.vdot(gs, ref)) ** 2
    banner("adiabatic", n, "ground-state overlap", ov_gpu, "oracle", ov_ref, "E", e)
    assert abs(ov_gpu - ov_ref) < 1e-12


# ---------------------------------------------------------------------------
# index arithmetic past 2^31 amplitudes: 32 and 33 qubits (complex64,
# 32 / 64 GiB), closed forms on sampled indices
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [32, 33])
def test_closed_forms_beyond_31_index_bits(api, n):
    import torch
    banner("index arithmetic", n)
    rng = np.random.default_rng(n)
    ys = np.concatenate([[0, 1, (1 << n) - 1, (1 << 31) - 1, 1 << 31, (1 << 32) - 1, 1 << (n - 1)],
                         rng.integers(0, 1 << n, 200_000)]).astype(np.int64)
    idx = torch.from_numpy(ys).cuda()
    st = api.State(n, "c64")
    # GHZ: 1/sqrt2 at 0 and 2^n - 1, zero elsewhere
    api.Circuit.from_spec(n, qsynth.ghz(n)).run(st)
    got = st.tensor[idx].cpu().numpy()
    exp = np.where((ys == 0) | (ys == (1 << n) - 1), 2 ** -0.5, 0.0)
    assert maxabs(got, exp) < TOL["c64"]
    # sampling the GHZ state: only the two ends
    y = api.sample(st.h, list(range(n)), 20000, seed=n)
    assert set(np.unique(y)) <= {0, (1 << n) - 1}
    assert 0.47 < np.mean(y == 0) < 0.53
    # one RY/RZ/CZ layer: the product-state closed form
    th, ph = rng.uniform(0, 2 * np.pi, n), rng.uniform(0, 2 * np.pi, n)
    params = np.stack([th, ph], axis=1)[None]
    st.set_basis(0)
    api.Circuit.from_spec(n, qsynth.ry_rz_cz_layers(n, params)).run(st, params.reshape(-1))
    got = st.tensor[idx].cpu().numpy()
    assert maxabs(got, ocirc.product_state_amplitudes(n, th, ph, ys)) < TOL["c64"]
    # QFT of a basis state above 2^32: the exact modular closed form
    x = (1 << (n - 1)) + int(rng.integers(0, 1 << (n - 1)))
    st.set_basis(x)
    api.Circuit.from_spec(n, qsynth.qft(n)).run(st)
    got = st.tensor[idx].cpu().numpy()
    assert maxabs(got, ocirc.qft_basis_amplitudes(n, x, ys.astype(np.uint64))) < TOL["c64"]
    assert abs(st.norm2() - 1) < 1e-5
    del st, idx
    _free()
