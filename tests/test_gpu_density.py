"""Density matrices and noise channels (Sec. 2.4.3) through the C ABI.

An n-qubit rho is a 2n-qubit state (rho[r][c] at r 2^n + c); gates act as
U rho U^dagger and channels as sum_i K_i rho K_i^dagger.  The GPU results are
compared element by element with the dense oracle (oracle.density, plain
2^n x 2^n matrix products), and at full size (30 state qubits) with closed
forms of product channels.  Tolerances: max-abs 1e-12 (complex128), 1e-5
(complex64); traces and Tr(H rho) 1e-12 / 1e-5 times the number of terms.
"""
import numpy as np
import pytest

import qsynth
from oracle import density as oden

from gpu_util import TOL, banner, maxabs

NPDT = {"c64": np.complex64, "c128": np.complex128}


@pytest.fixture(scope="module")
def api():
    from paper_2009_01845_amd import _lib, api as a
    import os
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2009_01845_amd import build
        build.build()
    return a


# ----------------------------------------------------------------- host side
def test_named_channels_are_trace_preserving_textbook_maps(api):
    """The library's Kraus sets against their definitions: sum K^dagger K = I,
    and the action on a generic 2x2 density matrix equals the textbook map."""
    from oracle import gates as og
    X, Z = og.PAULI["X"], og.PAULI["Z"]
    rng = np.random.default_rng(3)
    a = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    rho = a @ a.conj().T
    rho /= np.trace(rho)
    for p in (0.0, 0.13, 0.5, 1.0):
        for name in qsynth.CHANNELS:
            ks = api.channel_kraus(name, p)
            S = sum(K.conj().T @ K for K in ks)
            assert np.allclose(S, np.eye(2), atol=1e-15), (name, p)
            out = sum(K @ rho @ K.conj().T for K in ks)
            if name == "depolarizing":
                exp = (1 - p) * rho + p * np.trace(rho) * np.eye(2) / 2
            elif name == "bit_flip":
                exp = (1 - p) * rho + p * X @ rho @ X
            elif name == "phase_flip":
                exp = (1 - p) * rho + p * Z @ rho @ Z
            elif name == "amplitude_damping":
                exp = np.array([[rho[0, 0] + p * rho[1, 1], np.sqrt(1 - p) * rho[0, 1]],
                                [np.sqrt(1 - p) * rho[1, 0], (1 - p) * rho[1, 1]]])
            else:  # phase damping
                exp = np.array([[rho[0, 0], np.sqrt(1 - p) * rho[0, 1]],
                                [np.sqrt(1 - p) * rho[1, 0], rho[1, 1]]])
            assert np.allclose(out, exp, atol=1e-14), (name, p)
    with pytest.raises(Exception):
        api.channel_kraus("no_such_channel", 0.1)
    with pytest.raises(Exception):
        api.channel_kraus("depolarizing", 1.5)


def test_density_circuit_validation(api):
    c = api.circuit_create_density(3)
    try:
        with pytest.raises(Exception):  # qubit 3 is outside the 3-qubit system
            api.circuit_add_gate(c, np.eye(2), [3])
        with pytest.raises(Exception):
            api.circuit_add_channel(c, [np.eye(2)], [5])
        api.circuit_add_channel(c, api.channel_kraus("bit_flip", 0.2), [1])
        api.circuit_add_gate(c, np.eye(2), [2])
        g, _, _ = api.circuit_info(c)
        assert g == 3  # the gate became U on the rows and conj(U) on the columns
    finally:
        api.circuit_destroy(c)
    sv = api.circuit_create(3)
    try:
        with pytest.raises(Exception):  # channels need a density-matrix circuit
            api.circuit_add_channel(sv, [np.eye(2)], [0])
    finally:
        api.circuit_destroy(sv)


# ---------------------------------------------------------------- GPU parity
@pytest.mark.gpu
@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n,depth,seed", [(3, 3, 1), (5, 4, 2), (7, 3, 3), (8, 2, 4)])
def test_noisy_circuit_vs_dense_oracle(api, dt, n, depth, seed):
    banner("density noisy layers", n, depth, seed, dt)
    spec, params = qsynth.noisy_layers(n, depth, seed)
    c = api.DensityCircuit.from_spec(n, spec)
    rho = api.DensityMatrix(n, dt)
    c.run(rho, params)
    ref = oden.run(n, spec, None, params)
    got = rho.download()
    err = maxabs(got, ref)
    banner("density", n, dt, "max-abs", err)
    assert err < TOL[dt]
    assert abs(rho.trace() - 1.0) < 10 * TOL[dt]
    terms = qsynth.random_pauli_sum(n, 12, seed)
    H = api.Observable.pauli_sum(n, terms)
    e_ref = oden.expectation(ref, terms)
    assert abs(rho.expectation(H) - e_ref) < 12 * TOL[dt] * (1 + abs(e_ref))


@pytest.mark.gpu
@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_dense_blocks_on_rows_and_columns_share_matrix_core_passes(api, dt):
    # a 4-qubit gate becomes U on the row bits and conj(U) on the column bits:
    # two blocks on disjoint bits, which share one matrix-core launch
    n = 8
    banner("density mfma pairs", n, dt)
    rng = np.random.default_rng(21)
    spec = [qsynth.gate("MAT", (0, 1, 2, 3), mat=qsynth.haar_unitary(16, rng)),
            qsynth.gate("CH:depolarizing", (2,), theta=0.1),
            qsynth.gate("MAT", (4, 5, 6, 7), mat=qsynth.haar_unitary(16, rng)),
            qsynth.gate("MAT", (1, 3, 5, 7), mat=qsynth.haar_unitary(16, rng))]
    c = api.DensityCircuit.from_spec(n, spec, use_mfma=1)
    rho = api.DensityMatrix(n, dt)
    c.run(rho)
    assert any(k == 4 and nops == 2 for k, _, nops in c.passes())
    ref = oden.run(n, spec, None, None)
    assert maxabs(rho.download(), ref) < TOL[dt]
    assert abs(rho.trace() - 1.0) < 10 * TOL[dt]


@pytest.mark.gpu
@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_unitary_density_circuit_is_outer_product_of_state(api, dt):
    # no channel: rho(out) = |U psi><U psi| for rho(in) = |psi><psi|, here from
    # a random state (set_pure) through a mixed list of gates and controls
    n = 6
    banner("density pure", n, dt)
    spec = qsynth.random_mixed(n, 40, 5)
    psi0 = qsynth.random_state(n, 6)
    st = api.State(n, dt)
    st.upload(psi0.astype(NPDT[dt]))
    rho = api.DensityMatrix(n, dt)
    rho.set_pure(st)
    assert maxabs(rho.download(), oden.pure(psi0.astype(NPDT[dt]))) < TOL[dt]
    api.DensityCircuit.from_spec(n, spec).run(rho)
    ref = oden.run(n, spec, oden.pure(psi0.astype(NPDT[dt]).astype(complex)))
    assert maxabs(rho.download(), ref) < TOL[dt]


@pytest.mark.gpu
@pytest.mark.parametrize("n,dt", [(15, "c64"), (12, "c128")])
def test_product_channels_at_full_size_closed_form(api, n, dt):
    """RY(theta_q) on every qubit of |0..0>, then amplitude damping p_q and
    depolarising d_q on qubit q: rho is the Kronecker product of the one-qubit
    results, each from the oracle's 2x2 maps (2n = 30 / 24 state qubits)."""
    import torch
    banner("density product closed form", n, dt)
    rng = np.random.default_rng(n)
    th = rng.uniform(0, 2 * np.pi, n)
    pa, pd = rng.uniform(0, 0.4, n), rng.uniform(0, 0.4, n)
    spec = [qsynth.gate("RY", (q,), theta=th[q]) for q in range(n)]
    spec += [qsynth.gate("CH:amplitude_damping", (q,), theta=pa[q]) for q in range(n)]
    spec += [qsynth.gate("CH:depolarizing", (q,), theta=pd[q]) for q in range(n)]
    rho = api.DensityMatrix(n, dt)
    api.DensityCircuit.from_spec(n, spec).run(rho)
    ones = []
    for q in range(n):
        r = oden.run(1, [qsynth.gate("RY", (0,), theta=th[q]), qsynth.gate("CH:amplitude_damping", (0,), theta=pa[q]),
                         qsynth.gate("CH:depolarizing", (0,), theta=pd[q])])
        ones.append(r)
    idx = np.concatenate([[0, (1 << (2 * n)) - 1], rng.integers(0, 1 << (2 * n), 200_000)]).astype(np.int64)
    got = rho.state.tensor[torch.from_numpy(idx).cuda()].cpu().numpy()
    r, c = idx >> n, idx & ((1 << n) - 1)
    exp = np.ones(idx.size, dtype=complex)
    for q in range(n):
        b = n - 1 - q
        exp *= ones[q][(r >> b) & 1, (c >> b) & 1]
    err = maxabs(got, exp)
    banner("density product", n, dt, "max-abs", err)
    assert err < TOL[dt]
    assert abs(rho.trace() - 1.0) < (1e-5 if dt == "c64" else 1e-12)
    # Tr(Z_q rho) of a product state: the q-th factor's <Z>
    for q in (0, n // 2, n - 1):
        H = api.Observable.pauli_sum(n, [(1.0, qsynth.pauli_string(n, {q: "Z"}))])
        zq = (ones[q][0, 0] - ones[q][1, 1]).real
        assert abs(rho.expectation(H) - zq) < (1e-5 if dt == "c64" else 1e-12)
    del rho
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


@pytest.mark.gpu
def test_density_rejected_by_adjoint_and_batch(api):
    n = 3
    c = api.DensityCircuit(n)
    c.add_rot("Y", 0, 0)
    c.compile()
    H = api.Observable.pauli_sum(2 * n, [(1.0, "ZIIIII")])
    rho, lam = api.State(2 * n, "c128"), api.State(2 * n, "c128")
    with pytest.raises(Exception):
        api.adjoint(c.h, np.array([0.3]), H.h, rho.h, lam.h, 1)
    with pytest.raises(Exception):
        api.Batch([c], [H], "c64")
