"""Dense 3-5 qubit blocks applied on matrix cores (MFMA) against the oracle."""
import numpy as np
import pytest

import qsynth
from oracle import circuits as ocirc

from gpu_util import TOL, banner, gpu_state, maxabs, oracle_input

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available()
    from paper_2009_01845_amd import api as a
    return a


def blocks(n, seed, ks=(3, 4, 5), count=6, ctrl=True):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        k = ks[i % len(ks)]
        nc = int(rng.integers(0, 6 - k)) if ctrl else 0
        q = rng.permutation(n)[: k + nc]
        out.append(qsynth.gate("MAT", q[:k], q[k:], mat=qsynth.haar_unitary(1 << k, rng)))
        # interleave ordinary gates so tiled and MFMA passes alternate
        out.append(qsynth.gate("H", (int(rng.integers(0, n)),)))
        out.append(qsynth.gate("U1", (int(q[0]),), (int((q[0] + 1) % n),), theta=0.7))
    return out


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n", [12, 15])
def test_mfma_blocks_vs_oracle(api, dt, n):
    banner("mfma", dt, n)
    spec = blocks(n, 10 + n)
    c = api.Circuit.from_spec(n, spec, use_mfma=1)
    kinds = [k for k, _, _ in c.passes()]
    assert kinds.count(4) >= 6, kinds
    psi0 = qsynth.random_state(n, n)
    st = gpu_state(api, n, dt, psi0)
    c.run(st)
    ref = ocirc.run(n, spec, oracle_input(psi0, dt))
    assert maxabs(st.download(), ref) < TOL[dt]


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_mfma_uncontrolled_three_qubit_blocks(api, dt):
    # 3-qubit blocks are widened to 4 (G x I on a free bit) for matrix cores
    n = 13
    banner("mfma k3", dt)
    spec = blocks(n, 41, ks=(3,), count=5, ctrl=False)
    c = api.Circuit.from_spec(n, spec, use_mfma=1)
    assert [k for k, _, _ in c.passes()].count(4) == 5
    psi0 = qsynth.random_state(n, 3)
    st = gpu_state(api, n, dt, psi0)
    c.run(st)
    assert maxabs(st.download(), ocirc.run(n, spec, oracle_input(psi0, dt))) < TOL[dt]


def test_mfma_low_and_high_targets(api):
    n = 14
    banner("mfma targets")
    rng = np.random.default_rng(3)
    spec = []
    for tg in [(13, 12, 11, 10, 9), (0, 1, 2, 3, 4), (0, 13, 6, 7, 2), (5, 4, 3, 2)]:
        spec.append(qsynth.gate("MAT", tg, mat=qsynth.haar_unitary(1 << len(tg), rng)))
    psi0 = qsynth.random_state(n, 4)
    for dt in ("c64", "c128"):
        c = api.Circuit.from_spec(n, spec, use_mfma=1)
        st = gpu_state(api, n, dt, psi0)
        c.run(st)
        assert maxabs(st.download(), ocirc.run(n, spec, oracle_input(psi0, dt))) < TOL[dt]


def fused_pairs(n, seed):
    # consecutive blocks on disjoint bits: a 5-qubit low/high pair, a spread
    # block, a 4-qubit low/high pair, a spread block, another 4-qubit pair
    rng = np.random.default_rng(seed)
    sets = [tuple(range(n - 5, n)), tuple(range(5)), (0, n // 4, n // 2, 3 * n // 4, n - 1),
            tuple(range(n - 4, n)), tuple(range(4)), (3, n // 3 + 1, 2 * n // 3, n - 3),
            (1, 2, 3, 4), (n - 2, n - 3, n - 4, n - 5)]
    return [qsynth.gate("MAT", t, mat=qsynth.haar_unitary(1 << len(t), rng)) for t in sets]


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n", [12, 16, 20])
def test_mfma_fused_pairs_vs_oracle(api, dt, n):
    # two ready blocks of one size on disjoint bits that fit one tile share a
    # pass (5-qubit pairs only in complex64)
    banner("mfma fused pairs", dt, n)
    spec = fused_pairs(n, 70 + n)
    c = api.Circuit.from_spec(n, spec, use_mfma=1)
    psi0 = qsynth.random_state(n, 71 + n)
    st = gpu_state(api, n, dt, psi0)
    c.run(st)
    fused = sum(1 for k, _, nops in c.passes() if k == 4 and nops == 2)
    assert fused == (3 if dt == "c64" else 2)
    assert maxabs(st.download(), ocirc.run(n, spec, oracle_input(psi0, dt))) < TOL[dt]


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_mfma_fused_pairs_adjoint(api, dt):
    # the adjoint un-applies both blocks of a fused pass on psi and lambda
    from oracle import gradients as ograd
    n = 14
    banner("mfma fused adjoint", dt)
    rng = np.random.default_rng(9)
    spec = [qsynth.gate("RY", (q,), pidx=q) for q in range(n)]
    spec += fused_pairs(n, 12)
    spec += [qsynth.gate("RX", (q,), pidx=n + q) for q in range(n)]
    params = rng.uniform(0, 2 * np.pi, 2 * n)
    terms = qsynth.random_pauli_sum(n, 8, 2)
    c = api.Circuit.from_spec(n, spec, use_mfma=1)
    psi, lam = api.State(n, dt), api.State(n, dt)
    c.run(psi, params)
    assert any(k == 4 and nops == 2 for k, _, nops in c.passes())
    H = api.Observable.pauli_sum(n, terms)
    e, g = api.adjoint(c.h, params, H.h, psi.h, lam.h, c.nparams)
    e_ref, g_ref = ograd.adjoint(n, spec, params, terms)
    tol = 1e-10 if dt == "c128" else 2e-4
    assert abs(e - e_ref) < tol and np.max(np.abs(g - g_ref)) < tol


def test_mfma_adjoint_passes(api):
    # an energy gradient through a circuit with matrix-core blocks
    from oracle import gradients as ograd
    n = 12
    banner("mfma adjoint")
    rng = np.random.default_rng(5)
    spec = [qsynth.gate("RY", (q,), pidx=q) for q in range(n)]
    spec.append(qsynth.gate("MAT", (2, 5, 7, 9), mat=qsynth.haar_unitary(16, rng)))
    spec += [qsynth.gate("RX", (q,), pidx=n + q) for q in range(n)]
    params = rng.uniform(0, 2 * np.pi, 2 * n)
    terms = qsynth.random_pauli_sum(n, 8, 2)
    c = api.Circuit.from_spec(n, spec, use_mfma=1)
    assert 4 in [k for k, _, _ in c.passes()]
    psi, lam = api.State(n, "c128"), api.State(n, "c128")
    c.run(psi, params)
    H = api.Observable.pauli_sum(n, terms)
    e, g = api.adjoint(c.h, params, H.h, psi.h, lam.h, c.nparams)
    e_ref, g_ref = ograd.adjoint(n, spec, params, terms)
    assert abs(e - e_ref) < 1e-10 and np.max(np.abs(g - g_ref)) < 1e-10


@pytest.mark.parametrize("fuse_k", [2, 3, 4, 5])
@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_fused_circuits_vs_oracle(api, dt, fuse_k):
    # gate fusion (the paper's fuse step, widened to k qubits) must leave the
    # final state unchanged: random layers with controls, and the QFT
    n = 14
    banner("fuse", dt, fuse_k)
    psi0 = qsynth.random_state(n, 30 + fuse_k)
    for spec in (qsynth.random_mixed(n, 90, 40 + fuse_k), qsynth.qft(n)):
        c = api.Circuit.from_spec(n, spec, fuse_k=fuse_k)
        st = gpu_state(api, n, dt, psi0)
        c.run(st)
        ref = ocirc.run(n, spec, oracle_input(psi0, dt))
        assert maxabs(st.download(), ref) < TOL[dt]


def test_fused_variational_gradient(api):
    # rotations keep their parameters through fusion; the gradient is unchanged
    from oracle import gradients as ograd
    n = 10
    banner("fuse adjoint")
    n, spec, params, terms = qsynth.variational_10q(2)
    c = api.Circuit.from_spec(n, spec, fuse_k=4)
    psi, lam = api.State(n, "c128"), api.State(n, "c128")
    c.run(psi, params)
    H = api.Observable.pauli_sum(n, terms)
    e, g = api.adjoint(c.h, params, H.h, psi.h, lam.h, c.nparams)
    e_ref, g_ref = ograd.adjoint(n, spec, params, terms)
    assert abs(e - e_ref) < 1e-10 and np.max(np.abs(g - g_ref)) < 1e-10


def test_autotune_keeps_results_and_caches(api, tmp_path):
    n = 16
    banner("autotune")
    spec = qsynth.random_mixed(n, 120, 77, max_k=3)
    cache = str(tmp_path / "tune.txt")
    for dt in ("c64", "c128"):
        c = api.Circuit.from_spec(n, spec)
        st = api.State(n, dt)
        api.autotune(c.h, st.h, None, cache)
        lines = open(cache).read().splitlines()
        assert lines and ("dtype=" + dt) in lines[-1]
        api.autotune(c.h, st.h, None, cache)           # a cache hit appends nothing
        assert open(cache).read().splitlines() == lines
        psi0 = qsynth.random_state(n, 9)
        st.upload(psi0.astype(np.complex64 if dt == "c64" else np.complex128))
        c.run(st)
        assert maxabs(st.download(), ocirc.run(n, spec, oracle_input(psi0, dt))) < TOL[dt]
