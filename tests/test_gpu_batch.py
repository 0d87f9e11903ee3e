"""Batched persistent launch: every instance equals its own oracle run
(energy and adjoint gradient), replays are bitwise identical."""
import numpy as np
import pytest

import qsynth
from oracle import gradients as ograd

from gpu_util import banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available()
    from paper_2009_01845_amd import api as a
    return a


def build(api, insts, dt="c64"):
    circs = [api.Circuit.from_spec(n, spec) for n, spec, _, _ in insts]
    obs = [api.Observable.pauli_sum(n, terms) for n, _, _, terms in insts]
    return api.Batch(circs, obs, dt), np.concatenate([p for _, _, p, _ in insts])


@pytest.mark.parametrize("dt,tol", [("c64", 2e-4), ("c128", 1e-10)])
def test_batch_matches_oracle(api, dt, tol):
    banner("batch vs oracle", dt)
    insts = qsynth.batch_instances(seed=3, count=9, nmin=5, nmax=13, dmin=1, dmax=4)
    b, params = build(api, insts, dt)
    E, G = b.run(params)
    off = 0
    for i, (n, spec, p, terms) in enumerate(insts):
        e_ref, g_ref = ograd.adjoint(n, spec, p, terms)
        assert abs(E[i] - e_ref) < tol, (i, n)
        assert np.max(np.abs(G[off:off + p.size] - g_ref)) < tol, (i, n)
        off += p.size


def test_batch_graph_replay_and_new_parameters(api):
    banner("batch replay")
    insts = qsynth.batch_instances(seed=4, count=20, nmin=6, nmax=14, dmin=2, dmax=5)
    b, params = build(api, insts)
    E1, G1 = b.run(params)
    E2, G2 = b.run(params)  # graph replay
    assert np.array_equal(E1, E2) and np.array_equal(G1, G2)
    p2 = params + 0.3
    E3, G3 = b.run(p2)
    E4, G4 = b.run(p2)
    assert np.array_equal(E3, E4) and np.array_equal(G3, G4)
    # against the single-circuit path on the GPU for the new parameters
    off = 0
    for i, (n, spec, p, terms) in enumerate(insts):
        c = api.Circuit.from_spec(n, spec)
        H = api.Observable.pauli_sum(n, terms)
        pp = p2[off:off + p.size]
        psi, lam = api.State(n, "c64"), api.State(n, "c64")
        c.run(psi, pp)
        e, g = api.adjoint(c.h, pp, H.h, psi.h, lam.h, c.nparams)
        assert abs(e - E3[i]) < 1e-4 and np.max(np.abs(g - G3[off:off + p.size])) < 1e-4
        off += p.size


def test_full_512_instance_batch_sampled_against_oracle(api):
    banner("batch 512")
    insts = qsynth.batch_instances(seed=0)
    assert len(insts) == 512
    b, params = build(api, insts)
    E, G = b.run(params)
    E2, G2 = b.run(params)
    assert np.array_equal(E, E2) and np.array_equal(G, G2)
    offs = np.cumsum([0] + [p.size for _, _, p, _ in insts])
    rng = np.random.default_rng(0)
    small = [i for i, (n, _, _, _) in enumerate(insts) if n <= 12]
    for i in rng.choice(small, 4, replace=False):
        n, spec, p, terms = insts[i]
        e_ref, g_ref = ograd.adjoint(n, spec, p, terms)
        assert abs(E[i] - e_ref) < 2e-4
        assert np.max(np.abs(G[offs[i]:offs[i + 1]] - g_ref)) < 2e-4


def test_batch_autotune_per_size_class(api, tmp_path):
    banner("batch autotune")
    insts = qsynth.batch_instances(seed=5, count=24, nmin=8, nmax=15, dmin=2, dmax=6)
    b, params = build(api, insts)
    E0, G0 = b.run(params)
    cache = str(tmp_path / "batch_tune.txt")
    b.autotune(params, cache)
    lines = open(cache).read().strip().splitlines()
    classes = sorted({n for n, _, _, _ in insts})
    assert len(lines) == len(classes) and all(ln.startswith("batch-class n=") for ln in lines)
    for i, (n, _, _, _) in enumerate(insts):
        ch = b.choice(i)
        assert set(ch) == {"tile_bits", "fuse_k", "use_mfma", "low_bits", "lane_ops"}
        # one choice per size class
        assert ch == b.choice(next(j for j, it in enumerate(insts) if it[0] == n))
    E1, G1 = b.run(params)  # rebuilt batch, fresh graphs
    assert np.max(np.abs(E1 - E0)) < 1e-4 and np.max(np.abs(G1 - G0)) < 1e-4
    off = 0
    for i, (n, spec, p, terms) in enumerate(insts):
        if i % 6 == 0:
            e_ref, g_ref = ograd.adjoint(n, spec, p, terms)
            assert abs(E1[i] - e_ref) < 2e-4 and np.max(np.abs(G1[off:off + p.size] - g_ref)) < 2e-4
        off += p.size
    b.autotune(params, cache)  # every class from the cache: nothing appended
    assert len(open(cache).read().strip().splitlines()) == len(classes)
