"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point that include/qsim.h declares, validates arguments before
touching the device, and plans circuits into the expected passes."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import qsynth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qsim.h")


@pytest.fixture(scope="module")
def api():
    from paper_2009_01845_amd import _lib, api
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2009_01845_amd import build
        build.build()
    return api


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(qs_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for must in ["qs_state_create", "qs_apply", "qs_circuit_compile", "qs_circuit_run", "qs_pauli_sum_create",
                 "qs_expectation", "qs_sample", "qs_adiabatic_run", "qs_adjoint", "qs_batch_run"]:
        assert must in syms


def test_library_exports_every_declared_symbol(api):
    from paper_2009_01845_amd import _lib
    L = C.CDLL(_lib.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing
    assert set(declared_symbols()) == set(_lib.SIGNATURES), "binding signatures out of sync with the header"


def test_version_and_gate_matrices(api):
    assert "gfx950" in api.version()
    # the library's named matrices are the textbook ones (pinned against the
    # oracle's independent definitions, both checked by closed forms)
    from oracle import gates as og
    for name in ["H", "X", "Y", "Z", "S", "T", "SWAP"]:
        assert np.allclose(api.gate_matrix(name), og.matrix(name), atol=1e-15), name
    for name in ["RX", "RY", "RZ", "U1"]:
        for th in (0.0, 0.7, -2.3):
            assert np.allclose(api.gate_matrix(name, th), og.matrix(name, th), atol=1e-15), name
    # and directly against matrix exponentials: R_P(t) = exp(-i t P/2);
    # S and T are RZ(pi/2) and RZ(pi/4) times e^{i pi/4} and e^{i pi/8}
    import scipy.linalg as sla
    Z = np.diag([1.0, -1.0]).astype(complex)
    assert np.allclose(api.gate_matrix("S"), np.exp(0.25j * np.pi) * sla.expm(-0.25j * np.pi * Z), atol=1e-15)
    assert np.allclose(api.gate_matrix("T"), np.exp(0.125j * np.pi) * sla.expm(-0.125j * np.pi * Z), atol=1e-15)
    for p in "XYZ":
        assert np.allclose(api.gate_matrix("R" + p, 0.9), sla.expm(-0.45j * og.PAULI[p]), atol=1e-15), p
    with pytest.raises(api.QsError) as e:
        api.gate_matrix("NOPE")
    assert e.value.code == -1


@pytest.mark.parametrize("bad", [
    dict(targets=[0, 0]), dict(targets=[5]), dict(targets=[-1]), dict(targets=[0], controls=[0]),
    dict(targets=[0, 1, 2, 3, 4, 5]), dict(targets=[1], controls=[2, 2]),
])
def test_gate_validation(api, bad):
    c = api.circuit_create(4)
    k = len(bad["targets"])
    with pytest.raises(api.QsError) as e:
        api.circuit_add_gate(c, np.eye(1 << min(k, 5)), bad["targets"], bad.get("controls", ()))
    assert e.value.code == -1
    api.circuit_destroy(c)


def test_circuit_and_observable_validation(api):
    for n in (0, 36, -3):
        with pytest.raises(api.QsError):
            api.circuit_create(n)
    c = api.circuit_create(3)
    with pytest.raises(api.QsError):
        api.circuit_add_rot(c, "Q", 0, 0)
    with pytest.raises(api.QsError):
        api.circuit_add_rot(c, "X", 0, -1)
    with pytest.raises(api.QsError):
        api.circuit_compile(c, tile_bits=40)
    api.circuit_destroy(c)
    with pytest.raises(api.QsError):
        api.pauli_sum_create(3, [(1.0, "XQZ")])
    with pytest.raises(api.QsError):
        api.pauli_sum_create(3, [(1.0, "XZ")])
    o = api.pauli_sum_create(3, [(1.0, "XYZ"), (0.5, "IIZ")])
    api.obs_destroy(o)


def test_null_and_range_checks_do_not_touch_the_device(api):
    from paper_2009_01845_amd import _lib
    L = _lib.lib()
    h = C.c_void_p()
    assert L.qs_state_create(0, 1, None, C.byref(h)) == -1
    assert L.qs_state_create(36, 1, None, C.byref(h)) == -1
    assert L.qs_state_create(10, 7, None, C.byref(h)) == -1
    assert L.qs_state_create(10, 1, None, None) == -1
    assert L.qs_state_wrap(None, 10, 1, None, C.byref(h)) == -1
    assert L.qs_state_wrap(C.c_void_p(8), 10, 1, None, C.byref(h)) == -1  # misaligned
    assert L.qs_norm2(None, None) == -1
    assert L.qs_expectation(None, None, None) == -1
    assert "null" in L.qs_last_error().decode()
    assert L.qs_state_destroy(None) == 0


def test_memory_cap_forces_nomem(api, monkeypatch):
    from paper_2009_01845_amd import _lib
    monkeypatch.setenv("QS_MEM_LIMIT_BYTES", "1024")
    h = C.c_void_p()
    assert _lib.lib().qs_state_create(20, 1, None, C.byref(h)) == -2
    assert "QS_MEM_LIMIT_BYTES" in _lib.lib().qs_last_error().decode()


# ------------------------------------------------------------ planning (host)
def test_qft_plan_shape(api):
    for n, expect_max in [(28, 5), (30, 5)]:
        c = api.Circuit.from_spec(n, qsynth.qft(n))
        g, p, _ = c.info()
        assert g == n * (n + 1) // 2 + n // 2
        kinds = [k for k, _, _ in c.passes()]
        assert kinds.count(3) == 1        # the SWAP network is one bit-reversal pass
        assert p <= expect_max, c.passes()


def test_diagonal_only_circuit_is_one_pass(api):
    n = 20
    spec = [qsynth.gate("Z", (i + 1,), (i,)) for i in range(n - 1)] + [qsynth.gate("T", (3,)),
                                                                      qsynth.gate("RZ", (7,), theta=0.4)]
    c = api.Circuit.from_spec(n, spec)
    assert c.info()[1] == 1


def test_lookahead_bit_choice_shortens_layered_plans(api):
    # RY layers with a CZ ring, and RY/RZ layers with a CNOT chain: taking the
    # high bits that the first gates in index order ask for gives 19 and 23
    # passes; picking bits along the dependency light cone gives 13 and 11
    n = 30
    _, spec, _, _ = qsynth.gradient_20q(seed=0, n=n, layers=10)
    assert api.Circuit.from_spec(n, spec).info()[1] <= 13
    chain, k = [], 0
    for _ in range(5):
        for q in range(n):
            for r in ("RY", "RZ"):
                chain.append(qsynth.gate(r, (q,), theta=0.3, pidx=k))
                k += 1
        chain += [qsynth.gate("X", (q + 1,), (q,)) for q in range(n - 1)]
    assert api.Circuit.from_spec(n, chain).info()[1] <= 11
    # a brickwork of Haar 2-qubit gates, depth 12: 31 passes in index order
    rng = np.random.default_rng(5)
    brick = [qsynth.gate("MAT", (q, q + 1), mat=qsynth.haar_unitary(4, rng))
             for d in range(12) for q in range(d % 2, n - 1, 2)]
    assert api.Circuit.from_spec(n, brick).info()[1] <= 17


def test_tile_options_change_the_plan(api):
    n = 26
    spec = qsynth.random_layers(n, 4, 3)
    p12 = api.Circuit.from_spec(n, spec, tile_bits=12).info()[1]
    p8 = api.Circuit.from_spec(n, spec, tile_bits=8, low_bits=3).info()[1]
    assert p8 > p12


def test_swap_relabel_needs_no_pass_when_undone(api):
    n = 16
    spec = [qsynth.gate("SWAP", (0, 15)), qsynth.gate("SWAP", (0, 15))]
    assert api.Circuit.from_spec(n, spec).info()[1] == 0
    spec = [qsynth.gate("SWAP", (0, 5)), qsynth.gate("SWAP", (5, 9))]  # a 3-cycle: two involutions
    assert api.Circuit.from_spec(n, spec).info()[1] == 2


def test_dense_blocks_plan_onto_matrix_cores(api):
    rng = np.random.default_rng(0)
    spec = [qsynth.gate("MAT", (1, 4, 7, 9), mat=qsynth.haar_unitary(16, rng)),
            qsynth.gate("MAT", (0, 2, 3), (11,), mat=qsynth.haar_unitary(8, rng))]
    auto = api.Circuit.from_spec(14, spec)
    on = api.Circuit.from_spec(14, spec, use_mfma=1)
    off = api.Circuit.from_spec(14, spec, use_mfma=0)
    assert [k for k, _, _ in on.passes()].count(4) == 2
    assert [k for k, _, _ in auto.passes()].count(4) == 2   # k + controls >= 4 by default
    assert 4 not in [k for k, _, _ in off.passes()]


def test_three_qubit_blocks_widen_for_matrix_cores(api):
    rng = np.random.default_rng(2)
    spec = [qsynth.gate("MAT", (3, 8, 11), mat=qsynth.haar_unitary(8, rng))]
    on = api.Circuit.from_spec(14, spec, use_mfma=1)
    assert [k for k, _, _ in on.passes()] == [4]
    assert on.passes()[0][1] == 11          # tile = 4 widened targets + 7 other bits
    spec10 = [qsynth.gate("MAT", (3, 8, 9), mat=qsynth.haar_unitary(8, rng))]
    small = api.Circuit.from_spec(10, spec10, use_mfma=1)   # 4 + 7 > 10: no matrix cores
    assert 4 not in [k for k, _, _ in small.passes()]


def test_schedule_query_and_rollout_planning_time(api):
    import time
    n = 20
    _, spec, _, _ = qsynth.gradient_20q(seed=0, n=n, layers=12)
    c = api.Circuit.from_spec(n, spec, low_bits=6)
    assert c.schedule() == 2          # the one-step rollout gives the shortest plan here
    rng = np.random.default_rng(5)
    brick = [qsynth.gate("MAT", (q, q + 1), mat=qsynth.haar_unitary(4, rng))
             for d in range(8) for q in range(d % 2, 15, 2)]
    assert api.Circuit.from_spec(16, brick, tile_bits=8, low_bits=3).schedule() == 2
    assert api.Circuit.from_spec(16, qsynth.qft(16)).schedule() in (0, 1, 2)
    raw = api.circuit_create(4)
    with pytest.raises(api.QsError) as e:
        api.circuit_schedule(raw)
    assert e.value.code == -5
    api.circuit_destroy(raw)
    # planning cost stays bounded on long layered circuits (the rollout is
    # capped in first choices and skipped past a gate count)
    n = 30
    _, spec, _, _ = qsynth.gradient_20q(seed=1, n=n, layers=60)
    t = time.perf_counter()
    c = api.Circuit.from_spec(n, spec)
    assert time.perf_counter() - t < 60.0
    assert c.info()[0] == 3600


def test_default_row_length_follows_pass_count(api):
    # with low_bits left open the planner also plans rows one bit shorter and
    # keeps that plan only when it has fewer passes
    _, spec, _, _ = qsynth.gradient_20q(seed=0, n=30, layers=10)
    counts = {lb: api.Circuit.from_spec(30, spec, low_bits=lb).info()[1] for lb in (0, 5, 6)}
    assert counts == {0: 11, 5: 11, 6: 13}
    _, spec, _, _ = qsynth.gradient_20q(seed=0, n=20, layers=12)
    counts = {lb: api.Circuit.from_spec(20, spec, low_bits=lb).info()[1] for lb in (0, 5, 6)}
    assert counts == {0: 7, 5: 7, 6: 9}
    # the QFT needs five passes either way
    counts = {lb: api.Circuit.from_spec(30, qsynth.qft(30), low_bits=lb).info()[1] for lb in (0, 6)}
    assert counts == {0: 5, 6: 5}
