"""The no-allocation expectation entry point against the allocating one.

qs_expectation_noalloc runs the same kernels as qs_expectation_async with
its partial sums in the library's fixed per-GPU workspace.  Two calls in a
row, the second on a smaller state and observable, must each give what the
allocating entry point gives (same kernels, same fixed summation order: equal
bit for bit), and both must match the oracle's <psi|H|psi> within the
stated bar."""
import ctypes as C

import numpy as np
import pytest

import qsynth
from oracle import observables as oobs

from gpu_util import banner, gpu_state, oracle_input

pytestmark = pytest.mark.gpu
TOL_E = {"c64": 1e-5, "c128": 1e-12}


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2009_01845_amd import api as a
    return a


def _terms(n, seed):
    # diagonal ZZ ring, X on every qubit (tile sets), random Pauli strings
    # (far flip groups on the high qubits too)
    return qsynth.zz_ring_plus_x(n) + qsynth.random_pauli_sum(n, 12, seed)


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_noalloc_matches_allocating_entry_point(api, dt):
    import torch
    from paper_2009_01845_amd import _lib
    L = _lib.lib()
    for n, seed in [(22, 3), (13, 4)]:  # the second call is smaller
        banner("noalloc expectation", dt, n, seed)
        psi0 = qsynth.random_state(n, seed)
        st = gpu_state(api, n, dt, psi0)
        terms = _terms(n, seed)
        H = api.Observable.pauli_sum(n, terms)
        ref_dev = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        got_dev = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        api.expectation_async(st.h, H.h, ref_dev.data_ptr())  # also uploads the observable's tables
        assert L.qs_expectation_noalloc(st.h, H.h, C.c_void_p(got_dev.data_ptr())) == 0, L.qs_last_error()
        st.sync()
        torch.cuda.synchronize()
        ref, got = float(ref_dev.item()), float(got_dev.item())
        assert got == ref, (n, got, ref)
        e_or = oobs.expectation(oracle_input(psi0, dt), terms).real
        assert abs(got - e_or) < TOL_E[dt] * max(1.0, abs(e_or)), (n, got, e_or)


def test_noalloc_rejects_what_it_cannot_serve(api):
    import torch
    from paper_2009_01845_amd import _lib
    L = _lib.lib()
    n = 10
    banner("noalloc errors", n)
    st = gpu_state(api, n, "c64", qsynth.random_state(n, 1))
    H = api.Observable.pauli_sum(n, qsynth.zz_ring_plus_x(n))
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    # tables not yet on the device: an error, not an allocation
    assert L.qs_expectation_noalloc(st.h, H.h, C.c_void_p(out.data_ptr())) == -5
    assert b"upload" in L.qs_last_error()
    assert L.qs_expectation_noalloc(st.h, H.h, None) == -1
    H12 = api.Observable.pauli_sum(12, qsynth.z_sum(12))
    assert L.qs_expectation_noalloc(st.h, H12.h, C.c_void_p(out.data_ptr())) == -5
    # more reduction slots than the fixed workspace holds: random strings on
    # 20 qubits mostly flip more high bits than a tile holds: about a
    # hundred slots
    n2 = 20
    st2 = gpu_state(api, n2, "c64", qsynth.random_state(n2, 2))
    big = api.Observable.pauli_sum(n2, qsynth.random_pauli_sum(n2, 120, 5))
    api.expectation_async(st2.h, big.h, out.data_ptr())
    assert L.qs_expectation_noalloc(st2.h, big.h, C.c_void_p(out.data_ptr())) == -1
    assert b"reduction slots" in L.qs_last_error()
