"""Helpers shared by the GPU parity tests (test infrastructure)."""
import sys

import numpy as np

TOL = {"c64": 1e-5, "c128": 1e-12}
NPDT = {"c64": np.complex64, "c128": np.complex128}


def banner(*parts):
    print("[case]", *parts, flush=True)
    sys.stdout.flush()


def product_circuit(api, n, spec, **opts):
    return api.Circuit.from_spec(n, spec, **opts)


def gpu_state(api, n, dt, psi0=None):
    st = api.State(n, dt)
    if psi0 is not None:
        st.upload(np.asarray(psi0).astype(NPDT[dt]))
    return st


def oracle_input(psi0, dt):
    """What the oracle consumes for a run in precision dt: the input rounded
    to that precision, then widened to complex128."""
    return np.asarray(psi0).astype(NPDT[dt]).astype(np.complex128)


def maxabs(a, b):
    return float(np.max(np.abs(np.asarray(a, dtype=np.complex128) - np.asarray(b, dtype=np.complex128))))


def sampling_bound(n: int) -> float:
    """Largest CDF disagreement (relative to the total) that two float64
    prefix sums of the same 2^n non-negative terms can show in any summation
    order: each side is within (N - 1) u of the exact sum (u = 2^-53), and
    the per-term squares may differ by a few units in the last place."""
    return ((1 << n) + 8) * 2.0 ** -52


def assert_samples_match(got, psi_ref, qubits, u):
    """Shot-by-shot equality with the oracle's inverse-CDF draw, except where
    u_j * total lies within sampling_bound(n) of a CDF edge (there either
    neighbour is a correct draw under float64 rounding)."""
    from oracle import sampling as osamp
    n = int(np.log2(psi_ref.size))
    exp = osamp.sample(psi_ref, qubits, u)
    bad = np.nonzero(np.asarray(got) != exp)[0]
    if bad.size:
        idx = osamp.sample_indices(psi_ref, np.asarray(u)[bad])
        d = osamp.boundary_distance(psi_ref, np.asarray(u)[bad], idx)
        assert np.all(d < sampling_bound(n)), (bad[:10], d[:10])
    return bad.size
