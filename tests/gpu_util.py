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
