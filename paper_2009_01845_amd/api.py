"""Python binding of include/qsim.h.

Functions carry the C names without the ``qs_`` prefix and only marshal
arguments; every computation runs in libqsim.so's HIP kernels.  States live
in torch tensors (torch supplies device memory and the stream), wrapped by
``qs_state_wrap``.  The small classes below bundle a handle with its memory.
"""
from __future__ import annotations

import ctypes as C
from typing import Iterable, Sequence

import numpy as np

from . import _lib as _lib_mod
from ._lib import QS_C64, QS_C128, QsError, Tune, check, lib  # noqa: F401

_F64P = C.POINTER(C.c_double)


def _i32(seq: Sequence[int] | None):
    if not seq:
        return None
    return (C.c_int32 * len(seq))(*[int(v) for v in seq])


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_F64P)


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    if stream is not None:
        return C.c_void_p(int(stream))
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def dtype_code(dt) -> int:
    if dt in ("c64", QS_C64, np.complex64):
        return QS_C64
    if dt in ("c128", QS_C128, np.complex128):
        return QS_C128
    torch = _torch()
    if dt == torch.complex64:
        return QS_C64
    if dt == torch.complex128:
        return QS_C128
    raise ValueError(f"unsupported dtype {dt}")


# --------------------------------------------------------------------- raw ABI
def version() -> str:
    return lib().qs_version().decode()


def last_error() -> str:
    return lib().qs_last_error().decode()


def state_create(n: int, dt, stream=None):
    h = C.c_void_p()
    check(lib().qs_state_create(n, dtype_code(dt), _stream_ptr(stream), C.byref(h)))
    return h


def state_wrap(dev_ptr: int, n: int, dt, stream=None):
    h = C.c_void_p()
    check(lib().qs_state_wrap(C.c_void_p(dev_ptr), n, dtype_code(dt), _stream_ptr(stream), C.byref(h)))
    return h


def state_destroy(h):
    check(lib().qs_state_destroy(h))


def state_set_basis(h, x: int):
    check(lib().qs_state_set_basis(h, int(x)))


def state_set_plus(h):
    check(lib().qs_state_set_plus(h))


def state_upload(h, host: np.ndarray):
    host = np.ascontiguousarray(host)
    check(lib().qs_state_upload(h, host.ctypes.data_as(C.c_void_p)))


def state_download(h, n: int, dt) -> np.ndarray:
    out = np.empty(1 << n, dtype=np.complex128 if dtype_code(dt) == QS_C128 else np.complex64)
    check(lib().qs_state_download(h, out.ctypes.data_as(C.c_void_p)))
    return out


def state_copy(dst, src):
    check(lib().qs_state_copy(dst, src))


def state_sync(h):
    check(lib().qs_state_sync(h))


def gate_matrix(name: str, theta: float = 0.0) -> np.ndarray:
    buf = np.zeros(2 * 32 * 32)
    k = C.c_int32()
    check(lib().qs_gate_matrix(name.encode(), float(theta), buf.ctypes.data_as(_F64P), C.byref(k)))
    d = 1 << k.value
    return (buf[0:2 * d * d:2] + 1j * buf[1:2 * d * d:2]).reshape(d, d)


def _mat_arg(mat):
    m = np.ascontiguousarray(np.asarray(mat, dtype=np.complex128))
    flat = np.empty(2 * m.size)
    flat[0::2] = m.real.ravel()
    flat[1::2] = m.imag.ravel()
    return _f64(flat)


def apply(h, mat, targets: Sequence[int], controls: Sequence[int] = ()):
    keep, mp = _mat_arg(mat)
    check(lib().qs_apply(h, mp, len(targets), _i32(targets), len(controls), _i32(controls)))


def circuit_create(n: int):
    h = C.c_void_p()
    check(lib().qs_circuit_create(n, C.byref(h)))
    return h


def circuit_add_gate(c, mat, targets, controls=()):
    keep, mp = _mat_arg(mat)
    check(lib().qs_circuit_add_gate(c, mp, len(targets), _i32(targets), len(controls), _i32(controls)))


def circuit_add_rot(c, pauli: str, target: int, param_index: int, controls=()):
    check(lib().qs_circuit_add_rot(c, pauli.encode(), int(target), int(param_index), len(controls),
                                   _i32(controls)))


def circuit_compile(c, tile_bits=0, fuse_k=0, use_mfma=-1, low_bits=0, lane_ops=0):
    t = Tune(tile_bits, fuse_k, use_mfma, low_bits, int(lane_ops))
    check(lib().qs_circuit_compile(c, C.byref(t)))


def circuit_run(c, h, params=None, params_on_device: bool = False):
    if params is None:
        check(lib().qs_circuit_run(c, h, None, 0))
    elif params_on_device:
        check(lib().qs_circuit_run(c, h, C.c_void_p(int(params)), 1))
    else:
        keep, pp = _f64(params)
        check(lib().qs_circuit_run(c, h, C.cast(pp, C.c_void_p), 0))


def circuit_info(c):
    g, p, n = C.c_int32(), C.c_int32(), C.c_int32()
    check(lib().qs_circuit_info(c, C.byref(g), C.byref(p), C.byref(n)))
    return g.value, p.value, n.value


def circuit_pass_info(c, i: int):
    k, m, o = C.c_int32(), C.c_int32(), C.c_int32()
    check(lib().qs_circuit_pass_info(c, i, C.byref(k), C.byref(m), C.byref(o)))
    return k.value, m.value, o.value


def circuit_schedule(c) -> int:
    v = C.c_int32()
    check(lib().qs_circuit_schedule(c, C.byref(v)))
    return v.value


def circuit_destroy(c):
    check(lib().qs_circuit_destroy(c))


def circuit_create_density(n: int):
    h = C.c_void_p()
    check(lib().qs_circuit_create_density(n, C.byref(h)))
    return h


def channel_kraus(name: str, p: float) -> list:
    buf = np.zeros(2 * 4 * 16)
    nk, k = C.c_int32(), C.c_int32()
    check(lib().qs_channel_kraus(name.encode(), float(p), buf.ctypes.data_as(_F64P), C.byref(nk), C.byref(k)))
    d = 1 << k.value
    z = buf[0::2] + 1j * buf[1::2]
    return [z[i * d * d:(i + 1) * d * d].reshape(d, d) for i in range(nk.value)]


def circuit_add_channel(c, kraus, targets: Sequence[int]):
    mats = [np.asarray(K, dtype=np.complex128) for K in kraus]
    keep, mp = _mat_arg(np.concatenate([K.ravel() for K in mats]))
    check(lib().qs_circuit_add_channel(c, len(mats), mp, len(targets), _i32(targets)))


def density_set_pure(rho, psi):
    check(lib().qs_density_set_pure(rho, psi))


def density_expectation(rho, o) -> float:
    v = C.c_double()
    check(lib().qs_density_expectation(rho, o, C.byref(v)))
    return v.value


def density_trace(rho) -> float:
    v = C.c_double()
    check(lib().qs_density_trace(rho, C.byref(v)))
    return v.value


def pauli_sum_create(n: int, terms: Iterable):
    terms = list(terms)
    co = np.array([float(c) for c, _ in terms])
    arr = (C.c_char_p * max(1, len(terms)))(*[s.encode() for _, s in terms])
    h = C.c_void_p()
    keep, cp = _f64(co)
    check(lib().qs_pauli_sum_create(n, len(terms), cp, arr, C.byref(h)))
    return h


def ising_create(n: int, J, h_field):
    J = np.ascontiguousarray(J, dtype=np.float64).reshape(n, n)
    kj, jp = _f64(J)
    kh, hp = _f64(h_field)
    h = C.c_void_p()
    check(lib().qs_ising_create(n, jp, hp, C.byref(h)))
    return h


def obs_destroy(o):
    check(lib().qs_obs_destroy(o))


def expectation(h, o) -> float:
    v = C.c_double()
    check(lib().qs_expectation(h, o, C.byref(v)))
    return v.value


def expectation_async(h, o, dev_out: int):
    check(lib().qs_expectation_async(h, o, C.c_void_p(int(dev_out))))


def expectation_noalloc(h, o, dev_out: int):
    check(lib().qs_expectation_noalloc(h, o, C.c_void_p(int(dev_out))))


def norm2(h) -> float:
    v = C.c_double()
    check(lib().qs_norm2(h, C.byref(v)))
    return v.value


def sample(h, qubits: Sequence[int], shots: int, seed: int = 0, uniforms=None) -> np.ndarray:
    out = np.empty(max(1, shots), dtype=np.int64)
    if uniforms is not None:
        keep, up = _f64(uniforms)
    else:
        up = None
    check(lib().qs_sample(h, len(qubits), _i32(qubits), int(shots), int(seed), up,
                          out.ctypes.data_as(C.POINTER(C.c_int64))))
    return out[:shots]


def adiabatic_run(h, h1, T: float, dt: float, order: int = 2) -> float:
    e = C.c_double()
    check(lib().qs_adiabatic_run(h, h1, float(T), float(dt), int(order), C.byref(e)))
    return e.value


SOLVERS = {"exp": 1, "rk4": 2, "rk45": 3}


def _callbacks(K: int, every: int, energy=None, entropy_qubits: int = 0):
    """A qs_callbacks record and its output arrays (K / every values each)."""
    if not every:
        return None, None, None
    cnt = max(1, K // every)
    en = np.zeros(cnt)
    ent = np.zeros(cnt)
    cb = _lib_mod.Callbacks(int(every), int(entropy_qubits), energy.h if energy is not None else None,
                            en.ctypes.data_as(_F64P), ent.ctypes.data_as(_F64P))
    return cb, en, ent


def entanglement_entropy(h, a: int) -> float:
    v = C.c_double()
    check(lib().qs_entanglement_entropy(h, int(a), C.byref(v)))
    return v.value


def evolve(h, h0, h1, T: float, dt: float, solver: str = "exp", every: int = 0, energy=None,
           entropy_qubits: int = 0):
    """Integrate the Schroedinger equation (h0, h1: Observable).  Returns the
    recorded (energies, entropies) when every > 0, else (None, None)."""
    K = int(round(T / dt))
    cb, en, ent = _callbacks(K, every, energy, entropy_qubits)
    check(lib().qs_evolve(h, h0.h, h1.h, float(T), float(dt), SOLVERS[solver], C.byref(cb) if cb else None))
    return (en if energy is not None else None, ent if entropy_qubits else None) if cb else (None, None)


def adiabatic_run_callbacks(h, h1, T: float, dt: float, every: int, energy=None, entropy_qubits: int = 0,
                            order: int = 2):
    """Trotter evolution with callbacks; returns (final <H1>, energies, entropies)."""
    K = int(round(T / dt))
    cb, en, ent = _callbacks(K, every, energy, entropy_qubits)
    e = C.c_double()
    check(lib().qs_adiabatic_run_callbacks(h, h1.h, float(T), float(dt), int(order), C.byref(cb) if cb else None,
                                           C.byref(e)))
    return e.value, (en if energy is not None else None), (ent if entropy_qubits else None)


def adjoint(c, params, H, psi, lam, nparams: int):
    keep, pp = _f64(params if params is not None else np.zeros(0))
    grad = np.zeros(max(1, nparams))
    e = C.c_double()
    check(lib().qs_adjoint(c, pp, H, psi, lam, grad.ctypes.data_as(_F64P), C.byref(e)))
    return e.value, grad[:nparams]


def autotune(c, h, params=None, cache_path: str | None = None):
    keep, pp = _f64(params if params is not None else np.zeros(1))
    check(lib().qs_autotune(c, h, pp, cache_path.encode() if cache_path else None))


def profile_enable(on: bool = True):
    check(lib().qs_profile_enable(1 if on else 0))


def profile_reset():
    check(lib().qs_profile_reset())


def profile_read(family: int):
    n, ms = C.c_int64(), C.c_double()
    check(lib().qs_profile_read(family, C.byref(n), C.byref(ms)))
    return n.value, ms.value


PROFILE_FAMILIES = {"tile": 0, "phase": 1, "perm": 2, "mfma": 3, "dense": 4, "reduce": 5, "sample": 6,
                    "adjoint": 7, "batch": 8, "other": 9}


# --------------------------------------------------------------- conveniences
class State:
    """2^n amplitudes in a torch tensor on the current GPU, wrapped by the library."""

    def __init__(self, n: int, dtype="c64", tensor=None, stream=None):
        torch = _torch()
        self.n = n
        self.code = dtype_code(dtype)
        tdt = torch.complex128 if self.code == QS_C128 else torch.complex64
        if tensor is None:
            tensor = torch.zeros(1 << n, dtype=tdt, device="cuda")
            tensor[0] = 1.0
        if tensor.dtype != tdt or tensor.numel() != (1 << n) or not tensor.is_contiguous():
            raise ValueError("tensor must be a contiguous 2^n vector of the state dtype")
        self.tensor = tensor
        self.h = state_wrap(tensor.data_ptr(), n, self.code, stream)

    def set_basis(self, x: int):
        state_set_basis(self.h, x)

    def set_plus(self):
        state_set_plus(self.h)

    def upload(self, psi: np.ndarray):
        state_upload(self.h, np.ascontiguousarray(psi, dtype=np.complex128 if self.code == QS_C128 else np.complex64))

    def download(self) -> np.ndarray:
        return state_download(self.h, self.n, self.code)

    def sync(self):
        state_sync(self.h)

    def norm2(self) -> float:
        return norm2(self.h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                state_destroy(h)
            except Exception:
                pass
            self.h = None


class Observable:
    def __init__(self, h, n):
        self.h = h
        self.n = n

    @classmethod
    def pauli_sum(cls, n, terms):
        return cls(pauli_sum_create(n, terms), n)

    @classmethod
    def ising(cls, n, J, h_field):
        return cls(ising_create(n, J, h_field), n)

    def expectation(self, st: State) -> float:
        return expectation(st.h, self.h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                obs_destroy(h)
            except Exception:
                pass
            self.h = None


class Circuit:
    """A gate queue (paper Sec. 2.3) compiled into tiled passes."""

    def __init__(self, n: int):
        self.n = n
        self.h = circuit_create(n)

    @classmethod
    def from_spec(cls, n: int, spec, **compile_opts):
        """Build from ``qsynth.G`` records: named gates take their matrix from
        ``qs_gate_matrix``; trainable rotations become ``add_rot``."""
        c = cls(n)
        for g in spec:
            if g.pidx >= 0:
                circuit_add_rot(c.h, g.name[1], g.targets[0], g.pidx, g.controls)
            else:
                m = g.mat if g.name == "MAT" else gate_matrix(g.name, g.theta)
                circuit_add_gate(c.h, m, g.targets, g.controls)
        c.compile(**compile_opts)
        return c

    def add(self, mat, targets, controls=()):
        circuit_add_gate(self.h, mat, targets, controls)

    def add_rot(self, pauli, target, pidx, controls=()):
        circuit_add_rot(self.h, pauli, target, pidx, controls)

    def compile(self, **opts):
        circuit_compile(self.h, **opts)

    def run(self, st: State, params=None):
        circuit_run(self.h, st.h, params)

    def autotune(self, st: State, params=None, cache_path: str | None = None):
        """Pick the fastest plan for this circuit on st's precision (st is overwritten)."""
        autotune(self.h, st.h, params, cache_path)

    def info(self):
        return circuit_info(self.h)

    def passes(self):
        return [circuit_pass_info(self.h, i) for i in range(self.info()[1])]

    def schedule(self) -> int:
        return circuit_schedule(self.h)

    @property
    def nparams(self):
        return self.info()[2]

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                circuit_destroy(h)
            except Exception:
                pass
            self.h = None


class DensityMatrix:
    """An n-qubit density matrix held as a 2n-qubit state (rho[r][c] at
    r * 2^n + c), initialised to |0..0><0..0|."""

    def __init__(self, n: int, dtype="c64", stream=None):
        self.n = n
        self.state = State(2 * n, dtype, stream=stream)
        self.h = self.state.h

    def set_pure(self, psi: State):
        density_set_pure(self.h, psi.h)

    def set_basis(self, x: int):
        state_set_basis(self.h, (int(x) << self.n) | int(x))

    def expectation(self, obs: Observable) -> float:
        return density_expectation(self.h, obs.h)

    def trace(self) -> float:
        return density_trace(self.h)

    def download(self) -> np.ndarray:
        return self.state.download().reshape(1 << self.n, 1 << self.n)

    def upload(self, rho: np.ndarray):
        self.state.upload(np.asarray(rho).reshape(-1))


class DensityCircuit(Circuit):
    """A circuit acting on density matrices (Sec. 2.4.3): gates as
    U rho U^dagger, channels as sum_i K_i rho K_i^dagger."""

    def __init__(self, n: int):
        self.n = n
        self.h = circuit_create_density(n)

    @classmethod
    def from_spec(cls, n: int, spec, **compile_opts):
        """``qsynth.G`` records; ``CH:<channel>`` records are named channels
        with their parameter in theta."""
        c = cls(n)
        for g in spec:
            if g.name.startswith("CH:"):
                circuit_add_channel(c.h, channel_kraus(g.name[3:], g.theta), g.targets)
            elif g.pidx >= 0:
                circuit_add_rot(c.h, g.name[1], g.targets[0], g.pidx, g.controls)
            else:
                m = g.mat if g.name == "MAT" else gate_matrix(g.name, g.theta)
                circuit_add_gate(c.h, m, g.targets, g.controls)
        c.compile(**compile_opts)
        return c

    def add_channel(self, kraus, targets):
        circuit_add_channel(self.h, kraus, targets)

    def run(self, rho: DensityMatrix, params=None):
        circuit_run(self.h, rho.h, params)


# ---------------------------------------------------------------------- batch
def batch_create(circs, observables, dt="c64", stream=None):
    arr_c = (C.c_void_p * len(circs))(*[c.h.value for c in circs])
    arr_o = (C.c_void_p * len(observables))(*[o.h.value for o in observables])
    h = C.c_void_p()
    check(lib().qs_batch_create(len(circs), C.cast(arr_c, C.POINTER(C.c_void_p)),
                                C.cast(arr_o, C.POINTER(C.c_void_p)), dtype_code(dt),
                                C.c_void_p(int(stream)) if stream is not None else None, C.byref(h)))
    return h


def batch_run(h, params_packed, count: int, nparams: int, want_grads: bool = True):
    keep, pp = _f64(params_packed if nparams else np.zeros(1))
    e = np.zeros(count)
    g = np.zeros(max(1, nparams))
    check(lib().qs_batch_run(h, pp, e.ctypes.data_as(_F64P), g.ctypes.data_as(_F64P) if want_grads else None))
    return e, g[:nparams]


def batch_destroy(h):
    check(lib().qs_batch_destroy(h))


class Batch:
    """Many circuits with their own parameters and diagonal observables, run
    level by level (one pass of every instance per launch) and captured as a
    HIP graph on the first run.  stream: a HIP stream handle (int) or None
    for a stream of the batch's own."""

    def __init__(self, circuits, observables, dtype="c64", stream=None):
        self.circuits, self.observables = list(circuits), list(observables)  # keep the handles alive
        self.nparams = sum(c.nparams for c in self.circuits)
        self.h = batch_create(self.circuits, self.observables, dtype, stream)

    def run(self, params_packed, want_grads: bool = True):
        return batch_run(self.h, params_packed, len(self.circuits), self.nparams, want_grads)

    def autotune(self, params_packed, cache_path: str | None = None):
        keep, pp = _f64(params_packed if self.nparams else np.zeros(1))
        check(lib().qs_batch_autotune(self.h, pp, cache_path.encode() if cache_path else None))

    def choice(self, i: int) -> dict:
        t = Tune()
        check(lib().qs_batch_choice(self.h, i, C.byref(t)))
        return {"tile_bits": t.tile_bits, "fuse_k": t.fuse_k, "use_mfma": t.use_mfma, "low_bits": t.low_bits,
                "lane_ops": t.lane_ops}

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                batch_destroy(h)
            except Exception:
                pass
            self.h = None
