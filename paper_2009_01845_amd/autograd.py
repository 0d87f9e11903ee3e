"""<H> as a differentiable function of circuit angles.

Forward: ``qs_circuit_run`` then ``qs_expectation``.  Backward: the adjoint
sweep ``qs_adjoint`` (Jones & Gacon 2020), which un-applies the gates to the
state and to the co-state lambda = H psi and reads every rotation's
derivative Im<lambda|P psi> on the way; only two state vectors are held.
"""
from __future__ import annotations

import numpy as np

from .api import Circuit, Observable, State, adjoint, state_copy


def _torch():
    import torch
    return torch


def _make_fn():
    torch = _torch()

    class EnergyFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, params, circuit: Circuit, obs: Observable, dtype="c64"):
            p = np.ascontiguousarray(params.detach().to("cpu", torch.float64).numpy())
            st = State(circuit.n, dtype)
            circuit.run(st, p)
            e = obs.expectation(st)
            ctx.st, ctx.circuit, ctx.obs, ctx.p, ctx.dtype = st, circuit, obs, p, dtype
            ctx.pdtype, ctx.pdevice = params.dtype, params.device
            return torch.tensor(e, dtype=torch.float64)

        @staticmethod
        def backward(ctx, g):
            # the reverse sweep walks its state back to the circuit input, so
            # it runs on a copy: the saved output stays valid for a repeated
            # backward (retain_graph, autograd.grad twice, gradcheck)
            psi = State(ctx.circuit.n, ctx.dtype)
            state_copy(psi.h, ctx.st.h)
            lam = State(ctx.circuit.n, ctx.dtype)
            _, grad = adjoint(ctx.circuit.h, ctx.p, ctx.obs.h, psi.h, lam.h, ctx.circuit.nparams)
            out = torch.from_numpy(grad).to(device=ctx.pdevice, dtype=ctx.pdtype) * g.to(ctx.pdevice)
            return out, None, None, None

    return EnergyFn


_FN = None


def energy(params, circuit: Circuit, obs: Observable, dtype="c64"):
    """E(params) = <psi(params)|H|psi(params)> with an adjoint backward."""
    global _FN
    if _FN is None:
        _FN = _make_fn()
    return _FN.apply(params, circuit, obs, dtype)
