"""Per-result error of the HIP path against the float64 oracle, for each of
the benchmarked workloads at the largest size the oracle runs in seconds
(test infrastructure: it imports the oracle).

    python tests/precision_report.py [--out FILE.md]

Prints one JSON line per case and, with --out, a markdown table.  Errors:
max-abs amplitude error, 2-norm of the amplitude difference, |dE| of the
energy and max |d grad| of the gradient, complex64 (float64 accumulation)
and complex128."""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import qsynth  # noqa: E402
from oracle import adiabatic as oad  # noqa: E402
from oracle import circuits as ocirc  # noqa: E402
from oracle import gradients as ograd  # noqa: E402
from oracle import observables as oobs  # noqa: E402

NPDT = {"c64": np.complex64, "c128": np.complex128}


def _err(got, ref):
    d = np.asarray(got, dtype=np.complex128) - np.asarray(ref, dtype=np.complex128)
    return {"max_abs": float(np.max(np.abs(d))), "l2": float(np.linalg.norm(d))}


def _oracle_in(psi, dt):
    return np.asarray(psi).astype(NPDT[dt]).astype(np.complex128)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--quick", action="store_true", help="skip the 28-qubit QFT and the 20-qubit oracle adjoint")
    args = ap.parse_args()
    import torch
    from paper_2009_01845_amd import api
    rows = []

    def emit(row):
        rows.append(row)
        print(json.dumps(row), flush=True)

    for dt in ("c64", "c128"):
        # 10 qubits, depth 20: state and energy
        n, spec, params, terms = qsynth.variational_10q(0)
        c = api.Circuit.from_spec(n, spec)
        st = api.State(n, dt)
        c.run(st, params)
        ref = ocirc.run(n, spec, None, params)
        H = api.Observable.pauli_sum(n, terms)
        e = H.expectation(st)
        emit(dict(case="variational 10q depth 20", dtype=dt, **_err(st.download(), ref),
                  dE=abs(e - oobs.expectation(ref, terms).real)))
        # its gradient (400 parameters)
        psi, lam = api.State(n, dt), api.State(n, dt)
        c.run(psi, params)
        E, g = api.adjoint(c.h, params, H.h, psi.h, lam.h, c.nparams)
        E_ref, g_ref = ograd.adjoint(n, spec, params, terms)
        emit(dict(case="variational 10q adjoint", dtype=dt, dE=abs(E - E_ref), dgrad=float(np.max(np.abs(g - g_ref)))))
    if not args.quick:
        n = 28
        psi0 = qsynth.random_state(n, 2028)
        for dt in ("c64", "c128"):
            c = api.Circuit.from_spec(n, qsynth.qft(n))
            st = api.State(n, dt)
            st.upload(psi0.astype(NPDT[dt]))
            c.run(st)
            ref = ocirc.qft_via_fft(_oracle_in(psi0, dt))
            emit(dict(case="QFT-28 random state (vs FFT)", dtype=dt, **_err(st.download(), ref)))
            del st, ref
            torch.cuda.empty_cache()
        del psi0
        # 20 qubits, 200 parameters
        n, spec, params, terms = qsynth.gradient_20q(0)
        t = time.perf_counter()
        E_ref, g_ref = ograd.adjoint(n, spec, params, terms)
        psi_ref = ocirc.run(n, spec, None, params)
        for dt in ("c64", "c128"):
            c = api.Circuit.from_spec(n, spec)
            H = api.Observable.pauli_sum(n, terms)
            psi, lam = api.State(n, dt), api.State(n, dt)
            c.run(psi, params)
            st_err = _err(psi.download(), psi_ref)
            E, g = api.adjoint(c.h, params, H.h, psi.h, lam.h, c.nparams)
            emit(dict(case="gradient 20q (200 params)", dtype=dt, **st_err, dE=abs(E - E_ref),
                      dgrad=float(np.max(np.abs(g - g_ref))), oracle_s=time.perf_counter() - t))
    # batch: 32 instances spread over the sizes of the 512-instance workload
    insts = qsynth.batch_instances(seed=0)
    order = np.argsort([it[0] for it in insts], kind="stable")
    pick = [insts[i] for i in order[:: len(order) // 32]][:32]
    for dt in ("c64", "c128"):
        circs = [api.Circuit.from_spec(n, spec) for n, spec, _, _ in pick]
        obs = [api.Observable.pauli_sum(n, terms) for n, _, _, terms in pick]
        b = api.Batch(circs, obs, dt)
        P = np.concatenate([p for _, _, p, _ in pick])
        E, G = b.run(P)
        dE, dg, off = 0.0, 0.0, 0
        for i, (n, spec, p, terms) in enumerate(pick):
            e_ref, g_ref = ograd.adjoint(n, spec, p, terms)
            dE = max(dE, abs(E[i] - e_ref))
            dg = max(dg, float(np.max(np.abs(G[off:off + p.size] - g_ref))))
            off += p.size
        emit(dict(case=f"batch, {len(pick)} instances n={pick[0][0]}..{pick[-1][0]}", dtype=dt, dE=dE, dgrad=dg))
    # adiabatic evolution, 1000 steps
    for dt in ("c64", "c128"):
        n = 12
        J, h = qsynth.ising_couplings(n, 0)
        E = oobs.ising_energies(J, h)
        ref = oad.trotter(n, E, 10.0, 0.01)
        st = api.State(n, dt)
        st.set_plus()
        I = api.Observable.ising(n, J, h)
        e = api.adiabatic_run(st.h, I.h, 10.0, 0.01)
        emit(dict(case="adiabatic 12q, 1000 steps", dtype=dt, **_err(st.download(), ref), dE=abs(e - oad.energy(ref, E))))
    n = 24
    _, h = qsynth.ising_couplings(n, 24)
    st = api.State(n, "c128")
    st.set_plus()
    I = api.Observable.ising(n, np.zeros((n, n)), h)
    api.adiabatic_run(st.h, I.h, 10.0, 0.01)
    prod = np.array([1.0 + 0j])
    for q in range(n):
        prod = np.kron(prod, oad.single_qubit_trotter(h[q], 10.0, 0.01))
    emit(dict(case="adiabatic 24q J=0, 1000 steps (factorised)", dtype="c128", **_err(st.download(), prod)))
    del st
    # 30 qubits: product-state closed form of energy and gradient
    n = 30
    rng = np.random.default_rng(n + 1)
    th, ph = rng.uniform(0, 2 * np.pi, (3, n)), rng.uniform(0, 2 * np.pi, (3, n))
    spec = qsynth.ry_rz_layers(n, th, ph)
    params = np.concatenate([np.concatenate([th[l], ph[l]]) for l in range(3)])
    E_cf, g_cf = ograd.product_ring_energy(th, ph)
    c = api.Circuit.from_spec(n, spec)
    H = api.Observable.pauli_sum(n, qsynth.zz_ring_plus_x(n))
    psi, lam = api.State(n, "c64"), api.State(n, "c64")
    c.run(psi, params)
    E, g = api.adjoint(c.h, params, H.h, psi.h, lam.h, c.nparams)
    emit(dict(case="30q RY/RZ layers adjoint (closed form)", dtype="c64", dE=abs(E - E_cf),
              dgrad=float(np.max(np.abs(g - g_cf)))))
    del psi, lam
    torch.cuda.empty_cache()
    if args.out:
        cols = ["case", "dtype", "max_abs", "l2", "dE", "dgrad"]
        with open(args.out, "w") as f:
            f.write("# Error of the HIP path against the float64 oracle\n\n")
            f.write("Command: `python tests/precision_report.py --out " + args.out + "`\n\n")
            f.write("| " + " | ".join(cols) + " |\n|" + "---|" * len(cols) + "\n")
            for r in rows:
                f.write("| " + " | ".join(
                    (f"{r[k]:.2e}" if isinstance(r.get(k), float) else str(r.get(k, "")))
                    for k in cols) + " |\n")
    print("done", flush=True)


if __name__ == "__main__":
    main()
