#!/usr/bin/env python
"""Benchmark of the state-vector hot path on one MI355X.

One step = one pass of the whole 30-qubit hot path on seeded synthetic input,
complex64 amplitudes with float64 accumulation:
  1. QFT on 30 qubits (H, controlled phase, SWAP: 480 gates) on a random state;
  2. a 30-qubit variational circuit (10 layers of RY on every qubit + CZ ring,
     600 gates, 300 angles ~ U[0, 2pi)) from |0..0>;
  3. its energy <H>, H = sum Z_i Z_{i+1} (ring) + 0.5 sum X_i;
  4. the adjoint gradient of that energy (all 300 angles);
  5. 100000 measurement shots of the QFT output (all qubits).
value = forward gates (480 + 600) per second of the whole step.

Prints ONE JSON line.  Also measured in the same run (outside the timed
steps) and reported in the line: adjoint/forward time ratio, QFT-only gates/s,
the 24-qubit complex128 adiabatic run (1000 Trotter steps) and the batched
variational workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "state-vector GB/s & gates/s at 30 qubits; adjoint-grad / forward time ratio"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(n: int):
    """The CPU oracle on a bounded sample of the same workload: the first two
    QFT-30 gates (H, controlled phase) on a basis state, complex128."""
    import numpy as np
    import qsynth
    from oracle import gates as og, statevec as sv
    spec = qsynth.qft(n)[:2]
    psi = sv.basis(n, 12345)
    t = time.perf_counter()
    for g in spec:
        psi = sv.apply(psi, og.gate_matrix(g), g.targets, g.controls)
    dt = time.perf_counter() - t
    try:
        import threadpoolctl
        thr = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        thr = 1
    del psi
    return {"value": len(spec) / dt, "unit": "gates/s", "cores": int(thr), "kind": "oracle",
            "sample": f"first {len(spec)} QFT-{n} gates on a basis state, numpy complex128, {dt:.1f} s; "
                      f"host has {os.cpu_count()} logical CPUs"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--shots", type=int, default=100000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        sys.exit("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)")

    import numpy as np
    import torch

    import qsynth
    from paper_2009_01845_amd import api

    n = args.n
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()

    # ---- seeded synthetic inputs, resident in HBM before timing
    gen = torch.Generator(device=dev)
    gen.manual_seed(0)
    v = torch.randn(2 << n, generator=gen, device=dev, dtype=torch.float32)
    psi_in = torch.view_as_complex(v.view(-1, 2))
    psi_in /= torch.linalg.vector_norm(psi_in)
    del v
    qft = api.Circuit.from_spec(n, qsynth.qft(n))
    vn, vspec, vparams, vterms = qsynth.gradient_20q(seed=0, n=n, layers=10)
    var = api.Circuit.from_spec(n, vspec)
    H = api.Observable.pauli_sum(n, vterms)
    st_q = api.State(n, "c64")
    st_v = api.State(n, "c64")
    lam = api.State(n, "c64")
    qft_gates = qft.info()[0]
    var_gates = var.info()[0]
    log("n", n, "qft passes", qft.info()[1], "var passes", var.info()[1])

    comp = {"qft": 0.0, "var_fwd": 0.0, "energy": 0.0, "adjoint": 0.0, "sample": 0.0}

    def step(timed: bool):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        ev[0].record(stream)
        st_q.tensor.copy_(psi_in)
        qft.run(st_q)
        ev[1].record(stream)
        st_v.set_basis(0)
        var.run(st_v, vparams)
        ev[2].record(stream)
        H.expectation(st_v)
        ev[3].record(stream)
        api.adjoint(var.h, vparams, H.h, st_v.h, lam.h, var.nparams)
        ev[4].record(stream)
        api.sample(st_q.h, list(range(n)), args.shots, seed=7)
        ev[5].record(stream)
        if timed:
            torch.cuda.synchronize()
            for k, (a, b) in zip(comp, zip(ev[:-1], ev[1:])):
                comp[k] += a.elapsed_time(b)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    api.profile_reset()
    api.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
        log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    api.profile_enable(False)
    tile_n, tile_ms = api.profile_read(0)
    perm_n, perm_ms = api.profile_read(2)
    adj_n, adj_ms = api.profile_read(7)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = (qft_gates + var_gates) / (ms_per_step / 1e3)

    bytes_pass = 2 * (1 << n) * 8  # one read + one write of every complex64 amplitude
    tile_avg = tile_ms / max(tile_n, 1)
    achieved = bytes_pass / (tile_avg / 1e3) / 1e9
    per = {k: v / args.steps for k, v in comp.items()}
    fwd_ms = per["var_fwd"] + per["energy"]
    qft_gps = qft_gates / (per["qft"] / 1e3)
    passes_total = qft.info()[1] + var.info()[1]
    gbps_state = passes_total * bytes_pass / ((per["qft"] + per["var_fwd"]) / 1e3) / 1e9

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (fp32 pairs, fp64 accumulation)",
        "data": "synthetic (seeded)",
        "config": {"workload": f"QFT-{n} + variational-{n} energy and adjoint gradient + {args.shots} shots",
                   "n_qubits": n, "qft_gates": qft_gates, "variational_gates": var_gates,
                   "variational_params": var.nparams, "shots": args.shots, "parallelism": "single GPU"},
        "gbps_state_passes": gbps_state,
        "qft_gates_per_s": qft_gps,
        "adjoint_over_forward": per["adjoint"] / fwd_ms,
        "components_ms": per,
        "roofline": {"bound": "hbm", "kernel": "k_tile<float> (tiled pass)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "launches": tile_n, "avg_launch_ms": tile_avg,
                     "algorithmic_bytes_per_launch": bytes_pass},
        "perm_pass_avg_ms": perm_ms / max(perm_n, 1),
        "adjoint_pass_avg_ms": adj_ms / max(adj_n, 1),
    }
    del st_q, st_v, lam, psi_in
    torch.cuda.empty_cache()

    if not args.no_extras:
        ex = {}
        # adiabatic evolution, 24 qubits complex128, T = 10, dt = 0.01
        na, J, h, T, dta = qsynth.adiabatic_24q(0)
        st = api.State(na, "c128")
        st.set_plus()
        I = api.Observable.ising(na, J, h)
        torch.cuda.synchronize()
        t = time.perf_counter()
        e = api.adiabatic_run(st.h, I.h, T, dta)
        ex["adiabatic_24q_c128_s"] = time.perf_counter() - t
        ex["adiabatic_24q_energy"] = e
        ex["adiabatic_24q_overlap_ground"] = float(
            st.tensor[int(np.argmin(_ising_e_gpu(J, h, na)))].abs().item() ** 2)
        del st
        log("adiabatic done")
        out["extras"] = ex

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(n)
    print(json.dumps(out), flush=True)


def _ising_e_gpu(J, h, n):
    """Energies E(x) of the Ising problem for locating its ground state
    (computed with torch on the GPU; used only for the reported overlap)."""
    import torch
    x = torch.arange(1 << n, device="cuda", dtype=torch.int64)
    z = [(1 - 2 * ((x >> (n - 1 - q)) & 1)).to(torch.float64) for q in range(n)]
    E = torch.zeros(1 << n, device="cuda", dtype=torch.float64)
    for i in range(n):
        E += float(h[i]) * z[i]
        for j in range(i + 1, n):
            if J[i, j] != 0:
                E += float(J[i, j]) * z[i] * z[j]
    return E.cpu().numpy()


if __name__ == "__main__":
    main()
