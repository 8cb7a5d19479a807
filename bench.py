#!/usr/bin/env python3
"""Benchmark of the state-vector hot path on one MI355X.

Workload (one "step"): a 30-qubit complex64 state is reset to |0...0>, a
10-layer circuit of RX(theta) then RZ(phi) on every qubit followed by a CNOT
ladder (i -> i+1) is applied (890 gates), and <H> is evaluated for H = 200
random weight-4 Pauli strings with N(0, 1) coefficients, accumulated in FP64.
Inputs are seeded and synthetic (no dataset exists for this workload).

value = circuit gates per second over whole steps (expectation included);
extra fields give the HBM bandwidth and the split between the circuit and the
expectation. `roofline` reports the kernel family that takes the most time in
the timed steps, timed with HIP events recorded by the library on the stream
the kernels run on. `cpu_baseline` times the CPU oracle on a bounded sample of
the same circuit (the first gates of it, complex128).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode fused|unfused]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBPS = 8000.0
METRIC = "gates/s + HBM GB/s at 30q; adjoint grads/s vs plain finite-diff, 24q c64"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", choices=["fused", "unfused"], default="fused")
    ap.add_argument("--max-k", type=int, default=2)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--low", type=int, default=0)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def cpu_baseline(n, gates, budget_s):
    """Time the CPU oracle (complex128) on the first gates of the circuit."""
    from oracle import oracle as O
    lib = O.lib()
    psi = O.zero_state(n)
    done = 0
    t0 = time.perf_counter()
    for g in gates:
        O.apply_gate(psi, g)
        done += 1
        if time.perf_counter() - t0 > budget_s and done >= 3:
            break
    dt = time.perf_counter() - t0
    threads = int(lib.orc_num_threads())
    del psi
    return {"value": done / dt, "unit": "gates/s", "cores": threads, "kind": "oracle",
            "sample": f"first {done} of {len(gates)} gates of the {n}-qubit circuit, complex128, "
                      f"{dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is a "
                                   "design note, not an implementation", "n_gpus": args.gpus}))
        sys.exit(2)

    import paper_2011_13524_amd as Q
    from paper_2011_13524_amd import workloads as W

    n = args.n
    dt = "c64"
    S = 8
    N = 1 << n
    gates = W.layered_rx_rz_cnot(n, 10, seed_key=(2,))
    obs_terms = W.random_pauli_observable(n, 200, 4, seed_key=(2, 1))
    circ = Q.Circuit.from_records(n, gates)
    obs = Q.Observable(n, obs_terms)
    _, nterms, ngroups = obs.info()
    state = Q.State(n, dt)
    plan = None
    if args.mode == "fused":
        plan = Q.Plan(circ, dt, max_k=args.max_k, tile_qubits=args.tile, low_qubits=args.low)

    def run_circuit():
        if plan is not None:
            Q.apply_fused(state, plan)
        else:
            Q.apply_circuit(state, circ)

    def step():
        state.set_basis(0)
        run_circuit()
        return Q.expectation(state, obs)

    for _ in range(args.warmup):
        step()

    # split of one step (synchronised between the parts)
    state.set_basis(0)
    state.norm2()
    t0 = time.perf_counter()
    run_circuit()
    state.norm2()  # forces completion of the circuit
    t1 = time.perf_counter()
    Q.expectation(state, obs)
    t2 = time.perf_counter()
    circuit_ms_incl_norm = (t1 - t0) * 1e3
    expect_ms = (t2 - t1) * 1e3

    # timed region
    Q.prof_enable(True)
    state.norm2()
    t0 = time.perf_counter()
    energy = None
    for _ in range(args.steps):
        energy = step()
    state.norm2()
    t1 = time.perf_counter()
    Q.prof_enable(False)
    total = t1 - t0
    ms_per_step = total * 1e3 / args.steps

    fams = {}
    for fam in ("pair", "scale", "diag", "dense", "expect", "tile"):
        cnt, ms, by = Q.prof_read(fam)
        if cnt:
            fams[fam] = {"launches": cnt, "ms": ms, "bytes": by}
    dom = max(fams, key=lambda f: fams[f]["ms"])
    d = fams[dom]
    achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
    step_bytes = sum(f["bytes"] for f in fams.values()) / args.steps

    out = {
        "metric": METRIC,
        "value": len(gates) * args.steps / total,
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dt,
        "data": "synthetic",
        "config": {"workload": f"{n}-qubit complex64, 10 layers RX/RZ on every qubit + CNOT "
                               f"ladder ({len(gates)} gates), then <H> of 200 random weight-4 "
                               f"Pauli strings (FP64 accumulation)",
                   "mode": args.mode, "qubits": n, "gates": len(gates),
                   "plan": plan.info() if plan is not None else None,
                   "observable_terms": nterms, "flip_mask_groups": ngroups},
        "hbm_gbps_step": step_bytes / (ms_per_step * 1e-3) / 1e9,
        "circuit_ms": circuit_ms_incl_norm,
        "expectation_ms": expect_ms,
        "energy": energy,
        "kernel_families": {f: {"launches": v["launches"] // args.steps,
                                "ms_per_step": v["ms"] / args.steps,
                                "gbps": v["bytes"] / (v["ms"] * 1e-3) / 1e9}
                            for f, v in fams.items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": None,
                     "bytes_per_launch": d["bytes"] / d["launches"],
                     "avg_launch_ms": d["ms"] / d["launches"]},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n, gates, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
