#!/usr/bin/env python3
"""Benchmark of the state-vector hot path on one MI355X.

Headline workload (one "step"): a 30-qubit complex64 state is reset to
|0...0>, a 10-layer circuit of RX(theta) then RZ(phi) on every qubit followed
by a CNOT ladder (i -> i+1) is applied (890 gates, fused into tile passes),
and <H> is evaluated for H = 200 random weight-4 Pauli strings with N(0, 1)
coefficients, accumulated in FP64. Inputs are seeded and synthetic.

value = circuit gates per second over whole steps (expectation included).
`roofline` reports the kernel family that takes the most time in the timed
steps, timed with HIP events the library records on the stream its kernels run
on, against the 8 TB/s HBM peak. `cpu_baseline` times the CPU oracle on a
bounded sample of the same circuit (its first gates, complex128).

Extra legs (same JSON line):
  adjoint_24q   24 qubits, 20 layers RY/RZ + CNOT ring (960 parameters),
                500-term observable: adjoint gradient vs central finite
                differences on the same kernels (FD timed on a sample of
                parameters; both reported as gradient components per second)
  batch_vqe     512 hardware-efficient-ansatz items of 12..18 qubits: one
                persistent launch (graph replay, launch shape autotuned
                beforehand) vs one adjoint call per item
  random_26q    26-qubit Haar-1q + random-CZ circuit, fused vs unfused, and
                the plan the autotuner picks (fusion width, tile shape)
  adjoint_32q   32-qubit complex64 forward + adjoint pass (1920 gates, 1280
                parameters), one gradient component checked by the shift rule
  autotune_30q  the headline circuit's plan picked by the autotuner vs the
                default plan
  pauli_30q     multi-qubit Pauli rotations and transition amplitudes at 30
                qubits (GB/s of the state sweeps)
  sample_30q    marginal probabilities and Z-basis sampling at 30 qubits
  precision_30q_c128
                the headline step in complex128, and the complex64 energy and
                amplitudes' error against it
  small_10q     the 10-qubit complex128 layered circuit: microseconds per
                circuit (fused, unfused), state and <Z_0> against the oracle
  iqp_30q       a commuting RZ + CZ circuit at 30 qubits: light vs heavy
                (commutation-aware) planning, planning time included

Every leg states its results' error: against the CPU oracle where it runs in
seconds (10 and 26 qubits, sampled batch items), else against the complex128
GPU path (30-qubit headline, 24-qubit gradients), itself oracle-pinned in the
tests.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode fused|unfused]
                       [--quick] [--no-cpu] [--leg NAME]
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
FAMILIES = ("pair", "scale", "diag", "dense", "expect", "tile", "apply_obs", "adjoint", "batch")


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
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--fd-params", type=int, default=6)
    ap.add_argument("--batch-items", type=int, default=512)
    ap.add_argument("--leg", choices=["adjoint_24q", "batch_vqe", "random_26q", "adjoint_32q",
                                      "autotune_30q", "pauli_30q", "sample_30q", "small_10q",
                                      "iqp_30q"],
                    help="run only this extra leg and print its JSON (for profiling)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also copy the state once (a device copy of known size, used to "
                         "calibrate rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def traffic_from_profile(kernel_prefix):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when the kernel sources changed since it was taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "traffic_30q_c64_headline.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    h = hashlib.sha256()
    for name in rec.get("sources", []):
        h.update(open(os.path.join(ROOT, name), "rb").read())
    if h.hexdigest() != rec.get("sources_sha256") or not rec.get("kernel", "").startswith(kernel_prefix):
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def sync(Q, state):
    state.sync()  # the stream every kernel of the step runs on


def read_families(Q, steps):
    fams = {}
    for fam in FAMILIES:
        cnt, ms, by = Q.prof_read(fam)
        if cnt:
            fams[fam] = {"launches": cnt, "ms": ms, "bytes": by}
    return fams


def state_diff(a, b, chunk=1 << 24):
    """max |a - b| and ||a - b|| / ||b|| of two host complex128 vectors (chunked)."""
    mx, num, den = 0.0, 0.0, 0.0
    for i in range(0, a.size, chunk):
        d = a[i:i + chunk] - b[i:i + chunk]
        mx = max(mx, float(np.max(np.abs(d))))
        num += float(np.vdot(d, d).real)
        den += float(np.vdot(b[i:i + chunk], b[i:i + chunk]).real)
    return mx, (num / den) ** 0.5 if den > 0 else float("nan")


def companion_c128(Q, n, circ, obs, obs_terms, state64, e64, steps=3):
    """The headline step in complex128 on the GPU (the paper's precision), and
    the complex64 result's error against it: energy and amplitudes."""
    plan = Q.Plan(circ, "c128", max_k=2)
    s = Q.State(n, "c128")

    def step():
        s.set_basis(0)
        Q.apply_fused(s, plan)
        return Q.expectation(s, obs)

    step()
    sync(Q, s)
    t0 = time.perf_counter()
    for _ in range(steps):
        e = step()
    sync(Q, s)
    dt = (time.perf_counter() - t0) / steps
    ngates = circ.info()[1]
    a64 = state64.store()  # upcast to complex128 on the host
    a128 = s.store()
    mx, rel = state_diff(a64, a128)
    del a64, a128, s
    scale = sum(abs(c) for c, _ in obs_terms)
    return {"workload": "the headline circuit and observable in complex128 (FP64 amplitudes)",
            "ms_per_step": dt * 1e3, "gates_per_s": ngates / dt, "energy": e,
            "reference": "complex128 GPU path: oracle-pinned to 1e-12 (amplitudes up to 16 "
                         "qubits, expectations of 24-qubit states); the 30-qubit oracle needs "
                         "minutes per gate",
            "c64_abs_energy_error": abs(e64 - e),
            "c64_energy_error_over_sum_abs_alpha": abs(e64 - e) / scale,
            "c64_amp_max_abs_error": mx, "c64_amp_rel_l2_error": rel,
            "bars": {"amp_max_abs": 1e-5, "energy_over_sum_abs_alpha": 2e-5}}


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
    out = {"value": done / dt, "unit": "gates/s", "cores": threads, "kind": "oracle",
           "sample": f"first {done} of {len(gates)} gates of the {n}-qubit circuit, complex128, "
                     f"{dt:.1f} s"}
    # the same oracle on one thread (a bounded sample: the first gates)
    lib.orc_set_num_threads(1)
    done1 = 0
    t0 = time.perf_counter()
    for g in gates:
        O.apply_gate(psi, g)
        done1 += 1
        if time.perf_counter() - t0 > budget_s / 3 and done1 >= 1:
            break
    dt1 = time.perf_counter() - t0
    lib.orc_set_num_threads(threads)
    del psi
    out["one_thread"] = {"value": done1 / dt1, "unit": "gates/s", "cores": 1,
                         "sample": f"next {done1} gates of the same circuit, {dt1:.1f} s"}
    return out


def adjoint_leg(Q, W, fd_params):
    n = 24
    gates, npar = W.ry_rz_cnot_ring(n, 20)
    theta = W.uniform_angles(npar, (4, 0))
    obs_t = W.random_pauli_observable(n, 500, (1, 6), seed_key=(4, 1))
    circ = Q.Circuit.from_records(n, gates)
    obs = Q.Observable(n, obs_t)
    out = {"workload": "24 qubits, 20 layers RY/RZ + CNOT ring (1440 gates, 960 parameters), "
                       "500 random Pauli strings of weight 1..6", "params": npar}
    grads = {}
    for dt in ("c64", "c128"):
        plan = Q.Plan(circ, dt, max_k=2)
        psi, lam, s = Q.State(n, dt), Q.State(n, dt), Q.State(n, dt)
        Q.adjoint_gradient(circ, theta, obs, psi, lam, plan)  # warm-up
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            e, g = Q.adjoint_gradient(circ, theta, obs, psi, lam, plan)
        t_adj = (time.perf_counter() - t0) / reps

        def energy(th):
            s.set_basis(0)
            Q.apply_fused(s, plan, th)
            return Q.expectation(s, obs)

        energy(theta)
        h = 1e-6 if dt == "c128" else 4e-3
        slots = list(range(0, npar, max(1, npar // fd_params)))[:fd_params]
        t0 = time.perf_counter()
        fd = []
        for sl in slots:
            tp, tm = theta.copy(), theta.copy()
            tp[sl] += h
            tm[sl] -= h
            fd.append((energy(tp) - energy(tm)) / (2 * h))
        t_fd = (time.perf_counter() - t0) / len(slots)  # seconds per gradient component
        scale = sum(abs(c) for c, _ in obs_t)
        grads[dt] = (e, g)
        out[dt] = {"adjoint_s": t_adj, "grads_per_s": npar / t_adj,
                   "fd_grads_per_s": 1.0 / t_fd, "fd_sample_params": len(slots), "fd_h": h,
                   "speedup_vs_fd": (npar / t_adj) * t_fd,
                   "max_abs_adjoint_minus_fd_over_sum_abs_alpha":
                       float(np.max(np.abs(g[slots] - np.array(fd))) / scale),
                   "energy": e}
    # complex64 against the complex128 path (oracle-pinned at small sizes and,
    # for expectations, at 24 qubits); the 24-qubit oracle forward alone takes
    # seconds per gate, so the full gradient is not re-derived on the CPU here
    scale = sum(abs(c) for c, _ in obs_t)
    (e64, g64), (e128, g128) = grads["c64"], grads["c128"]
    out["c64_vs_c128"] = {"energy_error_over_sum_abs_alpha": abs(e64 - e128) / scale,
                          "grad_max_abs_error_over_sum_abs_alpha":
                              float(np.max(np.abs(g64 - g128))) / scale,
                          "bar_over_sum_abs_alpha": 2e-5}
    return out


def adjoint32_leg(Q, W):
    """32-qubit complex64 forward circuit and adjoint pass: psi, lambda and a
    third state (for a sampled shift-rule check) resident in HBM."""
    n = 32
    gates, npar = W.ry_rz_cnot_ring(n, 20)
    theta = W.uniform_angles(npar, (4, 2))
    obs_t = W.random_pauli_observable(n, 500, (1, 6), seed_key=(4, 3))
    circ = Q.Circuit.from_records(n, gates)
    obs = Q.Observable(n, obs_t)
    dt = "c64"
    plan = Q.Plan(circ, dt, max_k=2)
    psi, lam = Q.State(n, dt), Q.State(n, dt)
    t0 = time.perf_counter()
    psi.set_basis(0)
    Q.apply_fused(psi, plan, theta)
    sync(Q, psi)
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    e, g = Q.adjoint_gradient(circ, theta, obs, psi, lam, plan)
    t_adj = time.perf_counter() - t0
    s = Q.State(n, dt)

    def energy(th):
        s.set_basis(0)
        Q.apply_fused(s, plan, th)
        return Q.expectation(s, obs)

    slot = npar // 2
    tp, tm = theta.copy(), theta.copy()
    tp[slot] += np.pi / 2
    tm[slot] -= np.pi / 2
    shift = 0.5 * (energy(tp) - energy(tm))
    scale = sum(abs(c) for c, _ in obs_t)
    del s, psi, lam
    return {"workload": f"32 qubits complex64, 20 layers RY/RZ + CNOT ring ({len(gates)} gates, "
                        f"{npar} parameters), 500 random Pauli strings of weight 1..6; psi, lambda "
                        "and a check state (3 x 34.4 GB) in HBM",
            "forward_s": t_fwd, "forward_gates_per_s": len(gates) / t_fwd,
            "adjoint_s": t_adj, "grads_per_s": npar / t_adj, "energy": e,
            "shift_rule_check_slot": slot,
            "abs_adjoint_minus_shift_over_sum_abs_alpha": abs(g[slot] - shift) / scale,
            "passes": plan.info()["passes"]}


def batch_leg(Q, W, count):
    items = W.batch_items(count, seed=3)
    out = {"workload": f"{count} items, HEA 8 layers RY,RZ + CZ ladder, n uniform over "
                       "{12,14,16,18}, H = sum Z_i Z_i+1 + 0.7 sum X_i",
           "items": count, "params_total": int(sum(len(it["theta"]) for it in items))}
    b = Q.Batch()
    circs = []
    for it in items:
        c = Q.Circuit.from_records(it["n"], it["gates"])
        o = Q.Observable(it["n"], it["obs"])
        circs.append((c, o))
        b.add(c, o, it["theta"])
    # oracle references for sampled items (one per qubit count): energy and 4
    # gradient components by the exact two-term shift rule
    from oracle import oracle as O
    oracle_refs = {}
    for nq in sorted({it["n"] for it in items}):
        i = next(k for k, it in enumerate(items) if it["n"] == nq)
        it = items[i]
        npi = len(it["theta"])
        slots = [0, npi // 3, (2 * npi) // 3, npi - 1]
        oracle_refs[i] = (O.energy(nq, it["gates"], it["theta"], it["obs"]), slots,
                          O.param_shift_grad(nq, it["gates"], it["theta"], it["obs"], slots=slots),
                          sum(abs(c) for c, _ in it["obs"]))
    for dt in ("c64", "c128"):
        shape = b.autotune(dt, reps=1)  # launch shape by measurement (outside the timed runs)
        b.run(dt)  # builds device tables, captures the launch graph
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            e, g = b.run(dt)
        t_b = (time.perf_counter() - t0) / reps
        # plain per-circuit baseline: one adjoint call per item (per-gate launches), sampled
        sample = list(range(0, count, max(1, count // 32)))
        states = {}
        t_pc = 0.0
        for i in sample:
            n = items[i]["n"]
            if n not in states:
                states[n] = (Q.State(n, dt), Q.State(n, dt))
            psi, lam = states[n]
            c, o = circs[i]
            Q.adjoint_gradient(c, items[i]["theta"], o, psi, lam)
            t0 = time.perf_counter()
            e1, g1 = Q.adjoint_gradient(c, items[i]["theta"], o, psi, lam)
            t_pc += time.perf_counter() - t0
        per_item = t_pc / len(sample)
        # finite differences on the same kernels (fused forward + expectation per
        # energy), timed on a sample of parameters of the sampled items
        h = 1e-6 if dt == "c128" else 4e-3
        fd_t, fd_n = 0.0, 0
        for i in sample[:8]:
            n = items[i]["n"]
            c, o = circs[i]
            pl = Q.Plan(c, dt, max_k=2)
            s1 = states[n][0] if n in states else Q.State(n, dt)
            th = items[i]["theta"]
            for sl in (0, len(th) // 2):
                t0 = time.perf_counter()
                tp, tm = th.copy(), th.copy()
                tp[sl] += h
                tm[sl] -= h
                s1.set_basis(0)
                Q.apply_fused(s1, pl, tp)
                ep = Q.expectation(s1, o)
                s1.set_basis(0)
                Q.apply_fused(s1, pl, tm)
                em = Q.expectation(s1, o)
                fd_t += time.perf_counter() - t0
                fd_n += 1
        fd_grads_per_s = fd_n / fd_t
        # error against the oracle on sampled items (one per qubit count): energy
        # and 4 gradient components by the exact two-term shift rule
        e_err, g_err, checked = 0.0, 0.0, []
        for i, (e_ref, slots, g_ref, scale) in oracle_refs.items():
            e_err = max(e_err, abs(e[i] - e_ref) / scale)
            g_err = max(g_err, float(np.max(np.abs(g[i][slots] - g_ref))) / scale)
            checked.append(i)
        out[dt] = {"batch_s": t_b, "items_per_s": count / t_b, "launch_shape": shape,
                   "grads_per_s": out["params_total"] / t_b,
                   "per_circuit_items_per_s": 1.0 / per_item,
                   "speedup_vs_per_circuit": (count / t_b) * per_item,
                   "fd_grads_per_s": fd_grads_per_s, "fd_h": h,
                   "speedup_vs_fd": (out["params_total"] / t_b) / fd_grads_per_s,
                   "oracle_check": {"items": checked, "gradient_slots_per_item": 4,
                                    "energy_error_over_sum_abs_alpha": e_err,
                                    "grad_max_abs_error_over_sum_abs_alpha": g_err,
                                    "bar_over_sum_abs_alpha": 1e-10 if dt == "c128" else 2e-5}}
    return out


def random_leg(Q, W, check=True):
    n = 26
    gates = W.random_u_cz(n, 20, seed_key=(1,))
    circ = Q.Circuit.from_records(n, gates)
    out = {"workload": "26 qubits, 20 layers of Haar 1q on every qubit + CZ on a random "
                       "perfect matching (780 gates)"}
    ref = None
    if check:
        # one complex128 oracle run (1 GiB), all host threads
        from oracle import oracle as O
        t0 = time.perf_counter()
        ref = O.run_circuit(n, gates)
        out["oracle"] = {"s": time.perf_counter() - t0, "threads": int(O.lib().orc_num_threads())}
    for dt in ("c64", "c128"):
        s = Q.State(n, dt)
        plan = Q.Plan(circ, dt, max_k=2)
        t0 = time.perf_counter()
        tuned = Q.Plan.autotune(circ, s, reps=1)  # fusion width and tile shape by measurement
        t_tune = time.perf_counter() - t0
        r = {}
        for mode, pl in (("unfused", None), ("fused", plan), ("fused_autotuned", tuned)):
            f = (lambda: Q.apply_circuit(s, circ)) if pl is None else (lambda: Q.apply_fused(s, pl))
            f()
            sync(Q, s)
            t0 = time.perf_counter()
            f()
            sync(Q, s)
            t = time.perf_counter() - t0
            r[mode] = {"s": t, "gates_per_s": len(gates) / t,
                       "hbm_gb_per_s_algorithmic":
                           (2 * (1 << n) * (8 if dt == "c64" else 16) *
                            (pl.info()["passes"] if pl is not None else 0)) / t / 1e9
                           if pl is not None else None}
            if ref is not None:
                s.set_basis(0)
                f()
                mx, rel = state_diff(s.store(), ref)
                r[mode]["max_abs_error_vs_oracle"] = mx
                r[mode]["rel_l2_error_vs_oracle"] = rel
        r["passes"] = plan.info()["passes"]
        r["autotune"] = {"choice": tuned.choice, "passes": tuned.info()["passes"], "tuning_s": t_tune}
        out[dt] = r
    return out


def iqp_leg(Q, W, n=30, depth=20):
    """Commuting circuit (section 6.6: the random circuit with one RZ per qubit
    per layer, CZ brickwork): light vs heavy (commutation-aware) planning,
    complex64, with and without the planning time."""
    gates = W.iqp_rz_cz(n, depth, seed_key=(5,))
    circ = Q.Circuit.from_records(n, gates)
    s = Q.State(n, "c64")
    out = {"workload": f"{n} qubits complex64, {depth + 1} RZ layers on every qubit and {depth} "
                       f"CZ brickwork layers ({len(gates)} gates, all diagonal)"}
    for name, heavy in (("light", False), ("heavy", True)):
        t0 = time.perf_counter()
        pl = Q.Plan(circ, "c64", max_k=2, heavy=heavy)
        t_plan = time.perf_counter() - t0
        s.set_basis(0)
        Q.apply_fused(s, pl)
        sync(Q, s)
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            Q.apply_fused(s, pl)
        sync(Q, s)
        t = (time.perf_counter() - t0) / reps
        info = pl.info()
        out[name] = {"plan_ms": t_plan * 1e3, "blocks": info["blocks"], "passes": info["passes"],
                     "apply_ms": t * 1e3, "gates_per_s": len(gates) / t,
                     "gates_per_s_incl_plan": len(gates) / (t + t_plan),
                     "hbm_gb_per_s_algorithmic": 2 * (1 << n) * 8 * info["passes"] / t / 1e9}
    s.set_basis(0)
    Q.apply_fused(s, Q.Plan(circ, "c64", max_k=2, heavy=True))
    a = s.store()
    s.set_basis(0)
    Q.apply_fused(s, Q.Plan(circ, "c64", max_k=2))
    mx, rel = state_diff(a, s.store())
    out["heavy_vs_light_max_abs"] = mx
    out["heavy_vs_light_rel_l2"] = rel
    return out


def pauli_leg(Q, W, n=30):
    """Multi-qubit Pauli rotations and transition amplitudes at 30 qubits (complex64)."""
    rng = np.random.default_rng(91)
    s = Q.State(n, "c64")
    s.set_basis(0)
    N, S = 1 << n, 8
    out = {"workload": f"{n}-qubit complex64: exp(i t P/2) for random weight-4 strings (with X/Y) "
                       "and a weight-4 Z string; <a|O|b> for 8 random weight-4 strings"}
    rows = []
    for kind in ("xy", "xy", "z"):
        qs = [int(q) for q in rng.choice(n, size=4, replace=False)]
        ps = [int(p) for p in (rng.integers(1, 4, size=4) if kind == "xy" else [3] * 4)]
        if kind == "xy" and all(p == 3 for p in ps):
            ps[0] = 1
        Q.apply_pauli_rotation(s, qs, ps, 0.3)
        sync(Q, s)
        t0 = time.perf_counter()
        for _ in range(3):
            Q.apply_pauli_rotation(s, qs, ps, 0.3)
        sync(Q, s)
        t = (time.perf_counter() - t0) / 3
        rows.append({"qubits": qs, "paulis": ps, "ms": t * 1e3, "gbps": 2 * N * S / t / 1e9})
    out["rotations"] = rows
    other = Q.State(n, "c64")
    other.set_basis(3)
    obs = Q.Observable(n, W.random_pauli_observable(n, 8, 4, seed_key=(9, 1)))
    Q.transition_amplitude(s, obs, other)
    t0 = time.perf_counter()
    Q.transition_amplitude(s, obs, other)
    t = time.perf_counter() - t0
    out["transition"] = {"terms": 8, "ms": t * 1e3, "gbps": 8 * 2 * N * S / t / 1e9}
    return out


def sample_leg(Q, W, n=30, count=1 << 20):
    """Marginal probabilities and Z-basis sampling at 30 qubits (complex64)."""
    rng = np.random.default_rng(93)
    s = Q.State(n, "c64")
    s.set_basis(0)
    for q in range(n):
        s.apply_named("ry", [q], float(rng.uniform(0.2, 2.9)))
        s.apply_named("rz", [q], float(rng.uniform(-3.0, 3.0)))
    N, S = 1 << n, 8
    out = {"workload": f"{n}-qubit complex64 product state from RY/RZ on every qubit; marginals "
                       f"with 0 and 3 measured qubits; {count} samples from seeded uniforms"}
    for m in (0, 3):
        vals = [2] * n
        for q in range(m):
            vals[q] = q & 1
        s.marginal_probability(vals)
        t0 = time.perf_counter()
        prob = s.marginal_probability(vals)
        t = time.perf_counter() - t0
        out[f"marginal_{m}"] = {"prob": prob, "ms": t * 1e3, "gbps": (N >> m) * S / t / 1e9}
    u = rng.uniform(size=count)
    s.sample(u[:16])
    t0 = time.perf_counter()
    got = s.sample(u)
    t = time.perf_counter() - t0
    # the table build reads every amplitude once and writes one FP64 per amplitude
    out["sample"] = {"count": count, "ms": t * 1e3, "samples_per_s": count / t,
                     "table_gbps_lower_bound": N * (S + 8) / t / 1e9,
                     "distinct": int(np.unique(got).size)}
    return out


def small_leg(Q, W, reps=200):
    """The 10-qubit complex128 layered circuit (290 gates): time per circuit
    (state reset + circuit, one fused pass) against the paper's ~10 us per GPU
    call, and the unfused per-gate launches; state and <Z_0> against the oracle."""
    from oracle import oracle as O
    n = 10
    gates = W.layered_rx_rz_cnot(n, 10, seed_key=(0,))
    circ = Q.Circuit.from_records(n, gates)
    plan = Q.Plan(circ, "c128", max_k=2)
    s = Q.State(n, "c128")
    out = {"workload": "10 qubits complex128, 10 layers RX/RZ on every qubit + CNOT ladder "
                       f"({len(gates)} gates), from |0..0>", "passes": plan.info()["passes"]}
    for mode, f, r in (("fused", lambda: Q.apply_fused(s, plan), reps),
                       ("unfused", lambda: Q.apply_circuit(s, circ), max(1, reps // 10))):
        s.set_basis(0)
        f()
        sync(Q, s)
        t0 = time.perf_counter()
        for _ in range(r):
            s.set_basis(0)
            f()
        sync(Q, s)
        t = (time.perf_counter() - t0) / r
        out[mode] = {"us_per_circuit": t * 1e6, "gates_per_s": len(gates) / t}
    s.set_basis(0)
    Q.apply_fused(s, plan)
    ref = O.run_circuit(n, gates)
    z0 = [(1.0, [(0, 3)])]
    out["max_abs_error_vs_oracle"] = float(np.max(np.abs(s.store() - ref)))
    out["z0"] = Q.expectation(s, Q.Observable(n, z0))
    out["z0_error_vs_oracle"] = abs(out["z0"] - O.expectation(ref, z0))
    out["bar"] = 1e-12
    return out


def autotune_leg(Q, W, n=30):
    """The headline circuit's plan picked by the autotuner vs the default plan."""
    gates = W.layered_rx_rz_cnot(n, 10, seed_key=(2,))
    circ = Q.Circuit.from_records(n, gates)
    s = Q.State(n, "c64")
    t0 = time.perf_counter()
    tuned = Q.Plan.autotune(circ, s, reps=1)
    out = {"tuning_s": time.perf_counter() - t0, "choice": tuned.choice}
    for name, pl in (("default", Q.Plan(circ, "c64", max_k=2)), ("autotuned", tuned)):
        Q.apply_fused(s, pl)
        sync(Q, s)
        t0 = time.perf_counter()
        Q.apply_fused(s, pl)
        sync(Q, s)
        out[name + "_ms"] = (time.perf_counter() - t0) * 1e3
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the state-vector path runs on one GPU; sharding across GPUs "
                                   "is described, not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import paper_2011_13524_amd as Q
    from paper_2011_13524_amd import workloads as W

    if args.leg:
        legs = {"adjoint_24q": lambda: adjoint_leg(Q, W, args.fd_params),
                "batch_vqe": lambda: batch_leg(Q, W, args.batch_items),
                "random_26q": lambda: random_leg(Q, W), "adjoint_32q": lambda: adjoint32_leg(Q, W),
                "autotune_30q": lambda: autotune_leg(Q, W), "pauli_30q": lambda: pauli_leg(Q, W),
                "sample_30q": lambda: sample_leg(Q, W), "small_10q": lambda: small_leg(Q, W),
                "iqp_30q": lambda: iqp_leg(Q, W)}
        print(json.dumps({args.leg: legs[args.leg]()}), flush=True)
        return

    n = args.n
    dt = "c64"
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
    sync(Q, state)
    t0 = time.perf_counter()
    run_circuit()
    sync(Q, state)
    t1 = time.perf_counter()
    Q.expectation(state, obs)
    t2 = time.perf_counter()

    # timed region
    Q.prof_enable(True)
    sync(Q, state)
    t_start = time.perf_counter()
    energy = None
    for _ in range(args.steps):
        energy = step()
    sync(Q, state)
    t_end = time.perf_counter()
    Q.prof_enable(False)
    total = t_end - t_start
    ms_per_step = total * 1e3 / args.steps

    fams = read_families(Q, args.steps)
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
        "circuit_ms": (t1 - t0) * 1e3,
        "expectation_ms": (t2 - t1) * 1e3,
        "energy": energy,
        "kernel_families": {f: {"launches": v["launches"] // args.steps,
                                "ms_per_step": v["ms"] / args.steps,
                                "gbps": v["bytes"] / (v["ms"] * 1e-3) / 1e9}
                            for f, v in fams.items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": traffic_from_profile("qsv::k_tile_reg") if dom == "tile" else None,
                     "bytes_per_launch": d["bytes"] / d["launches"],
                     "avg_launch_ms": d["ms"] / d["launches"]},
    }
    if args.calib_copy:
        other = Q.State(n, dt)
        other.copy_from(state)  # device-to-device copy of 2^n x 8 bytes
        other.norm2()
        del other
    if not args.quick:
        out["precision_30q_c128"] = companion_c128(Q, n, circ, obs, obs_terms, state, energy)
    del state
    if not args.quick:
        out["small_10q"] = small_leg(Q, W)
        out["adjoint_24q"] = adjoint_leg(Q, W, args.fd_params)
        out["batch_vqe"] = batch_leg(Q, W, args.batch_items)
        out["random_26q"] = random_leg(Q, W)
        out["adjoint_32q"] = adjoint32_leg(Q, W)
        out["autotune_30q"] = autotune_leg(Q, W)
        out["pauli_30q"] = pauli_leg(Q, W)
        out["iqp_30q"] = iqp_leg(Q, W)
        out["sample_30q"] = sample_leg(Q, W)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n, gates, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
