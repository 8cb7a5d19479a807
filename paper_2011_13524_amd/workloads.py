"""Seeded synthetic inputs: circuits, parameters and observables.

This module only draws random numbers and lists gates; it holds none of the
simulation arithmetic, so that both the GPU library and the CPU oracle can be
fed the same inputs without sharing any code that computes a result.

A circuit is a list of gate records (plain dicts):

  {"op": "rx"|"ry"|"rz", "q": [q], "angle": a}            fixed rotation
  {"op": "rx"|"ry"|"rz", "q": [q], "slot": s}             parametric rotation,
                                                          angle = theta[s]
  {"op": "h"|"x"|"y"|"z", "q": [q]}
  {"op": "cnot", "q": [control, target]}
  {"op": "cz", "q": [a, b]}
  {"op": "dense", "q": [t0, t1, ...], "mat": complex ndarray (2^k, 2^k),
   "controls": [...], "ctrl_vals": [...]}                 bit j of the matrix
                                                          index <-> q[j]

Rotations follow the paper's table of named gates: R_P(t) = exp(+i t P / 2).

An observable is a list of terms (coef, [(qubit, pauli_id), ...]) with
pauli ids 0..3 = I, X, Y, Z (section 4.3.2, Pauli gate) and real coefficients
(section 4.5).

Workloads (sizes are parameters so that tests can run small instances of the
same structure):
  layered_rx_rz_cnot  n-qubit layers of RX then RZ on every qubit and a CNOT
                      ladder (i -> i+1); 10 layers at n=10 (c128) and at n=30
                      (c64) are the two headline forward circuits.
  random_u_cz         layers of a Haar-random one-qubit unitary per qubit and
                      CZ on a random perfect matching of the qubits (n=26, 20
                      layers), modelled on the paper's random-circuit benchmark
                      (section 6.6).
  hea_ry_rz_cz        hardware-efficient ansatz: layers of parametric RY, RZ on
                      every qubit and a CZ ladder (batched VQE items).
  ry_rz_cnot_ring     layers of parametric RY, RZ on every qubit and a CNOT ring
                      (i -> i+1 mod n) (24-qubit adjoint workload).
  iqp_rz_cz           RZ layers and CZ brickwork only: every gate commutes
                      (section 6.6, circuits dominated by commuting gates).
"""
from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi


def rng_for(*key: int) -> np.random.Generator:
    """numpy PCG64 generator seeded by an integer key, e.g. (config, item)."""
    return np.random.default_rng(list(key))


def haar_unitary(rng: np.random.Generator, d: int) -> np.ndarray:
    """Haar-random d x d unitary: QR of a complex Ginibre matrix with the
    phases of R's diagonal folded into Q (Mezzadri 2007)."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diagonal(r) / np.abs(np.diagonal(r))
    return q * ph[None, :]


def layered_rx_rz_cnot(n: int, layers: int, seed_key=(0,)):
    """Each layer: RX(theta_q) then RZ(phi_q) on every qubit q (angles drawn
    qubit-major, uniform in [0, 2 pi)), then CNOT(i -> i+1) for i = 0..n-2."""
    rng = rng_for(*seed_key)
    gates = []
    for _ in range(layers):
        ang = rng.uniform(0.0, TWO_PI, size=(n, 2))
        for q in range(n):
            gates.append({"op": "rx", "q": [q], "angle": float(ang[q, 0])})
            gates.append({"op": "rz", "q": [q], "angle": float(ang[q, 1])})
        for i in range(n - 1):
            gates.append({"op": "cnot", "q": [i, i + 1]})
    return gates


def random_u_cz(n: int, layers: int, seed_key=(1,)):
    """Each layer: a Haar one-qubit unitary on every qubit, then CZ on the
    pairs (pi_{2j}, pi_{2j+1}) of a random permutation pi of the qubits."""
    rng = rng_for(*seed_key)
    gates = []
    for _ in range(layers):
        for q in range(n):
            gates.append({"op": "dense", "q": [q], "mat": haar_unitary(rng, 2),
                          "controls": [], "ctrl_vals": []})
        perm = rng.permutation(n)
        for j in range(n // 2):
            gates.append({"op": "cz", "q": [int(perm[2 * j]), int(perm[2 * j + 1])]})
    return gates


def iqp_rz_cz(n: int, depth: int, seed_key=(5,)):
    """Commuting (IQP-like) circuit: depth + 1 layers of RZ with uniform angles
    on every qubit, separated by depth brickwork layers of CZ(i, i+1) (even i
    in even layers, odd i in odd ones): the random circuit of section 6.6 with
    each qubit's three rotations replaced by one RZ, so that every gate is
    diagonal."""
    rng = rng_for(*seed_key)
    gates = []
    for layer in range(depth + 1):
        for q in range(n):
            gates.append({"op": "rz", "q": [q], "angle": float(rng.uniform(0.0, TWO_PI))})
        if layer == depth:
            break
        for q in range(layer % 2, n - 1, 2):
            gates.append({"op": "cz", "q": [q, q + 1]})
    return gates


def hea_ry_rz_cz(n: int, layers: int):
    """Hardware-efficient ansatz: per layer parametric RY then RZ on every
    qubit and CZ(i, i+1), i = 0..n-2. Parameter slots run 0..2*n*layers-1."""
    gates = []
    slot = 0
    for _ in range(layers):
        for q in range(n):
            gates.append({"op": "ry", "q": [q], "slot": slot})
            gates.append({"op": "rz", "q": [q], "slot": slot + 1})
            slot += 2
        for i in range(n - 1):
            gates.append({"op": "cz", "q": [i, i + 1]})
    return gates, slot


def ry_rz_cnot_ring(n: int, layers: int):
    """Per layer parametric RY then RZ on every qubit, then CNOT(i -> (i+1) mod n)
    applied in ascending i (the ring closes with CNOT(n-1 -> 0))."""
    gates = []
    slot = 0
    for _ in range(layers):
        for q in range(n):
            gates.append({"op": "ry", "q": [q], "slot": slot})
            gates.append({"op": "rz", "q": [q], "slot": slot + 1})
            slot += 2
        for i in range(n):
            gates.append({"op": "cnot", "q": [i, (i + 1) % n]})
    return gates, slot


def uniform_angles(count: int, seed_key) -> np.ndarray:
    return rng_for(*seed_key).uniform(0.0, TWO_PI, size=count)


def random_pauli_observable(n: int, terms: int, weight, seed_key):
    """`terms` random Pauli strings. weight: an int (fixed weight) or a tuple
    (lo, hi) for a weight uniform in lo..hi. Qubits distinct and uniform,
    letters uniform over {X, Y, Z}, coefficients N(0, 1)."""
    rng = rng_for(*seed_key)
    obs = []
    for _ in range(terms):
        w = weight if isinstance(weight, int) else int(rng.integers(weight[0], weight[1] + 1))
        qs = rng.choice(n, size=w, replace=False)
        ps = rng.integers(1, 4, size=w)
        coef = float(rng.standard_normal())
        obs.append((coef, [(int(q), int(p)) for q, p in zip(qs, ps)]))
    return obs


def tfim_chain(n: int, hx: float = 0.7):
    """H = sum_{i<n-1} Z_i Z_{i+1} + hx * sum_i X_i (open chain)."""
    obs = [(1.0, [(i, 3), (i + 1, 3)]) for i in range(n - 1)]
    obs += [(hx, [(i, 1)]) for i in range(n)]
    return obs


def batch_items(count: int, qubit_choices=(12, 14, 16, 18), layers: int = 8, seed: int = 3):
    """Batched-VQE items: qubit count uniform over qubit_choices, HEA circuit,
    angles uniform in [0, 2 pi), TFIM-chain Hamiltonian."""
    items = []
    for it in range(count):
        rng = rng_for(seed, it)
        n = int(rng.choice(np.asarray(qubit_choices)))
        gates, npar = hea_ry_rz_cz(n, layers)
        theta = rng.uniform(0.0, TWO_PI, size=npar)
        items.append({"n": n, "gates": gates, "theta": theta, "obs": tfim_chain(n)})
    return items


def gate_count(gates) -> int:
    return len(gates)
