"""CPU-only checks of the C ABI: the library loads and exports every symbol
include/qsv.h declares, and every host-side validation path returns the
documented error code without touching a device (no compute is launched).
"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2011_13524_amd as Q
from paper_2011_13524_amd import binding as B
from paper_2011_13524_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qsv.h")

EINVAL, ERANGE, EDUP, ENOMEM, EHIP, EDTYPE, ENODEV = -1, -2, -3, -4, -5, -6, -7


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(qsv_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported_and_bound():
    L = Q.lib()
    names = declared()
    assert len(names) >= 30
    for name in names:
        assert hasattr(L, name), name
        assert name in B.declared_symbols(), name


def test_version_and_last_error():
    L = Q.lib()
    assert L.qsv_version() >= 100
    h = ctypes.c_void_p()
    assert L.qsv_circuit_create(0, ctypes.byref(h)) == ERANGE
    assert b"qubit count" in L.qsv_last_error()


def _code(fn, *a):
    with pytest.raises(Q.QsvError) as ei:
        fn(*a)
    return ei.value.code


def test_circuit_validation():
    c = Q.Circuit(4)
    assert _code(c.add_record, {"op": "dense", "q": [4], "mat": np.eye(2)}) == ERANGE
    assert _code(c.add_record, {"op": "dense", "q": [1, 1], "mat": np.eye(4)}) == EDUP
    assert _code(c.add_record, {"op": "dense", "q": [0], "mat": np.eye(2), "controls": [0],
                                "ctrl_vals": [1]}) == EDUP
    assert _code(c.add_record, {"op": "dense", "q": [0], "mat": np.eye(2), "controls": [1],
                                "ctrl_vals": [2]}) == EINVAL
    assert _code(c.add_record, {"op": "cnot", "q": [3, 3]}) == EDUP
    L = Q.lib()
    assert L.qsv_circuit_add_rotation(c.h, 4, 0, 0) == EINVAL
    assert L.qsv_circuit_add_rotation(c.h, 1, 9, 0) == ERANGE
    assert L.qsv_circuit_add_rotation(c.h, 1, 0, -1) == ERANGE
    m = np.eye(64, dtype=np.complex128)
    t = np.arange(6, dtype=np.int32)
    assert L.qsv_circuit_add_gate(c.h, m.ctypes.data_as(B._dp), t.ctypes.data_as(B._ip), 6, None,
                                  None, 0) == EINVAL
    assert c.info() == (4, 0, 0)


def test_observable_validation():
    o = Q.Observable(3)
    assert _code(o.add_term, 1.0, [(3, 1)]) == ERANGE
    assert _code(o.add_term, 1.0, [(0, 4)]) == EINVAL
    assert _code(o.add_term, 1.0, [(1, 1), (1, 3)]) == EDUP
    o.add_term(0.5, [(0, 1), (1, 2)])
    o.add_term(0.5, [(0, 1), (1, 1), (2, 3)])
    o.add_term(0.1, [])
    # X0Y1 and X0X1Z2 share the flip mask {0, 1}; the identity has flip mask 0
    assert o.info() == (3, 3, 2)


def test_state_without_device():
    L = Q.lib()
    h = ctypes.c_void_p()
    rc = L.qsv_state_alloc(4, 1, None, ctypes.byref(h))
    assert rc in (ENODEV, 0)
    if rc == 0:  # a device is present: nothing more to check here
        L.qsv_state_free(h)
        return
    assert L.qsv_state_alloc(0, 1, None, ctypes.byref(h)) == ERANGE
    assert L.qsv_state_alloc(35, 1, None, ctypes.byref(h)) == ERANGE  # 2^35 amplitudes: beyond 34
    assert L.qsv_state_alloc(4, 7, None, ctypes.byref(h)) == EDTYPE


def test_validation_before_any_launch_on_wrapped_memory():
    # a wrapped host buffer is never touched: each call fails validation first
    L = Q.lib()
    buf = np.zeros(32 + 4, dtype=np.float64)
    addr = (buf.ctypes.data + 15) // 16 * 16
    h = ctypes.c_void_p()
    assert L.qsv_state_wrap(ctypes.c_void_p(addr), 4, 2, None, ctypes.byref(h)) == 0
    s = Q.State(4, "c128", _handle=h)
    assert _code(s.apply_gate, np.eye(2), [4]) == ERANGE
    assert _code(s.apply_gate, np.eye(4), [2, 2]) == EDUP
    assert _code(s.apply_gate, np.eye(2), [0], [1], [3]) == EINVAL
    assert L.qsv_apply_gate(s.h, np.eye(2).ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            (ctypes.c_int * 11)(*range(11)), 11, None, None, 0) == EINVAL
    assert _code(s.apply_named, "cnot", [1]) == EINVAL
    assert _code(s.set_basis, 16) == ERANGE
    h2 = ctypes.c_void_p()
    assert L.qsv_state_wrap(ctypes.c_void_p(addr + 8), 4, 2, None, ctypes.byref(h2)) == EINVAL
    assert h2.value is None
    c = Q.Circuit(5)
    assert L.qsv_apply_circuit(s.h, c.h, None) == ERANGE
    o = Q.Observable(5)
    out = ctypes.c_double()
    assert L.qsv_expectation(s.h, o.h, ctypes.byref(out)) == ERANGE
    assert _code(s.marginal_probability, [0, 1, 3, 2]) == EINVAL
    assert _code(s.sample, [0.5, 1.0]) == ERANGE
    assert _code(s.sample, [float("nan")]) == ERANGE
    assert _code(s.sample, [-0.25]) == ERANGE
    assert L.qsv_sample(s.h, None, -1, None) == EINVAL
    np.testing.assert_array_equal(buf, 0.0)


def test_planner_on_host():
    n = 30
    gates = W.layered_rx_rz_cnot(n, 10, seed_key=(2,))
    c = Q.Circuit.from_records(n, gates)
    info = Q.Plan(c, "c64", max_k=2).info()
    assert info["gates"] == 890
    # RX/RZ pairs merged per qubit (300 one-qubit blocks); the 290 ladder CNOTs
    # stay exchanges: a two-qubit dense block would cost more arithmetic
    assert info["blocks"] == 590
    assert info["passes"] <= 40
    small = Q.Circuit.from_records(10, W.layered_rx_rz_cnot(10, 10, seed_key=(0,)))
    assert Q.Plan(small, "c128", max_k=2).info()["passes"] == 1
    assert _code(Q.Plan, c, "c64", 0) == EINVAL
    assert _code(Q.Plan, c, "c128", 2, 14) == EINVAL
    assert _code(Q.Plan, c, "c64", 5, 8, 6) == EINVAL


def test_observable_pass_packing_on_host():
    # flip masks of the 200-term weight-4 observable on 30 qubits packed into
    # 2^12-amplitude tiles: far fewer passes than distinct masks
    o = Q.Observable(30, W.random_pauli_observable(30, 200, 4, seed_key=(2, 1)))
    n, terms, groups = o.info()
    assert (n, terms, groups) == (30, 200, 186)
    assert o.passes("c64") <= 21 and o.passes("c128") <= 22
    assert Q.Observable(4, [(1.0, [(0, 3)])]).passes("c64") == 1  # pure Z: one pass
    assert Q.Observable(4, []).passes("c64") == 0
    # masks that share qubits land in one pass: X on every pair of 8 high
    # qubits (28 masks) fits one 2^12 tile with the 4 low qubits
    pairs = [(1.0, [(a, 1), (b, 1)]) for a in range(20, 28) for b in range(a + 1, 28)]
    assert Q.Observable(30, pairs).passes("c64") == 1
    # a mask with more flip qubits than a tile holds (with the low ones) is
    # evaluated on its own: one more state read, and packing terminates
    wide = [(1.0, [(q, 1) for q in range(10, 22)])]
    assert Q.Observable(30, wide).passes("c64") == 1
    assert Q.Observable(30, wide + pairs).passes("c64") == 2
    assert Q.Observable(30, wide + pairs).passes("c128") == 2


def test_merge_never_raises_arithmetic():
    rng = np.random.default_rng(3)
    u1 = W.haar_unitary(rng, 2)
    u2 = W.haar_unitary(rng, 4)

    def blocks(recs, k=2):
        return Q.Plan(Q.Circuit.from_records(3, recs), "c128", max_k=k).info()["blocks"]

    U = {"op": "dense", "q": [0], "mat": u1}
    U1 = {"op": "dense", "q": [1], "mat": u1}
    U01 = {"op": "dense", "q": [0, 1], "mat": u2}
    cx = {"op": "cnot", "q": [0, 1]}
    cz = {"op": "cz", "q": [0, 1]}
    assert blocks([U, cx]) == 2          # an exchange never widens a dense block
    assert blocks([U01, cx]) == 1        # ... but is absorbed by one covering it
    assert blocks([cx, U01]) == 1        # a dense gate absorbs an exchange it covers
    assert blocks([cx, U]) == 2
    assert blocks([cz, cx]) == 2         # diagonal x exchange would be dense
    assert blocks([cx, cx]) == 2
    assert blocks([cz, {"op": "rz", "q": [1], "slot": 0}]) == 1  # diagonal products stay diagonal
    assert blocks([{"op": "rz", "q": [0], "slot": 0}, {"op": "rx", "q": [0], "slot": 1}]) == 1
    assert blocks([U, U1]) == 2          # no shared qubit: independent blocks
    assert blocks([U, U01]) == 1
    assert blocks([U, U01], k=1) == 2


X_, Y_, Z_ = 1, 2, 4


def test_commute_metadata():
    # per-qubit commuting Paulis (section 5.4): pinned by the algebra of each
    # gate (a controlled gate is diagonal on its control; X-type targets
    # commute with X; H and SWAP with none of X, Y, Z on a single qubit)
    rng = np.random.default_rng(8)
    u = W.haar_unitary(rng, 2)
    recs = [{"op": "cnot", "q": [0, 1]}, {"op": "cz", "q": [1, 2]}, {"op": "h", "q": [0]},
            {"op": "swap", "q": [0, 2]}, {"op": "rx", "q": [1], "slot": 0},
            {"op": "ry", "q": [2], "slot": 1}, {"op": "rz", "q": [0], "angle": 0.4},
            {"op": "x", "q": [1]}, {"op": "y", "q": [1]}, {"op": "z", "q": [1]},
            {"op": "dense", "q": [0, 1], "mat": np.kron(np.eye(2), u)},
            {"op": "dense", "q": [1, 0], "mat": np.array([[1, 0, 0, 0], [0, 1, 0, 0],
                                                          [0, 0, 0, 1], [0, 0, 1, 0]])},
            {"op": "dense", "q": [2], "mat": Q.binding.np.array(
                [[np.cos(0.3), 1j * np.sin(0.3)], [1j * np.sin(0.3), np.cos(0.3)]]),
             "controls": [0], "ctrl_vals": [0]},
            {"op": "pauli_rot", "q": [0, 2], "paulis": [1, 3], "angle": 0.7}]
    c = Q.Circuit.from_records(3, recs)
    want = [(Z_, X_, 7), (7, Z_, Z_), (0, 7, 7), (0, 7, 0), (7, X_, 7), (7, 7, Y_), (Z_, 7, 7),
            (7, X_, 7), (7, Y_, 7), (7, Z_, 7),
            (0, 7, 7),            # kron(I, u): u on qubit 0 (bit 0 <-> q[0]), identity on 1
            (Z_, X_, 7),          # App. A matrix on targets [1, 0]: CNOT control 0, target 1
            (Z_, 7, X_),          # X rotation on 2 controlled by qubit 0
            (X_, 7, Z_)]
    for gi, w in enumerate(want):
        got = tuple(c.commute(gi, q) for q in range(3))
        assert got == w, (gi, recs[gi]["op"], got, w)
    assert _code(c.commute, len(recs), 0) == ERANGE
    assert _code(c.commute, 0, 3) == ERANGE


def test_heavy_merge_on_host():
    def blocks(n, recs, heavy, k=2):
        return Q.Plan(Q.Circuit.from_records(n, recs), "c128", max_k=k, heavy=heavy).info()["blocks"]

    rz0 = {"op": "rz", "q": [0], "angle": 0.3}
    rx0 = {"op": "rx", "q": [0], "angle": 0.3}
    rx1 = {"op": "rx", "q": [1], "angle": 0.3}
    cx = {"op": "cnot", "q": [0, 1]}
    h0 = {"op": "h", "q": [0]}
    cz = {"op": "cz", "q": [0, 1]}
    # a Z rotation passes the CNOT's control, an X rotation its target
    assert (blocks(2, [rz0, cx, rz0], False), blocks(2, [rz0, cx, rz0], True)) == (3, 2)
    assert (blocks(2, [rx1, cx, rx1], False), blocks(2, [rx1, cx, rx1], True)) == (3, 2)
    # ... but not the other way round, and nothing passes H (no shared Pauli)
    assert blocks(2, [rx0, cx, rx0], True) == 3
    assert blocks(2, [h0, cz, h0], True) == 3
    # commuting (IQP-like) circuits compress to constant depth: the block count
    # no longer grows with the number of layers
    n = 16
    for depth in (4, 16):
        g = W.iqp_rz_cz(n, depth, seed_key=(5, depth))
        light, heavy = blocks(n, g, False), blocks(n, g, True)
        assert heavy <= 2 * n, (depth, heavy)
        assert light >= depth * (n - 1) // 2, (depth, light)
    # on the headline circuit heavy planning never needs more blocks
    g = W.layered_rx_rz_cnot(12, 4, seed_key=(2,))
    assert blocks(12, g, True) <= blocks(12, g, False)
    with pytest.raises(Q.QsvError):
        Q.lib()  # (library loaded)
        B.check(Q.lib().qsv_plan_fused_ex(Q.Circuit.from_records(2, [cx]).h, 2, 2, 0, 0, 2,
                                          ctypes.byref(ctypes.c_void_p())))


def test_batch_validation():
    b = Q.Batch()
    c = Q.Circuit(3)
    o = Q.Observable(4)
    assert _code(b.add, c, o) == ERANGE
    c1 = Q.Circuit(1)
    assert _code(b.add, c1, Q.Observable(1)) == ERANGE
    c3 = Q.Circuit.from_records(3, [{"op": "ry", "q": [0], "slot": 1}])
    L = Q.lib()
    assert L.qsv_batch_add(b.h, c3.h, Q.Observable(3).h, None) == EINVAL
    b.add(c3, Q.Observable(3), [0.1, 0.2])
    items, tot = ctypes.c_int(), ctypes.c_int()
    assert L.qsv_batch_info(b.h, ctypes.byref(items), ctypes.byref(tot)) == 0
    assert (items.value, tot.value) == (1, 2)
    assert L.qsv_batch_set_theta(b.h, 1, None) == ERANGE
