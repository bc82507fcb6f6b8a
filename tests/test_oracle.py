"""Pins for the CPU oracle (no GPU).

Each oracle function is checked against something other than itself:
closed forms, a Kronecker-product construction of the full unitary, the
worked example of Sec. 2.2.1 with its naive sum (Eq. naive_summation), the
printed step costs of Eq. sequence, the grey-node instance counts of Fig. 3/5,
the printed m=10 shared-work numbers, and finite differences.
"""

import json
import os

import numpy as np
import pytest

from oracle import grad as ograd
from oracle import statevector as sv
from oracle import taskgraph, tn_oracle
from tngen import circuits, gates, network, path as tpath, slicing

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- gates -----
def test_gates_unitary_and_closed_forms():
    for u in (gates.SQRT_X, gates.SQRT_Y, gates.SQRT_W, gates.fsim(0.3, 1.1), gates.H,
              gates.CNOT, gates.haar_unitary(16, np.random.default_rng(0))):
        assert np.allclose(u @ u.conj().T, np.eye(u.shape[0]), atol=1e-14)
    assert np.allclose(gates.fsim(0.0, 0.0), np.eye(4))
    e01 = np.zeros(4, complex)
    e01[1] = 1
    out = gates.fsim(np.pi / 2, 0.0) @ e01
    assert np.allclose(out, [0, 0, -1j, 0])
    for s, p in ((gates.SQRT_X, gates.X), (gates.SQRT_Y, gates.Y), (gates.SQRT_W, gates.W)):
        assert np.allclose(s @ s, p, atol=1e-14)
    # printed form of sqrt(W) under the stated convention
    assert np.allclose(gates.SQRT_W, [[(1 + 1j) / 2, -1j / np.sqrt(2)], [1 / np.sqrt(2), (1 + 1j) / 2]])
    # the oracle's own fSim equals the generator's
    assert np.allclose(sv.fsim_matrix(0.7, 0.2), gates.fsim(0.7, 0.2))


def test_grid_generator_counts_and_seed():
    c1 = circuits.grid_rqc(3, 4, 8, seed=0)
    c2 = circuits.grid_rqc(3, 4, 8, seed=0)
    c3 = circuits.grid_rqc(3, 4, 8, seed=1)
    n2 = sum(1 for o in c1.ops if len(o.qudits) == 2)
    n1 = sum(1 for o in c1.ops if len(o.qudits) == 1)
    assert n1 == 12 * 9
    assert n2 == 34
    assert [o.name for o in c1.ops] == [o.name for o in c2.ops]
    assert [o.name for o in c1.ops] != [o.name for o in c3.ops]
    _, cl = circuits.grid_couplers(5, 6)
    for k, pairs in cl.items():                        # each class is a matching
        flat = [q for p in pairs for q in p]
        assert len(flat) == len(set(flat)), k
    c53 = circuits.grid_rqc(6, 9, 12, seed=0, inactive=((0, 4),))
    assert c53.n == 53 and sum(1 for o in c53.ops if len(o.qudits) == 2) == 270
    c30 = circuits.grid_rqc(5, 6, 14, seed=0)
    assert sum(1 for o in c30.ops if len(o.qudits) == 2) == 171
    g = circuits.gbs_like(4, 4, 6, seed=0)
    assert len(g.ops) == 144 and all(o.matrix.shape == (16, 16) for o in g.ops)


# ------------------------------------------------------------ state vector --
def _full_unitary(circ):
    """Independent construction: each gate as a d^n x d^n matrix built from a
    Kronecker product and an explicit basis permutation (integer digit maths)."""
    n, d = circ.n, circ.d
    dim = d ** n
    idx = np.arange(dim)
    digits = np.stack([(idx // d ** (n - 1 - q)) % d for q in range(n)], 1)
    full = np.eye(dim, dtype=complex)
    for op in circ.ops:
        k = len(op.qudits)
        order = list(op.qudits) + [q for q in range(n) if q not in op.qudits]
        # basis map: state with qudits reordered so that gate qudits lead
        perm_digits = digits[:, order]
        pidx = (perm_digits * (d ** np.arange(n - 1, -1, -1))).sum(1)
        p = np.zeros((dim, dim))
        p[pidx, idx] = 1.0
        g = np.kron(op.matrix, np.eye(d ** (n - k)))
        full = p.T @ g @ p @ full
    return full


@pytest.mark.parametrize("maker", [
    lambda: circuits.grid_rqc(2, 2, 4, seed=3),
    lambda: circuits.grid_rqc(1, 5, 6, seed=4),
    lambda: circuits.ghz(4),
    lambda: circuits.gbs_like(1, 3, 1, seed=5, d=4, literal=True),
])
def test_statevector_matches_kron_unitary(maker):
    circ = maker()
    # add a gate on non-adjacent qudits listed in descending order
    rng = np.random.default_rng(9)
    if circ.n >= 3:
        circ.add((circ.n - 1, 0), gates.haar_unitary(circ.d ** 2, rng))
    psi = sv.final_state(circ).reshape(-1)
    u = _full_unitary(circ)
    assert np.allclose(psi, u[:, 0], atol=1e-12)


def test_statevector_closed_forms():
    for n in (2, 5, 9):
        psi = sv.final_state(circuits.ghz(n)).reshape(-1)
        ref = np.zeros(2 ** n, complex)
        ref[0] = ref[-1] = 1 / np.sqrt(2)
        assert np.allclose(psi, ref, atol=1e-14)
    pc = circuits.product(6, seed=2)
    x = np.array([1, 0, 1, 1, 0, 1])
    expect = np.prod([op.matrix[x[q], 0] for q, op in enumerate(pc.ops)])
    assert np.isclose(sv.amplitudes(pc, x)[0], expect, atol=1e-14)
    vv = circuits.v_vdag(circuits.grid_rqc(3, 3, 5, seed=1))
    psi = sv.final_state(vv).reshape(-1)
    assert np.isclose(psi[0], 1.0, atol=1e-12)
    assert np.isclose(np.sum(np.abs(sv.final_state(circuits.grid_rqc(3, 4, 8, 0))) ** 2), 1.0,
                      atol=1e-12)


# ------------------------------------------------------------- TN oracle ----
def _tn_amp(circ, outcome, seed=None):
    tn = network.relabel_compact(network.circuit_network(circ, outcome=outcome))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open, seed=seed,
                          temperature=0.5 if seed is not None else 0.0)
    assert tpath.check_path(tn.n_tensors, p)
    return tn, p, tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p)


@pytest.mark.parametrize("name,maker", [
    ("grid3x4d8", lambda: circuits.grid_rqc(3, 4, 8, seed=0)),
    ("grid4x4d6", lambda: circuits.grid_rqc(4, 4, 6, seed=1)),
    ("gbs2x4d4", lambda: circuits.gbs_like(2, 4, 2, seed=2, d=4)),
    ("ghz7", lambda: circuits.ghz(7)),
])
def test_tn_oracle_matches_statevector(name, maker):
    circ = maker()
    outs = circuits.random_bitstrings(circ.n, circ.d, 3, seed=7)
    if name == "ghz7":
        outs = np.array([[0] * 7, [1] * 7, [0, 1, 0, 0, 0, 0, 0]])
    ref = sv.amplitudes(circ, outs)
    for x, r in zip(outs, ref):
        _, _, a = _tn_amp(circ, x)
        assert abs(a - r) <= 1e-12 * max(1.0, abs(r)) + 1e-15, (a, r)


def test_tn_oracle_path_independent_and_sliced_sum():
    circ = circuits.grid_rqc(3, 4, 8, seed=0)
    x = circuits.random_bitstrings(12, 2, 1, seed=0)[0]
    tn, p0, a0 = _tn_amp(circ, x)
    _, p1, a1 = _tn_amp(circ, x, seed=5)
    assert p0 != p1
    assert abs(a0 - a1) < 1e-13
    ts = slicing.TreeSets(tn.labels, tn.dims, tn.open, p0)
    sl = slicing.greedy_slices(ts, n_slice=4)
    parts = tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p0, sl, per_slice=True)
    assert parts.shape[0] == 16
    assert abs(parts.sum() - a0) < 1e-13
    # a slice is not the whole amplitude (the sum is not trivial)
    assert np.max(np.abs(parts - a0)) > 1e-6


def test_tn_oracle_batch_and_unitarity():
    circ = circuits.grid_rqc(3, 4, 8, seed=2)
    allx = np.array([[(j >> (11 - q)) & 1 for q in range(12)] for j in range(4096)])
    tn = network.relabel_compact(network.circuit_network(circ, batch=allx))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    amps = tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p)
    assert amps.shape == (4096,)
    assert abs(np.sum(np.abs(amps) ** 2) - 1.0) < 1e-12
    psi = sv.final_state(circ).reshape(-1)
    assert np.allclose(amps, psi, atol=1e-13)


def _worked_example(D, rng):
    g = json.load(open(os.path.join(GOLD, "worked_example.json")))
    names = g["leaf_order"]
    letters = sorted({c for n in names for c in g["tensors"][n]})
    ids = {c: i for i, c in enumerate(letters)}
    labels = [[ids[c] for c in g["tensors"][n]] for n in names]
    tensors = [rng.standard_normal([D] * len(l)) + 1j * rng.standard_normal([D] * len(l))
               for l in labels]
    dims = {i: D for i in ids.values()}
    return g, ids, labels, tensors, dims


@pytest.mark.parametrize("D", [2, 3])
def test_worked_example_naive_sequence_sliced(D):
    """Eq. naive_summation == Eq. sequence == sum of Eq. sliced_sum over e."""
    g, ids, labels, tensors, dims = _worked_example(D, np.random.default_rng(D))
    path = [tuple(p) for p in g["path_ssa"]]
    naive = tn_oracle.naive_sum(tensors, labels)
    seq = tn_oracle.contract(tensors, labels, dims, [], path)
    parts = tn_oracle.contract(tensors, labels, dims, [], path, sliced=[ids["e"]], per_slice=True)
    assert abs(naive - seq) < 1e-12 * abs(naive)
    assert len(parts) == D
    assert abs(parts.sum() - naive) < 1e-12 * abs(naive)
    # brute force: explicit loops over all six indices for D=2
    if D == 2:
        S1, S2, B, k0a, k0d, b1, b2 = tensors
        tot = 0
        for a, b, c, d, e, f in np.ndindex(2, 2, 2, 2, 2, 2):
            tot += b1[c] * b2[f] * B[c, f, b, e] * S1[b, a] * S2[e, d] * k0a[a] * k0d[d]
        assert abs(tot - naive) < 1e-12 * abs(naive)


@pytest.mark.parametrize("D", [2, 3])
def test_taskgraph_worked_example(D):
    g, ids, labels, tensors, dims = _worked_example(D, np.random.default_rng(0))
    path = [tuple(p) for p in g["path_ssa"]]
    st = taskgraph.enumerate_tasks(labels, dims, [], path, [])
    assert st["step_cost"] == [D ** p for p in g["step_cost_power_of_D"]]
    st = taskgraph.enumerate_tasks(labels, dims, [], path, [ids["e"]])
    expect = [1 if c == 1 else D for c in g["instances_when_e_sliced"]]
    assert st["instances"] == expect


def test_taskgraph_agrees_with_generator_statistics():
    circ = circuits.grid_rqc(3, 4, 8, seed=1)
    tn = network.relabel_compact(network.circuit_network(circ, outcome=[0] * 12))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    ts = slicing.TreeSets(tn.labels, tn.dims, tn.open, p)
    sl = slicing.greedy_slices(ts, n_slice=5)
    a = taskgraph.enumerate_tasks(tn.labels, tn.dims, tn.open, p, sl)
    b = ts.stats(sl)
    assert a["flop_reuse"] == pytest.approx(b["flop_reuse"], rel=1e-12)
    assert a["flop_noreuse"] == pytest.approx(b["flop_noreuse"], rel=1e-12)
    assert a["flop_reuse"] < a["flop_noreuse"]


def test_shared_work_formula_reproduces_printed_m10_numbers():
    g = json.load(open(os.path.join(GOLD, "m10_shared_work.json")))
    n_sl = g["n_slices"]
    total = g["flop_total_gflop"]
    reuse = total - g["flop_saved_gflop"]
    flop_sl = total / n_sl
    f = taskgraph.shared_fraction(reuse, flop_sl, n_sl)
    assert taskgraph.task_based_flops(f, flop_sl, n_sl) == pytest.approx(reuse)
    # the quoted saving (~47 %) is f_sl (N-1)/N of the no-reuse total
    assert abs(100 * f * (n_sl - 1) / n_sl - g["saving_percent_quoted"]) < 1.0
    assert 0.46 < f < 0.48
    # endpoints of Eq. task_based_amplitude_flops: f=0 is Eq. sliced_flops, f=1 one slice
    assert taskgraph.task_based_flops(0.0, flop_sl, n_sl) == pytest.approx(total)
    assert taskgraph.task_based_flops(1.0, flop_sl, n_sl) == pytest.approx(flop_sl)


# --------------------------------------------------------------- gradient ---
def test_adjoint_gradient_matches_finite_differences():
    circ = circuits.grid_rqc(2, 3, 4, seed=3, trainable=True)
    batch = circuits.random_bitstrings(circ.n, 2, 8, seed=3)
    loss, g = sv.nll_grad(circ, batch)
    assert loss == pytest.approx(sv.nll_loss(circ, batch))
    fd = ograd.fd_grad(circ, batch, h=1e-4)
    scale = max(1.0, np.max(np.abs(fd)))
    # central differences carry an O(h^2 f''') truncation error; at h=1e-4 and
    # a log-loss this is ~1e-6 relative, so h=1e-4 is checked at 1e-5 ...
    assert np.max(np.abs(g - fd)) <= 1e-5 * scale
    # ... and the Richardson combination (4 D(h/2) - D(h)) / 3, which cancels
    # the h^2 term, pins the adjoint to 1e-8.
    fd2 = ograd.fd_grad(circ, batch, h=5e-5)
    rich = (4 * fd2 - fd) / 3
    assert np.max(np.abs(g - rich)) <= 1e-8 * scale
    assert np.max(np.abs(g)) > 1e-3


def test_network_leaves_are_selected_gate_entries():
    circ = circuits.grid_rqc(2, 2, 2, seed=0)
    x = [1, 0, 1, 1]
    tn = network.circuit_network(circ, outcome=x)
    for t, oi in zip(tn.tensors, tn.leaf_op):
        vals = set(np.round(circ.ops[oi].matrix.reshape(-1), 12))
        assert set(np.round(t.reshape(-1), 12)) <= vals
