"""Backward schedule (checkpoint policies, outer iterations, slice subsets)
executed on the CPU exactly as tn_contract_backward runs it
(``plan_exec.execute_backward``: every value and gradient at the plan's
workspace offsets), against the oracle.

The contraction is linear in each leaf, so for leaf j, output-gradient w and
any direction D, the leaf gradient g_j (PyTorch convention) satisfies
    sum(conj(g_j) * D) = sum_o conj(w_o) * contraction_o(leaf j := D),
with the contraction summed over the selected slices (Eq. sliced_sum); the
right side is computed by the oracle.
"""

import numpy as np
import pytest

from oracle import tn_oracle
from tngen import circuits, network, path as tpath, slicing

from paper_2107_09793_amd.binding import Plan, TN_CKPT_ALL, TN_CKPT_RECOMPUTE

from .plan_exec import execute_backward


def _net(seed, rows, cols, depth, n_slice, batch=None):
    circ = circuits.grid_rqc(rows, cols, depth, seed=seed)
    if batch:
        b = circuits.random_bitstrings(circ.n, 2, batch, seed)
        tn = network.relabel_compact(network.circuit_network(circ, batch=b))
    else:
        x = circuits.random_bitstrings(circ.n, 2, 1, seed)[0]
        tn = network.relabel_compact(network.circuit_network(circ, outcome=x))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    sl = slicing.greedy_slices(slicing.TreeSets(tn.labels, tn.dims, tn.open, p), n_slice=n_slice)
    return tn, p, sl


def _check(pl, tn, p, sl, slice_ids=None, n_leaves=10, seed=0):
    rng = np.random.default_rng(seed)
    n_out = int(np.prod([tn.dims[i] for i in tn.open], dtype=np.int64)) if tn.open else 1
    w = rng.standard_normal(n_out) + 1j * rng.standard_normal(n_out)
    grads = execute_backward(pl, tn, w, slice_ids=slice_ids)
    for j in rng.choice(len(tn.tensors), size=min(n_leaves, len(tn.tensors)), replace=False):
        D = rng.standard_normal(tn.tensors[j].shape) + 1j * rng.standard_normal(tn.tensors[j].shape)
        ts = list(tn.tensors)
        ts[j] = D
        lin = tn_oracle.contract(ts, tn.labels, tn.dims, tn.open, p, sl, slice_ids=slice_ids)
        expect = np.sum(np.conj(w) * np.asarray(lin).reshape(-1))
        got = np.sum(np.conj(grads[j]) * D.reshape(-1))
        scale = np.sqrt(np.sum(np.abs(w) ** 2) * np.sum(np.abs(lin) ** 2))
        assert abs(got - expect) <= 1e-10 * scale, (j, got, expect)


@pytest.mark.parametrize("policy", ["all", "recompute"])
def test_backward_resident(policy):
    tn, p, sl = _net(5, 4, 4, 8, 5)
    pl = Plan(tn.labels, tn.dims, tn.open, p, sl, checkpoint=policy, workspace_limit=0)
    info = pl.info()
    assert info["backward_policy"] == (TN_CKPT_ALL if policy == "all" else TN_CKPT_RECOMPUTE)
    _check(pl, tn, p, sl)


def test_backward_recompute_under_budget_with_chains():
    """A workspace limit below the store-everything backward forces
    recomputation; chains of the forward run fused in the backward's forward
    pass where a block holds them."""
    tn, p, sl = _net(7, 4, 4, 14, 2, batch=32)
    full = Plan(tn.labels, tn.dims, tn.open, p, sl, checkpoint="all", workspace_limit=0).info()
    lim = max(full["workspace_bytes"] + (1 << 16), full["workspace_backward_bytes"] // 2)
    pl = Plan(tn.labels, tn.dims, tn.open, p, sl, workspace_limit=lim)
    info = pl.info()
    assert info["n_outer_bits"] == 0
    assert info["backward_policy"] == TN_CKPT_RECOMPUTE
    assert info["cmac_backward_recompute"] > 0
    assert info["workspace_backward_bytes"] < full["workspace_backward_bytes"]
    T = pl.backward_tables()
    assert (T["keep"] == 0).any()
    if info["n_chains"]:
        assert T["fuse_chain"][:info["n_chains"]].any()
    _check(pl, tn, p, sl)


@pytest.mark.parametrize("policy", ["all", "recompute"])
def test_backward_outer_iterations(policy):
    tn, p, sl = _net(5, 4, 4, 8, 5)
    pl = Plan(tn.labels, tn.dims, tn.open, p, sl, max_resident_bits=2, checkpoint=policy,
              workspace_limit=0)
    info = pl.info()
    assert info["n_outer_bits"] >= 2
    T = pl.backward_tables()
    assert T["frontier"].any()
    _check(pl, tn, p, sl)


def test_backward_slice_subset_with_repeats():
    tn, p, sl = _net(5, 4, 4, 8, 5)
    pl = Plan(tn.labels, tn.dims, tn.open, p, sl, max_resident_bits=3, workspace_limit=0)
    _check(pl, tn, p, sl, slice_ids=[7, 0, 31, 12, 5, 7])


def test_backward_batch_outputs_outer():
    tn, p, sl = _net(3, 3, 5, 8, 3, batch=16)
    pl = Plan(tn.labels, tn.dims, tn.open, p, sl, max_resident_bits=1, checkpoint="recompute",
              workspace_limit=0)
    assert pl.info()["n_outer_bits"] >= 2
    _check(pl, tn, p, sl, slice_ids=[1, 6, 2])
