"""Shared-work-aware refinement of path and slices (tngen.refine), on the CPU.

* it never raises the objective it descends on (multiply-adds with reuse,
  Eq. task_based_amplitude_flops, or the roofline time estimate), keeps every
  per-slice intermediate within the cap, and returns a full binary tree;
* the refined path contracts to the same value as the original one (the
  contraction does not depend on the path, Sec. 2.3) -- oracle on both;
* the stored refined paths of the workloads belong to their networks and
  meet the workloads' caps, and lower the multiply-adds with reuse against
  the greedy search alone.
"""

import numpy as np
import pytest

from oracle import tn_oracle
from tngen import circuits, network, path as tpath, refine, slicing, workloads


def _net(seed, rows, cols, depth, batch=None):
    circ = circuits.grid_rqc(rows, cols, depth, seed=seed)
    if batch:
        tn = network.circuit_network(circ, batch=circuits.random_bitstrings(circ.n, 2, batch, seed))
    else:
        tn = network.circuit_network(circ, outcome=circuits.random_bitstrings(circ.n, 2, 1, seed)[0])
    return network.relabel_compact(tn)


@pytest.mark.parametrize("objective", ["cmac", "time"])
@pytest.mark.parametrize("case", [(3, 3, 4, 8, None, 4), (4, 4, 4, 10, 8, 3)])
def test_refine_lowers_objective_and_keeps_value(objective, case):
    seed, rows, cols, depth, batch, n_slice = case
    tn = _net(seed, rows, cols, depth, batch)
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    ts = slicing.TreeSets(tn.labels, tn.dims, tn.open, p)
    sl = slicing.greedy_slices(ts, n_slice=n_slice)
    st = ts.stats(sl)
    cap = st["max_log2"]
    p2, sl2, obj2 = refine.refine(tn.labels, tn.dims, tn.open, p, sl, cap_log2=cap,
                                  objective=objective, rounds=3, tree_moves=20000,
                                  slice_moves=500, seed=seed)
    assert tpath.check_path(len(tn.tensors), p2)
    assert len(sl2) == len(sl) and len(set(sl2)) == len(sl2)
    st2 = slicing.TreeSets(tn.labels, tn.dims, tn.open, p2).stats(sl2)
    assert st2["max_log2"] <= cap
    t1 = refine._Tree(tn.labels, tn.dims, tn.open, p)
    t1.timed, t1.rate, t1.bw = objective == "time", 19.66e12, 8e12
    assert obj2 <= t1.total(t1.mask(sl)) * (1 + 1e-12)
    if objective == "cmac":
        assert obj2 == pytest.approx(st2["flop_reuse"], rel=1e-12)
    a = tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p, sl)
    b = tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p2, sl2)
    assert np.allclose(a, b, rtol=1e-10, atol=1e-13)


@pytest.mark.parametrize("name", ["sliced", "precision", "gradient"])
def test_stored_refined_paths(name):
    w = workloads.build(name, seed=0)
    cfg = workloads.CONFIGS[name]
    assert w.meta["path_key"]["network"] == workloads.network_hash(w.tn)
    assert tpath.check_path(len(w.tn.tensors), w.path)
    if cfg.get("cap_log2") is not None:
        assert w.stats["max_log2"] <= cfg["cap_log2"]
    assert len(w.sliced) == cfg["n_slice"]
    greedy = workloads.build(name, seed=0, refine=False)
    # the time objective trades some multiply-adds for traffic, never all
    assert w.stats["flop_reuse"] < greedy.stats["flop_reuse"]
