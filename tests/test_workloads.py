"""Workload generators and the stored oracle values that depend on them.

* The 53-qubit depth-12 workload must still be the one the stored complex128
  slice values were computed on (path and sliced indices fingerprint), with
  1024 slices and per-slice intermediates <= 2^30 entries (Sec. 2.4 slicing to
  bound memory).
* The oracle's per-step hook stops a slice early and otherwise leaves the
  result unchanged.
"""

import json
import os

import numpy as np
import pytest

from oracle import tn_oracle
from tngen import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden", "precision_slices_seed0.json")


@pytest.mark.skipif(not os.path.exists(GOLD), reason="oracle values not generated")
def test_precision_workload_matches_stored_oracle_values():
    from .golden.make_precision_slices import fingerprint
    doc = json.load(open(GOLD))
    w = workloads.build("precision", seed=0)
    assert fingerprint(w) == doc["fingerprint"]
    assert w.stats["n_slices"] == 1024 and w.stats["max_log2"] <= 30
    assert w.circuit.n == 53
    vals = np.array([s[1] + 1j * s[2] for s in doc["slices"]])
    # a slice can be exactly zero (its fixed values select zero gate entries)
    assert np.all(np.isfinite(vals)) and np.sum(np.abs(vals) > 0) >= len(vals) // 2


def test_oracle_step_hook_prefix_and_full():
    w = workloads.build("plain", seed=2, trials=1)
    args = (w.tn.tensors, w.tn.labels, w.tn.open, w.path, [], [])
    full = tn_oracle.contract_slice(*args)
    seen = []
    again = tn_oracle.contract_slice(*args, on_step=lambda k: seen.append(k))
    assert seen == list(range(len(w.path)))
    assert np.array_equal(full, again)
    assert tn_oracle.contract_slice(*args, on_step=lambda k: k < 3) is None


def test_open_output_network_is_the_state_vector():
    """Every output index open: the contraction (any path, here the
    time-ordered one and the greedy one) is the state vector U|0>, with the
    open indices in qudit order (row-major state index)."""
    import numpy as np
    from oracle import statevector as sv
    from oracle import tn_oracle
    from tngen import circuits, network, path as tpath
    for circ in (circuits.gbs_like(2, 4, 2, seed=3, d=4), circuits.grid_rqc(3, 4, 6, seed=2)):
        tn = network.relabel_compact(network.circuit_network(circ, open_outputs=True))
        psi = sv.final_state(circ).reshape(-1)
        for p in (tpath.time_ordered_path(len(tn.tensors)),
                  tpath.greedy_path(tn.labels, tn.dims, tn.open)):
            assert tpath.check_path(len(tn.tensors), p)
            got = tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p).reshape(-1)
            assert np.allclose(got, psi, atol=1e-12)
