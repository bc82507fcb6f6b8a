"""The bosonic workload (16 modes on a 4x4 lattice, Fock cutoff 4, depth 6,
two sliced dimension-4 indices = 16 slices), on the CPU.

* Slicing cannot bound its memory: on the workload's path, every pair of
  indices leaves a per-slice intermediate of 2^32 entries = 4^16, the full
  Fock space of the 16 modes (Sec. 2.4 slices to bound intermediates; here
  the path's widest tensors are states of all 16 modes, and a pair of sliced
  indices is shared by only some of them).  The slicer therefore keeps its
  tie-break, the least work with shared reuse (Eq. task_based_amplitude_flops).
* At a fixed cutoff the plan does not depend on the output pattern (Sec. 4,
  GBS experiment: runtime independent of the measured photon numbers): the
  schedule, kernels, strides and launch count are identical for 5 seeded
  patterns; only leaf values differ.
"""

import numpy as np
import pytest

from tngen import circuits, network, slicing, workloads

from paper_2107_09793_amd.binding import Plan


@pytest.fixture(scope="module")
def wl():
    return workloads.build("bosonic", seed=0)


def test_no_index_pair_bounds_the_bosonic_intermediates(wl):
    tn = wl.tn
    ts = slicing.TreeSets(tn.labels, tn.dims, tn.open, wl.path)
    inter = ts.open[ts.n:].astype(float) * ts.w[None, :]      # log2 per (node, index)
    tot = inter.sum(1)
    cand = np.where(~ts.kept)[0]
    best = np.inf
    for i, e in enumerate(cand):
        if i + 1 < len(cand):
            m = (tot[:, None] - inter[:, [e]] - inter[:, cand[i + 1:]]).max(0)
            best = min(best, m.min())
    assert best == 32.0 == 2 * 16                                 # 4^16 entries
    assert tot.max() == 32.0
    assert len(wl.sliced) == 2 and all(tn.dims[e] == 4 for e in wl.sliced)
    assert wl.stats["n_slices"] == 16 and wl.stats["max_log2"] == 32.0


def test_plan_independent_of_output_pattern(wl):
    circ = wl.circuit
    ref = None
    for s in range(5):
        x = circuits.random_bitstrings(circ.n, circ.d, 1, 100 + s)[0]
        tn = network.relabel_compact(network.circuit_network(circ, outcome=x))
        assert tn.labels == wl.tn.labels and tn.dims == wl.tn.dims
        pl = Plan.from_network(tn, wl.path, wl.sliced, workspace_limit=200 << 30)
        info = pl.info()
        key = (info["n_launches"], info["workspace_bytes"], info["cmac_exec"],
               tuple(pl.schedule()),
               tuple(tuple((k, tuple(v) if isinstance(v, list) else v) for k, v in st.items())
                     for st in pl.steps()),
               tuple(str(c) for c in pl.chains()))
        if ref is None:
            ref = key
        assert key == ref, s
