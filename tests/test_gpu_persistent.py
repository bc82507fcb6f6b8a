"""Persistent segments of small steps (one launch per run of small steps,
workgroups claiming items in topological order and waiting on completion
counters) against per-step launches: the two execute the same multiply-add
sequence per output, so results must agree bit for bit; both are also
checked against the complex128 oracle (1e-5)."""

import numpy as np
import pytest

from oracle import tn_oracle
from tngen import circuits, network, path as tpath, slicing, workloads

pytestmark = [pytest.mark.gpu, pytest.mark.skip(
    reason="persistent segments are opt-in (TN_FLAG_PERSISTENT) and off by default: the first "
           "full-size GPU run of a plan with segments did not finish and the cause is not yet "
           "shown; the segment kernel stays off the GPU until it is")]
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _cases():
    out = []
    w = workloads.build("plain", seed=1, trials=2)
    out.append(("plain", w.tn, w.path, w.sliced, {}))
    circ = circuits.grid_rqc(4, 4, 8, seed=5)
    x = circuits.random_bitstrings(16, 2, 1, 5)[0]
    tn = network.relabel_compact(network.circuit_network(circ, outcome=x))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    sl = slicing.greedy_slices(slicing.TreeSets(tn.labels, tn.dims, tn.open, p), n_slice=5)
    out.append(("sliced_outer", tn, p, sl, dict(max_resident_bits=2)))
    circ = circuits.grid_rqc(3, 5, 8, seed=3)
    batch = circuits.random_bitstrings(15, 2, 64, 3)
    tn = network.relabel_compact(network.circuit_network(circ, batch=batch))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    sl = slicing.greedy_slices(slicing.TreeSets(tn.labels, tn.dims, tn.open, p), n_slice=2)
    out.append(("batch", tn, p, sl, {}))
    return out


@pytest.mark.parametrize("case", range(3))
def test_persistent_bitwise_equals_per_step(case):
    from paper_2107_09793_amd import Plan
    dev = _dev()
    name, tn, p, sl, kw = _cases()[case]
    leaves = [torch.from_numpy(t.astype(np.complex64)).to(dev) for t in tn.tensors]
    pp = Plan(tn.labels, tn.dims, tn.open, p, sl, persistent=True, **kw)
    ps = Plan(tn.labels, tn.dims, tn.open, p, sl, persistent=False, **kw)
    assert pp.info()["n_launches"] < ps.info()["n_launches"]
    a = pp.contract(leaves, per_slice=True).cpu().numpy()
    b = ps.contract(leaves, per_slice=True).cpu().numpy()
    assert np.array_equal(a, b), name
    a2 = pp.contract(leaves, per_slice=True).cpu().numpy()
    assert np.array_equal(a, a2), "run-to-run"
    ref = tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p, sl, per_slice=True)
    ref = np.asarray(ref).reshape(a.shape)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    assert np.max(np.abs(a - ref)) <= 1e-5 * rms
