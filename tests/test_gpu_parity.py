"""GPU parity: the HIP path (through the C ABI) against the complex128 oracle.

Tolerance: complex64 results within 1e-5 relative of the oracle (scalar:
|a_gpu - a| / |a|; vectors: ||a_gpu - a||_2 / ||a||_2 and per-element
|a_gpu - a| <= 1e-5 max|a|).  Per-slice results are compared with the same
bound relative to the rms slice magnitude, because single slices can be
close to zero.
"""

import numpy as np
import pytest

from oracle import statevector as sv
from oracle import tn_oracle
from tngen import circuits, network, path as tpath, slicing, workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _leaves(tn, dev):
    return [torch.from_numpy(np.ascontiguousarray(t, dtype=np.complex64)).to(dev)
            for t in tn.tensors]


def _rel(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _plan(*a, **k):
    from paper_2107_09793_amd import Plan
    return Plan(*a, **k)


def _perm_ref(x, pin, pout):
    """Definition: logical element i (bits i_j) is read at sum_j i_j 2^pin[j]
    and written at sum_j i_j 2^pout[j]."""
    idx = np.arange(x.size, dtype=np.int64)
    src = np.zeros_like(idx)
    dst = np.zeros_like(idx)
    for j in range(len(pin)):
        src |= ((idx >> j) & 1) << int(pin[j])
        dst |= ((idx >> j) & 1) << int(pout[j])
    ref = np.empty_like(x)
    ref[dst] = x[src]
    return ref


@pytest.mark.parametrize("nbits", [1, 5, 9, 10, 11, 12, 13, 20, 26])
def test_permute_bitwise(nbits):
    """Plain kernel below 10 bits, LDS-tiled (10- and 12-bit tiles) above;
    random permutations on both sides, plus identity and full reversal."""
    from paper_2107_09793_amd import permute
    dev = _dev()
    rng = np.random.default_rng(nbits)
    x = (rng.standard_normal(1 << nbits) + 1j * rng.standard_normal(1 << nbits)).astype(np.complex64)
    xd = torch.from_numpy(x).to(dev)
    cases = [(list(range(nbits)), list(rng.permutation(nbits))),
             (list(rng.permutation(nbits)), list(rng.permutation(nbits))),
             (list(range(nbits)), list(range(nbits))),
             (list(range(nbits)), list(reversed(range(nbits))))]
    for pin, pout in cases:
        y = permute(xd, pin, pout).cpu().numpy()
        assert np.array_equal(y, _perm_ref(x, pin, pout)), (pin, pout)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plain_amplitude(seed):
    dev = _dev()
    w = workloads.build("plain", seed=seed, trials=2)
    ref = complex(tn_oracle.contract(w.tn.tensors, w.tn.labels, w.tn.dims, w.tn.open, w.path))
    pl = _plan(w.tn.labels, w.tn.dims, w.tn.open, w.path)
    got = complex(pl.contract(_leaves(w.tn, dev)).cpu().item())
    assert abs(got - ref) <= 1e-5 * abs(ref), (got, ref)
    # the state-vector simulation gives the same amplitude
    a_sv = sv.amplitudes(w.circuit, w.outcome)[0]
    assert abs(got - a_sv) <= 1e-5 * abs(a_sv)


def test_unitarity_all_bitstrings():
    dev = _dev()
    circ = circuits.grid_rqc(3, 4, 8, seed=0)
    allx = np.array([[(j >> (11 - q)) & 1 for q in range(12)] for j in range(4096)])
    tn = network.relabel_compact(network.circuit_network(circ, batch=allx))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    pl = _plan(tn.labels, tn.dims, tn.open, p)
    amps = pl.contract(_leaves(tn, dev))
    norm = float(torch.sum(torch.abs(amps) ** 2).item())   # float64 on the device
    assert abs(norm - 1.0) <= 1e-5
    ref = sv.final_state(circ).reshape(-1)
    a = amps.cpu().numpy()
    assert _rel(a, ref) <= 1e-5
    assert np.max(np.abs(a - ref)) <= 1e-5 * np.max(np.abs(ref))


@pytest.mark.parametrize("variant", ["resident", "outer", "noreuse", "simple"])
def test_sliced_small_matches_oracle(variant):
    dev = _dev()
    circ = circuits.grid_rqc(4, 4, 8, seed=5)
    x = circuits.random_bitstrings(16, 2, 1, 5)[0]
    tn = network.relabel_compact(network.circuit_network(circ, outcome=x))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    ts = slicing.TreeSets(tn.labels, tn.dims, tn.open, p)
    sl = slicing.greedy_slices(ts, n_slice=5)
    kw = dict(resident={}, outer=dict(max_resident_bits=2), noreuse=dict(no_reuse=True),
              simple=dict(simple=True))[variant]
    pl = _plan(tn.labels, tn.dims, tn.open, p, sl, **kw)
    leaves = _leaves(tn, dev)
    parts = tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p, sl, per_slice=True)
    ref = parts.sum()
    got = complex(pl.contract(leaves).cpu().item())
    assert abs(got - ref) <= 1e-5 * abs(ref)
    per = pl.contract(leaves, per_slice=True).cpu().numpy()
    rms = np.sqrt(np.mean(np.abs(parts) ** 2))
    assert np.max(np.abs(per - parts)) <= 1e-5 * rms
    # a subset of slices, in a scrambled order
    ids = [7, 0, 31, 12, 5]
    sub = pl.contract(leaves, slice_ids=ids, per_slice=True).cpu().numpy()
    assert np.max(np.abs(sub - parts[ids])) <= 1e-5 * rms
    s = complex(pl.contract(leaves, slice_ids=ids).cpu().item())
    assert abs(s - parts[ids].sum()) <= 1e-5 * rms * len(ids)


def test_batched_outcomes_match_statevector():
    dev = _dev()
    circ = circuits.grid_rqc(3, 5, 8, seed=3)
    batch = circuits.random_bitstrings(15, 2, 64, 3)
    tn = network.relabel_compact(network.circuit_network(circ, batch=batch))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    ts = slicing.TreeSets(tn.labels, tn.dims, tn.open, p)
    sl = slicing.greedy_slices(ts, n_slice=2)
    pl = _plan(tn.labels, tn.dims, tn.open, p, sl)
    got = pl.contract(_leaves(tn, dev)).cpu().numpy()
    ref = sv.amplitudes(circ, batch)
    assert _rel(got, ref) <= 1e-5
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))


def test_batch_option_matches_statevector():
    """The same 64 outcomes through tn_plan_options.batch: the network is
    given without the batch index and the output leaves are flagged as
    batched (leading axis of 64 variants)."""
    dev = _dev()
    circ = circuits.grid_rqc(3, 5, 8, seed=3)
    batch = circuits.random_bitstrings(15, 2, 64, 3)
    tn = network.relabel_compact(network.circuit_network(circ, batch=batch))
    bi = tn.batch_index
    others = sorted(i for i in tn.dims if i != bi)
    mp = {i: j for j, i in enumerate(others)}
    batched = [t for t, l in enumerate(tn.labels) if bi in l]
    labels = [[mp[i] for i in l if i != bi] for l in tn.labels]
    dims = {mp[i]: v for i, v in tn.dims.items() if i != bi}
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    ts = slicing.TreeSets(tn.labels, tn.dims, tn.open, p)
    sl = [mp[i] for i in slicing.greedy_slices(ts, n_slice=2)]
    from paper_2107_09793_amd import Plan
    pl = Plan(labels, dims, [], p, sl, batch=64, batched_leaves=batched)
    got = pl.contract(_leaves(tn, dev)).cpu().numpy()
    assert got.shape == (64,)
    ref = sv.amplitudes(circ, batch)
    assert _rel(got, ref) <= 1e-5
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))


@pytest.mark.parametrize("seed", [0, 1])
def test_batches_of_tiny_steps(seed):
    """The 3x4 circuit with a batch of 8 outcomes and 2 sliced indices: every
    slice with tiny steps batched into single-workgroup launches, and with
    one launch per step, against the oracle (1e-5 of the rms slice)."""
    dev = _dev()
    circ = circuits.grid_rqc(3, 4, 8, seed=20 + seed)
    batch = circuits.random_bitstrings(12, 2, 8, 20 + seed)
    tn = network.relabel_compact(network.circuit_network(circ, batch=batch))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    sl = slicing.greedy_slices(slicing.TreeSets(tn.labels, tn.dims, tn.open, p), n_slice=2)
    on = _plan(tn.labels, tn.dims, tn.open, p, sl)
    off = _plan(tn.labels, tn.dims, tn.open, p, sl, tiny=False)
    assert on.info()["n_launches"] < off.info()["n_launches"]
    leaves = _leaves(tn, dev)
    ref = np.asarray(tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p, sl,
                                        per_slice=True)).reshape(4, -1)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    for pl in (on, off):
        got = pl.contract(leaves, per_slice=True).cpu().numpy().reshape(4, -1)
        assert np.max(np.abs(got - ref)) <= 1e-5 * rms


def test_bosonic_small_matches_oracle():
    dev = _dev()
    circ = circuits.gbs_like(2, 4, 2, seed=1, d=4)
    x = circuits.random_bitstrings(8, 4, 1, 1)[0]
    tn = network.relabel_compact(network.circuit_network(circ, outcome=x))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    ts = slicing.TreeSets(tn.labels, tn.dims, tn.open, p)
    sl = slicing.greedy_slices(ts, n_slice=1)
    pl = _plan(tn.labels, tn.dims, tn.open, p, sl)
    got = complex(pl.contract(_leaves(tn, dev)).cpu().item())
    ref = sv.amplitudes(circ, x)[0]
    assert abs(got - ref) <= 1e-5 * abs(ref)


def test_sliced_workload_full_size_all_slices():
    """The 30-qubit depth-14 workload at full size: all 64 slices on the GPU
    in one call against complex128 oracle values of every slice
    (tests/golden/sliced_slices_seed0.json, written by make_sliced_slices.py
    from the oracle alone), so the full amplitude is pinned too."""
    import json
    import os
    from .golden.make_sliced_slices import fingerprint
    dev = _dev()
    doc = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      "sliced_slices_seed0.json")))
    w = workloads.build("sliced", seed=0)
    assert fingerprint(w) == doc["fingerprint"], "workload differs from the one the oracle used"
    assert w.stats["max_log2"] <= 26 and len(w.sliced) == 6
    ref = np.array([r + 1j * i for _, r, i in doc["slices"]])
    amp_ref = complex(*doc["amplitude"])
    pl = _plan(w.tn.labels, w.tn.dims, w.tn.open, w.path, w.sliced)
    leaves = _leaves(w.tn, dev)
    per = pl.contract(leaves, per_slice=True).cpu().numpy().reshape(-1)
    total = complex(pl.contract(leaves).cpu().item())
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    err = np.abs(per - ref) / rms
    print("per-slice error / rms: max", err.max(), "amplitude rel. error",
          abs(total - amp_ref) / abs(amp_ref))
    assert np.all(err <= 1e-5), err
    assert abs(total - amp_ref) <= 1e-5 * abs(amp_ref)
