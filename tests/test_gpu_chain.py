"""Fused chains of stream steps on the GPU against the same steps launched
one by one.  With the chain on the vector units each output value is formed
by the same complex FMAs in the same order either way, so results must agree
bit for bit.  With the matrix-core chain steps (the default) the sums run in
another order, so both are checked against the complex128 oracle (1e-5 of
the rms slice value).  The small networks here are planned without batches
of tiny steps (tiny=False), which would otherwise take all of their steps
out of chains."""

import numpy as np
import pytest

from oracle import tn_oracle
from tngen import circuits, network, path as tpath, slicing, workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _batch_net(seed, rows, cols, depth, batch, n_slice):
    circ = circuits.grid_rqc(rows, cols, depth, seed=seed)
    b = circuits.random_bitstrings(circ.n, 2, batch, seed)
    tn = network.relabel_compact(network.circuit_network(circ, batch=b))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    sl = slicing.greedy_slices(slicing.TreeSets(tn.labels, tn.dims, tn.open, p), n_slice=n_slice)
    return tn, p, sl


@pytest.mark.parametrize("cfg", [(3, 4, 4, 12, 16, 2), (7, 4, 4, 14, 32, 2), (9, 4, 4, 10, 16, 3),
                                 (3, 4, 5, 12, 16, 2), (7, 4, 5, 14, 32, 2), (5, 4, 5, 12, 64, 2)])
def test_chain_bitwise_equals_per_step(cfg):
    from paper_2107_09793_amd import Plan
    dev = _dev()
    tn, p, sl = _batch_net(*cfg)
    leaves = [torch.from_numpy(t.astype(np.complex64)).to(dev) for t in tn.tensors]
    fused = Plan.from_network(tn, p, sl, tiny=False, chain_mfma=False)
    plain = Plan.from_network(tn, p, sl, tiny=False, chain_mfma=False, chain_fused=False)
    mfma = Plan.from_network(tn, p, sl, tiny=False)
    assert fused.info()["n_chains"] > 0
    assert plain.info()["n_chains"] == fused.info()["n_chains"]
    assert plain.info()["n_launches"] > fused.info()["n_launches"]
    a = fused.contract(leaves, per_slice=True).cpu().numpy()
    b = plain.contract(leaves, per_slice=True).cpu().numpy()
    c = mfma.contract(leaves, per_slice=True).cpu().numpy()
    assert np.array_equal(a, b)
    ref = tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p, sl, per_slice=True)
    ref = np.asarray(ref).reshape(a.shape)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    assert np.max(np.abs(a - ref)) <= 1e-5 * rms
    assert np.max(np.abs(c - ref)) <= 1e-5 * rms


def test_chain_sliced_workload_bitwise():
    """The 30-qubit 64-slice workload with its default plan (chains, no
    persistent segments) against the same plan without chains."""
    from paper_2107_09793_amd import Plan
    dev = _dev()
    w = workloads.build("sliced", seed=0)
    leaves = [torch.from_numpy(np.ascontiguousarray(t, dtype=np.complex64)).to(dev)
              for t in w.tn.tensors]
    fused = Plan.from_network(w.tn, w.path, w.sliced, chain_mfma=False)
    plain = Plan.from_network(w.tn, w.path, w.sliced, chain_mfma=False, chain_fused=False)
    a = fused.contract(leaves, per_slice=True).cpu().numpy()
    del fused
    torch.cuda.empty_cache()
    b = plain.contract(leaves, per_slice=True).cpu().numpy()
    assert np.array_equal(a, b)
    del plain
    torch.cuda.empty_cache()
    mfma = Plan.from_network(w.tn, w.path, w.sliced)
    c = mfma.contract(leaves, per_slice=True).cpu().numpy()
    rms = np.sqrt(np.mean(np.abs(b) ** 2))
    assert np.max(np.abs(c - b)) <= 1e-5 * rms
    del mfma
    torch.cuda.empty_cache()
    # split-BF16 (its matrix-core chain steps include shapes 4x3 and 4x5)
    sb = Plan.from_network(w.tn, w.path, w.sliced, precision="split_bf16")
    d = sb.contract(leaves, per_slice=True).cpu().numpy()
    assert np.max(np.abs(d - b)) <= 1e-3 * rms


@pytest.mark.parametrize("cfg", [(3, 4, 4, 12, 16, 2), (7, 4, 4, 14, 32, 2), (9, 4, 4, 10, 16, 3),
                                 (7, 4, 5, 14, 32, 2)])
def test_chain_split_bf16(cfg):
    """Split-BF16 matrix-core chain steps (three BF16 products, float32
    accumulation) against the complex128 oracle at 1e-3 of the rms slice
    value, and against the vector-unit chain of the same plan."""
    from paper_2107_09793_amd import Plan
    dev = _dev()
    tn, p, sl = _batch_net(*cfg)
    leaves = [torch.from_numpy(t.astype(np.complex64)).to(dev) for t in tn.tensors]
    sb = Plan.from_network(tn, p, sl, tiny=False, precision="split_bf16")
    assert sb.info()["n_chains"] > 0
    assert any(2 <= len(d["kslot"]) <= 6 and 3 <= len(d["nslot"]) <= 5
               and len(d["kslot"]) + len(d["nslot"]) <= 9 and d["nrow"] >= 4
               for ch in sb.chains() for d in ch["st"])
    got = sb.contract(leaves, per_slice=True).cpu().numpy()
    ref = tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p, sl, per_slice=True)
    ref = np.asarray(ref).reshape(got.shape)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    assert np.max(np.abs(got - ref)) <= 1e-3 * rms


@pytest.mark.parametrize("cfg", [(7, 4, 4, 14, 32, 2), (9, 4, 4, 10, 16, 3)])
def test_one_step_chains_bitwise(cfg):
    """A lone stream step run as a one-step chain on the vector units forms
    every value by the same complex FMAs in the same order as the stream
    kernel: identical results with and without one-step chains."""
    from paper_2107_09793_amd import Plan
    dev = _dev()
    tn, p, sl = _batch_net(*cfg)
    leaves = [torch.from_numpy(t.astype(np.complex64)).to(dev) for t in tn.tensors]
    single = Plan.from_network(tn, p, sl, tiny=False, chain_mfma=False)
    multi = Plan.from_network(tn, p, sl, tiny=False, chain_mfma=False, chain_single=False)
    assert any(ch["first"] == ch["last"] for ch in single.chains())
    assert all(ch["first"] < ch["last"] for ch in multi.chains())
    a = single.contract(leaves, per_slice=True).cpu().numpy()
    b = multi.contract(leaves, per_slice=True).cpu().numpy()
    assert np.array_equal(a, b)
