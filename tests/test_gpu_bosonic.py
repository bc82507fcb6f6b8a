"""The bosonic workload (16 modes on a 4x4 lattice, Fock cutoff 4, depth 6,
2 sliced dimension-4 indices = 16 slices) on the GPU.

At full size the complex128 oracle cannot run on the host (its widest
intermediates are the 4^16 = 2^32-entry Fock space: 64 GiB each in
complex128, about 2e13 multiply-adds per slice), so full size is checked
through properties that hold at any size, with the oracle at reduced depth:

* full size: the 16 per-slice results sum to the summed output; the same
  circuit with every output open, contracted along the time-ordered path
  (a different network and path), gives the state U|0>, whose norm is 1
  (unitarity, float64 sum on the GPU); the sliced amplitude of three output
  patterns equals the state's entry (path independence, Sec. 2.3);
* depth 2 on the same lattice: every slice against the oracle.
Tolerance: complex64, 1e-5 (of the rms entry for single entries and slices).
"""

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


def _leaves(tn, dev):
    return [torch.from_numpy(np.ascontiguousarray(t, dtype=np.complex64)).to(dev)
            for t in tn.tensors]


def test_bosonic_reduced_depth_every_slice_against_oracle():
    from paper_2107_09793_amd import Plan
    dev = _dev()
    circ = circuits.gbs_like(4, 4, 2, seed=0, d=4)
    x = circuits.random_bitstrings(16, 4, 1, 0)[0]
    tn = network.relabel_compact(network.circuit_network(circ, outcome=x))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    sl = slicing.greedy_slices(slicing.TreeSets(tn.labels, tn.dims, tn.open, p), n_slice=2)
    assert all(tn.dims[e] == 4 for e in sl)
    pl = Plan(tn.labels, tn.dims, tn.open, p, sl)
    assert pl.info()["n_slices"] == 16
    got = pl.contract(_leaves(tn, dev), per_slice=True).cpu().numpy().reshape(-1)
    ref = np.asarray(tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p, sl,
                                        per_slice=True)).reshape(-1)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    assert np.max(np.abs(got - ref)) <= 1e-5 * rms


def test_bosonic_full_size_unitarity_and_path_independence():
    from paper_2107_09793_amd import Plan
    dev = _dev()
    wl = workloads.build("bosonic", seed=0)
    circ = wl.circuit
    pats = [wl.outcome] + [circuits.random_bitstrings(16, 4, 1, 200 + s)[0] for s in range(2)]
    amps = []
    for x in pats:
        tn = network.relabel_compact(network.circuit_network(circ, outcome=x))
        pl = Plan.from_network(tn, wl.path, wl.sliced)
        info = pl.info()
        assert info["n_slices"] == 16 and info["max_log2_per_slice"] == 32
        leaves = _leaves(tn, dev)
        per = pl.contract(leaves, per_slice=True).cpu().numpy().reshape(-1)
        amp = complex(pl.contract(leaves).cpu().item())
        assert abs(amp - per.sum()) <= 1e-6 * np.sqrt(np.sum(np.abs(per) ** 2)) * 4
        amps.append(amp)
        pl.release_workspace()
        del pl, leaves
        torch.cuda.empty_cache()
    tn = network.relabel_compact(network.circuit_network(circ, open_outputs=True))
    ps = Plan.from_network(tn, tpath.time_ordered_path(len(tn.tensors)), [])
    assert ps.info()["out_elems"] == 4 ** 16
    psi = ps.contract(_leaves(tn, dev)).reshape(-1)
    ps.release_workspace()
    torch.cuda.empty_cache()
    norm2 = torch.zeros((), dtype=torch.float64, device=dev)
    for ch in psi.split(1 << 26):
        norm2 += (ch.real ** 2 + ch.imag ** 2).sum()
    norm2 = float(norm2.item())
    rms = np.sqrt(norm2 / psi.numel())
    print("bosonic: |psi|^2 - 1 =", norm2 - 1.0)
    assert abs(norm2 - 1.0) <= 1e-5
    for x, amp in zip(pats, amps):
        idx = int(sum(int(v) * 4 ** (15 - q) for q, v in enumerate(x)))
        ref = complex(psi[idx].item())
        print("bosonic: pattern", list(map(int, x)), "sliced", amp, "state", ref)
        assert abs(amp - ref) <= 1e-5 * max(abs(ref), rms)
    del psi
    torch.cuda.empty_cache()
