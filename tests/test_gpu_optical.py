"""Optical GBS circuits of Alg. 1 (squeezers and beam splitters in the
truncated Fock basis, r = 0.5) on the GPU.

* GBS-88-m1 at cutoff 4 (Sec. 4): the amplitude of three output patterns
  against the complex128 oracle on the same path; the plan is identical for
  every pattern (Sec. 4: at a fixed cutoff the run time does not depend on
  the photon numbers).
* Cutoff 8 (three bits per index): a 2x4-mode circuit against the state
  vector; GBS-88-m1 at cutoff 8 at full size (2^33-entry intermediates, too
  large for the host oracle) through a property that holds at any size: the
  per-slice results of the same network with two sliced indices add up to
  the unsliced amplitude.
Tolerance: complex64, 1e-5 relative.
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


def test_gbs88_cutoff4_against_oracle():
    from paper_2107_09793_amd import Plan
    dev = _dev()
    w = workloads.build("gbs", seed=0)
    ref_steps = None
    for s in range(3):
        x = w.outcome if s == 0 else circuits.gbs_pattern(w.circuit.n, 4, 0.5, 10 + s)
        tn = network.relabel_compact(network.circuit_network(w.circuit, outcome=x))
        assert tn.labels == w.tn.labels
        pl = Plan.from_network(tn, w.path, w.sliced)
        steps = pl.steps()
        if ref_steps is None:
            ref_steps = steps
        assert steps == ref_steps
        got = complex(pl.contract(_leaves(tn, dev)).cpu().item())
        ref = complex(tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, w.path,
                                         w.sliced))
        print("gbs88 cutoff 4: photons", int(x.sum()), "gpu", got, "oracle", ref)
        assert abs(got - ref) <= 1e-5 * abs(ref)


def test_cutoff8_small_against_state_vector():
    from paper_2107_09793_amd import Plan
    dev = _dev()
    circ = circuits.gbs_optical(2, 4, 1, seed=3, d=8, r=0.5)
    for s in range(2):
        x = circuits.gbs_pattern(8, 8, 0.5, s)
        tn = network.relabel_compact(network.circuit_network(circ, outcome=x))
        p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
        sl = slicing.greedy_slices(slicing.TreeSets(tn.labels, tn.dims, tn.open, p), n_slice=1)
        pl = Plan(tn.labels, tn.dims, tn.open, p, sl)
        got = complex(pl.contract(_leaves(tn, dev)).cpu().item())
        ref = complex(sv.amplitudes(circ, [x])[0])
        assert abs(got - ref) <= 1e-5 * abs(ref), (got, ref)


def test_gbs88_cutoff8_full_size_sliced_sum():
    from paper_2107_09793_amd import Plan
    dev = _dev()
    w = workloads.build("gbs8", seed=0)
    leaves = _leaves(w.tn, dev)
    pl = Plan.from_network(w.tn, w.path, [])
    assert pl.info()["max_log2_per_slice"] == 33
    amp = complex(pl.contract(leaves).cpu().item())
    pl.release_workspace()
    del pl
    torch.cuda.empty_cache()
    ts = slicing.TreeSets(w.tn.labels, w.tn.dims, w.tn.open, w.path)
    sl = slicing.greedy_slices(ts, n_slice=2)
    ps = Plan.from_network(w.tn, w.path, sl)
    assert ps.info()["n_slices"] == 64
    per = ps.contract(leaves, per_slice=True).cpu().numpy().reshape(-1)
    print("gbs88 cutoff 8: amplitude", amp, "sum of 64 slices", per.sum())
    assert abs(per.sum() - amp) <= 1e-5 * abs(amp)
    ps.release_workspace()
    del ps
    torch.cuda.empty_cache()
