"""Contractions replayed as HIP graphs (tn_graph_create / tn_graph_launch).

The graph records the kernels tn_contract launches; the leaves are changed
in place between replays (new output patterns of the same circuit: same
shapes, new values), with eager work and synchronizations in between, and
every replay is compared with tn_contract on the same leaves -- bit for bit,
the kernels and their order being the same -- and with the state vector
(complex64, 1e-5 relative).
"""

import numpy as np
import pytest

from oracle import statevector as sv
from tngen import circuits, network, path as tpath, slicing

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _tensors(tn):
    return [torch.from_numpy(np.ascontiguousarray(t, dtype=np.complex64)) for t in tn.tensors]


def test_graph_replays_match_eager_and_statevector():
    from paper_2107_09793_amd import Plan
    dev = _dev()
    circ = circuits.grid_rqc(3, 4, 8, seed=11)
    xs = circuits.random_bitstrings(12, 2, 4, 11)
    tns = [network.relabel_compact(network.circuit_network(circ, outcome=x)) for x in xs]
    p = tpath.greedy_path(tns[0].labels, tns[0].dims, tns[0].open)
    pl = Plan(tns[0].labels, tns[0].dims, tns[0].open, p)
    leaves = [t.to(dev) for t in _tensors(tns[0])]
    g = pl.graph(leaves)
    ref = sv.amplitudes(circ, xs)
    for rep in range(3):
        for i, tn in enumerate(tns):
            for dst, src in zip(leaves, _tensors(tn)):
                dst.copy_(src.to(dev))
            got = g.launch().clone()
            # eager work between replays: the same contraction through tn_contract
            eager = pl.contract(leaves)
            torch.cuda.synchronize()
            assert torch.equal(got, eager), (rep, i)
            a = complex(got.cpu().item())
            assert abs(a - ref[i]) <= 1e-5 * abs(ref[i]), (rep, i, a, ref[i])


def test_graph_per_slice_subset():
    from paper_2107_09793_amd import Plan
    dev = _dev()
    circ = circuits.grid_rqc(3, 5, 8, seed=12)
    batch = circuits.random_bitstrings(15, 2, 16, 12)
    tn = network.relabel_compact(network.circuit_network(circ, batch=batch))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    sl = slicing.greedy_slices(slicing.TreeSets(tn.labels, tn.dims, tn.open, p), n_slice=3)
    pl = Plan(tn.labels, tn.dims, tn.open, p, sl)
    leaves = [t.to(dev) for t in _tensors(tn)]
    ids = [5, 0, 7, 5]
    g = pl.graph(leaves, slice_ids=ids, per_slice=True)
    for rep in range(3):
        got = g.launch().clone()
        eager = pl.contract(leaves, slice_ids=ids, per_slice=True)
        torch.cuda.synchronize()
        assert got.shape == (4, 16)
        assert torch.equal(got, eager), rep
    full = pl.contract(leaves, per_slice=True).cpu().numpy()
    assert np.array_equal(got.cpu().numpy(), full[ids])
    # the sum over all slices: the state vector's amplitudes
    gs = pl.graph(leaves)
    amp = gs.launch().cpu().numpy()
    ref = sv.amplitudes(circ, batch)
    assert np.linalg.norm(amp - ref) <= 1e-5 * np.linalg.norm(ref)


def test_graph_refuses_persistent_segments():
    from paper_2107_09793_amd import Plan
    from paper_2107_09793_amd.binding import TN_E_UNSUPPORTED, TnError
    dev = _dev()
    circ = circuits.grid_rqc(3, 4, 8, seed=13)
    x = circuits.random_bitstrings(12, 2, 1, 13)[0]
    tn = network.relabel_compact(network.circuit_network(circ, outcome=x))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    pl = Plan(tn.labels, tn.dims, tn.open, p, persistent=True)
    if pl.info()["n_segments"] == 0:
        pytest.skip("no segment in this plan")
    with pytest.raises(TnError) as e:
        pl.graph([t.to(dev) for t in _tensors(tn)])
    assert e.value.status == TN_E_UNSUPPORTED


@pytest.mark.parametrize("policy", ["all", "recompute"])
def test_backward_graph_replays_match_eager(policy):
    """tn_graph_create_backward: the adjoint of the trainable 4x5 workload
    (256 outcome strings) recorded once and replayed with new leaf values and
    new output gradients written in place, the gradient buffers cleared
    between replays, and eager forward and backward calls in between; every
    replay equals tn_contract_backward on the same inputs bit for bit (the
    same kernels in the same order)."""
    from paper_2107_09793_amd import Plan
    from tngen import workloads
    dev = _dev()
    wl = workloads.build("gradient", seed=0)
    tn = wl.tn
    pl = Plan.from_network(tn, wl.path, wl.sliced, checkpoint=policy)
    rng = np.random.default_rng(21)
    leaves = [t.to(dev) for t in _tensors(tn)]
    gout = torch.zeros(256, dtype=torch.complex128, device=dev)
    grads = [torch.zeros_like(x) for x in leaves]
    g = pl.backward_graph(leaves, gout, grads)
    for rep in range(3):
        for x in leaves:        # new leaf values of the same shapes
            x.mul_(complex(np.exp(1j * rng.uniform(0, 2 * np.pi))))
        gout.copy_(torch.from_numpy(rng.standard_normal(256) + 1j * rng.standard_normal(256)))
        for x in grads:
            x.zero_()
        g.launch()
        got = [x.clone() for x in grads]
        pl.contract(leaves)     # eager work between replays
        ref = [torch.zeros_like(x) for x in leaves]
        pl.backward(leaves, gout, ref)
        torch.cuda.synchronize()
        for j, (a, b) in enumerate(zip(got, ref)):
            assert torch.equal(a, b), (rep, j)
        assert any(torch.count_nonzero(a) > 0 for a in got)
