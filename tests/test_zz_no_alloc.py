"""tn_contract_noalloc (the library's static per-GPU workspace, no device
allocation in the call) against tn_contract with a caller workspace, through
the C ABI: two calls in a row, the second on a smaller network, per-slice and
summed results within the complex64 tolerance (1e-5 of the rms slice); a plan
whose workspace exceeds the static array is rejected with TN_E_WORKSPACE."""

import numpy as np
import pytest

from tngen import circuits, network, path as tpath, slicing

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _net(rows, cols, depth, seed, n_slice):
    circ = circuits.grid_rqc(rows, cols, depth, seed=seed)
    x = circuits.random_bitstrings(circ.n, 2, 1, seed)[0]
    tn = network.relabel_compact(network.circuit_network(circ, outcome=x))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    sl = slicing.greedy_slices(slicing.TreeSets(tn.labels, tn.dims, tn.open, p),
                               n_slice=n_slice)
    return tn, p, sl


def test_noalloc_matches_contract_two_calls():
    from paper_2107_09793_amd import Plan
    from paper_2107_09793_amd.binding import NOALLOC_WORKSPACE_BYTES
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    # the second call's network is smaller (fewer qubits, fewer slices)
    for rows, cols, depth, seed, n_slice in ((4, 4, 8, 5, 5), (3, 4, 8, 1, 2)):
        tn, p, sl = _net(rows, cols, depth, seed, n_slice)
        pl = Plan(tn.labels, tn.dims, tn.open, p, sl)
        assert pl.info()["workspace_bytes"] <= NOALLOC_WORKSPACE_BYTES
        leaves = [torch.from_numpy(np.ascontiguousarray(t, dtype=np.complex64)).to(dev)
                  for t in tn.tensors]
        ref = pl.contract(leaves, per_slice=True)
        out = torch.full_like(ref, float("nan"))
        pl.contract_noalloc(leaves, out, per_slice=True)
        ref_sum = pl.contract(leaves)
        out_sum = torch.full_like(ref_sum, float("nan"))
        pl.contract_noalloc(leaves, out_sum)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy().reshape(-1), ref.cpu().numpy().reshape(-1)
        rms = np.sqrt(np.mean(np.abs(b) ** 2))
        assert np.all(np.isfinite(a))
        assert np.max(np.abs(a - b)) <= 1e-5 * rms, (rows, cols)
        s, r = complex(out_sum.cpu().item()), complex(ref_sum.cpu().item())
        assert abs(s - r) <= 1e-5 * rms * len(b), (rows, cols)


def test_noalloc_rejects_plan_larger_than_static_workspace():
    from paper_2107_09793_amd import Plan
    from paper_2107_09793_amd.binding import NOALLOC_WORKSPACE_BYTES, TN_E_WORKSPACE, TnError
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    tn, p, sl = _net(5, 5, 10, 2, 0)
    big = Plan(tn.labels, tn.dims, tn.open, p, sl)
    if big.info()["workspace_bytes"] <= NOALLOC_WORKSPACE_BYTES:
        pytest.skip("network too small for the rejection case")
    leaves = [torch.from_numpy(np.ascontiguousarray(t, dtype=np.complex64)).to(dev)
              for t in tn.tensors]
    out = torch.empty((), dtype=torch.complex128, device=dev)
    with pytest.raises(TnError) as e:
        big.contract_noalloc(leaves, out)
    assert e.value.status == TN_E_WORKSPACE
