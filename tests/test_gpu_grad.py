"""Adjoint (tn_contract_backward) and the autograd path on the GPU.

1. Leaf gradients: the amplitude is linear in every leaf, so for a direction
   D the oracle's contraction with leaf j replaced by D is exactly
   sum(env_j * D); the library's leaf gradient g_j (PyTorch convention, with
   output gradient w) must satisfy sum(conj(g_j) * D) = sum_o conj(w_o) *
   contraction_o(leaf_j := D).
2. Gate-parameter gradients of L = -mean log|amp|^2 for the trainable fSim
   circuit (4x5 grid, depth 10, 256 outcomes) through Amplitude.apply and
   torch autograd, against the state-vector adjoint (complex128) and central
   finite differences (h = 1e-4, float64).
Tolerance: 1e-5 relative for complex64 leaf gradients (norm-wise); the
parameter gradient, which divides by |amp|^2, is checked at 1e-4 norm-wise.
"""

import numpy as np
import pytest

from oracle import grad as ograd
from oracle import statevector as sv
from oracle import tn_oracle
from tngen import circuits, network, path as tpath, slicing, workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("precision,tol", [("c64", 1e-5), ("split_bf16", 1e-3)])
def test_leaf_gradients_directional(precision, tol):
    from paper_2107_09793_amd import Plan
    dev = _dev()
    circ = circuits.grid_rqc(3, 4, 8, seed=6)
    batch = circuits.random_bitstrings(12, 2, 16, 6)
    tn = network.relabel_compact(network.circuit_network(circ, batch=batch))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    ts = slicing.TreeSets(tn.labels, tn.dims, tn.open, p)
    sl = slicing.greedy_slices(ts, n_slice=3)
    pl = Plan(tn.labels, tn.dims, tn.open, p, sl, precision=precision)
    leaves = [torch.from_numpy(t.astype(np.complex64)).to(dev) for t in tn.tensors]
    rng = np.random.default_rng(11)
    w = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    grads = [torch.zeros_like(x) for x in leaves]
    pl.backward(leaves, torch.from_numpy(w).to(dev), grads)
    torch.cuda.synchronize()
    for j in rng.choice(len(leaves), size=8, replace=False):
        D = rng.standard_normal(tn.tensors[j].shape) + 1j * rng.standard_normal(tn.tensors[j].shape)
        ts2 = list(tn.tensors)
        ts2[j] = D
        lin = tn_oracle.contract(ts2, tn.labels, tn.dims, tn.open, p, sl)
        expect = np.sum(np.conj(w) * lin)
        g = grads[j].cpu().numpy().astype(np.complex128)
        got = np.sum(np.conj(g) * D)
        scale = np.sqrt(np.sum(np.abs(w) ** 2) * np.sum(np.abs(lin) ** 2))
        assert abs(got - expect) <= tol * scale, (j, got, expect)


def test_gate_parameter_gradients():
    from paper_2107_09793_amd import Plan
    from paper_2107_09793_amd.autograd import Amplitude, circuit_leaves
    dev = _dev()
    wl = workloads.build("gradient", seed=0)
    circ, tn = wl.circuit, wl.tn
    pl = Plan.from_network(tn, wl.path, wl.sliced)
    params = torch.tensor(circ.params, dtype=torch.float64, requires_grad=True)
    leaves = circuit_leaves(tn, circ, params, dev)
    amp = Amplitude.apply(pl, *leaves)
    loss = -torch.mean(torch.log(torch.abs(amp) ** 2))
    loss.backward()
    g_gpu = params.grad.numpy()
    ref_loss, g_ref = sv.nll_grad(circ, wl.batch)
    assert abs(loss.item() - ref_loss) <= 1e-5 * abs(ref_loss)
    err = np.linalg.norm(g_gpu - g_ref) / np.linalg.norm(g_ref)
    assert err <= 1e-4, err
    # finite differences on a few parameters (the oracle's own loss)
    sub = [0, 1, 17, 88, 155]
    fd = ograd.fd_grad(circ, wl.batch, subset=sub)
    idx = [(k // 2, k % 2) for k in sub]
    fdv = np.array([fd[i] for i in idx])
    gv = np.array([g_gpu[i] for i in idx])
    assert np.max(np.abs(gv - fdv)) <= 1e-4 * max(1.0, np.max(np.abs(fdv)))
