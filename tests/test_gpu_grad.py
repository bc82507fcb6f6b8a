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
Tolerance: the stated complex64 tolerance, 1e-5 (1e-3 for split-BF16),
norm-wise: a directional derivative sum(conj(g) * D) is compared within
tol * ||g|| ||D|| (the Cauchy-Schwarz bound of the inner product, so a result
that cancels is not judged against its own small size), the parameter
gradient within tol of its norm, and each checked parameter against finite
differences within tol * max(1, |gradient|).
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


CASES = [("c64", "all", -1, None), ("split_bf16", "all", -1, None),
         ("c64", "recompute", -1, None), ("c64", "recompute", 1, None),
         ("c64", "all", 1, [5, 0, 6, 2, 5]), ("split_bf16", "recompute", 1, [3, 4])]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_leaf_gradients_directional(case):
    """Checkpoint policies (store everything / recompute inside blocks),
    outer iterations (max_resident_bits=1) and slice subsets (a slice listed
    twice counts twice), against the oracle."""
    from paper_2107_09793_amd import Plan
    precision, policy, mrb, sids = CASES[case]
    tol = 1e-5 if precision == "c64" else 1e-3
    dev = _dev()
    circ = circuits.grid_rqc(3, 4, 8, seed=6)
    batch = circuits.random_bitstrings(12, 2, 16, 6)
    tn = network.relabel_compact(network.circuit_network(circ, batch=batch))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    ts = slicing.TreeSets(tn.labels, tn.dims, tn.open, p)
    sl = slicing.greedy_slices(ts, n_slice=3)
    pl = Plan(tn.labels, tn.dims, tn.open, p, sl, precision=precision, checkpoint=policy,
              max_resident_bits=mrb)
    if mrb >= 0:
        assert pl.info()["n_outer_bits"] >= 2
    leaves = [torch.from_numpy(t.astype(np.complex64)).to(dev) for t in tn.tensors]
    rng = np.random.default_rng(11)
    w = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    grads = [torch.zeros_like(x) for x in leaves]
    pl.backward(leaves, torch.from_numpy(w).to(dev), grads, slice_ids=sids)
    torch.cuda.synchronize()
    for j in rng.choice(len(leaves), size=8, replace=False):
        D = rng.standard_normal(tn.tensors[j].shape) + 1j * rng.standard_normal(tn.tensors[j].shape)
        ts2 = list(tn.tensors)
        ts2[j] = D
        lin = tn_oracle.contract(ts2, tn.labels, tn.dims, tn.open, p, sl, slice_ids=sids)
        expect = np.sum(np.conj(w) * lin)
        g = grads[j].cpu().numpy().astype(np.complex128)
        got = np.sum(np.conj(g) * D)
        # norm-wise bound on an inner product: tol * ||g|| ||D|| (Cauchy-Schwarz)
        scale = np.linalg.norm(g) * np.linalg.norm(D)
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
    print("parameter gradient: norm-wise relative error", err)
    assert err <= 1e-5, err
    # finite differences on a few parameters (the oracle's own loss)
    sub = [0, 1, 17, 88, 155]
    fd = ograd.fd_grad(circ, wl.batch, subset=sub)
    idx = [(k // 2, k % 2) for k in sub]
    fdv = np.array([fd[i] for i in idx])
    gv = np.array([g_gpu[i] for i in idx])
    fd_err = np.max(np.abs(gv - fdv)) / max(1.0, np.max(np.abs(fdv)))
    print("parameter gradient vs finite differences:", fd_err)
    assert fd_err <= 1e-5, fd_err


def _full_size_directional(pl, w_tn, n_dirs=3, seed=3):
    """Adjoint identity at full size: sum(conj(g_j) * D) equals
    conj(w) . contraction(leaf j := D), the contraction by the library's
    forward path (itself compared with the oracle on every slice of this
    workload)."""
    dev = _dev()
    leaves = [torch.from_numpy(np.ascontiguousarray(t, dtype=np.complex64)).to(dev)
              for t in w_tn.tensors]
    rng = np.random.default_rng(seed)
    w = complex(rng.standard_normal(), rng.standard_normal())
    grads = [torch.zeros_like(x) for x in leaves]
    pl.backward(leaves, torch.tensor([w], dtype=torch.complex128, device=dev), grads)
    torch.cuda.synchronize()
    for j in rng.choice(len(leaves), size=n_dirs, replace=False):
        D = (rng.standard_normal(w_tn.tensors[j].shape) +
             1j * rng.standard_normal(w_tn.tensors[j].shape)).astype(np.complex64)
        l2 = list(leaves)
        l2[j] = torch.from_numpy(D).to(dev)
        lin = complex(pl.contract(l2).cpu().item())
        expect = np.conj(w) * lin
        g = grads[j].cpu().numpy().astype(np.complex128)
        got = np.sum(np.conj(g) * D)
        # norm-wise bound on an inner product: 1e-5 ||g|| ||D|| (Cauchy-Schwarz)
        scale = np.linalg.norm(g) * np.linalg.norm(D.astype(np.complex128))
        print("leaf", j, "adjoint", got, "forward", expect, "error / scale",
              abs(got - expect) / scale)
        assert abs(got - expect) <= 1e-5 * scale, (j, got, expect)


def test_full_size_gradient_with_recomputation():
    """The 30-qubit workload under a workspace cap (28 GiB) that the
    store-everything backward (about 35 GiB) exceeds: values used inside a
    block are recomputed."""
    from paper_2107_09793_amd import Plan
    _dev()
    wl = workloads.build("sliced", seed=0)
    full = Plan.from_network(wl.tn, wl.path, wl.sliced, workspace_limit=0, checkpoint="all")
    assert full.info()["workspace_backward_bytes"] > 28 << 30
    del full
    pl = Plan.from_network(wl.tn, wl.path, wl.sliced, workspace_limit=28 << 30)
    info = pl.info()
    assert info["backward_policy"] == 2 and info["cmac_backward_recompute"] > 0
    assert info["workspace_backward_bytes"] <= 28 << 30
    _full_size_directional(pl, wl.tn)


def test_full_size_gradient_with_outer_iterations():
    """The 30-qubit workload with a 20 GiB cap that the backward must also
    fit: part of the slices become outer iterations whose gradients
    accumulate."""
    from paper_2107_09793_amd import Plan
    _dev()
    wl = workloads.build("sliced", seed=0)
    pl = Plan.from_network(wl.tn, wl.path, wl.sliced, workspace_limit=20 << 30,
                           fit_backward=True)
    info = pl.info()
    assert info["n_outer_bits"] >= 1
    assert info["workspace_backward_bytes"] <= 20 << 30
    _full_size_directional(pl, wl.tn, seed=4)


@pytest.mark.parametrize("policy", ["all", "recompute"])
def test_backward_tiny_batches(policy):
    """The adjoint's tiny products (values, recomputations, adjoint products)
    run in batches of one workgroup, each product one level above the
    earlier ones of its batch whose memory it shares: the leaf gradients of
    the trainable workload (256 outcomes, every leaf) equal those of one
    launch per product within the complex64 tolerance, norm-wise, and leaf
    gradients accumulate into what the caller passes in."""
    from paper_2107_09793_amd import Plan
    dev = _dev()
    wl = workloads.build("gradient", seed=0)
    tn = wl.tn
    leaves = [torch.from_numpy(np.ascontiguousarray(t, dtype=np.complex64)).to(dev)
              for t in tn.tensors]
    rng = np.random.default_rng(7)
    gout = torch.from_numpy(rng.standard_normal(256) + 1j * rng.standard_normal(256)).to(dev)
    res = {}
    for tiny in (True, False):
        pl = Plan.from_network(tn, wl.path, wl.sliced, tiny=tiny, checkpoint=policy)
        g = [torch.zeros_like(x) for x in leaves]
        pl.backward(leaves, gout, g)
        torch.cuda.synchronize()
        res[tiny] = [x.cpu().numpy().astype(np.complex128) for x in g]
        if tiny:
            base = [torch.ones_like(x) for x in leaves]
            pl.backward(leaves, gout, base)
            torch.cuda.synchronize()
            acc = [x.cpu().numpy().astype(np.complex128) for x in base]
    a = np.concatenate([x.ravel() for x in res[True]])
    b = np.concatenate([x.ravel() for x in res[False]])
    err = np.linalg.norm(a - b) / np.linalg.norm(b)
    print(policy, "tiny batches vs one launch per product:", err)
    assert err <= 1e-5, err
    c = np.concatenate([x.ravel() for x in acc]) - 1.0
    assert np.linalg.norm(c - a) <= 1e-5 * np.linalg.norm(a)


def test_circuit_amplitude_parameter_gradients():
    """The stacked-gate path (CircuitLeaves + CircuitAmplitude: one device
    tensor of fSim leaves, gate gradients written straight into one tensor)
    gives the loss and parameter gradient of the state-vector adjoint, twice
    in a row on the same builder."""
    from paper_2107_09793_amd import Plan
    from paper_2107_09793_amd.autograd import CircuitAmplitude, CircuitLeaves
    dev = _dev()
    wl = workloads.build("gradient", seed=0)
    circ, tn = wl.circuit, wl.tn
    pl = Plan.from_network(tn, wl.path, wl.sliced)
    builder = CircuitLeaves(tn, circ, dev)
    ref_loss, g_ref = sv.nll_grad(circ, wl.batch)
    for _ in range(2):
        params = torch.tensor(circ.params, dtype=torch.float64, requires_grad=True)
        amp = CircuitAmplitude.apply(pl, builder, builder.gates(params))
        loss = -torch.mean(torch.log(torch.abs(amp) ** 2))
        loss.backward()
        assert abs(loss.item() - ref_loss) <= 1e-5 * abs(ref_loss)
        err = np.linalg.norm(params.grad.numpy() - g_ref) / np.linalg.norm(g_ref)
        print("stacked gates: parameter gradient norm-wise relative error", err)
        assert err <= 1e-5, err
