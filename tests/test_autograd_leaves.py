"""The torch glue of the gradient path, on the CPU: the batched fSim leaves
equal the per-gate construction and the generator's gate tensors (the network
builder's own fSim), and the builder puts every parameterised leaf where the
network has it."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2107_09793_amd.autograd import CircuitLeaves, fsim, fsim_batch  # noqa: E402
from tngen import gates, workloads  # noqa: E402


def test_fsim_batch_matches_single_gates_and_generator():
    rng = np.random.default_rng(0)
    th = torch.tensor(rng.uniform(0, np.pi, 7), dtype=torch.float64)
    ph = torch.tensor(rng.uniform(0, np.pi, 7), dtype=torch.float64)
    b = fsim_batch(th, ph)
    assert b.shape == (7, 2, 2, 2, 2) and b.dtype == torch.complex64
    for i in range(7):
        assert torch.equal(b[i], fsim(th[i], ph[i]))
        ref = gates.fsim(float(th[i]), float(ph[i])).reshape(2, 2, 2, 2)
        assert np.allclose(b[i].numpy(), ref, atol=1e-7)


def test_circuit_leaves_reproduce_the_network():
    w = workloads.build("gradient", seed=0)
    params = torch.tensor(w.circuit.params, dtype=torch.float64, requires_grad=True)
    cl = CircuitLeaves(w.tn, w.circuit, torch.device("cpu"))
    g = cl.gates(params)
    assert g.shape[0] == len(cl.gate_leaf) == len(w.circuit.params)
    leaves = cl.assemble(g)
    assert len(leaves) == len(w.tn.tensors)
    for t, x in zip(w.tn.tensors, leaves):
        assert np.allclose(x.detach().numpy(), t, atol=1e-6)
    # the parameters reach the loss through the stacked gates
    (g.real.sum() + g.imag.sum()).backward()
    assert params.grad is not None and torch.count_nonzero(params.grad) > 0
