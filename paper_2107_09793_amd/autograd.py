"""torch.autograd face of the library.

``Amplitude.apply(plan, *leaves)`` returns the contraction (complex128) and,
on backward, calls tn_contract_backward for the leaf gradients (PyTorch's
convention for complex tensors: dL/dRe + i dL/dIm).  Gradients with respect
to gate parameters follow from torch's chain rule through the differentiable
leaf construction below.
"""

import torch


class Amplitude(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, *leaves):
        ctx.plan = plan
        ctx.save_for_backward(*leaves)
        return plan.contract(list(leaves))

    @staticmethod
    def backward(ctx, grad_out):
        leaves = ctx.saved_tensors
        grads = [torch.zeros_like(x) if ctx.needs_input_grad[i + 1] else None
                 for i, x in enumerate(leaves)]
        ctx.plan.backward(list(leaves), grad_out, grads)
        return (None, *grads)


def fsim(theta, phi):
    """fSim(theta, phi) in the basis |00>,|01>,|10>,|11> as a complex64 tensor
    of shape (2, 2, 2, 2) = [out_a, out_b, in_a, in_b], differentiable in
    theta and phi (real float64 scalars)."""
    c = torch.cos(theta)
    s = torch.sin(theta)
    zero = torch.zeros_like(c)
    one = torch.ones_like(c)
    re = torch.stack([one, zero, zero, zero,
                      zero, c, zero, zero,
                      zero, zero, c, zero,
                      zero, zero, zero, torch.cos(phi)])
    im = torch.stack([zero, zero, zero, zero,
                      zero, zero, -s, zero,
                      zero, -s, zero, zero,
                      zero, zero, zero, -torch.sin(phi)])
    return torch.complex(re, im).to(torch.complex64).reshape(2, 2, 2, 2)


def circuit_leaves(tn, circuit, params, device):
    """Leaves of a network built from a trainable circuit: every fSim leaf
    with a parameter index is rebuilt from ``params`` (n_param x 2 float64
    tensor, requires_grad for gradients); the other leaves are constants."""
    out = []
    for t, oi in zip(tn.tensors, tn.leaf_op):
        op = circuit.ops[oi]
        if op.param is not None and t.shape == (2, 2, 2, 2):
            out.append(fsim(params[op.param, 0], params[op.param, 1]).to(device))
        else:
            out.append(torch.from_numpy(t.astype("complex64")).to(device))
    return out


def fsim_batch(theta, phi):
    """fSim gates of a vector of angles: an (n, 2, 2, 2, 2) complex64 tensor,
    entry i equal to ``fsim(theta[i], phi[i])``, differentiable in both."""
    c = torch.cos(theta)
    s = torch.sin(theta)
    zero = torch.zeros_like(c)
    one = torch.ones_like(c)
    re = torch.stack([one, zero, zero, zero,
                      zero, c, zero, zero,
                      zero, zero, c, zero,
                      zero, zero, zero, torch.cos(phi)], dim=1)
    im = torch.stack([zero, zero, zero, zero,
                      zero, zero, -s, zero,
                      zero, -s, zero, zero,
                      zero, zero, zero, -torch.sin(phi)], dim=1)
    return torch.complex(re, im).to(torch.complex64).reshape(-1, 2, 2, 2, 2)


class CircuitLeaves:
    """Leaves of a trainable circuit's network for repeated evaluation: the
    constant leaves go to the device once; the parameterised fSim leaves are
    formed from the parameters in one batched expression and travel to the
    device as one tensor (rows in ``gate_leaf`` order)."""

    def __init__(self, tn, circuit, device):
        self.device = device
        self.n = len(tn.tensors)
        self.gate_leaf, gate_param = [], []
        self.const = [None] * self.n
        for j, (t, oi) in enumerate(zip(tn.tensors, tn.leaf_op)):
            op = circuit.ops[oi]
            if op.param is not None and t.shape == (2, 2, 2, 2):
                self.gate_leaf.append(j)
                gate_param.append(op.param)
            else:
                self.const[j] = torch.from_numpy(t.astype("complex64")).to(device)
        self.gate_param = torch.tensor(gate_param, dtype=torch.long)

    def gates(self, params):
        """(n_gates, 2, 2, 2, 2) device tensor of the fSim leaves."""
        p = params[self.gate_param]
        return fsim_batch(p[:, 0], p[:, 1]).to(self.device)

    def assemble(self, gates):
        leaves = list(self.const)
        for i, j in enumerate(self.gate_leaf):
            leaves[j] = gates[i]
        return leaves


class CircuitAmplitude(torch.autograd.Function):
    """The contraction as a function of the stacked fSim leaves: forward is
    tn_contract on the assembled leaves, backward one tn_contract_backward
    that writes the gate gradients straight into one (n_gates, 2, 2, 2, 2)
    tensor (no gradients are formed for the constant leaves)."""

    @staticmethod
    def forward(ctx, plan, builder, gates):
        ctx.plan = plan
        ctx.builder = builder
        ctx.save_for_backward(gates)
        return plan.contract(builder.assemble(gates))

    @staticmethod
    def backward(ctx, grad_out):
        (gates,) = ctx.saved_tensors
        b = ctx.builder
        g = torch.zeros_like(gates)
        grads = [None] * b.n
        for i, j in enumerate(b.gate_leaf):
            grads[j] = g[i]
        ctx.plan.backward(b.assemble(gates), grad_out, grads)
        return None, None, g
