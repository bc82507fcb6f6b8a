"""O1: brute-force state-vector simulation in complex128.

The amplitude <x|U|0...0> (Sec. 2.2) computed by applying every gate of the
circuit, in order, to the full state stored as an array of shape [d]*n.
Qudit q is axis q; the outcome string x indexes the array directly, so the
flat state index is sum_q x_q d^(n-1-q).

Gradient: the adjoint method (Jones & Gacon, "Efficient calculation of
gradients in classical simulations of variational quantum algorithms", 2020):
one forward pass, then the gates are undone one by one while a co-state is
carried backwards; dL/dp = 2 Re <chi| dU/dp |psi_before> (times the loss's
prefactor).
"""

import numpy as np


def apply_gate(psi, u, qudits, d):
    k = len(qudits)
    ut = np.asarray(u).reshape([d] * (2 * k))
    out = np.tensordot(ut, psi, axes=(list(range(k, 2 * k)), list(qudits)))
    return np.moveaxis(out, list(range(k)), list(qudits))


def final_state(circ):
    psi = np.zeros([circ.d] * circ.n, dtype=np.complex128)
    psi[(0,) * circ.n] = 1.0
    for op in circ.ops:
        psi = apply_gate(psi, op.matrix, op.qudits, circ.d)
    return psi


def amplitudes(circ, outcomes):
    psi = final_state(circ)
    outcomes = np.atleast_2d(np.asarray(outcomes, np.int64))
    return np.array([psi[tuple(x)] for x in outcomes])


def fsim_matrix(theta, phi):
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[1, 0, 0, 0], [0, c, -1j * s, 0], [0, -1j * s, c, 0],
                     [0, 0, 0, np.exp(-1j * phi)]], dtype=np.complex128)


def dfsim(theta, phi):
    """Partial derivatives of fsim_matrix with respect to theta and phi."""
    c, s = np.cos(theta), np.sin(theta)
    dt = np.array([[0, 0, 0, 0], [0, -s, -1j * c, 0], [0, -1j * c, -s, 0], [0, 0, 0, 0]],
                  dtype=np.complex128)
    dp = np.zeros((4, 4), np.complex128)
    dp[3, 3] = -1j * np.exp(-1j * phi)
    return dt, dp


def with_params(circ, params):
    """Copy of a trainable circuit whose fSim gates take ``params`` (n, 2)."""
    import copy
    c2 = copy.copy(circ)
    c2.ops = []
    for op in circ.ops:
        o = copy.copy(op)
        if op.param is not None:
            o.matrix = fsim_matrix(*params[op.param])
        c2.ops.append(o)
    c2.params = np.array(params, dtype=np.float64)
    return c2


def nll_loss(circ, batch):
    """L = -mean_b log |amp(x_b)|^2."""
    a = amplitudes(circ, batch)
    return float(-np.mean(np.log(np.abs(a) ** 2)))


def nll_grad(circ, batch):
    """(L, dL/d(theta, phi)) by the adjoint method; shape (n_param, 2)."""
    d, n = circ.d, circ.n
    batch = np.asarray(batch, np.int64)
    nb = batch.shape[0]
    psi = final_state(circ)
    amps = np.array([psi[tuple(x)] for x in batch])
    loss = float(-np.mean(np.log(np.abs(amps) ** 2)))
    # dL = -(2/B) Re sum_b c_b d(amp_b),  c_b = conj(amp_b) / |amp_b|^2
    c = np.conj(amps) / np.abs(amps) ** 2
    chi = np.zeros_like(psi)
    for b in range(nb):
        chi[tuple(batch[b])] += np.conj(c[b])
    grad = np.zeros((len(circ.params), 2))
    for op in reversed(circ.ops):
        udag = op.matrix.conj().T
        psi = apply_gate(psi, udag, op.qudits, d)
        if op.param is not None:
            th, ph = circ.params[op.param]
            for j, du in enumerate(dfsim(th, ph)):
                g = np.vdot(chi, apply_gate(psi, du, op.qudits, d))
                grad[op.param, j] += -2.0 / nb * g.real
        chi = apply_gate(chi, udag, op.qudits, d)
    return loss, grad
