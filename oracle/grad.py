"""O3: central finite differences (h = 1e-4, float64) of the state-vector
loss L = -mean log|amp|^2 with respect to every fSim (theta, phi)."""

import numpy as np

from . import statevector as sv


def fd_grad(circ, batch, h=1e-4, subset=None):
    params = np.array(circ.params, dtype=np.float64)
    grad = np.full(params.shape, np.nan)
    idx = [(i, j) for i in range(params.shape[0]) for j in range(2)]
    if subset is not None:
        idx = [idx[k] for k in subset]
    for (i, j) in idx:
        p = params.copy()
        p[i, j] += h
        lp = sv.nll_loss(sv.with_params(circ, p), batch)
        p[i, j] -= 2 * h
        lm = sv.nll_loss(sv.with_params(circ, p), batch)
        grad[i, j] = (lp - lm) / (2 * h)
    return grad
