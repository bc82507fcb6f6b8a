"""Optical GBS gates in the truncated Fock basis (Alg. 1: squeezer S(r) and
beam splitter BS(theta, phi)) and the GBS circuit built from them, on the
CPU, pinned against closed forms and an independent derivation:

* S(r e^{i psi})|0> = cosh(r)^-1/2 sum_n (-e^{i psi} tanh r)^n sqrt((2n)!)
  / (2^n n!) |2n> (the squeezed vacuum);
* BS conserves the total photon number; BS(0, phi) = I; on one photon it is
  the mode rotation [[cos t, -e^{-i phi} sin t], [e^{i phi} sin t, cos t]];
  a 50:50 splitter never sends |1,1> to |1,1> (Hong-Ou-Mandel); every block
  of total photon number below the cutoff is unitary; all entries agree
  with the binomial expansion of the transformed creation operators;
* Alg. 1's gate counts, and the network's contraction (oracle, greedy path)
  equals the state vector of a small GBS circuit; odd-total patterns have
  amplitude zero.
"""

import math

import numpy as np
import pytest

from oracle import statevector as sv
from oracle import tn_oracle
from tngen import circuits, gates as G, network, path as tpath


@pytest.mark.parametrize("r,psi,d", [(0.5, 0.0, 8), (0.3, 1.1, 4), (0.8, -0.4, 8)])
def test_squeezed_vacuum_closed_form(r, psi, d):
    S = G.squeezer(r, d, psi)
    ref = np.zeros(d, np.complex128)
    for n in range((d + 1) // 2):
        ref[2 * n] = ((-np.exp(1j * psi) * np.tanh(r)) ** n * math.sqrt(math.factorial(2 * n))
                      / (2 ** n * math.factorial(n) * math.sqrt(np.cosh(r))))
    assert np.allclose(S[:, 0], ref, atol=1e-13)
    # the block has converged in the space it is computed in
    assert np.allclose(S, G.squeezer(r, d, psi, extra=200), atol=1e-13)
    # S(z) S(-z) = I on photon numbers far below the cutoff of the product space
    big = G.squeezer(r, d + 100, psi) @ G.squeezer(r, d + 100, psi + np.pi)
    assert np.allclose(big[:d, :d], np.eye(d), atol=1e-9)


def _bs_formula(theta, phi, d):
    """<m_a m_b|U|n_a n_b> from U adag U^-1 = c adag + e^{i phi} s bdag and
    U bdag U^-1 = -e^{-i phi} s adag + c bdag, expanded binomially."""
    c, s = np.cos(theta), np.sin(theta)
    U = np.zeros((d * d, d * d), np.complex128)
    for na in range(d):
        for nb in range(d):
            for j in range(na + 1):          # j of the n_a factors give adag
                for k in range(nb + 1):      # k of the n_b factors give adag
                    ma, mb = j + k, na - j + nb - k
                    if ma >= d or mb >= d:
                        continue
                    coef = (math.comb(na, j) * math.comb(nb, k) * c ** j *
                            (np.exp(1j * phi) * s) ** (na - j) * (-np.exp(-1j * phi) * s) ** k *
                            c ** (nb - k))
                    U[d * ma + mb, d * na + nb] += coef * math.sqrt(
                        math.factorial(ma) * math.factorial(mb) /
                        (math.factorial(na) * math.factorial(nb)))
    return U


@pytest.mark.parametrize("theta,phi,d", [(0.7, 2.1, 4), (np.pi / 4, 0.3, 8), (2.9, 5.0, 8)])
def test_beam_splitter(theta, phi, d):
    U = G.beam_splitter(theta, phi, d)
    assert np.allclose(U, _bs_formula(theta, phi, d), atol=1e-12)
    tot = np.array([a + b for a in range(d) for b in range(d)])
    assert np.all(np.abs(U[tot[:, None] != tot[None, :]]) < 1e-14)
    for n in range(d):
        blk = np.where(tot == n)[0]
        B = U[np.ix_(blk, blk)]
        assert np.allclose(B.conj().T @ B, np.eye(len(blk)), atol=1e-12)
    one = [d * 1 + 0, d * 0 + 1]                   # |1,0>, |0,1>
    c, s = np.cos(theta), np.sin(theta)
    rot = np.array([[c, -np.exp(-1j * phi) * s], [np.exp(1j * phi) * s, c]])
    assert np.allclose(U[np.ix_(one, one)], rot, atol=1e-13)
    assert np.allclose(G.beam_splitter(0.0, phi, d), np.eye(d * d), atol=1e-14)
    hom = G.beam_splitter(np.pi / 4, phi, d)[d + 1, d + 1]
    assert abs(hom) < 1e-13


def test_gbs_circuit_and_network():
    circ = circuits.gbs_optical(2, 3, 2, seed=1, d=4, r=0.5)
    modes = 6
    assert sum(op.name == "squeezer" for op in circ.ops) == modes
    assert sum(op.name == "bs" for op in circ.ops) == 2 * ((modes - 1) + (modes - 3))
    psi = sv.final_state(circ).reshape(-1)
    for seed in range(3):
        x = circuits.gbs_pattern(modes, 4, 0.5, seed)
        assert int(x.sum()) % 2 == 0
        tn = network.relabel_compact(network.circuit_network(circ, outcome=x))
        p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
        got = complex(tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p))
        idx = int(sum(int(v) * 4 ** (modes - 1 - q) for q, v in enumerate(x)))
        assert abs(got - psi[idx]) <= 1e-12
    odd = np.where(np.array([sum(np.base_repr(i, 4).rjust(modes, "0")[q] != "0" and
                                 int(np.base_repr(i, 4).rjust(modes, "0")[q]) for q in
                                 range(modes)) % 2 for i in range(4 ** modes)]))[0]
    assert np.max(np.abs(psi[odd])) < 1e-14


def test_three_dimensional_lattice():
    """Alg. 1 with dim = 3: strides 1, width and width^2, wraps included; the
    tensor network of a 2x2x2 lattice equals the state vector."""
    circ = circuits.gbs_optical(2, 2, 1, seed=4, d=4, r=0.5, layers=2)
    modes = 8
    pairs = [op.qudits for op in circ.ops if op.name == "bs"]
    assert pairs == ([(i, i + 1) for i in range(7)] + [(i, i + 2) for i in range(6)] +
                     [(i, i + 4) for i in range(4)])
    psi = sv.final_state(circ)
    for seed in range(2):
        x = circuits.gbs_pattern(modes, 4, 0.5, seed)
        tn = network.relabel_compact(network.circuit_network(circ, outcome=x))
        p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
        got = complex(tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p))
        assert abs(got - psi[tuple(x)]) <= 1e-12
