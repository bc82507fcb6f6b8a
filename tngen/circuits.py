"""Seeded circuit generators.

A circuit is a list of gate applications on qudits of one dimension ``d``,
applied to |0...0>.  Gate matrices act on the listed qudits with the first
listed qudit most significant (``U[d*out_a + out_b, d*in_a + in_b]``).

Generators
----------
* ``grid_rqc``   Sycamore-style random circuit on a rectangular grid (Sec. 4:
                 Sycamore-53 circuits with fSim two-qubit gates, Fig. 6).
                 Coupler classes A-D and the cycle sequence ABCDCDAB are the
                 reading used for a rectangular lattice (the paper's circuit
                 files are not reproduced).
* ``gbs_like``   bosonic-mode network following the loop order of Alg. 1
                 (random n-dimensional GBS circuit) with Haar-random
                 two-mode gates in a truncated Fock space of dimension d.
* ``ghz``, ``v_vdag``, ``product``  closed-form circuits used as pins.

Seeds: ``numpy.random.default_rng([seed, 0])`` draws the circuit; draw order is
cycle-major, sites row-major, gates in application order.
"""

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

from . import gates as G


@dataclass
class Op:
    qudits: Tuple[int, ...]
    matrix: np.ndarray               # (d^k, d^k) complex128
    name: str = ""
    param: Optional[int] = None      # trainable fSim: index of (theta, phi) pair


@dataclass
class Circuit:
    n: int
    d: int
    ops: List[Op] = field(default_factory=list)
    params: Optional[np.ndarray] = None   # (n_param, 2) theta, phi for trainable fSim
    meta: dict = field(default_factory=dict)

    def add(self, qudits, matrix, name="", param=None):
        self.ops.append(Op(tuple(int(q) for q in qudits), np.asarray(matrix, np.complex128), name, param))


def grid_couplers(rows, cols, inactive=()):
    """Active-site numbering and the four coupler classes of a grid.

    Site (r, c) becomes qubit q = its row-major rank among active sites.
    A: (r,c)-(r,c+1) with r+c even; B: same with r+c odd;
    C: (r,c)-(r+1,c) with r+c even; D: same with r+c odd.
    Each class is a matching.  Couplers touching an inactive site are dropped.
    """
    inactive = set(tuple(s) for s in inactive)
    sites = [(r, c) for r in range(rows) for c in range(cols) if (r, c) not in inactive]
    qid = {s: i for i, s in enumerate(sites)}
    classes = {"A": [], "B": [], "C": [], "D": []}
    for (r, c) in sites:
        even = (r + c) % 2 == 0
        if (r, c + 1) in qid:
            classes["A" if even else "B"].append((qid[(r, c)], qid[(r, c + 1)]))
        if (r + 1, c) in qid:
            classes["C" if even else "D"].append((qid[(r, c)], qid[(r + 1, c)]))
    return sites, classes


def grid_rqc(rows, cols, depth, seed, inactive=(), pattern="ABCDCDAB",
             theta=np.pi / 2, phi=np.pi / 6, trainable=False, no_repeat=False):
    """Sycamore-style random circuit.

    Each cycle: a layer of single-qubit gates drawn uniformly from
    {sqrt(X), sqrt(Y), sqrt(W)} on every active qubit, then fSim on every
    coupler of class ``pattern[t % len(pattern)]``.  One final single-qubit
    layer closes the circuit.  With ``trainable`` every fSim gets its own
    (theta_i, phi_i) ~ U(0, pi) (drawn after the circuit, in gate order).
    """
    rng = np.random.default_rng([seed, 0])
    sites, classes = grid_couplers(rows, cols, inactive)
    n = len(sites)
    circ = Circuit(n=n, d=2, meta=dict(kind="grid_rqc", rows=rows, cols=cols, depth=depth,
                                       seed=seed, inactive=[list(s) for s in inactive],
                                       pattern=pattern))
    last = [-1] * n

    def one_qubit_layer():
        for q in range(n):
            if no_repeat and last[q] >= 0:
                k = int(rng.integers(0, 2))
                k = [i for i in range(3) if i != last[q]][k]
            else:
                k = int(rng.integers(0, 3))
            last[q] = k
            circ.add((q,), G.ONE_QUBIT_SET[k], G.ONE_QUBIT_NAMES[k])

    two_qubit = []
    for t in range(depth):
        one_qubit_layer()
        for (a, b) in classes[pattern[t % len(pattern)]]:
            two_qubit.append(len(circ.ops))
            circ.add((a, b), G.fsim(theta, phi), "fsim")
    one_qubit_layer()
    if trainable:
        prng = np.random.default_rng([seed, 4])
        params = prng.uniform(0.0, np.pi, size=(len(two_qubit), 2))
        for i, oi in enumerate(two_qubit):
            circ.ops[oi].param = i
            circ.ops[oi].matrix = G.fsim(params[i, 0], params[i, 1])
        circ.params = params
    return circ


def gbs_like(rows, cols, depth, seed, d=4, literal=False):
    """Bosonic-mode network with the loop order of Alg. 1 (dim = 2 lattice).

    For each cycle, for l = 1, 2 (stride width^(l-1)), for i ascending, a gate
    acts on modes (i, i + stride).  Pairs that wrap around a row end are
    skipped unless ``literal`` (then every pair of Alg. 1 is kept).  Each gate
    is a Haar-random d^2 x d^2 unitary; the input is the vacuum |0>^modes and
    no squeezers are applied (their Fock matrix elements are not given).
    """
    rng = np.random.default_rng([seed, 0])
    modes = rows * cols
    llens = [1, cols]
    circ = Circuit(n=modes, d=d, meta=dict(kind="gbs_like", rows=rows, cols=cols, depth=depth,
                                           seed=seed, d=d, literal=literal))
    for _ in range(depth):
        for stride in llens:
            for i in range(modes - stride):
                if stride == 1 and not literal and (i + 1) % cols == 0:
                    continue
                circ.add((i, i + stride), G.haar_unitary(d * d, rng), "haar")
    return circ


def gbs_optical(rows, cols, cycles, seed, d=4, r=0.5, layers=1):
    """Random GBS circuit of Alg. 1 on a rows x cols lattice (dim = 2, width =
    ``cols``) or, with ``layers`` > 1, on a layers x rows x cols lattice
    (dim = 3, strides 1, cols and rows*cols): a squeezer S(r) on every mode,
    then per cycle, for each stride in ascending order and i ascending, a
    beam splitter BS(theta, phi) on modes (i, i + stride) with theta, phi ~
    U(0, 2 pi) -- every pair of the algorithm, wraps included.  Gates are the
    truncated Fock-space operators at cutoff ``d`` (``gates.squeezer``,
    ``gates.beam_splitter``).  The paper's GBS-88-m1 is
    ``gbs_optical(8, 8, 1, seed, d, r=0.5)`` and its GBS-444-m1 is
    ``gbs_optical(4, 4, 1, seed, 4, r, layers=4)``."""
    rng = np.random.default_rng([seed, 0])
    modes = layers * rows * cols
    llens = [1, cols] + ([rows * cols] if layers > 1 else [])
    circ = Circuit(n=modes, d=d, meta=dict(kind="gbs_optical", rows=rows, cols=cols,
                                           layers=layers, cycles=cycles, seed=seed, d=d,
                                           r=r))
    S = G.squeezer(r, d)
    for k in range(modes):
        circ.add((k,), S, "squeezer")
    for _ in range(cycles):
        for stride in llens:
            for i in range(modes - stride):
                theta = float(rng.uniform(0.0, 2.0 * np.pi))
                phi = float(rng.uniform(0.0, 2.0 * np.pi))
                circ.add((i, i + stride), G.beam_splitter(theta, phi, d), "bs")
    return circ


def gbs_pattern(n, d, r, seed):
    """A seeded GBS output pattern of typical size: each mode's photon count
    drawn from a geometric distribution with the mean photon number of a
    squeezed vacuum, sinh(r)^2, cut at d - 1, then made even in total
    (``even_total``)."""
    rng = np.random.default_rng([seed, 1])
    mean = np.sinh(r) ** 2
    p = 1.0 / (1.0 + mean)                  # geometric on {0, 1, ...} with that mean
    x = np.minimum(rng.geometric(p, size=n) - 1, d - 1)
    return even_total(x)


def even_total(pattern):
    """A GBS output pattern with an even total photon number: squeezed vacua
    hold even photon numbers only and beam splitters conserve the total, so
    any pattern with an odd total has amplitude exactly 0.  An odd total is
    made even by flipping the last entry between 2k and 2k + 1."""
    x = np.array(pattern, dtype=np.int64)
    if int(x.sum()) % 2:
        x[-1] ^= 1
    return x


def ghz(n):
    circ = Circuit(n=n, d=2, meta=dict(kind="ghz", n=n))
    circ.add((0,), G.H, "h")
    for q in range(n - 1):
        circ.add((q, q + 1), G.CNOT, "cnot")
    return circ


def product(n, seed):
    """Random single-qubit Haar gate on every qubit: amplitude factorises."""
    rng = np.random.default_rng([seed, 0])
    circ = Circuit(n=n, d=2, meta=dict(kind="product", n=n, seed=seed))
    for q in range(n):
        circ.add((q,), G.haar_unitary(2, rng), "haar1")
    return circ


def v_vdag(base):
    """Circuit V followed by V^dagger: the final state is |0...0>."""
    circ = Circuit(n=base.n, d=base.d, meta=dict(kind="v_vdag", base=base.meta))
    for op in base.ops:
        circ.add(op.qudits, op.matrix, op.name)
    for op in reversed(base.ops):
        circ.add(op.qudits, op.matrix.conj().T, op.name + "_dag")
    return circ


def random_bitstrings(n, d, count, seed):
    """``count`` seeded outcome strings, uniform over {0..d-1}^n."""
    rng = np.random.default_rng([seed, 1])
    return rng.integers(0, d, size=(count, n)).astype(np.int64)
