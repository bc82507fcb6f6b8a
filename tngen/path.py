"""Greedy pairwise contraction paths (input generation; the paper takes its
paths from an external path finder, Sec. 3, and so does this library).

Path format: SSA pairs.  Leaves are ids ``0..n-1``; step ``k`` creates id
``n+k`` from the two ids it lists.  ``n-1`` steps contract a connected network
to one tensor.

Greedy rule: among pairs of live tensors that share at least one contracted
(non-open) index, take the pair minimising ``size(out) - size(a) - size(b)``;
ties go to the smaller multiply-add count, then the smaller id pair.  Seeded
trials perturb the score with Gumbel noise.  Tensors left with no contractable
neighbour are joined smallest first at the end.
"""

import heapq
import math

import numpy as np


def _logdim(dims):
    return {i: math.log2(d) for i, d in dims.items()}


class _Tree:
    def __init__(self, labels, dims, kept):
        self.lw = _logdim(dims)
        self.kept = set(kept)
        self.sets = {i: frozenset(l) for i, l in enumerate(labels)}

    def out_of(self, a, b):
        sa, sb = self.sets[a], self.sets[b]
        common = sa & sb
        return (sa | sb) - (common - self.kept)

    def logsize(self, s):
        return sum(self.lw[i] for i in s)


def greedy_path(labels, dims, kept=(), seed=None, temperature=0.0, alpha=1.0):
    """Greedy SSA path.  ``seed=None`` -> deterministic plain greedy."""
    n = len(labels)
    tr = _Tree(labels, dims, kept)
    rng = np.random.default_rng([seed, 2]) if seed is not None else None
    holders = {}
    for t, s in tr.sets.items():
        for i in s:
            holders.setdefault(i, set()).add(t)
    alive = set(range(n))
    heap = []

    def push(a, b):
        if a > b:
            a, b = b, a
        out = tr.out_of(a, b)
        la, lb, lo = tr.logsize(tr.sets[a]), tr.logsize(tr.sets[b]), tr.logsize(out)
        score = 2.0 ** lo - alpha * (2.0 ** la + 2.0 ** lb)
        if rng is not None and temperature > 0:
            score = score / (2.0 ** la + 2.0 ** lb) - temperature * rng.gumbel()
        lmnk = tr.logsize(tr.sets[a] | tr.sets[b])
        heapq.heappush(heap, (score, lmnk, a, b))

    def neighbours(t):
        nb = set()
        for i in tr.sets[t]:
            if i in tr.kept:
                continue
            nb |= holders[i]
        nb.discard(t)
        return nb

    for t in range(n):
        for u in neighbours(t):
            if u > t:
                push(t, u)
    path = []
    nxt = n
    while heap:
        score, lmnk, a, b = heapq.heappop(heap)
        if a not in alive or b not in alive:
            continue
        out = tr.out_of(a, b)
        tr.sets[nxt] = frozenset(out)
        for i in tr.sets[a] | tr.sets[b]:
            holders[i].discard(a)
            holders[i].discard(b)
        for i in out:
            holders[i].add(nxt)
        alive -= {a, b}
        alive.add(nxt)
        path.append((a, b))
        for u in neighbours(nxt):
            push(u, nxt)
        nxt += 1
    # join disconnected remainders, smallest first
    rest = sorted(alive, key=lambda t: (tr.logsize(tr.sets[t]), t))
    while len(rest) > 1:
        a, b = rest[0], rest[1]
        out = tr.out_of(a, b)
        tr.sets[nxt] = frozenset(out)
        path.append((a, b))
        rest = sorted(rest[2:] + [nxt], key=lambda t: (tr.logsize(tr.sets[t]), t))
        nxt += 1
    return path


def check_path(n, path):
    """A path is valid iff it is a full binary tree over all n leaves."""
    used = set()
    if len(path) != n - 1:
        return False
    for k, (a, b) in enumerate(path):
        if a == b or a in used or b in used or a >= n + k or b >= n + k or a < 0 or b < 0:
            return False
        used.add(a)
        used.add(b)
    return True


def time_ordered_path(n):
    """The Schroedinger-style path: leaves absorbed one by one, in leaf order
    (circuit order for networks built by ``network.circuit_network``), into
    one running tensor, which after every gate is the state on the modes
    reached so far.  For a network with every output open its largest
    intermediate is the full state."""
    if n < 2:
        return []
    path = [(0, 1)]
    for k in range(1, n - 1):
        path.append((n + k - 1, k + 1))
    return path
