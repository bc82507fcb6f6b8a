"""Shared-work-aware refinement of a contraction tree and its sliced indices
(input generation).

Objective: the multiply-adds with shared work reused, Eq.
task_based_amplitude_flops -- every step runs once per assignment of the
sliced indices that occur below it, so its cost is 2^(sliced bits below) x
(product of the dims of its operands' other indices) -- subject to the
per-slice cap on intermediates (Sec. 2.4).  The paper slices greedily along
a fixed path (Sec. 4) and leaves finding path and slices together for later
(Sec. 5); here a seeded descent does it with two moves:

* tree rotation at a step v = (u, w) with u = (x, y): v becomes (x, (y, w));
  only the costs of v and of the new inner step change (the indices below v,
  hence its result, are unchanged), so a move is evaluated in O(1) on bit
  masks of index sets;
* slice swap: one sliced index is replaced by another index, evaluated over
  the whole tree.

A move is kept when it lowers the objective and keeps every per-slice
intermediate within the cap; moves that leave it unchanged are kept with
probability 1/2 (drifting along plateaus).  Index sets are Python integers
used as bit sets; an index of dimension 2^w weighs w.

``objective="time"`` replaces the multiply-add count by a roofline estimate
of each step on one GPU: max(multiply-adds / R, 8 bytes x (operand and
result entries, instance bits included) / BW), with R and BW the device's
complex multiply-add rate and memory bandwidth, so that steps which stream
large tensors past small ones are not taken as free.
"""

import numpy as np


class _Tree:
    def __init__(self, labels, dims, kept, path):
        self.n = len(labels)
        ids = sorted(dims)
        self.col = {i: c for c, i in enumerate(ids)}
        self.ids = ids
        wmask = {}
        for i in ids:
            w = int(dims[i]).bit_length() - 1
            wmask[w] = wmask.get(w, 0) | (1 << self.col[i])
        self.wmask = sorted(wmask.items())
        self.K = self.mask(kept)
        self.ch = {}
        self.opn, self.sub = {}, {}
        for t, lab in enumerate(labels):
            m = self.mask(lab)
            self.opn[t] = m
            self.sub[t] = m
        for k, (a, b) in enumerate(path):
            v = self.n + k
            self.ch[v] = [a, b]
            self.opn[v] = self.join(a, b)
            self.sub[v] = self.sub[a] | self.sub[b]

    def mask(self, idx):
        m = 0
        for i in idx:
            m |= 1 << self.col[i]
        return m

    def size(self, m):
        """log2 of the product of the dims of the indices in m"""
        return sum(w * bin(m & wm).count("1") for w, wm in self.wmask)

    def join(self, a, b):
        sh = self.opn[a] & self.opn[b]
        return (self.opn[a] | self.opn[b]) & ~(sh & ~self.K)

    def step_log(self, a, b, subv, S):
        return self.size((self.opn[a] | self.opn[b]) & ~S) + self.size(subv & S)

    def elems_log(self, x, S):
        """log2 entries of node x as held with every resident slice bit"""
        return self.size(self.opn[x] & ~S) + self.size(self.sub[x] & S)

    def cost(self, a, b, v, S):
        """cost of the step (a, b) -> v with the objective in effect"""
        c = 2.0 ** self.step_log(a, b, self.sub[v], S)
        if not self.timed:
            return c
        by = 8.0 * (2.0 ** self.elems_log(a, S) + 2.0 ** self.elems_log(b, S) +
                    2.0 ** self.elems_log(v, S))
        return max(c / self.rate, by / self.bw)

    def total(self, S):
        return sum(self.cost(a, b, v, S) for v, (a, b) in self.ch.items())

    def max_per_slice(self, S):
        return max((self.size(self.opn[v] & ~S) for v in self.ch), default=0)

    def path(self):
        par = set()
        for a, b in self.ch.values():
            par.add(a)
            par.add(b)
        root = [v for v in self.ch if v not in par]
        assert len(root) == 1
        out = []
        stack = [(root[0], False)]
        made = {}
        while stack:   # iterative post-order (trees can be deep)
            v, seen = stack.pop()
            if v < self.n:
                made[v] = v
                continue
            a, b = self.ch[v]
            if not seen:
                stack.append((v, True))
                stack.append((b, False))
                stack.append((a, False))
            else:
                out.append((made[a], made[b]))
                made[v] = self.n + len(out) - 1
        return out


def refine(labels, dims, kept, path, sliced, cap_log2=None, rounds=6, tree_moves=60000,
           slice_moves=1500, seed=0, objective="cmac", rate=19.66e12, bw=8e12):
    """Returns (path, sliced, objective) with an objective no larger than the
    input's; every per-slice intermediate stays within 2^cap_log2 (or within
    the input's largest, if no cap is given).  ``rate`` (complex multiply-adds
    per second) and ``bw`` (bytes per second) are used by ``objective="time"``
    (defaults: MI355X FP32 matrix cores, 157.3 TFLOP/s / 8, and 8 TB/s)."""
    tr = _Tree(labels, dims, kept, path)
    tr.timed = objective == "time"
    tr.rate, tr.bw = rate, bw
    rng = np.random.default_rng([seed, 6])
    sl = list(sliced)
    S = tr.mask(sl)
    cap = tr.max_per_slice(S) if cap_log2 is None else cap_log2
    cap = max(cap, tr.max_per_slice(S))
    cand = [i for i in tr.ids if not (tr.K >> tr.col[i]) & 1]
    internal = list(tr.ch)
    n = tr.n
    cur = tr.total(S)
    for _ in range(rounds):
        # tree rotations
        for _ in range(tree_moves):
            v = internal[rng.integers(len(internal))]
            a, b = tr.ch[v]
            u, w = (a, b) if rng.integers(2) == 0 else (b, a)
            if u < n:
                continue
            x, y = tr.ch[u]
            if rng.integers(2):
                x, y = y, x
            o_u = tr.join(y, w)
            if tr.size(o_u & ~S) > cap:
                continue
            old = tr.cost(tr.ch[u][0], tr.ch[u][1], u, S) + tr.cost(a, b, v, S)
            saved = (tr.opn[u], tr.sub[u])
            tr.opn[u] = o_u
            tr.sub[u] = tr.sub[y] | tr.sub[w]
            new = tr.cost(y, w, u, S) + tr.cost(x, u, v, S)
            d = new - old
            if d < 0 or (d == 0 and rng.integers(2)):
                tr.ch[u] = [y, w]
                tr.ch[v] = [x, u]
                cur += d
            else:
                tr.opn[u], tr.sub[u] = saved
        # slice swaps
        if sl:
            for _ in range(slice_moves):
                j = int(rng.integers(len(sl)))
                e = cand[rng.integers(len(cand))]
                if e in sl:
                    continue
                new_sl = sl[:j] + [e] + sl[j + 1:]
                S2 = tr.mask(new_sl)
                if tr.max_per_slice(S2) > cap:
                    continue
                t2 = tr.total(S2)
                if t2 < cur:
                    sl, S, cur = new_sl, S2, t2
    cur = tr.total(S)   # exact, without accumulated rounding of the deltas
    return tr.path(), sl, cur
