"""Greedy slice selection along a fixed path (input generation).

Sec. 4 (m=10 runs) selects sliced edges greedily along a fixed contraction
path so that shared work is as large as possible; Sec. 2.4 slices to bound the
size of intermediates.  The slicer here adds one index at a time, choosing the
index that minimises (largest per-slice intermediate, then the multiply-add
count with shared work reused, then the index id).

The quantities are the ones of Eqs. (sliced_flops) and
(task_based_amplitude_flops), evaluated per node of the contraction tree:

* per-slice size of a node: product of dims of its open indices not sliced;
* per-slice cost of a step: product of dims of all distinct indices of its two
  operands that are not sliced (multiply-adds of the pairwise contraction);
* instances of a step: product of dims of the sliced indices that occur in any
  leaf below it (a step depending on no sliced index runs once).
"""

import numpy as np

from .path import greedy_path


class TreeSets:
    """Index-incidence matrices of a contraction tree (unsliced)."""

    def __init__(self, labels, dims, kept, path):
        n = len(labels)
        ids = sorted(dims)
        self.ids = ids
        col = {i: c for c, i in enumerate(ids)}
        self.w = np.array([np.log2(dims[i]) for i in ids])
        kept = set(kept)
        nn = n + len(path)
        self.open = np.zeros((nn, len(ids)), bool)     # open indices of each node
        self.sub = np.zeros((nn, len(ids)), bool)      # indices in leaves below
        self.uni = np.zeros((len(path), len(ids)), bool)  # all indices of a step's operands
        for t, lab in enumerate(labels):
            for i in lab:
                self.open[t, col[i]] = True
                self.sub[t, col[i]] = True
        keptm = np.zeros(len(ids), bool)
        for i in kept:
            if i in col:
                keptm[col[i]] = True
        self.kept = keptm
        for k, (a, b) in enumerate(path):
            v = n + k
            common = self.open[a] & self.open[b]
            self.open[v] = (self.open[a] | self.open[b]) & ~(common & ~keptm)
            self.sub[v] = self.sub[a] | self.sub[b]
            self.uni[k] = self.open[a] | self.open[b]
        self.n = n
        self.path = path

    def stats(self, sliced):
        s = np.zeros(len(self.ids), bool)
        col = {i: c for c, i in enumerate(self.ids)}
        for i in sliced:
            s[col[i]] = True
        ws = self.w * s
        node_log = (self.open * (self.w - ws)).sum(1)
        inter = node_log[self.n:]
        step_log = (self.uni * (self.w - ws)).sum(1)
        inst_log = (self.sub[self.n:] * ws).sum(1)
        nsl_log = ws.sum()
        flop_reuse = float(np.sum(2.0 ** (step_log + inst_log)))
        flop_sl = float(np.sum(2.0 ** step_log))
        return dict(max_log2=float(inter.max()) if len(inter) else 0.0,
                    flop_reuse=flop_reuse, flop_noreuse=flop_sl * 2.0 ** nsl_log,
                    flop_sl=flop_sl, n_slices=int(round(2.0 ** nsl_log)))


def greedy_slices(ts, n_slice=None, cap_log2=None, max_slices=64, initial=()):
    """Pick sliced indices greedily; stop after ``n_slice`` indices, or once the
    largest per-slice intermediate is at most ``2**cap_log2``.  ``initial``:
    indices already sliced (kept first in the returned list)."""
    cand = ~ts.kept
    inter_open = ts.open[ts.n:]
    chosen = np.zeros(len(ts.ids), bool)
    col = {i: c for c, i in enumerate(ts.ids)}
    out = []
    for i in initial:
        chosen[col[i]] = True
        out.append(i)
    while True:
        ws = ts.w * chosen
        cur = (inter_open * (ts.w - ws)).sum(1)
        if n_slice is not None and len(out) >= n_slice:
            break
        if n_slice is None and cap_log2 is not None and cur.max() <= cap_log2 + 1e-9:
            break
        if len(out) >= max_slices:
            break
        # max per-slice intermediate if index e is added
        red = cur[:, None] - inter_open * ts.w[None, :]
        newmax = red.max(0)
        newmax[~cand | chosen] = np.inf
        best = newmax.min()
        if not np.isfinite(best):
            break
        tied = np.where(newmax <= best + 1e-9)[0]
        step_log = (ts.uni * (ts.w - ws)).sum(1)
        inst_log = (ts.sub[ts.n:] * ws).sum(1)
        base = step_log + inst_log
        fl = []
        for e in tied:
            lg = base - ts.uni[:, e] * ts.w[e] + ts.sub[ts.n:, e] * ts.w[e]
            fl.append(np.sum(2.0 ** lg))
        e = tied[int(np.argmin(np.array(fl)))]
        chosen[e] = True
        out.append(ts.ids[e])
    return out


def search(labels, dims, kept, n_slice=None, cap_log2=None, trials=8, seed=0):
    """Best of a deterministic greedy path plus ``trials`` seeded randomised
    ones (temperature drawn from a fixed list, cost weight alpha ~ U(0.5, 2)),
    each sliced greedily; ranked by (meets the cap, multiply-adds with reuse,
    largest per-slice intermediate)."""
    best = None
    temps = (0.0, 0.05, 0.1, 0.2, 0.3, 0.5, 1.0)
    for t in range(trials + 1):
        if t == 0:
            path = greedy_path(labels, dims, kept)
        else:
            rng = np.random.default_rng([seed, 2, t])
            temp = float(rng.choice(temps))
            alpha = float(rng.uniform(0.5, 2.0))
            path = greedy_path(labels, dims, kept, seed=seed * 100000 + t,
                               temperature=temp, alpha=alpha)
        ts = TreeSets(labels, dims, kept, path)
        sl = greedy_slices(ts, n_slice=n_slice)
        st = ts.stats(sl)
        ok = cap_log2 is None or st["max_log2"] <= cap_log2 + 1e-9
        key = (not ok, st["flop_reuse"], st["max_log2"])
        if best is None or key < best[0]:
            best = (key, path, sl, st)
    return best[1], best[2], best[3]
