"""Brute-force task enumeration for multi-contractions (Sec. 3.2, Fig. 5).

Each slice's contraction is written out as tasks, one per path step.  A task
is named by its path order number and the values of the sliced indices its
result depends on; tasks with equal names are computed once (shared work).
The result of a step depends on a sliced index iff some leaf below it carries
that index (the grey-node rule of Fig. 3, applied recursively up the tree).

From the distinct names this module counts, per step, how many instances run,
and the multiply-add totals with and without reuse, as in Eq. sliced_flops
(every slice pays every step) and Eq. task_based_amplitude_flops (shared
tasks paid once).  The per-slice cost of a step is the product of the
dimensions of all distinct unsliced indices of its two operands (the
D^4, D^2, ... orders of Eq. sequence).
"""

import itertools

import numpy as np


def enumerate_tasks(labels, dims, open_ids, path, sliced):
    n = len(labels)
    open_ids = set(open_ids)
    sliced = list(sliced)
    sets = {t: set(l) for t, l in enumerate(labels)}
    below = {t: set(l) for t, l in enumerate(labels)}    # indices of leaves below
    step_cost = []
    for k, (a, b) in enumerate(path):
        v = n + k
        uni = sets[a] | sets[b]
        common = sets[a] & sets[b]
        sets[v] = uni - (common - open_ids)
        below[v] = below[a] | below[b]
        step_cost.append(int(np.prod([dims[i] for i in uni if i not in sliced], dtype=np.int64)))
    names = [set() for _ in path]
    radix = [range(dims[e]) for e in sliced]
    for values in itertools.product(*radix):
        assign = dict(zip(sliced, values))
        for k in range(len(path)):
            dep = tuple(sorted((e, assign[e]) for e in sliced if e in below[n + k]))
            names[k].add((k, dep))
    inst = [len(s) for s in names]
    n_sl = int(np.prod([dims[e] for e in sliced], dtype=np.int64)) if sliced else 1
    flop_reuse = sum(c * m for c, m in zip(step_cost, inst))
    flop_sl = sum(step_cost)
    return dict(instances=inst, step_cost=step_cost, flop_reuse=flop_reuse,
                flop_noreuse=n_sl * flop_sl, flop_sl=flop_sl, n_slices=n_sl)


def shared_fraction(flop_reuse, flop_sl, n_sl):
    """f_sl solving Eq. task_based_amplitude_flops for a given reuse total:
    FLOP_amp = f FLOP_sl + N_sl (1 - f) FLOP_sl."""
    return (n_sl * flop_sl - flop_reuse) / ((n_sl - 1) * flop_sl)


def task_based_flops(f_sl, flop_sl, n_sl):
    """Eq. task_based_amplitude_flops."""
    return f_sl * flop_sl + n_sl * (1.0 - f_sl) * flop_sl
