"""Circuit -> tensor network of one amplitude (or a batch of amplitudes).

Sec. 2.2 and its worked example: a one-qudit gate is a rank-2 tensor, a
two-qudit gate a rank-4 tensor, the input |0> and the output <a| are rank-1
tensors, and the amplitude <a|U|0> is the contraction of all of them.

Here the rank-1 boundary tensors are not kept as separate leaves: fixing an
index of a gate tensor to a basis value is a *selection* of entries (no
multiply-add), so the first gate on each qudit has its input axis taken at 0
and the last gate has its output axis taken at the requested outcome.  All
remaining leaves are gate tensors with axes ``[out_0..out_{k-1}, in_0..in_{k-1}]``
(first listed qudit first), exactly ``matrix.reshape([d]*2k)``.

Batch of outcomes: the output axes of last gates are replaced by one shared
*batch index* of size ``B`` (an open index that several leaves carry, i.e. a
hyperedge); entry ``[beta, ...]`` of such a leaf is the gate entry selected at
outcome ``beta``.  A leaf that is the last gate of several qudits selects them
jointly, so it carries the batch index once.

File format (``save``/``load``): ``<stem>.json`` (labels, dims, open, path,
sliced, metadata) + ``<stem>.npz`` (leaf arrays ``t0, t1, ...``).
"""

import json
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np


@dataclass
class TensorNetwork:
    tensors: List[np.ndarray]
    labels: List[List[int]]
    dims: Dict[int, int]
    open: List[int] = field(default_factory=list)
    leaf_op: List[int] = field(default_factory=list)    # circuit op index of each leaf
    batch_index: Optional[int] = None
    meta: dict = field(default_factory=dict)

    @property
    def n_tensors(self):
        return len(self.tensors)

    def index_ids(self):
        return sorted(self.dims)

    def check(self):
        count = {}
        for t, lab in zip(self.tensors, self.labels):
            assert t.ndim == len(lab), (t.shape, lab)
            assert len(set(lab)) == len(lab), lab
            for ax, i in enumerate(lab):
                assert t.shape[ax] == self.dims[i], (i, t.shape, self.dims[i])
                count[i] = count.get(i, 0) + 1
        for i, c in count.items():
            if i not in self.open:
                assert c == 2, f"index {i} appears in {c} tensors"
        return True


def circuit_network(circ, outcome=None, batch=None, open_outputs=False):
    """Tensor network of <outcome| U |0> (``outcome``: (n,) ints), of a batch
    (``batch``: (B, n) ints; the batch index is open and listed in ``open``),
    or of the whole output state U|0> (``open_outputs``: every qudit's output
    index stays open, listed in qudit order, so the result is the state in
    the row-major order of the state vector)."""
    if (outcome is not None) + (batch is not None) + bool(open_outputs) != 1:
        raise ValueError("give exactly one of outcome / batch / open_outputs")
    n, d = circ.n, circ.d
    next_id = [0]

    def new_id():
        next_id[0] += 1
        return next_id[0] - 1

    dims = {}
    wire = [None] * n          # current wire index of each qudit (None: still |0>)
    tensors, labels, leaf_op = [], [], []
    for oi, op in enumerate(circ.ops):
        k = len(op.qudits)
        t = op.matrix.reshape([d] * (2 * k))
        lab = []
        for _ in range(k):
            i = new_id()
            dims[i] = d
            lab.append(i)
        for q in op.qudits:
            lab.append(wire[q])
        # select input value 0 on axes whose wire is still the initial |0>
        for ax in reversed(range(k, 2 * k)):
            if lab[ax] is None:
                t = np.take(t, 0, axis=ax)
                del lab[ax]
        for j, q in enumerate(op.qudits):
            wire[q] = lab[j]
        tensors.append(np.ascontiguousarray(t))
        labels.append(lab)
        leaf_op.append(oi)
    if any(w is None for w in wire):
        raise ValueError("every qudit needs at least one gate")

    where = {}                 # output wire id -> tensor holding it
    for ti, lab in enumerate(labels):
        for i in lab:
            where.setdefault(i, []).append(ti)
    per_tensor = {}
    for q in range(n):
        ti = [x for x in where[wire[q]]][0]
        per_tensor.setdefault(ti, []).append(q)

    tn_open = []
    batch_index = None
    if open_outputs:
        tn = TensorNetwork(tensors=tensors, labels=labels, dims=dict(dims),
                           open=[wire[q] for q in range(n)], leaf_op=leaf_op,
                           meta=dict(circuit=circ.meta, output_leaves=sorted(per_tensor)))
        tn.check()
        return tn
    if batch is not None:
        batch = np.asarray(batch, np.int64)
        batch_index = new_id()
        dims[batch_index] = batch.shape[0]
        tn_open = [batch_index]
    for ti, qs in per_tensor.items():
        t, lab = tensors[ti], labels[ti]
        axes = [lab.index(wire[q]) for q in qs]
        if batch is None:
            for ax, q in sorted(zip(axes, qs), reverse=True):
                t = np.take(t, int(outcome[q]), axis=ax)
                del lab[ax]
        else:
            # joint selection over all output axes of this leaf -> one batch axis
            perm = axes + [a for a in range(t.ndim) if a not in axes]
            t = np.transpose(t, perm)
            idx = tuple(batch[:, q] for q in qs)
            t = t[idx]                                # (B, remaining axes...)
            lab = [batch_index] + [lab[a] for a in range(len(lab)) if a not in axes]
        tensors[ti] = np.ascontiguousarray(t)
        labels[ti] = lab
    used = set(i for lab in labels for i in lab)
    dims = {i: dims[i] for i in used}
    tn = TensorNetwork(tensors=tensors, labels=labels, dims=dims, open=tn_open,
                       leaf_op=leaf_op, batch_index=batch_index,
                       meta=dict(circuit=circ.meta, output_leaves=sorted(per_tensor)))
    tn.check()
    return tn


def relabel_compact(tn):
    """Renumber index ids to 0..n_index-1 (order of first appearance)."""
    mp = {}
    for lab in tn.labels:
        for i in lab:
            if i not in mp:
                mp[i] = len(mp)
    for i in tn.open:
        if i not in mp:
            mp[i] = len(mp)
    return TensorNetwork(tensors=list(tn.tensors),
                         labels=[[mp[i] for i in lab] for lab in tn.labels],
                         dims={mp[i]: v for i, v in tn.dims.items()},
                         open=[mp[i] for i in tn.open], leaf_op=list(tn.leaf_op),
                         batch_index=None if tn.batch_index is None else mp[tn.batch_index],
                         meta=dict(tn.meta))


def save(stem, tn, path=None, sliced=None):
    doc = dict(labels=tn.labels, dims={str(k): v for k, v in tn.dims.items()}, open=tn.open,
               leaf_op=tn.leaf_op, batch_index=tn.batch_index, meta=tn.meta,
               path=[list(p) for p in path] if path is not None else None,
               sliced=list(sliced) if sliced is not None else None)
    with open(stem + ".json", "w") as f:
        json.dump(doc, f)
    np.savez(stem + ".npz", **{f"t{i}": t for i, t in enumerate(tn.tensors)})


def load(stem):
    with open(stem + ".json") as f:
        doc = json.load(f)
    z = np.load(stem + ".npz", allow_pickle=False)
    tensors = [z[f"t{i}"] for i in range(len(doc["labels"]))]
    tn = TensorNetwork(tensors=tensors, labels=doc["labels"],
                       dims={int(k): v for k, v in doc["dims"].items()}, open=doc["open"],
                       leaf_op=doc["leaf_op"], batch_index=doc["batch_index"], meta=doc["meta"])
    path = [tuple(p) for p in doc["path"]] if doc["path"] is not None else None
    return tn, path, doc["sliced"]
