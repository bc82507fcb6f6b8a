"""O2: plain sliced pairwise contraction in complex128 (no reuse).

Follows Sec. 2.3-2.4:

* a slice fixes the value of every sliced index (Eq. sliced_sum); slice id
  ``i`` is decoded in mixed radix with the first listed sliced index most
  significant;
* each slice's network is contracted pairwise along the path (Eq. sequence):
  a step sums over the indices its two operands share, except open indices,
  which stay as a common (batch) axis;
* the slice partial sums s_i are added in complex128 in slice-id order.

Every slice is recomputed from the leaves: this is the "no shared work"
contraction whose total cost is Eq. sliced_flops.  The pairwise step is the
definition written out with one library primitive: operands are transposed to
(batch, free, summed) / (batch, summed, free) and multiplied with numpy's
batched matmul.
"""

import numpy as np


def decode_slice(sid, radix):
    vals = []
    for r in reversed(radix):
        vals.append(sid % r)
        sid //= r
    return list(reversed(vals))


def pairwise(a, la, b, lb, open_ids):
    common = [i for i in la if i in lb]
    batch = [i for i in common if i in open_ids]
    summed = [i for i in common if i not in open_ids]
    fa = [i for i in la if i not in common]
    fb = [i for i in lb if i not in common]
    sa = dict(zip(la, a.shape))
    sb = dict(zip(lb, b.shape))
    nb = int(np.prod([sa[i] for i in batch], dtype=np.int64))
    nk = int(np.prod([sa[i] for i in summed], dtype=np.int64))
    nfa = int(np.prod([sa[i] for i in fa], dtype=np.int64))
    nfb = int(np.prod([sb[i] for i in fb], dtype=np.int64))
    at = np.transpose(a, [la.index(i) for i in batch + fa + summed]).reshape(nb, nfa, nk)
    bt = np.transpose(b, [lb.index(i) for i in batch + summed + fb]).reshape(nb, nk, nfb)
    c = np.matmul(at, bt)
    shape = [sa[i] for i in batch] + [sa[i] for i in fa] + [sb[i] for i in fb]
    return c.reshape(shape), batch + fa + fb


def contract_slice(tensors, labels, open_ids, path, sliced, values, on_step=None):
    """One slice: leaves with sliced indices fixed, contracted along ``path``.
    Returns the result with axes in ``open_ids`` order.  ``on_step(k)``, if
    given, is called after step k; returning False stops the contraction early
    (the function then returns None), which lets a caller time a prefix."""
    fixed = dict(zip(sliced, values))
    pool = {}
    n = len(tensors)
    for t, (x, lab) in enumerate(zip(tensors, labels)):
        x = np.asarray(x, np.complex128)
        lab = list(lab)
        for ax in reversed(range(len(lab))):
            if lab[ax] in fixed:
                x = np.take(x, fixed[lab[ax]], axis=ax)
                del lab[ax]
        pool[t] = (x, lab)
    for k, (i, j) in enumerate(path):
        a, la = pool.pop(i)
        b, lb = pool.pop(j)
        pool[n + k] = pairwise(a, la, b, lb, open_ids)
        if on_step is not None and on_step(k) is False:
            return None
    if len(pool) != 1:
        raise ValueError("path does not contract the network to one tensor")
    (x, lab), = pool.values()
    if sorted(lab) != sorted(open_ids):
        raise ValueError(f"result indices {lab} differ from open indices {open_ids}")
    return np.transpose(x, [lab.index(i) for i in open_ids])


def contract(tensors, labels, dims, open_ids, path, sliced=(), slice_ids=None,
             per_slice=False):
    """Sum over slices (or the list of per-slice results) in complex128."""
    sliced = list(sliced)
    radix = [dims[e] for e in sliced]
    n_sl = int(np.prod(radix, dtype=np.int64)) if sliced else 1
    ids = range(n_sl) if slice_ids is None else [int(s) for s in slice_ids]
    parts = []
    total = None
    for sid in ids:
        s = contract_slice(tensors, labels, open_ids, path, sliced, decode_slice(sid, radix))
        if per_slice:
            parts.append(s)
        else:
            total = s.copy() if total is None else total + s
    if per_slice:
        return np.stack(parts)
    return total


def naive_sum(tensors, labels, open_ids=()):
    """Eq. naive_summation: the whole network as one sum over every index
    (numpy einsum with no path optimisation).  Tiny networks only."""
    letters = {}
    for lab in labels:
        for i in lab:
            letters.setdefault(i, chr(ord("a") + len(letters)) if len(letters) < 26
                               else chr(ord("A") + len(letters) - 26))
    spec = ",".join("".join(letters[i] for i in lab) for lab in labels)
    spec += "->" + "".join(letters[i] for i in open_ids)
    return np.einsum(spec, *[np.asarray(t, np.complex128) for t in tensors], optimize=False)
