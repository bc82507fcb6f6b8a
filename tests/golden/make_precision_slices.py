"""Writes precision_slices_seed0.json: complex128 oracle values of sampled
slices of the 53-qubit depth-12 workload (seed 0).

Calls only the oracle (tn_oracle.contract) on inputs from the seeded
generators.  Each requested slice is contracted as the sum of its 4
sub-slices over two further sliced indices, which bounds host memory; the
sum of sub-slices is exactly the slice (Eq. sliced_sum).  The two indices
are the pair, among the indices of the per-slice intermediates of 2^28 or
more entries, with the smallest (largest sub-slice intermediate, sub-slice
multiply-adds).

    python tests/golden/make_precision_slices.py [slice ids ...]

Default: 16 slices, ids 0, 1, 513, 1023 and 12 more drawn with
numpy.random.default_rng([0, 5]) from the rest.
"""

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import tn_oracle  # noqa: E402
from tngen import slicing, workloads  # noqa: E402


def fingerprint(w):
    h = hashlib.sha256()
    h.update(json.dumps([list(map(int, p)) for p in w.path]).encode())
    h.update(json.dumps(list(map(int, w.sliced))).encode())
    return h.hexdigest()[:16]


def extra_pair(ts, base):
    col = {i: c for c, i in enumerate(ts.ids)}
    s0 = np.zeros(len(ts.ids), bool)
    for i in base:
        s0[col[i]] = True
    node = (ts.open[ts.n:] * (ts.w - ts.w * s0)).sum(1)
    big = np.where(node >= 28)[0]
    cand = sorted(set(np.where(ts.open[ts.n:][big].any(0) & ~ts.kept & ~s0)[0]))
    best = None
    for i, a in enumerate(cand):
        for b in cand[i + 1:]:
            st = ts.stats(base + [ts.ids[a], ts.ids[b]])
            key = (st["max_log2"], st["flop_sl"], a, b)
            if best is None or key < best:
                best = key
    return [ts.ids[best[2]], ts.ids[best[3]]]


def default_ids():
    fixed = [0, 1, 513, 1023]
    rest = np.setdiff1d(np.arange(1024), fixed)
    more = np.random.default_rng([0, 5]).choice(rest, size=12, replace=False)
    return fixed + sorted(int(x) for x in more)


def main():
    ids = [int(x) for x in sys.argv[1:]] or default_ids()
    w = workloads.build("precision", seed=0)
    ts = slicing.TreeSets(w.tn.labels, w.tn.dims, w.tn.open, w.path)
    extra = extra_pair(ts, list(w.sliced))
    n_sub = int(np.prod([w.tn.dims[e] for e in extra]))
    out = []
    for sid in ids:
        t0 = time.time()
        sub = [sid * n_sub + j for j in range(n_sub)]
        v = tn_oracle.contract(w.tn.tensors, w.tn.labels, w.tn.dims, w.tn.open, w.path,
                               list(w.sliced) + list(extra), slice_ids=sub)
        v = complex(v)
        out.append([sid, v.real, v.imag])
        print(f"slice {sid}: {v!r} ({time.time() - t0:.0f} s)", flush=True)
    doc = dict(source="oracle/tn_oracle.contract, complex128, sub-sliced over 2 extra indices",
               workload="precision", seed=0, fingerprint=fingerprint(w),
               extra_sliced=list(map(int, extra)), slices=out)
    with open(os.path.join(HERE, "precision_slices_seed0.json"), "w") as f:
        json.dump(doc, f, indent=1)


if __name__ == "__main__":
    main()
