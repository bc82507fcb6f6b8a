"""Writes sliced_slices_seed0.json: complex128 oracle values of all 64 slices
of the 30-qubit depth-14 workload (seed 0), hence its full amplitude (their
sum, Eq. sliced_sum).

Calls only the oracle (tn_oracle.contract) on inputs from the seeded
generators.

    python tests/golden/make_sliced_slices.py
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
from tngen import workloads  # noqa: E402


def fingerprint(w):
    h = hashlib.sha256()
    h.update(json.dumps([list(map(int, p)) for p in w.path]).encode())
    h.update(json.dumps(list(map(int, w.sliced))).encode())
    return h.hexdigest()[:16]


def main():
    w = workloads.build("sliced", seed=0)
    n_sl = int(np.prod([w.tn.dims[e] for e in w.sliced]))
    out = []
    t0 = time.time()
    for sid in range(n_sl):
        v = complex(tn_oracle.contract(w.tn.tensors, w.tn.labels, w.tn.dims, w.tn.open, w.path,
                                       w.sliced, slice_ids=[sid]))
        out.append([sid, v.real, v.imag])
        print(f"slice {sid}: {v!r} ({time.time() - t0:.0f} s)", flush=True)
    amp = sum(complex(r, i) for _, r, i in out)   # slice-id order, complex128
    doc = dict(source="oracle/tn_oracle.contract, complex128, one slice at a time",
               workload="sliced", seed=0, fingerprint=fingerprint(w),
               amplitude=[amp.real, amp.imag], slices=out)
    with open(os.path.join(HERE, "sliced_slices_seed0.json"), "w") as f:
        json.dump(doc, f, indent=1)


if __name__ == "__main__":
    main()
