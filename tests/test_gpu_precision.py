"""The 53-qubit depth-12 workload (1024 slices, per-slice intermediates <=
2^30) at full size on the GPU, complex64 and split-BF16, against complex128
oracle values of sampled slices (tests/golden/precision_slices_seed0.json,
written by make_precision_slices.py from the oracle alone).

Per-slice bound: |s_gpu - s_oracle| <= tol * rms(oracle slices), tol 1e-5
(complex64) and 1e-3 (split-BF16), the stated tolerances.
"""

import json
import os

import numpy as np
import pytest

from tngen import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden", "precision_slices_seed0.json")


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(GOLD):
        pytest.skip("oracle values not generated")
    from .golden.make_precision_slices import fingerprint
    doc = json.load(open(GOLD))
    w = workloads.build("precision", seed=0)
    assert fingerprint(w) == doc["fingerprint"], "workload differs from the one the oracle used"
    dev = torch.device("cuda:0")
    leaves = [torch.from_numpy(np.ascontiguousarray(t, dtype=np.complex64)).to(dev)
              for t in w.tn.tensors]
    ids = [s[0] for s in doc["slices"]]
    ref = np.array([s[1] + 1j * s[2] for s in doc["slices"]])
    return w, leaves, ids, ref


@pytest.mark.parametrize("precision,tol", [("c64", 1e-5), ("split_bf16", 1e-3)])
def test_precision_workload_sampled_slices(setup, precision, tol):
    from paper_2107_09793_amd import Plan
    w, leaves, ids, ref = setup
    pl = Plan.from_network(w.tn, w.path, w.sliced, precision=precision)
    info = pl.info()
    assert info["max_log2_per_slice"] <= 30 and info["n_slices"] == 1024
    got = pl.contract(leaves, slice_ids=ids, per_slice=True).cpu().numpy().reshape(-1)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    err = np.abs(got - ref) / rms
    print(precision, "per-slice error / rms:", err)
    assert np.all(err <= tol), err
    del pl
    torch.cuda.empty_cache()
