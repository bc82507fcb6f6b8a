"""One tn_contract of a workload preceded by a plain 1 GiB device copy.

Run under ``rocprofv3 --pmc FETCH_SIZE`` (then ``WRITE_SIZE``): the copy reads
and writes exactly 1 GiB, which calibrates the counters; the contraction's
dispatches then give the HBM traffic of each step.

    python -m paper_2107_09793_amd.traffic_probe [--workload sliced] [--precision c64]
"""

import argparse
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="sliced")
    ap.add_argument("--precision", default="c64")
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    import torch
    from paper_2107_09793_amd import Plan
    from tngen import workloads

    dev = torch.device("cuda:0")
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)    # 1 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    w = workloads.build(args.workload, seed=args.seed)
    plan = Plan.from_network(w.tn, w.path, w.sliced, precision=args.precision)
    leaves = [torch.from_numpy(np.ascontiguousarray(t, dtype=np.complex64)).to(dev)
              for t in w.tn.tensors]
    out = plan.contract(leaves)
    torch.cuda.synchronize()
    print("traffic probe done", complex(out.cpu().item()), flush=True)


if __name__ == "__main__":
    main()
