"""Writes the stored refined paths of the workloads that use one
(tngen/paths/<name>_seed<seed>.json): the seeded greedy search followed by
the shared-work-aware refinement, exactly as workloads.build runs it.

    python -m tngen.make_paths [name ...]
"""

import sys
import time

from . import workloads


def main():
    names = sys.argv[1:] or [n for n, c in workloads.CONFIGS.items() if c.get("refine")]
    for name in names:
        t0 = time.time()
        w = workloads.store_path(name)
        print(f"{name}: multiply-adds with reuse {w.stats['flop_reuse']:.4g}, largest per-slice "
              f"2^{w.stats['max_log2']:.0f} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
