"""GEMM tile autotuner.

For the heaviest GEMM step shapes of a workload, time every compiled tile
configuration of each precision on the device (HIP events around the step,
through tn_contract_probe) and write the winners to tune/gfx950.json, which
Plan loads by default.  Entries: [precision, nm, nn, nk, config] with the
shape as log2 (rows, columns, summed); the plan applies an entry to steps
with the same precision and column count and the nearest (rows, summed).

    python -m paper_2107_09793_amd.autotune [--workload sliced precision] [--shapes 6]

With several workloads the entries of all of them go into one table.  Steps
are timed on a contraction of slice 0 only (the slice-independent steps plus
one pass of the per-slice steps), which holds every step once.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

N_CONFIGS = 10
CONFIG_NAMES = {0: "128x64 k16", 1: "128x32 k16", 2: "256x16 k16", 3: "128x128 k16",
                4: "256x64 k16", 5: "128x64 k32 (c64) / k16 (split)",
                6: "128x32 k8 (c64) / k16 (split)", 7: "128x16 k16",
                8: "stream: 32-row bands past a resident B block",
                9: "stream, three real products per complex product (c64; else as 8)"}
PREC_ID = {"c64": 0, "split_bf16": 1}


def time_step(plan, leaves, step, reps, torch):
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        plan.contract(leaves, slice_ids=[0], probe=(step, e0, e1))
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def tune(workload="sliced", seed=0, n_shapes=6, reps=3, precisions=("c64", "split_bf16"),
         out=None, log=print):
    import torch
    from paper_2107_09793_amd.binding import Plan, default_workspace_limit
    from tngen import workloads

    w = workloads.build(workload, seed=seed)
    dev = torch.device("cuda:0")
    leaves = [torch.from_numpy(np.ascontiguousarray(t, dtype=np.complex64)).to(dev)
              for t in w.tn.tensors]
    # one workspace limit for every plan: the same outer split, so a step
    # index has the same shape in every configuration
    ws_limit = default_workspace_limit()
    base = Plan.from_network(w.tn, w.path, w.sliced, tune=[], workspace_limit=ws_limit)
    steps = base.steps()
    # GEMM launches only: a step inside a fused chain runs on the chain kernel
    gem = [k for k, s in enumerate(steps) if s["kind_name"] == "gemm" and s["chain"] < 0]
    gem.sort(key=lambda k: -steps[k]["cmac"])
    shapes, chosen = [], []
    for k in gem:
        sh = (steps[k]["nm"], steps[k]["nn"], steps[k]["nk"])
        if sh not in shapes:
            shapes.append(sh)
            chosen.append(k)
        if len(chosen) >= n_shapes:
            break
    raw = []
    entries = []
    for prec in precisions:
        times = {k: {} for k in chosen}
        for cfg in range(N_CONFIGS):
            pl = Plan.from_network(w.tn, w.path, w.sliced, precision=prec, gemm_config=cfg,
                                   tune=[], workspace_limit=ws_limit)
            for k in chosen:
                got = pl.step(k)
                assert (got["nb"], got["nm"], got["nn"], got["nk"]) == \
                    (steps[k]["nb"], steps[k]["nm"], steps[k]["nn"], steps[k]["nk"])
            pl.contract(leaves, slice_ids=[0])
            torch.cuda.synchronize()
            for k in chosen:
                ms = time_step(pl, leaves, k, reps, torch)
                times[k][cfg] = ms
                s = steps[k]
                tf = 8.0 * s["cmac"] / (ms * 1e-3) / 1e12
                raw.append(dict(precision=prec, step=k, nb=s["nb"], nm=s["nm"], nn=s["nn"],
                                nk=s["nk"], config=cfg, ms=ms, tflops=tf))
                log(f"{prec:10s} step {k:4d} b{s['nb']} m{s['nm']} n{s['nn']} k{s['nk']} "
                    f"cfg {cfg} ({CONFIG_NAMES[cfg]}): {ms:9.3f} ms  {tf:7.2f} TFLOP/s")
            pl.release_workspace()
            del pl
            torch.cuda.empty_cache()
        for k in chosen:
            best = min(times[k], key=times[k].get)
            s = steps[k]
            entries.append([PREC_ID[prec], s["nm"], s["nn"], s["nk"], best])
    doc = dict(device="MI355X (gfx950)", workload=workload, seed=seed,
               generated=time.strftime("%Y-%m-%d %H:%M:%S"),
               configs=CONFIG_NAMES, entries=entries, measurements=raw)
    write(doc, out)
    return doc


def write(doc, out):
    for path in ([out] if isinstance(out, str) else list(out or [])):
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as f:
            json.dump(doc, f, indent=1)


def merge(docs):
    """One table from several workloads' results (an entry per distinct
    (precision, shape); the first workload's choice wins a tie of shapes)."""
    seen, entries, raw = set(), [], []
    for d in docs:
        for e in d["entries"]:
            if tuple(e[:4]) not in seen:
                seen.add(tuple(e[:4]))
                entries.append(e)
        raw += [dict(m, workload=d["workload"]) for m in d["measurements"]]
    return dict(device=docs[0]["device"], workload=[d["workload"] for d in docs],
                seed=docs[0]["seed"], generated=docs[-1]["generated"],
                configs=CONFIG_NAMES, entries=entries, measurements=raw)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", nargs="+", default=["sliced"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--shapes", type=int, default=6)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", nargs="+", default=[os.path.join(HERE, "tune", "gfx950.json")])
    args = ap.parse_args()
    docs = [tune(wl, args.seed, args.shapes, args.reps, out=None,
                 log=lambda s: print(s, flush=True)) for wl in args.workload]
    write(merge(docs), args.out)


if __name__ == "__main__":
    main()
