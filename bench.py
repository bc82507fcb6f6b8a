"""Benchmark: sliced contraction of one amplitude on one MI355X.

Workload (default): 30-qubit 5x6 grid random circuit, depth 14, one
amplitude, 6 sliced indices = 64 slices, all slices in one tn_contract call
with slice-independent work done once.  A step is one full tn_contract (all
64 slices, every contraction step, the float64 slice sum) with leaves already
resident in HBM.

Prints one JSON line: complex GFLOP/s (2 x multiply-adds executed / time),
slices/s, the roofline of the dominant step (timed with HIP events on the
launch stream during the timed region) and the CPU oracle timed on a bounded
sample of slices.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published peaks
    "hbm": 8000.0,                 # GB/s
    "mfma_c64": 157.3,             # TFLOP/s, FP32 matrix
    "mfma_split_bf16": 2516.6,     # TFLOP/s, BF16 dense matrix
    "alu": 78.6,                   # TFLOP/s, FP32 vector FMA without packed math
}

WORKLOAD_DESC = {
    "sliced": "30-qubit 5x6 grid random circuit, depth 14, fSim(pi/2,pi/6) + sqrt(X/Y/W), "
              "one amplitude, 6 sliced dim-2 indices (64 slices), per-slice rank <= 26",
    "plain": "12-qubit 3x4 grid random circuit, depth 8, one amplitude, no slicing",
    "precision": "53-qubit 6x9 grid (site (0,4) inactive) random circuit, depth 12, "
                 "one amplitude, 10 sliced indices (1024 slices)",
    "bosonic": "16-mode 4x4 lattice, Fock cutoff 4, depth 6, Haar two-mode gates, 16 slices",
    "gradient": "20-qubit 4x5 grid, depth 10, batch of 256 outcome strings (forward)",
}


def dominant_step(plan, leaves, info, steps, torch):
    """Step with the longest single execution among the heaviest candidates."""
    cand = sorted(range(len(steps)), key=lambda k: -steps[k]["cmac"])[:3]
    cand += sorted(range(len(steps)), key=lambda k: -steps[k]["bytes"])[:2]
    best, best_ms = None, -1.0
    for k in dict.fromkeys(cand):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        plan.contract(leaves, probe=(k, e0, e1))
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        if ms > best_ms:
            best, best_ms = k, ms
    return best


def roofline(step, avg_s, precision):
    kind = step["kind_name"]
    if kind == "gemm":
        peak = PEAKS["mfma_" + precision]
        ach = 8.0 * step["cmac"] / avg_s / 1e12
        return dict(bound="mfma", achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak)
    if kind in ("stream", "splitk"):
        ach = step["bytes"] / avg_s / 1e9
        return dict(bound="hbm", achieved=ach, peak=PEAKS["hbm"], unit="GB/s",
                    frac=ach / PEAKS["hbm"])
    ach = 8.0 * step["cmac"] / avg_s / 1e12
    return dict(bound="alu", achieved=ach, peak=PEAKS["alu"], unit="TFLOP/s",
                frac=ach / PEAKS["alu"])


def measured_traffic(step, precision):
    """HBM bytes of the dominant step from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the summary is
    for another step shape or precision, or the GEMM source changed since."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_gemm_{precision}_sliced30q.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_b = re.search(r"traffic_bytes:\s*([0-9.eE+]+)", txt)
    m_h = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    m_s = re.search(r"step_shape:\s*b(\d+) m(\d+) n(\d+) k(\d+)", txt)
    if not (m_b and m_h and m_s):
        return None
    h = hashlib.sha256()
    for f in ("paper_2107_09793_amd/csrc/kernels_gemm.h", "paper_2107_09793_amd/csrc/kernels_common.h"):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    shape = tuple(int(x) for x in m_s.groups())
    if h.hexdigest()[:16] != m_h.group(1) or shape != (step["nb"], step["nm"], step["nn"], step["nk"]):
        return None
    return float(m_b.group(1))


def cpu_baseline(w, n_sample, gpu_per_slice):
    """The oracle (numpy complex128, one slice at a time, no reuse) on a
    bounded sample of slices; returns its throughput and the GPU's relative
    error on the same slices."""
    from oracle import tn_oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        cores = len(os.sched_getaffinity(0))
    n_sl = 1
    for e in w.sliced:
        n_sl *= w.tn.dims[e]
    ids = list(range(min(n_sample, n_sl)))
    t0 = time.perf_counter()
    ref = tn_oracle.contract(w.tn.tensors, w.tn.labels, w.tn.dims, w.tn.open, w.path, w.sliced,
                             slice_ids=ids, per_slice=True)
    dt = time.perf_counter() - t0
    ref = np.asarray(ref).reshape(len(ids), -1)
    got = gpu_per_slice.reshape(gpu_per_slice.shape[0], -1)[ids]
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    err = float(np.max(np.abs(got - ref)) / rms)
    return dt, len(ids), cores, err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sliced", choices=sorted(WORKLOAD_DESC))
    ap.add_argument("--precision", default="c64", choices=["c64", "split_bf16"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=3, help="slices the oracle times (0 = skip)")
    ap.add_argument("--no-reuse", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): slices are independent, "
              "so the multi-GPU layout is one slice range per GPU plus one all-reduce of the "
              "float64 partial sums; this build measures the single-GPU share.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2107_09793_amd import Plan
    from tngen import workloads

    dev = torch.device("cuda:0")
    w = workloads.build(args.workload, seed=args.seed)
    plan = Plan.from_network(w.tn, w.path, w.sliced, precision=args.precision,
                             no_reuse=args.no_reuse)
    info = plan.info()
    leaves = [torch.from_numpy(np.ascontiguousarray(t, dtype=np.complex64)).to(dev)
              for t in w.tn.tensors]
    steps = plan.steps()
    for s in steps:
        ea = 1 << (s["nb"] + s["nm"] + s["nk"])
        eb = 1 << (s["nb"] + s["nk"] + s["nn"])
        ec = 1 << (s["nb"] + s["nm"] + s["nn"])
        s["bytes"] = 8.0 * (ea + eb + ec)
    print(f"# plan: {info['n_steps']} steps, {info['n_slices']} slices, "
          f"cmac_exec={info['cmac_exec']:.4g}, arena={info['arena_bytes'] / 2**30:.2f} GiB",
          file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        plan.contract(leaves)
    torch.cuda.synchronize()
    dom = dominant_step(plan, leaves, info, steps, torch)

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for i in range(args.steps):
        out = plan.contract(leaves, probe=(dom, evs[i][0], evs[i][1]))
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    dom_s = float(np.mean([a.elapsed_time(b) for a, b in evs])) / 1e3

    value = 2.0 * info["cmac_exec"] / t / 1e9
    rec = dict(metric="complex GFLOP/s and slices/sec at 1 GPU, split-BF16 vs complex64 at "
                      "stated rel error",
               value=value, unit="complex GFLOP/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=t * 1e3, higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="c64" if args.precision == "c64" else "split_bf16",
               data="synthetic",
               config=dict(workload=WORKLOAD_DESC[args.workload], name=args.workload,
                           seed=args.seed, n_slices=info["n_slices"], precision=args.precision,
                           reuse=not args.no_reuse),
               slices_per_s=info["n_slices"] / t,
               amplitude=[float(out.real.item()), float(out.imag.item())] if out.numel() == 1 else None)
    d = steps[dom]
    rl = roofline(d, dom_s, args.precision)
    rl.update(traffic=measured_traffic(d, args.precision), step=dom, kernel=d["kind_name"],
              cmac=d["cmac"],
              bytes=d["bytes"], avg_ms=dom_s * 1e3,
              shape=dict(nb=d["nb"], nm=d["nm"], nn=d["nn"], nk=d["nk"]))
    rec["roofline"] = rl
    rec["plan"] = dict(cmac_reuse=info["cmac_reuse"], cmac_noreuse=info["cmac_noreuse"],
                       cmac_exec=info["cmac_exec"], f_sl=info["f_sl"],
                       arena_bytes=info["arena_bytes"], n_launches=info["n_launches"])
    if args.cpu_sample > 0:
        per = plan.contract(leaves, per_slice=True).cpu().numpy()
        dt, k, cores, err = cpu_baseline(w, args.cpu_sample, per)
        cps = 2.0 * info["cmac_per_slice"] * k / dt / 1e9
        rec["cpu_baseline"] = dict(value=cps, unit="complex GFLOP/s", cores=cores, kind="oracle",
                                   sample=f"{k} of {info['n_slices']} slices, numpy complex128, "
                                          f"no reuse, {dt:.1f} s",
                                   slices_per_s=k / dt)
        rec["rel_err_vs_oracle"] = err
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
