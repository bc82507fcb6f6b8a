"""Benchmark: sliced contraction of one amplitude on one MI355X.

Workload (default): 53-qubit random circuit on a 6x9 grid (site (0,4)
inactive), depth 12, one amplitude, 10 sliced indices = 1024 slices, per-slice
intermediates <= 2^30 entries; all slices in one tn_contract call with the
slice-independent work done once.  A step is one full tn_contract (all 1024
slices, every contraction step, the float64 slice sum) with leaves already
resident in HBM.  Both precisions run by default: complex64 (the reported
value) and split-BF16, each with its relative error against complex128 oracle
values of sampled slices (stored under tests/golden/).

Prints one JSON line: complex GFLOP/s (2 x multiply-adds executed / time),
slices/s, the roofline of the dominant step (timed with HIP events on the
launch stream during the timed region) and the CPU oracle timed on a bounded
sample of the same workload.
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
                                   # (256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz)
}

WORKLOAD_DESC = {
    "sliced": "30-qubit 5x6 grid random circuit, depth 14, fSim(pi/2,pi/6) + sqrt(X/Y/W), "
              "one amplitude, 6 sliced dim-2 indices (64 slices), per-slice rank <= 26",
    "plain": "12-qubit 3x4 grid random circuit, depth 8, one amplitude, no slicing",
    "precision": "53-qubit 6x9 grid (site (0,4) inactive) random circuit, depth 12, "
                 "one amplitude, 10 sliced indices (1024 slices)",
    "bosonic": "16-mode 4x4 lattice, Fock cutoff 4, depth 6, Haar two-mode gates, 16 slices",
    "gradient": "20-qubit 4x5 grid, depth 10, batch of 256 outcome strings (forward; forward + backward and the training step in the record's gradient entry)",
    "gbs": "GBS-88-m1: 64-mode 8x8 optical GBS circuit, squeezers r=0.5 + one cycle of "
           "random beam splitters, Fock cutoff 4, one output pattern",
    "gbs8": "GBS-88-m1: 64-mode 8x8 optical GBS circuit, squeezers r=0.5 + one cycle of "
            "random beam splitters, Fock cutoff 8, one output pattern, no slicing",
}


def launch_units(plan, steps):
    """What one launch computes: a fused chain (all its steps) or one step.
    Returns {first step of the unit: dict(kind, cmac, bytes, phase, steps)} with
    the algorithmic HBM bytes (each operand read once, the result written
    once; a chain's intermediates stay on chip)."""
    units = {}
    chains = plan.chains() if plan.info()["n_chains"] else []
    for k, s in enumerate(steps):
        if s["chain"] >= 0:
            continue
        units[k] = dict(kind=s["kind_name"], cmac=s["cmac"], bytes=s["bytes"], phase=s["phase"],
                        steps=[k], shape=dict(nb=s["nb"], nm=s["nm"], nn=s["nn"], nk=s["nk"]),
                        tile_run=s["tile_run"])
    for ch in chains:
        mem = [steps[d["step"]] for d in ch["st"]]
        f, l = mem[0], mem[-1]
        el = 2 ** (f["nb"] + f["nm"] + f["nk"]) + 2 ** (l["nb"] + l["nm"] + l["nn"])
        el += sum(2 ** (m["nb"] + m["nk"] + m["nn"]) for m in mem)
        # steps the chain runs on the matrix cores (the plan's rule, see
        # kernels_chain.h): 2^nk >= 4, 2^nn >= 8, at least 16 rows
        on_mfma = [len(d["kslot"]) >= 2 and len(d["nslot"]) >= 3 and d["nrow"] >= 4
                   and not plan.chain_valu for d in ch["st"]]
        units[ch["first"]] = dict(kind="chain", cmac=sum(m["cmac"] for m in mem), bytes=8.0 * el,
                                  phase=ch["phase"], steps=[d["step"] for d in ch["st"]],
                                  cmac_mfma=sum(m["cmac"] for m, f in zip(mem, on_mfma) if f),
                                  shape=[dict(nb=m["nb"], nm=m["nm"], nn=m["nn"], nk=m["nk"])
                                         for m in mem])
    return units


def dominant_unit(plan, leaves, info, units, torch):
    """Launch with the largest total time (first execution's duration times
    its executions per contraction) among the heaviest candidates; returns
    (first step of the unit, executions)."""
    n_outer = 1 << info["n_outer_bits"]
    execs = {k: (n_outer if u["phase"] == 1 else 1) for k, u in units.items()}
    keys = list(units)
    cand = sorted(keys, key=lambda k: -units[k]["cmac"] * execs[k])[:4]
    cand += sorted(keys, key=lambda k: -units[k]["bytes"] * execs[k])[:4]
    best, best_ms = None, -1.0
    for k in dict.fromkeys(cand):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        plan.contract(leaves, probe=(k, e0, e1))
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) * execs[k]
        if ms > best_ms:
            best, best_ms = k, ms
    return best, execs[best]


# complex64 GEMM tile configurations that form three real products per
# complex product (the others use the real embedding)
GAUSS_CONFIGS = (0, 1, 3, 4, 5, 6, 9)


def roofline(unit, avg_s, precision):
    """The unit's bound is the larger of its HBM time (algorithmic bytes at
    8 TB/s) and its compute time (the MFMA work its kernel executes at the
    precision's peak: 8 real flops per complex multiply-add in the real
    embedding (tile configurations 2, 7 and 8), 6 with three real products
    per complex product (configuration 9 and the complex64 tiles 0, 1, 3-6),
    three BF16 products of 8 in split-BF16; for chain steps
    MFMA at the precision's peak or FP32 vector FMA, as the chain runs them;
    FP32 vector FMA for the others).  Achieved is measured in that bound's
    unit: algorithmic bytes, or algorithmic flops (8 per complex multiply-add,
    the complex GEMM's 2 M N K complex flops) against the peak of the units
    doing most of the work; a GEMM also reports the executed MFMA flops per
    complex multiply-add and the matrix cores' use (executed flops / peak)."""
    kind = unit["kind"]
    extra = {}
    if kind == "gemm":
        flops = 8.0 * unit["cmac"]
        per = 24.0 if precision == "split_bf16" else \
            (6.0 if unit.get("tile_run") in GAUSS_CONFIGS else 8.0)
        peak, cbound = PEAKS["mfma_" + precision], "mfma"
        t_cmp = per * unit["cmac"] / (peak * 1e12)
        extra = dict(executed_flops_per_cmac=per,
                     mfma_util=per * unit["cmac"] / avg_s / 1e12 / peak)
    elif kind == "chain":
        # chain steps run on the matrix cores (FP32, or three BF16 products
        # in split-BF16 plans) or on the FP32 vector units
        fm = 8.0 * unit["cmac_mfma"]
        fv = 8.0 * unit["cmac"] - fm
        mpeak = PEAKS["mfma_" + precision]
        fm_exec = fm * (3.0 if precision == "split_bf16" else 1.0)
        t_cmp = fm_exec / (mpeak * 1e12) + fv / (PEAKS["alu"] * 1e12)
        if fm_exec / mpeak >= fv / PEAKS["alu"]:
            flops, peak, cbound = fm_exec + fv, mpeak, "mfma"
        else:
            flops, peak, cbound = fm_exec + fv, PEAKS["alu"], "alu"
    else:
        flops = 8.0 * unit["cmac"]
        peak, cbound = PEAKS["alu"], "alu"
        t_cmp = flops / (peak * 1e12)
    t_mem = unit["bytes"] / (PEAKS["hbm"] * 1e9)
    if t_mem >= t_cmp:
        ach = unit["bytes"] / avg_s / 1e9
        return dict(bound="hbm", achieved=ach, peak=PEAKS["hbm"], unit="GB/s",
                    frac=ach / PEAKS["hbm"], **extra)
    ach = flops / avg_s / 1e12
    return dict(bound=cbound, achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak, **extra)


KERNEL_SOURCES = {
    "gemm": ("paper_2107_09793_amd/csrc/kernels_gemm.h",
             "paper_2107_09793_amd/csrc/kernels_gemm_stream.h",
             "paper_2107_09793_amd/csrc/kernels_common.h"),
    "stream": ("paper_2107_09793_amd/csrc/kernels_basic.h", "paper_2107_09793_amd/csrc/kernels_common.h"),
    "chain": ("paper_2107_09793_amd/csrc/kernels_chain.h", "paper_2107_09793_amd/csrc/kernels_common.h"),
}


def kernel_sha(kind):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kind, KERNEL_SOURCES["stream"]):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload, unit, precision):
    """HBM bytes per launch of the dominant launch from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when there is
    no summary for this workload and precision, none of its entries is this
    launch, or the kernel source changed since the counters were taken."""
    import re
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}_{precision}.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_h = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    if not m_h or kernel_sha(unit["kind"]) != m_h.group(1):
        return None
    launch = None
    for line in txt.splitlines():
        m_s = re.match(r"launch:\s*(\w+) steps ([0-9,]+)", line)
        if m_s:
            launch = (m_s.group(1), [int(x) for x in m_s.group(2).split(",")])
        m_b = re.match(r"traffic_bytes:\s*([0-9.eE+]+)", line)
        if m_b and launch == (unit["kind"], unit["steps"]):
            return float(m_b.group(1))
    return None


def oracle_cores():
    try:
        from threadpoolctl import threadpool_info
        return max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        return len(os.sched_getaffinity(0))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_step_costs(labels, dims, open_ids, path, fixed):
    """Multiply-adds of each pairwise step as the oracle runs it (product of
    the dims of all indices of both operands, the ``fixed`` ones excluded) and
    the largest intermediate (entries)."""
    fixed = set(fixed)
    labs = {t: set(l) - fixed for t, l in enumerate(labels)}
    opn = set(open_ids)
    n = len(labels)
    costs, big = [], 1.0
    for k, (i, j) in enumerate(path):
        a, b = labs.pop(i), labs.pop(j)
        costs.append(float(np.prod([dims[x] for x in a | b], dtype=np.float64)))
        labs[n + k] = (a | b) - ((a & b) - opn)
        big = max(big, float(np.prod([dims[x] for x in labs[n + k]], dtype=np.float64)))
    return costs, big


def zgemm_rate():
    """Multiply-adds per second of numpy's complex128 matrix product here
    (a short calibration used only to size the oracle sample)."""
    rng = np.random.default_rng(0)
    a = rng.standard_normal((1024, 1024)) + 1j * rng.standard_normal((1024, 1024))
    a @ a
    t0, reps = time.perf_counter(), 0
    while time.perf_counter() - t0 < 0.5:
        a @ a
        reps += 1
    return reps * 1024.0 ** 3 / (time.perf_counter() - t0)


def cpu_baseline(w, budget_s, max_entries=2 ** 30):
    """The oracle (numpy complex128, one slice at a time, no reuse) on a
    bounded sample of the same contraction: whole slices if one fits the time
    budget (at most 3), else one whole sub-slice of slice 0 -- every step of
    the path, with just enough further indices fixed (chosen by the same
    greedy slicer) that its estimated time fits the budget and its largest
    intermediate fits host memory.  Sub-slices of a slice sum to the slice
    (Eq. sliced_sum), so the sample is a part of the real work, large steps
    included."""
    from oracle import tn_oracle
    tn, path, sliced = w.tn, w.path, list(w.sliced)
    est_rate = 0.1 * zgemm_rate()    # the oracle's rate is well below the bare product's
    slice_cost = sum(oracle_step_costs(tn.labels, tn.dims, tn.open, path, sliced)[0])
    n_sl = int(np.prod([tn.dims[e] for e in sliced])) if sliced else 1
    fix = list(sliced)
    costs, big = oracle_step_costs(tn.labels, tn.dims, tn.open, path, fix)
    opn = set(tn.open)
    # fix indices of the costliest step, one at a time, each the one that
    # lowers the total most, until the sample fits the budget and memory
    while sum(costs) / est_rate > budget_s or big > max_entries:
        labs = {t: set(l) for t, l in enumerate(tn.labels)}
        n = len(tn.labels)
        worst, worst_set = -1.0, set()
        for k, (i, j) in enumerate(path):
            a, b = labs.pop(i), labs.pop(j)
            if costs[k] > worst:
                worst, worst_set = costs[k], (a | b)
            labs[n + k] = (a | b) - ((a & b) - opn)
        cand = [e for e in sorted(worst_set) if e not in opn and e not in fix]
        if not cand:
            break
        trial = [(sum(oracle_step_costs(tn.labels, tn.dims, tn.open, path, fix + [e])[0]), e)
                 for e in cand]
        fix.append(min(trial)[1])
        costs, big = oracle_step_costs(tn.labels, tn.dims, tn.open, path, fix)
    sub = fix[len(sliced):]
    t0 = time.perf_counter()
    if not sub:
        # whole slices, one at a time, while the next one fits the budget
        m = 0
        while m < min(3, n_sl):
            tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, path, fix, slice_ids=[m])
            m += 1
            el = time.perf_counter() - t0
            if el * (m + 1) / m > budget_s:
                break
        ids = list(range(m))
        what = f"{m} whole slice{'s' if m > 1 else ''}"
    else:
        ids = [0]                         # slice 0, sub-slice 0 (mixed radix, first most significant)
        n_sub = int(np.prod([tn.dims[e] for e in sub]))
        what = (f"sub-slice 0 of {n_sub} of slice 0 ({len(sub)} more indices fixed; every "
                f"step of the path)")
        tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, path, fix, slice_ids=ids)
    dt = time.perf_counter() - t0
    cmac = sum(costs) * len(ids)
    rate = cmac / dt
    return dict(value=2.0 * rate / 1e9, unit="complex GFLOP/s", cores=oracle_cores(),
                cpu=cpu_model(), kind="oracle",
                sample=f"{what}: {cmac:.3e} multiply-adds ({cmac / slice_cost:.3f} of a slice "
                       f"of {slice_cost:.3e}), numpy complex128, no reuse, {dt:.1f} s",
                slices_per_s=rate / slice_cost, n_slices=n_sl)


def path_fingerprint(w):
    """Hash of the path and the sliced indices (as the scripts that write the
    stored oracle values compute it)."""
    import hashlib
    h = hashlib.sha256()
    h.update(json.dumps([list(map(int, p)) for p in w.path]).encode())
    h.update(json.dumps(list(map(int, w.sliced))).encode())
    return h.hexdigest()[:16]


def golden(workload, seed, w):
    """complex128 oracle values of sampled slices of this very path and slice
    set, written by the scripts in tests/golden/ (oracle only), or None."""
    path = os.path.join(ROOT, "tests", "golden", f"{workload}_slices_seed{seed}.json")
    if not os.path.exists(path):
        return None
    doc = json.load(open(path))
    if doc.get("fingerprint") != path_fingerprint(w):
        return None
    return [s[0] for s in doc["slices"]], np.array([s[1] + 1j * s[2] for s in doc["slices"]])


def permute_roofline(torch, nbits=28, reps=10, seed=0):
    """The LDS-tiled bit permutation (tn_permute) on a 2^nbits complex64
    tensor under a seeded random permutation of its bits: 16 bytes moved per
    element (read + write), timed with HIP events on the current stream."""
    from paper_2107_09793_amd import permute
    rng = np.random.default_rng([seed, 5])
    pin = list(range(nbits))
    pout = [int(v) for v in rng.permutation(nbits)]
    x = torch.randn(1 << nbits, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    permute(x, pin, pout, out=y)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        permute(x, pin, pout, out=y)
    e1.record()
    torch.cuda.synchronize()
    avg = e0.elapsed_time(e1) / reps / 1e3
    gbs = 16.0 * (1 << nbits) / avg / 1e9
    del x, y
    torch.cuda.empty_cache()
    return dict(bound="hbm", achieved=gbs, peak=PEAKS["hbm"], unit="GB/s",
                frac=gbs / PEAKS["hbm"], traffic=None, avg_ms=avg * 1e3,
                elements=1 << nbits, permutation=pout)


def run_precision(args, w, precision, leaves, torch, ws_limit):
    """Plan, warm up, find the dominant launch, time ``args.steps`` contractions."""
    from paper_2107_09793_amd import Plan
    plan = Plan.from_network(w.tn, w.path, w.sliced, precision=precision,
                             no_reuse=args.no_reuse, workspace_limit=ws_limit)
    info = plan.info()
    steps = plan.steps()
    for s in steps:
        ea = 1 << (s["nb"] + s["nm"] + s["nk"])
        eb = 1 << (s["nb"] + s["nk"] + s["nn"])
        ec = 1 << (s["nb"] + s["nm"] + s["nn"])
        s["bytes"] = 8.0 * (ea + eb + ec)
    print(f"# {precision}: {info['n_steps']} steps, {info['n_launches']} launches, "
          f"{info['n_slices']} slices, cmac_exec={info['cmac_exec']:.4g}, "
          f"arena={info['arena_bytes'] / 2**30:.2f} GiB", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        plan.contract(leaves)
    torch.cuda.synchronize()
    units = launch_units(plan, steps)
    dom, dom_execs = dominant_unit(plan, leaves, info, units, torch)
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
    print(f"# {precision}: {t * 1e3:.1f} ms per contraction", file=sys.stderr, flush=True)
    d = units[dom]
    rl = roofline(d, dom_s, precision)
    rl.update(traffic=measured_traffic(args.workload, d, precision), steps=d["steps"],
              kernel=d["kind"], executions_per_step=dom_execs, cmac=d["cmac"],
              bytes=d["bytes"], avg_ms=dom_s * 1e3,
              share_of_step=dom_s * dom_execs / t, shape=d["shape"])
    res = dict(value=2.0 * info["cmac_exec"] / t / 1e9, slices_per_s=info["n_slices"] / t,
               ms_per_step=t * 1e3, roofline=rl,
               amplitude=[float(out.real.item()), float(out.imag.item())]
               if out.numel() == 1 else None,
               plan=dict(cmac_reuse=info["cmac_reuse"], cmac_noreuse=info["cmac_noreuse"],
                         cmac_exec=info["cmac_exec"], f_sl=info["f_sl"],
                         arena_bytes=info["arena_bytes"], n_launches=info["n_launches"],
                         n_steps=info["n_steps"], outer_bits=info["n_outer_bits"]))
    gold = golden(args.workload, args.seed, w)
    if gold is not None:
        ids, ref = gold
        got = plan.contract(leaves, slice_ids=ids, per_slice=True).cpu().numpy().reshape(-1)
        rms = np.sqrt(np.mean(np.abs(ref) ** 2))
        res["rel_err_vs_oracle"] = float(np.max(np.abs(got - ref)) / rms)
        res["rel_err_slices"] = ids
    res["tolerance"] = 1e-5 if precision == "c64" else 1e-3
    if info["n_segments"] == 0:
        # the same contraction replayed as a HIP graph (tn_graph_create):
        # the launch sequence without the per-launch host work
        g = plan.graph(leaves)
        g.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.launch()
        torch.cuda.synchronize()
        res["graph_ms_per_step"] = (time.perf_counter() - t0) / args.steps * 1e3
        del g
    return plan, info, res


def gradient_step(args, w, plan, leaves, torch):
    """Timed gradients of the trainable workload (loss = -mean log|amp|^2 over
    the batch of outcome strings).  ``fwd_bwd``: one ``tn_contract`` plus one
    ``tn_contract_backward`` (every leaf's gradient) on resident leaves;
    ``fwd_bwd_graph``: the same two calls replayed as HIP graphs
    (``tn_graph_create``, ``tn_graph_create_backward``);
    ``train``: the whole step through torch -- the fSim leaves formed from
    the gate parameters, ``CircuitAmplitude.apply``, the loss, and the chain
    rule back to the parameters."""
    from paper_2107_09793_amd.autograd import CircuitAmplitude, CircuitLeaves
    info = plan.info()
    grads = [torch.zeros_like(x) for x in leaves]
    gout = torch.ones(info["out_elems"], dtype=torch.complex128, device=leaves[0].device)

    def fwd_bwd():
        plan.contract(leaves)
        plan.backward(leaves, gout, grads)

    params = torch.tensor(w.circuit.params, dtype=torch.float64, requires_grad=True)
    builder = CircuitLeaves(w.tn, w.circuit, leaves[0].device)

    def train():
        params.grad = None
        amp = CircuitAmplitude.apply(plan, builder, builder.gates(params))
        loss = -torch.mean(torch.log(torch.abs(amp) ** 2))
        loss.backward()

    # the same forward + backward replayed as two HIP graphs
    fg = plan.graph(leaves)
    bg = plan.backward_graph(leaves, gout, grads)

    def fwd_bwd_graph():
        fg.launch()
        bg.launch()

    out = {}
    for name, fn in (("fwd_bwd", fwd_bwd), ("fwd_bwd_graph", fwd_bwd_graph), ("train", train)):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        out[name + "_ms_per_step"] = (time.perf_counter() - t0) / args.steps * 1e3
    # the adjoint of a step is two products of the step's size (dA = dC B^H,
    # dB = A^H dC), plus the forward values it recomputes
    cmac = 3.0 * info["cmac_exec"] + info["cmac_backward_recompute"]
    out.update(cmac=cmac, value=2.0 * cmac / (out["fwd_bwd_ms_per_step"] * 1e-3) / 1e9,
               unit="complex GFLOP/s", n_params=int(params.numel()),
               workspace_backward_bytes=info["workspace_backward_bytes"],
               backward_policy=info["backward_policy"])
    del fg, bg
    print(f"# gradient: forward + backward {out['fwd_bwd_ms_per_step']:.3f} ms "
          f"({out['fwd_bwd_graph_ms_per_step']:.3f} ms as graphs), "
          f"training step {out['train_ms_per_step']:.3f} ms", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed contractions (default 3 "
                    "for the 53-qubit workload, 10 otherwise)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="precision", choices=sorted(WORKLOAD_DESC))
    ap.add_argument("--precision", default="both", choices=["both", "c64", "split_bf16"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=20.0,
                    help="seconds of oracle work for cpu_baseline (0 = skip)")
    ap.add_argument("--no-reuse", action="store_true")
    ap.add_argument("--path", default="default", choices=["default", "greedy", "cmac", "time"],
                    help="contraction path: the workload's default, the seeded greedy "
                         "search alone, or followed by the shared-work-aware refinement "
                         "(multiply-adds with reuse; then the roofline time estimate)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): slices are independent, "
              "so the multi-GPU layout is one slice range per GPU plus one all-reduce of the "
              "float64 partial sums; this benchmark measures the single-GPU share.", file=sys.stderr)
        sys.exit(2)
    if args.steps is None:
        args.steps = 3 if args.workload == "precision" else 10

    import torch
    from tngen import workloads

    dev = torch.device("cuda:0")
    w = workloads.build(args.workload, seed=args.seed,
                        refine={"default": None, "greedy": False}.get(args.path, args.path))
    leaves = [torch.from_numpy(np.ascontiguousarray(t, dtype=np.complex64)).to(dev)
              for t in w.tn.tensors]
    perm = permute_roofline(torch)
    precs = ["c64", "split_bf16"] if args.precision == "both" else [args.precision]
    from paper_2107_09793_amd.binding import default_workspace_limit
    ws_limit = default_workspace_limit()   # the same limit (and outer split) for both
    results = {}
    keep = None
    for prec in precs:
        plan, info, res = run_precision(args, w, prec, leaves, torch, ws_limit)
        results[prec] = res
        plan.release_workspace()
        if prec == precs[0]:
            keep = (plan, info)
        else:
            del plan
        torch.cuda.empty_cache()
    main_prec = precs[0]
    r0 = results[main_prec]
    plan, info = keep
    rec = dict(metric="complex GFLOP/s and slices/sec at 1 GPU, split-BF16 vs complex64 at "
                      "stated rel error",
               value=r0["value"], unit="complex GFLOP/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=r0["ms_per_step"], higher_is_better=True,
               scaling="weak", vs_baseline=None,
               dtype="c64" if main_prec == "c64" else "split_bf16",
               data="synthetic",
               config=dict(workload=WORKLOAD_DESC[args.workload], name=args.workload,
                           seed=args.seed, n_slices=info["n_slices"], precision=main_prec,
                           reuse=not args.no_reuse),
               slices_per_s=r0["slices_per_s"], amplitude=r0["amplitude"],
               roofline=r0["roofline"], plan=r0["plan"])
    for key in ("rel_err_vs_oracle", "rel_err_slices", "tolerance"):
        if key in r0:
            rec[key] = r0[key]
    rec["permute_roofline"] = perm
    if "split_bf16" in results and main_prec != "split_bf16":
        sb = results["split_bf16"]
        rec["split_bf16"] = {k: sb[k] for k in ("value", "slices_per_s", "ms_per_step",
                                                "roofline", "rel_err_vs_oracle", "tolerance",
                                                "amplitude") if k in sb}
        rec["speedup_split_bf16_vs_c64"] = r0["ms_per_step"] / sb["ms_per_step"]
    rec["launches"] = info["n_launches"]
    rec["us_per_amplitude"] = r0["ms_per_step"] * 1e3 / info["out_elems"]
    if "graph_ms_per_step" in r0:
        rec["graph_ms_per_step"] = r0["graph_ms_per_step"]
        rec["graph_us_per_amplitude"] = r0["graph_ms_per_step"] * 1e3 / info["out_elems"]
    if getattr(w.circuit, "params", None) is not None and w.batch is not None:
        rec["gradient"] = gradient_step(args, w, plan, leaves, torch)
    if args.cpu_budget > 0:
        print(f"# cpu baseline (oracle, budget {args.cpu_budget:.0f} s)", flush=True)
        rec["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
