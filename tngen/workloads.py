"""The five synthetic workloads (seeded), each returned as a ``Workload``:
circuit, tensor network, SSA path, sliced index ids and path statistics.

1. plain      3x4 grid, depth 8, one amplitude, greedy path, no slicing.
2. sliced     5x6 grid, depth 14, one amplitude, 6 sliced dim-2 indices
              (64 slices) chosen to cap per-slice intermediates at 2^26.
3. precision  53 active sites of a 6x9 grid (site (0,4) inactive), depth 12,
              10 sliced indices (1024 slices), per-slice cap 2^30.
4. bosonic    4x4 modes, depth 6, Fock cutoff 4, Haar two-mode gates,
              2 sliced dim-4 indices (16 slices).
5. gradient   4x5 grid, depth 10, trainable fSim(theta_i, phi_i) on every
              two-qubit gate, batch of 256 outcome strings.

Sycamore-style circuits stand in for the Sycamore-53 circuit files and the
GBS-like network for the GBS circuits of Sec. 4 (same gate counts per cycle
and lattice shapes as described there; no external data is used).
Seeds: circuit ``[seed, 0]``, outcomes ``[seed, 1]``, path trials
``[seed, 2, t]``.
"""

import hashlib
import json
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import circuits, network, refine as refine_mod, slicing


@dataclass
class Workload:
    name: str
    circuit: object
    tn: object
    path: list
    sliced: List[int]
    stats: dict
    outcome: Optional[np.ndarray] = None
    batch: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)


CONFIGS = {
    "plain": dict(kind="grid", rows=3, cols=4, depth=8, n_slice=0, trials=8),
    "sliced": dict(kind="grid", rows=5, cols=6, depth=14, n_slice=6, cap_log2=26, trials=64,
                   refine="time"),
    "precision": dict(kind="grid", rows=6, cols=9, depth=12, inactive=((0, 4),),
                      n_slice=10, cap_log2=30, trials=96, refine="time"),
    "bosonic": dict(kind="gbs", rows=4, cols=4, depth=6, d=4, n_slice=2, trials=96),
    "gradient": dict(kind="grid", rows=4, cols=5, depth=10, batch=256, trainable=True,
                     n_slice=0, trials=8, refine="time"),
    # GBS-88-m1 of Sec. 4 (Alg. 1 with squeezers and beam splitters, r = 0.5),
    # Fock cutoff 4 and 8; output patterns of typical photon numbers
    # (circuits.gbs_pattern)
    "gbs": dict(kind="gbs_optical", rows=8, cols=8, cycles=1, d=4, r=0.5, n_slice=0,
                trials=64, refine="time"),
    "gbs8": dict(kind="gbs_optical", rows=8, cols=8, cycles=1, d=8, r=0.5, n_slice=0,
                 trials=64, refine="time"),
}

# Refined paths are stored (input data, not results): the search takes minutes
# for the 53-qubit network.  A stored path is used only when it was made for
# the same network (hash of leaf labels, dims and open indices) and the same
# greedy search and refinement settings.
PATHS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paths")


def network_hash(tn):
    h = hashlib.sha256()
    h.update(json.dumps([list(map(int, l)) for l in tn.labels]).encode())
    h.update(json.dumps(sorted((int(k), int(v)) for k, v in tn.dims.items())).encode())
    h.update(json.dumps(list(map(int, tn.open))).encode())
    return h.hexdigest()[:16]


def build(name, seed=0, trials=None, refine=None, use_stored=True, **over):
    """``refine``: follow the greedy search with the shared-work-aware
    refinement of tree and slices (``tngen.refine``): False (greedy search
    only), "cmac" (descent on the multiply-adds with reuse), or "time" (that
    descent, then one on the per-step roofline time estimate); default per
    workload (``CONFIGS[name]["refine"]``)."""
    cfg = dict(CONFIGS[name])
    mode = cfg.pop("refine", False) if refine is None else refine
    cfg.pop("refine", None)
    cfg.update(over)
    kind = cfg.pop("kind")
    n_slice = cfg.pop("n_slice", 0)
    cap = cfg.pop("cap_log2", None)
    batch_n = cfg.pop("batch", None)
    trainable = cfg.pop("trainable", False)
    n_trials = cfg.pop("trials", 8) if trials is None else trials
    if kind == "grid":
        circ = circuits.grid_rqc(cfg["rows"], cfg["cols"], cfg["depth"], seed,
                                 inactive=cfg.get("inactive", ()), trainable=trainable)
    elif kind == "gbs_optical":
        circ = circuits.gbs_optical(cfg["rows"], cfg["cols"], cfg["cycles"], seed, d=cfg["d"],
                                    r=cfg["r"])
    else:
        circ = circuits.gbs_like(cfg["rows"], cfg["cols"], cfg["depth"], seed, d=cfg["d"])
    levels = min(circ.d, 4) if kind == "gbs_optical" else circ.d
    outcome = batch = None
    if batch_n:
        batch = circuits.random_bitstrings(circ.n, levels, batch_n, seed)
        tn = network.circuit_network(circ, batch=batch)
    elif kind == "gbs_optical":
        outcome = circuits.gbs_pattern(circ.n, circ.d, cfg["r"], seed)
        tn = network.circuit_network(circ, outcome=outcome)
    else:
        outcome = circuits.random_bitstrings(circ.n, levels, 1, seed)[0]
        tn = network.circuit_network(circ, outcome=outcome)
    tn = network.relabel_compact(tn)
    key = dict(network=network_hash(tn), trials=n_trials, n_slice=n_slice, cap_log2=cap,
               refine=mode or "none")
    stored = os.path.join(PATHS, f"{name}_seed{seed}.json")
    if mode and use_stored and not over and os.path.exists(stored):
        doc = json.load(open(stored))
        if doc.get("key") == key:
            path = [tuple(p) for p in doc["path"]]
            sliced = list(doc["sliced"])
            st = slicing.TreeSets(tn.labels, tn.dims, tn.open, path).stats(sliced)
            return Workload(name=name, circuit=circ, tn=tn, path=path, sliced=sliced, stats=st,
                            outcome=outcome, batch=batch,
                            meta=dict(seed=seed, cap_log2=cap, path_key=key))
    path, sliced, st = slicing.search(tn.labels, tn.dims, tn.open,
                                      n_slice=n_slice if n_slice else 0,
                                      cap_log2=cap, trials=n_trials, seed=seed)
    if mode:
        path, sliced, _ = refine_mod.refine(tn.labels, tn.dims, tn.open, path, sliced,
                                            cap_log2=cap, seed=seed)
        if mode == "time":
            path, sliced, _ = refine_mod.refine(tn.labels, tn.dims, tn.open, path, sliced,
                                                cap_log2=cap, seed=seed, objective="time",
                                                rounds=4)
        st = slicing.TreeSets(tn.labels, tn.dims, tn.open, path).stats(sliced)
    return Workload(name=name, circuit=circ, tn=tn, path=path, sliced=sliced, stats=st,
                    outcome=outcome, batch=batch, meta=dict(seed=seed, cap_log2=cap, path_key=key))


def store_path(name, seed=0):
    """Runs the search (no stored path) and writes tngen/paths/<name>_seed<seed>.json."""
    w = build(name, seed=seed, use_stored=False)
    os.makedirs(PATHS, exist_ok=True)
    doc = dict(key=w.meta["path_key"], path=[list(map(int, p)) for p in w.path],
               sliced=list(map(int, w.sliced)),
               stats={k: float(v) for k, v in w.stats.items()})
    with open(os.path.join(PATHS, f"{name}_seed{seed}.json"), "w") as f:
        json.dump(doc, f)
    return w
