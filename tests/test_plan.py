"""Plan (host side of the library) through the C ABI, on the CPU.

* the library loads and exports every function include/tn.h declares;
* malformed input is rejected with the documented status codes;
* instance counts and multiply-add totals equal the brute-force enumeration
  of named tasks over all slices (Sec. 3.2) done by the oracle;
* executing the plan's own step descriptors on the CPU reproduces the
  oracle's amplitude (layouts, folding of instances, arena offsets).
"""

import json
import os
import re

import numpy as np
import pytest

from oracle import taskgraph, tn_oracle
from tngen import circuits, network, path as tpath, slicing

from paper_2107_09793_amd import binding
from paper_2107_09793_amd.binding import Plan, TnError

from .plan_exec import execute

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_library_exports_every_declared_function():
    hdr = open(os.path.join(ROOT, "include", "tn.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    names = set(re.findall(r"\b(tn_[a-z_0-9]+)\s*\(", hdr))
    assert {"tn_plan_create", "tn_contract", "tn_contract_backward"} <= names
    L = binding.lib()
    for nm in sorted(names):
        assert hasattr(L, nm), nm
    assert set(binding.EXPORTS) == names


def _small_net(seed=0, rows=3, cols=4, depth=8, batch=None):
    circ = circuits.grid_rqc(rows, cols, depth, seed=seed)
    if batch:
        b = circuits.random_bitstrings(circ.n, 2, batch, seed)
        tn = network.relabel_compact(network.circuit_network(circ, batch=b))
    else:
        x = circuits.random_bitstrings(circ.n, 2, 1, seed)[0]
        tn = network.relabel_compact(network.circuit_network(circ, outcome=x))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    return tn, p


def test_rejects_malformed_input():
    tn, p = _small_net()
    with pytest.raises(TnError) as e:
        Plan(tn.labels, tn.dims, tn.open, p[:-1])
    assert e.value.status == binding.TN_E_INVALID
    bad = list(p)
    bad[3] = (bad[3][0], bad[3][0])
    with pytest.raises(TnError) as e:
        Plan(tn.labels, tn.dims, tn.open, bad)
    assert e.value.status == binding.TN_E_INVALID
    dims = dict(tn.dims)
    dims[0] = 3
    with pytest.raises(TnError) as e:
        Plan(tn.labels, dims, tn.open, p)
    assert e.value.status == binding.TN_E_UNSUPPORTED
    labels = [list(l) for l in tn.labels]
    labels[5] = labels[5] + [labels[0][0]] if labels[0][0] not in labels[5] else labels[5]
    with pytest.raises(TnError) as e:
        Plan(labels, tn.dims, tn.open, p)
    assert e.value.status == binding.TN_E_INVALID
    with pytest.raises(TnError) as e:
        Plan(tn.labels, tn.dims, tn.open, p, sliced=[10**6])
    assert e.value.status == binding.TN_E_INVALID


def _worked(D):
    g = json.load(open(os.path.join(GOLD, "worked_example.json")))
    names = g["leaf_order"]
    letters = sorted({c for n in names for c in g["tensors"][n]})
    ids = {c: i for i, c in enumerate(letters)}
    labels = [[ids[c] for c in g["tensors"][n]] for n in names]
    dims = {i: D for i in ids.values()}
    return g, ids, labels, dims, [tuple(x) for x in g["path_ssa"]]


@pytest.mark.parametrize("D", [2, 4])
def test_worked_example_instances(D):
    g, ids, labels, dims, path = _worked(D)
    pl = Plan(labels, dims, [], path, sliced=[ids["e"]])
    inst = [2 ** s["inst_bits"] for s in pl.steps()]
    expect = [1 if c == 1 else D for c in g["instances_when_e_sliced"]]
    assert inst == expect
    info = pl.info()
    # the printed orders D^p are the sizes of the steps' index sets
    assert [len(s) for s in g["step_indices"]] == g["step_cost_power_of_D"]
    # per slice, e is fixed: D^(|set| - [e in set]); with reuse each step
    # additionally runs once per instance (Sec. 2.4 slicing overhead shows
    # at step 6, which does not touch e unsliced but runs for both slices)
    per_slice = [D ** (len(s) - ("e" in s)) for s in g["step_indices"]]
    assert info["cmac_noreuse"] == pytest.approx(D * sum(per_slice))
    assert info["cmac_reuse"] == pytest.approx(sum(i * c for i, c in zip(expect, per_slice)))


@pytest.mark.parametrize("n_slice,batch", [(0, None), (3, None), (5, None), (2, 16)])
def test_statistics_equal_task_enumeration(n_slice, batch):
    tn, p = _small_net(seed=n_slice, batch=batch)
    ts = slicing.TreeSets(tn.labels, tn.dims, tn.open, p)
    sl = slicing.greedy_slices(ts, n_slice=n_slice) if n_slice else []
    pl = Plan.from_network(tn, p, sl)
    info = pl.info()
    ref = taskgraph.enumerate_tasks(tn.labels, tn.dims, tn.open, p, sl)
    assert info["cmac_reuse"] == pytest.approx(ref["flop_reuse"], rel=1e-12)
    assert info["cmac_noreuse"] == pytest.approx(ref["flop_noreuse"], rel=1e-12)
    assert info["cmac_per_slice"] == pytest.approx(ref["flop_sl"], rel=1e-12)
    assert info["n_slices"] == ref["n_slices"]
    # batch counts as instances too: the per-step instance count of the
    # enumeration (slices only) times the batch carried by the step
    steps = pl.steps()
    for k, s in enumerate(steps):
        assert 2 ** s["inst_bits"] == ref["instances"][k]
    if n_slice:
        f = taskgraph.shared_fraction(ref["flop_reuse"], ref["flop_sl"], ref["n_slices"])
        assert info["f_sl"] == pytest.approx(f, rel=1e-12)


@pytest.mark.parametrize("case", ["plain", "sliced3", "sliced6", "batch", "worked", "bosonic"])
def test_cpu_execution_of_plan_matches_oracle(case):
    rng = np.random.default_rng(1)
    if case == "worked":
        g, ids, labels, dims, path = _worked(2)
        tensors = [rng.standard_normal([2] * len(l)) + 1j * rng.standard_normal([2] * len(l))
                   for l in labels]
        open_ids, sl = [], [ids["e"]]
    else:
        if case == "bosonic":
            circ = circuits.gbs_like(2, 3, 2, seed=4, d=4)
            x = circuits.random_bitstrings(circ.n, 4, 1, 4)[0]
            tn = network.relabel_compact(network.circuit_network(circ, outcome=x))
            path = tpath.greedy_path(tn.labels, tn.dims, tn.open)
        else:
            tn, path = _small_net(seed=2, batch=8 if case == "batch" else None)
        labels, dims, tensors, open_ids = tn.labels, tn.dims, tn.tensors, tn.open
        ns = {"plain": 0, "batch": 2, "sliced3": 3, "sliced6": 6, "bosonic": 2}[case]
        ts = slicing.TreeSets(labels, dims, open_ids, path)
        sl = slicing.greedy_slices(ts, n_slice=ns) if ns else []
    pl = Plan(labels, dims, open_ids, path, sl)
    got, per, _ = execute(pl, tensors)
    ref = tn_oracle.contract(tensors, labels, dims, open_ids, path, sl)
    ref = np.asarray(ref).reshape(-1)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-14 * np.max(np.abs(ref)))
    if sl:
        info = pl.info()
        parts = tn_oracle.contract(tensors, labels, dims, open_ids, path, sl, per_slice=True)
        parts = np.asarray(parts).reshape(parts.shape[0], -1)
        # column r of the root holds slice id sum_j bit_j(r) << res_slicebit[j]
        rb = info["n_resident_bits"]
        for r in range(1 << rb):
            sid = sum(((r >> j) & 1) << info["res_slicebit"][j] for j in range(rb))
            assert np.allclose(per[:, r], parts[sid], rtol=1e-12, atol=1e-14)


def _batch_net(seed, rows, cols, depth, batch, n_slice):
    circ = circuits.grid_rqc(rows, cols, depth, seed=seed)
    b = circuits.random_bitstrings(circ.n, 2, batch, seed)
    tn = network.relabel_compact(network.circuit_network(circ, batch=b))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    sl = slicing.greedy_slices(slicing.TreeSets(tn.labels, tn.dims, tn.open, p), n_slice=n_slice)
    return tn, p, sl


@pytest.mark.parametrize("cfg", [(7, 4, 4, 14, 32, 2), (9, 4, 4, 10, 16, 3), (7, 4, 5, 14, 32, 2)])
def test_cpu_execution_of_fused_chains_matches_oracle(cfg):
    """Chains (consecutive stream steps run as one tiled pass) executed on the
    CPU from their descriptors: tile loads through the input strides, LDS
    slots, per-step small operands selected by passive batch bits, tile
    stores through the output strides.  With batches of tiny steps off, every
    step outside a persistent segment may join a chain, so small networks
    have chains with passive and batch bits."""
    tn, p, sl = _batch_net(*cfg)
    pl = Plan.from_network(tn, p, sl, tiny=False, persistent=False)
    info = pl.info()
    chains = pl.chains()
    assert info["n_chains"] == len(chains) > 0
    assert any(ch["pas_in"] for ch in chains)
    steps = pl.steps()
    for ch in chains:
        assert 1 <= len(ch["st"]) <= 8 and ch["tile_bits"] <= 12
        for k in range(ch["first"], ch["last"]):
            assert steps[k + 1]["a"] == pl.n_tensors + k and steps[k]["c_offset"] == -1
        # staged small operands: 4 floats per entry on the matrix cores (k
        # padded to 8 complex values), 2 on the vector units, 4096 floats in all
        def staged(d):
            nk, nn = len(d["kslot"]), len(d["nslot"])
            if 2 <= nk <= 6 and 3 <= nn <= 5 and nk + nn <= 9 and d["nrow"] >= 4:
                return 4 * max(2 ** nk, 8) * 2 ** nn
            return 2 * 2 ** (nk + nn)
        used = sum(staged(d) for d in ch["st"])
        assert used <= 4096
    got, _, _ = execute(pl, tn.tensors)
    ref = np.asarray(tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p, sl)).reshape(-1)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-13 * np.max(np.abs(ref)))
    stepwise = Plan.from_network(tn, p, sl, tiny=False, chain_fused=False)
    assert stepwise.info()["n_chains"] == info["n_chains"]
    assert all(s["c_offset"] >= 0 for s in stepwise.steps())
    got2, _, _ = execute(stepwise, tn.tensors)
    assert np.allclose(got2, ref, rtol=1e-12, atol=1e-13 * np.max(np.abs(ref)))
    # lone chainable steps run as one-step chains unless switched off
    multi = Plan.from_network(tn, p, sl, tiny=False, chain_single=False)
    mch = multi.chains()
    assert all(len(ch["st"]) >= 2 for ch in mch)
    assert len(mch) == sum(len(ch["st"]) >= 2 for ch in chains)
    got3, _, _ = execute(multi, tn.tensors)
    assert np.allclose(got3, ref, rtol=1e-12, atol=1e-13 * np.max(np.abs(ref)))
    unfused = Plan.from_network(tn, p, sl, tiny=False, persistent=False, chains=False)
    assert unfused.info()["n_chains"] == 0
    assert unfused.info()["n_launches"] - info["n_launches"] == sum(
        ch["last"] - ch["first"] for ch in chains) * (1 << info["n_outer_bits"])


def test_some_chain_selects_small_operands_by_batch_bits():
    """Across the chain test networks, some chain step has batch bits (slice
    or output bits held by both operands), which pick the small operand per
    tile; the CPU execution above covers them."""
    found = False
    for cfg in [(7, 4, 4, 14, 32, 2), (9, 4, 4, 10, 16, 3), (7, 4, 5, 14, 32, 2)]:
        tn, p, sl = _batch_net(*cfg)
        pl = Plan.from_network(tn, p, sl, tiny=False)
        found |= any(d["bB"] for ch in pl.chains() for d in ch["st"])
    assert found


def test_chain_descriptors_hold_wide_matrix_core_steps():
    """GEMM-kind steps with up to 2^6 summed and 2^5 new values join chains
    on the matrix-core path (not on the vector-unit path); their descriptors
    carry every summed and new bit, and the CPU execution still matches."""
    circ = circuits.grid_rqc(3, 4, 8, seed=2)
    b = circuits.random_bitstrings(circ.n, 2, 8, 2)
    tn = network.relabel_compact(network.circuit_network(circ, batch=b))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    sl = slicing.greedy_slices(slicing.TreeSets(tn.labels, tn.dims, tn.open, p), n_slice=2)
    pl = Plan(tn.labels, tn.dims, tn.open, p, sl, tiny=False)
    steps = pl.steps()
    wide = [(d, steps[d["step"]]) for ch in pl.chains() for d in ch["st"]
            if steps[d["step"]]["nn"] > 4 or steps[d["step"]]["nk"] > 4]
    assert wide
    for d, s in wide:
        assert len(d["kslot"]) == s["nk"] and len(d["nslot"]) == s["nn"] and d["nrow"] >= 4
    valu = Plan(tn.labels, tn.dims, tn.open, p, sl, tiny=False, chain_mfma=False)
    vsteps = valu.steps()
    for ch in valu.chains():
        for d in ch["st"]:
            assert vsteps[d["step"]]["nk"] <= 4 and vsteps[d["step"]]["nn"] <= 4
    got, _, _ = execute(pl, tn.tensors)
    ref = np.asarray(tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p, sl)).reshape(-1)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-13 * np.max(np.abs(ref)))


def _live_ranges(pl):
    """(produced, last used, start byte, end byte) of every stored result in
    execution order; a chain produces its output and reads all its inputs at
    the position of its last step."""
    steps = pl.steps()
    n = pl.n_tensors
    chains = pl.chains()
    order = [k for k in range(n - 1) if steps[k]["phase"] == 0] + \
            [k for k in range(n - 1) if steps[k]["phase"] == 1]
    order = [k for k in order if steps[k]["chain"] < 0 or chains[steps[k]["chain"]]["last"] == k]
    pos = {k: i for i, k in enumerate(order)}
    consumer = {}
    for k, s in enumerate(steps):
        at = k if s["chain"] < 0 else chains[s["chain"]]["last"]
        consumer[s["a"]] = at
        consumer[s["b"]] = at
    live = []
    for k in order:
        s = steps[k]
        end = pos[consumer[n + k]] if (n + k) in consumer else len(order)
        live.append((pos[k], end, s["c_offset"], s["c_offset"] + s["c_bytes"]))
    return live


@pytest.mark.parametrize("fused", [False, True])
def test_liveness_never_overlaps_live_results(fused):
    if fused:
        tn, p, sl = _batch_net(7, 4, 4, 14, 32, 2)
        pl = Plan.from_network(tn, p, sl, tiny=False, persistent=False)
        assert pl.info()["n_chains"] > 0
    else:
        tn, p = _small_net(seed=3, rows=4, cols=4, depth=8)
        ts = slicing.TreeSets(tn.labels, tn.dims, tn.open, p)
        sl = slicing.greedy_slices(ts, n_slice=3)
        pl = Plan.from_network(tn, p, sl, tiny=False)
    live = _live_ranges(pl)
    for i in range(len(live)):
        for j in range(i + 1, len(live)):
            a, b = live[i], live[j]
            if a[0] <= b[1] and b[0] <= a[1]:      # lifetimes overlap
                assert a[3] <= b[2] or b[3] <= a[2], (a, b)
    info = pl.info()
    assert info["arena_bytes"] <= info["bytes_no_deletion"]


def test_outer_split_and_no_reuse_statistics():
    tn, p = _small_net(seed=4, rows=4, cols=4, depth=10)
    ts = slicing.TreeSets(tn.labels, tn.dims, tn.open, p)
    sl = slicing.greedy_slices(ts, n_slice=4)
    full = Plan.from_network(tn, p, sl).info()
    assert full["n_outer_bits"] == 0 and full["n_resident_bits"] == 4
    assert full["cmac_exec"] == pytest.approx(full["cmac_reuse"])
    capped = Plan.from_network(tn, p, sl, max_resident_bits=2).info()
    assert capped["n_resident_bits"] <= 2 and capped["n_outer_bits"] >= 2
    assert capped["cmac_exec"] >= full["cmac_exec"]
    assert capped["cmac_exec"] <= full["cmac_noreuse"] + 1e-6
    nr = Plan.from_network(tn, p, sl, no_reuse=True).info()
    assert nr["cmac_exec"] == pytest.approx(full["cmac_noreuse"])
    lim = Plan.from_network(tn, p, sl, workspace_limit=full["arena_bytes"] // 3).info()
    assert lim["arena_bytes"] <= full["arena_bytes"] // 3


def test_workspace_too_small_is_reported():
    """TN_E_WORKSPACE before any device work: the status is returned while
    the pointers are only checked for NULL (fake addresses are never used)."""
    import ctypes
    tn, p = _small_net(seed=2)
    ts = slicing.TreeSets(tn.labels, tn.dims, tn.open, p)
    pl = Plan.from_network(tn, p, slicing.greedy_slices(ts, n_slice=2))
    info = pl.info()
    L = binding.lib()
    fake = (ctypes.c_void_p * pl.n_tensors)(*([0x1000] * pl.n_tensors))
    for ws_bytes in (0, info["workspace_bytes"] - 1):
        st = L.tn_contract(pl._h, fake, None, 0, binding.TN_OUT_SUM, ctypes.c_void_p(0x2000),
                           ctypes.c_void_p(0x3000), ws_bytes, None)
        assert st == binding.TN_E_WORKSPACE
        assert b"workspace" in L.tn_last_error()
    grads = (ctypes.c_void_p * pl.n_tensors)(*([0x4000] * pl.n_tensors))
    st = L.tn_contract_backward(pl._h, fake, ctypes.c_void_p(0x2000), grads, None, 0,
                                ctypes.c_void_p(0x3000), info["workspace_backward_bytes"] - 1,
                                None)
    assert st == binding.TN_E_WORKSPACE


@pytest.mark.parametrize("batch", [None, 8])
def test_invariant_results_reused_across_calls(batch):
    """Variable leaves (the output leaves): the steps depending on none of
    them run first; their results consumed later stay in the arena, so a
    second run from position n_invariant with new output leaves reuses them
    (Sec. 3.2, shared work kept across amplitudes).  The reused run ignores
    the leaves only invariant steps read (they are zeroed here), which shows
    the invariant steps really are skipped."""
    circ = circuits.grid_rqc(3, 4, 8, seed=4)
    outs = circuits.random_bitstrings(circ.n, 2, 3 * (batch or 1), 4)
    nets = []
    for i in range(3):
        if batch:
            tn = network.circuit_network(circ, batch=outs[i * batch:(i + 1) * batch])
        else:
            tn = network.circuit_network(circ, outcome=outs[i])
        nets.append(network.relabel_compact(tn))
    tn = nets[0]
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    sl = slicing.greedy_slices(slicing.TreeSets(tn.labels, tn.dims, tn.open, p), n_slice=3)
    var = tn.meta["output_leaves"]
    pl = Plan(tn.labels, tn.dims, tn.open, p, sl, variable_leaves=var)
    info = pl.info()
    steps, sched = pl.steps(), pl.schedule()
    n = pl.n_tensors
    below = [set() for _ in range(2 * n - 1)]
    for t in range(n):
        below[t] = {t}
    for k, s in enumerate(steps):
        below[n + k] = below[s["a"]] | below[s["b"]]
    inv = [k for k in range(n - 1) if not below[n + k] & set(var)]
    assert sorted(sched[:info["n_invariant"]]) == sorted(inv) and 0 < len(inv) < n - 1
    assert info["n_launches_reuse"] < info["n_launches"]
    got, _, arena = execute(pl, tn.tensors)
    ref = tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p, sl)
    assert np.allclose(got, np.asarray(ref).reshape(-1), rtol=1e-12)
    inv_set = set(inv)
    only_inv = [t for t in range(n)
                if any(k in inv_set for k, s in enumerate(steps) if t in (s["a"], s["b"]))]
    assert only_inv
    for other in nets[1:]:
        assert other.labels == tn.labels
        leaves = [np.zeros_like(x) if t in only_inv else x for t, x in enumerate(other.tensors)]
        got, _, arena = execute(pl, leaves, arena=arena, start=info["n_invariant"])
        ref = tn_oracle.contract(other.tensors, tn.labels, tn.dims, tn.open, p, sl)
        assert np.allclose(got, np.asarray(ref).reshape(-1), rtol=1e-12)


def _pair(nb, nm, nn, nk):
    """Two tensors A[b, m, k], B[b, k, n] of dimension-2 indices, every free
    and batch index open: one pairwise step of that shape."""
    ids = list(range(nb + nm + nn + nk))
    bat, row = ids[:nb], ids[nb:nb + nm]
    col, summ = ids[nb + nm:nb + nm + nn], ids[nb + nm + nn:]
    dims = {i: 2 for i in ids}
    return [bat + row + summ, bat + summ + col], dims, bat + row + col


# (precision, configuration, nb, nm, nn, nk) -> configuration that runs
STREAM_FALLBACKS = [
    ("c64", 9, 0, 17, 7, 6, 9), ("c64", 9, 0, 13, 6, 5, 9), ("c64", 9, 0, 11, 9, 6, 9),
    ("c64", 9, 0, 10, 5, 5, 9),
    ("c64", 9, 0, 17, 4, 9, 8),       # too many summed values for three products
    ("c64", 9, 0, 16, 5, 8, 8),
    ("c64", 9, 0, 11, 7, 4, 8),       # k tile of 32 needs nk >= 5
    ("c64", 9, 0, 12, 4, 6, 8),       # 16 columns: below a 32-column tile
    ("c64", 9, 1, 12, 7, 6, 0),       # a batch bit: the rule's 128 x 64
    ("c64", 9, 0, 12, 4, 9, 7),       # few tiles, long sum: split over k, no stream
    ("c64", 8, 0, 17, 4, 9, 8),       # 16 x 512 B entries = 2^13
    ("c64", 8, 0, 16, 5, 9, 1),       # 2^14 B entries: the rule's 128 x 32
    ("c64", 8, 0, 9, 6, 6, 0),        # fewer than 2^10 rows
    ("split_bf16", 9, 0, 17, 7, 6, 8),   # column tiles of 64, 2^12 B entries
    ("split_bf16", 8, 0, 16, 5, 8, 8),
    ("split_bf16", 8, 0, 17, 4, 9, 7),   # 2^(12 - 9) columns: below 16
    ("split_bf16", 8, 0, 11, 7, 4, 0),   # k tile of 32 needs nk >= 5
]


@pytest.mark.parametrize("case", STREAM_FALLBACKS, ids=lambda c: "%s_cfg%d_b%dm%dn%dk%d" % c[:6])
def test_stream_tile_fallbacks(case):
    """The stream configurations fall back 9 -> 8 -> the rule's configuration
    on shapes they do not take; the step reports the one that runs."""
    precision, cfg, nb, nm, nn, nk, want = case
    labels, dims, open_ids = _pair(nb, nm, nn, nk)
    pl = Plan(labels, dims, open_ids, [(0, 1)], precision=precision, gemm_config=cfg)
    st = pl.step(0)
    assert st["kind_name"] == "gemm" and st["tile"] == cfg
    assert (st["nb"], st["nm"], st["nn"], st["nk"]) == (nb, nm, nn, nk)
    assert st["tile_run"] == want


def test_amplitude_batch_option_matches_explicit_batch_index():
    """tn_plan_options.batch / batched_leaves: the library adds the batch index
    (id n_index) as the leading axis of the listed leaves and the leading open
    index.  The plan equals the one of the network that carries that index
    explicitly, and its CPU execution equals the oracle on the same leaves
    (8 outcomes of a 3x4 circuit, 2 sliced indices)."""
    tn, p, sl = _batch_net(seed=3, rows=3, cols=4, depth=6, batch=8, n_slice=2)
    bi = tn.batch_index
    # move the batch index to the last id, then drop it from the description
    others = sorted(i for i in tn.dims if i != bi)
    mp = {i: j for j, i in enumerate(others)}
    mp[bi] = len(others)
    labels = [[mp[i] for i in l] for l in tn.labels]
    dims = {mp[i]: v for i, v in tn.dims.items()}
    open_ids = [mp[i] for i in tn.open]
    sliced = [mp[i] for i in sl]
    bid = mp[bi]
    assert open_ids == [bid]
    batched = [t for t, l in enumerate(labels) if bid in l]
    assert all(labels[t][0] == bid for t in batched)   # leading axis
    plain_labels = [l[1:] if t in batched else l for t, l in enumerate(labels)]
    plain_dims = {i: v for i, v in dims.items() if i != bid}
    explicit = Plan(labels, dims, open_ids, p, sliced)
    opt = Plan(plain_labels, plain_dims, [], p, sliced, batch=8, batched_leaves=batched)
    for key in ("n_index", "cmac_reuse", "cmac_noreuse", "n_slices", "arena_bytes", "n_launches"):
        assert opt.info()[key] == explicit.info()[key], key
    assert opt.steps() == explicit.steps()
    assert opt.labels == labels and opt.open_ids == open_ids
    got, _, _ = execute(opt, tn.tensors)
    ref = np.asarray(tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p, sl)).reshape(-1)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-14 * np.max(np.abs(ref)))
    # errors: not a power of two, bad leaf lists
    with pytest.raises(TnError) as e:
        Plan(plain_labels, plain_dims, [], p, sliced, batch=6, batched_leaves=batched)
    assert e.value.status == binding.TN_E_UNSUPPORTED
    for bad in ([], [batched[0], batched[0]], [len(labels)]):
        with pytest.raises(TnError) as e:
            Plan(plain_labels, plain_dims, [], p, sliced, batch=8, batched_leaves=bad)
        assert e.value.status == binding.TN_E_INVALID


def test_batches_of_tiny_steps():
    """Tiny steps (at most 2^13 multiply-adds and 2^11 outputs, so that one
    workgroup gives each thread a few outputs) run in batches of up to 20
    consecutive ones per launch of one workgroup: they never join chains, the
    batches stay inside one schedule group, the launch count drops by the
    batched steps, and the CPU execution of the schedule (the order the
    batches run in) matches the oracle.  TN_FLAG_NO_TINY and persistent
    segments switch batches off."""
    tn, p, sl = _batch_net(3, 4, 4, 12, 16, 2)
    on = Plan.from_network(tn, p, sl)
    off = Plan.from_network(tn, p, sl, tiny=False)
    assert on.info()["n_launches"] < off.info()["n_launches"]
    steps = on.steps()
    tiny = [k for k, s in enumerate(steps) if s["tiny_batch"] >= 0]
    assert tiny and all(steps[k]["chain"] < 0 for k in tiny)
    assert all(steps[k]["cmac"] <= 2 ** 13 and steps[k]["nb"] + steps[k]["nm"] + steps[k]["nn"] <= 11
               and steps[k]["chunks"] <= 1 and steps[k]["kind_name"] != "splitk" for k in tiny)
    assert all(s["tiny_batch"] < 0 for s in off.steps())
    got, _, _ = execute(on, tn.tensors)
    ref = np.asarray(tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p, sl)).reshape(-1)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-13 * np.max(np.abs(ref)))
    # the 3x4 circuit of one amplitude: a few launches in all
    circ = circuits.grid_rqc(3, 4, 8, seed=0)
    x = circuits.random_bitstrings(12, 2, 1, 0)[0]
    t1 = network.relabel_compact(network.circuit_network(circ, outcome=x))
    p1 = tpath.greedy_path(t1.labels, t1.dims, t1.open)
    a = Plan.from_network(t1, p1)
    b = Plan.from_network(t1, p1, tiny=False)
    assert a.info()["n_launches"] <= 16 < b.info()["n_launches"]
    assert Plan.from_network(t1, p1, persistent=True).info()["n_launches"] == \
        Plan.from_network(t1, p1, persistent=True, tiny=False).info()["n_launches"]


@pytest.mark.parametrize("net", ["batch", "plain", "sliced"])
def test_tiny_levels_are_safe_to_run_at_once(net):
    """Inside a batch of tiny steps the steps of one level run at the same
    time: every operand produced in the batch comes from a lower level, the
    results of one level overlap neither each other nor any buffer a step of
    that level reads, and no result overlaps a buffer still to be read later
    in the batch (the batch's frees are deferred to its end)."""
    if net == "batch":
        tn, p, sl = _batch_net(3, 4, 4, 12, 16, 2)
    else:
        circ = circuits.grid_rqc(3, 4, 8, seed=4) if net == "plain" else \
            circuits.grid_rqc(4, 4, 10, seed=4)
        x = circuits.random_bitstrings(circ.n, 2, 1, 4)[0]
        tn = network.relabel_compact(network.circuit_network(circ, outcome=x))
        p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
        sl = [] if net == "plain" else \
            slicing.greedy_slices(slicing.TreeSets(tn.labels, tn.dims, tn.open, p), n_slice=3)
    pl = Plan.from_network(tn, p, sl)
    steps = pl.steps()
    n = pl.n_tensors
    sched = pl.schedule()
    batches = {}
    for pos, k in enumerate(sched):
        b = steps[k]["tiny_batch"]
        if b >= 0:
            batches.setdefault(b, []).append((pos, k))
    assert batches
    for b, mem in batches.items():
        pos = [q for q, _ in mem]
        assert pos == list(range(pos[0], pos[0] + len(pos)))   # consecutive
        assert 2 <= len(mem) <= 20
        level = {n + k: steps[k]["tiny_level"] for _, k in mem}
        levels = [steps[k]["tiny_level"] for _, k in mem]
        assert levels == sorted(levels)

        def rng(node):
            s = steps[node - n]
            return (s["c_offset"], s["c_offset"] + s["c_bytes"])

        def overlap(x, y):
            return x[0] < y[1] and y[0] < x[1]
        for _, k in mem:
            s = steps[k]
            for x in (s["a"], s["b"]):
                if x in level:
                    assert level[x] < s["tiny_level"]
        for _, k in mem:
            out = rng(n + k)
            for _, k2 in mem:
                if k2 == k:
                    continue
                s2 = steps[k2]
                if s2["tiny_level"] == steps[k]["tiny_level"]:
                    assert not overlap(out, rng(n + k2))
                # a later or concurrent reader's operand produced before the batch
                if s2["tiny_level"] >= steps[k]["tiny_level"]:
                    for x in (s2["a"], s2["b"]):
                        if x >= n and x not in level and x != n + k:
                            assert not overlap(out, rng(x)), (k, k2, x)
    got, _, _ = execute(pl, tn.tensors)
    ref = np.asarray(tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p, sl)).reshape(-1)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-13 * np.max(np.abs(ref)))
