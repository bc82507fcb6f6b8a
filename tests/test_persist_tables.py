"""Persistent segments (TN_FLAG_PERSISTENT), checked on the CPU from the
control tables tn_contract uploads (``tn_plan_segment_tables``).

For the 30-qubit workload (the plan whose first GPU run with segments did not
finish) and for three small networks:

* every descriptor's producer dependencies point to earlier positions of the
  same segment, and an operand read inside a segment is exactly the result
  of the dependency it names (pointer equality), never of a later step;
* results written inside a segment overlap no buffer another step of the
  segment reads or writes (steps of a segment run concurrently);
* every operand's bit strides stay inside its buffer;
* the item table lists each step's items contiguously, in segment order, and
  each counter's wait target equals the number of items that publish to it;
* the tables sit inside the workspace, after the arena and the split-k
  scratch, with zeroed counters and error word;
* a simulation of the ticket / counter protocol with many workers under
  random interleavings always drains;
* for the small networks, the descriptors executed as the kernel reads them
  (item -> outputs, bit-stride addressing) reproduce the oracle.
"""

import numpy as np
import pytest

from oracle import tn_oracle
from tngen import circuits, network, path as tpath, slicing, workloads

from paper_2107_09793_amd.binding import Plan

from .plan_exec import bit_offsets

DESC = np.dtype([("A", "<u8"), ("B", "<u8"), ("C", "<u8"),
                 ("nb", "<i4"), ("nm", "<i4"), ("nn", "<i4"), ("nk", "<i4"),
                 ("n_items", "<i4"), ("item0", "<i4"), ("dep0", "<i4"), ("dep1", "<i4")] +
                [(k, "i1", (24,)) for k in ("sA_b", "sB_b", "sC_b", "sA_m", "sC_m", "sB_n",
                                            "sC_n", "sA_k", "sB_k")])
assert DESC.itemsize == 272
CTR_STRIDE = 32
WS_BASE = 0x7000_0000_0000
LEAF_BASE = 0x1000_0000_0000


def _small_cases():
    out = []
    w = workloads.build("plain", seed=1, trials=2)
    out.append(("plain", w.tn, w.path, w.sliced, {}))
    circ = circuits.grid_rqc(4, 4, 8, seed=5)
    x = circuits.random_bitstrings(16, 2, 1, 5)[0]
    tn = network.relabel_compact(network.circuit_network(circ, outcome=x))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    sl = slicing.greedy_slices(slicing.TreeSets(tn.labels, tn.dims, tn.open, p), n_slice=5)
    out.append(("sliced_outer", tn, p, sl, dict(max_resident_bits=2)))
    circ = circuits.grid_rqc(3, 5, 8, seed=3)
    batch = circuits.random_bitstrings(15, 2, 64, 3)
    tn = network.relabel_compact(network.circuit_network(circ, batch=batch))
    p = tpath.greedy_path(tn.labels, tn.dims, tn.open)
    sl = slicing.greedy_slices(slicing.TreeSets(tn.labels, tn.dims, tn.open, p), n_slice=2)
    out.append(("batch", tn, p, sl, {}))
    return out


def _leaf_layout(tn):
    """Fake, disjoint device addresses of the leaves (never dereferenced)."""
    sizes = [int(np.prod([tn.dims[i] for i in lab], dtype=np.int64)) for lab in tn.labels]
    bases = [LEAF_BASE + t * (1 << 32) for t in range(len(sizes))]
    return bases, sizes


def _tables(pl, tn):
    bases, sizes = _leaf_layout(tn)
    blob, lays = pl.segment_tables(bases, WS_BASE)
    segs = []
    for L in lays:
        d = np.frombuffer(blob, DESC, count=L["n_steps"], offset=L["off_desc"]).copy()
        items = np.frombuffer(blob, "<i4", count=L["n_items"], offset=L["off_items"]).copy()
        ctr = np.frombuffer(blob, "<i4", count=CTR_STRIDE * (L["n_steps"] + 2),
                            offset=L["off_ctr"]).copy()
        segs.append((L, d, items, ctr))
    return blob, segs, bases, sizes


def _check_tables(pl, tn):
    info = pl.info()
    assert info["n_segments"] > 0
    blob, segs, bases, sizes = _tables(pl, tn)
    assert len(blob) == info["segment_table_bytes"]
    assert np.frombuffer(blob, "<i4", count=64).sum() == 0        # header / error word
    off = info["segment_table_offset"]
    arena = info["arena_bytes"]
    assert off >= arena and off % 256 == 0
    assert off + info["segment_table_bytes"] <= info["workspace_bytes"]
    sched = pl.schedule()
    steps = pl.steps()
    n = pl.n_tensors

    def operand_range(ptr, nbits, strides):
        """Check a read stays inside its buffer; return (lo, hi) if in the arena."""
        span = int(sum(1 << int(s) for s in strides))   # largest element offset
        if WS_BASE <= ptr < WS_BASE + arena:
            o = ptr - WS_BASE
            assert o % 8 == 0
            assert sorted(int(s) for s in strides) == list(range(nbits)), "dense operand"
            assert o + 8 * (1 << nbits) <= arena
            return (o, o + 8 * (1 << nbits))
        t = (ptr - LEAF_BASE) >> 32
        assert 0 <= t < n and ptr >= bases[t]
        assert (ptr - bases[t]) // 8 + span < sizes[t]
        return None

    n_execs = {}
    for L, d, items, ctr in segs:
        ln = L["n_steps"]
        n_execs[L["segment"]] = n_execs.get(L["segment"], 0) + 1
        assert ctr.sum() == 0
        # item table: contiguous per step, in segment order
        assert d["item0"][0] == 0
        assert np.all(d["item0"][1:] == d["item0"][:-1] + d["n_items"][:-1])
        assert d["item0"][-1] + d["n_items"][-1] == L["n_items"] == len(items)
        assert np.array_equal(items, np.repeat(np.arange(ln), d["n_items"]))
        outs = 1 << (d["nb"] + d["nm"] + d["nn"]).astype(np.int64)
        assert np.array_equal(d["n_items"], (outs + 255) // 256)
        # schedule: the descriptors are the plan's steps at these positions
        for i in range(ln):
            s = steps[sched[L["first_pos"] + i]]
            assert (d["nb"][i], d["nm"][i], d["nn"][i], d["nk"][i]) == \
                (s["nb"], s["nm"], s["nn"], s["nk"])
            assert d["C"][i] == WS_BASE + s["c_offset"]
        c_rng = []
        reads = []
        for i in range(ln):
            nb, nm, nn, nk = (int(d[k][i]) for k in ("nb", "nm", "nn", "nk"))
            deps = [int(x) for x in (d["dep0"][i], d["dep1"][i]) if x >= 0]
            assert all(0 <= x < i for x in deps)
            assert (d["dep1"][i] < 0) or (d["dep0"][i] >= 0)
            ra = operand_range(int(d["A"][i]), nb + nm + nk,
                               list(d["sA_b"][i][:nb]) + list(d["sA_m"][i][:nm]) +
                               list(d["sA_k"][i][:nk]))
            rb = operand_range(int(d["B"][i]), nb + nn + nk,
                               list(d["sB_b"][i][:nb]) + list(d["sB_n"][i][:nn]) +
                               list(d["sB_k"][i][:nk]))
            rc = operand_range(int(d["C"][i]), nb + nm + nn,
                               list(d["sC_b"][i][:nb]) + list(d["sC_m"][i][:nm]) +
                               list(d["sC_n"][i][:nn]))
            assert rc is not None
            # an operand produced inside the segment is named as a dependency
            named = []
            for ptr in (int(d["A"][i]), int(d["B"][i])):
                prod = [j for j in range(ln) if int(d["C"][j]) == ptr]
                assert all(j < i for j in prod), "reads a result produced later in the segment"
                named += prod
            assert sorted(named) == sorted(deps)
            c_rng.append(rc)
            reads.append([(r, j) for r, j in ((ra, d["dep0"][i]), (rb, d["dep1"][i])) if r])
        # concurrent steps: a result overlaps nothing else of the segment
        for i in range(ln):
            lo, hi = c_rng[i]
            for j in range(ln):
                if j != i:
                    assert hi <= c_rng[j][0] or c_rng[j][1] <= lo, ("results overlap", i, j)
                for (rlo, rhi), _ in reads[j]:
                    if (rlo, rhi) == (lo, hi):
                        continue          # reads exactly this result (a named dependency)
                    assert rhi <= lo or hi <= rlo, ("result overlaps a read", i, j)
        _simulate(d, items, workers=min(L["n_items"], 256), seed=L["segment"])
    return segs, bases


def _simulate(d, items, workers, seed):
    """The kernel's protocol: a worker takes the next ticket, waits until the
    items of its step's producers are all published, then publishes.  Random
    interleavings of many workers must always drain."""
    rng = np.random.default_rng(seed)
    ln = len(d)
    need = d["n_items"].astype(np.int64)
    deps = [[int(x) for x in (d["dep0"][i], d["dep1"][i]) if x >= 0] for i in range(ln)]
    cnt = np.zeros(ln, np.int64)
    ticket = 0
    held = []                      # tickets claimed and not yet published
    free = workers
    while ticket < len(items) or held:
        ready = [t for t in held if all(cnt[x] == need[x] for x in deps[items[t]])]
        can_claim = free > 0 and ticket < len(items)
        assert ready or can_claim, "protocol deadlock"
        if can_claim and (not ready or rng.random() < 0.5):
            held.append(ticket)
            ticket += 1
            free -= 1
        else:
            t = ready[rng.integers(len(ready))]
            held.remove(t)
            cnt[items[t]] += 1
            free += 1
    assert np.array_equal(cnt, need)


def _emulate(pl, tn, segs, bases):
    """Execute the plan in schedule order, segment steps from their
    descriptors exactly as the kernel indexes them; returns per-slice rows."""
    info = pl.info()
    assert info["n_outer_bits"] == 0, "leaf offsets per outer iteration are not emulated"
    n = pl.n_tensors
    steps = pl.steps()
    sched = pl.schedule()
    leaves = [np.asarray(x, np.complex128).reshape(-1) for x in tn.tensors]
    arena = np.full(max(info["arena_bytes"] // 8, 1), np.nan + 0j)
    seg_at = {}
    for L, d, items, ctr in segs:
        seg_at.setdefault(L["first_pos"], {})[L["execution"]] = (L, d)

    def mem(ptr):
        if WS_BASE <= ptr < WS_BASE + info["arena_bytes"]:
            return arena, (ptr - WS_BASE) // 8
        t = (ptr - LEAF_BASE) >> 32
        return leaves[t], (ptr - bases[t]) // 8

    pos = 0
    while pos < len(sched):
        if pos in seg_at:
            L, d = seg_at[pos][0]
            for i in range(L["n_steps"]):
                _run_desc(d[i], mem)
            pos += L["n_steps"]
            continue
        k = sched[pos]
        assert steps[k]["chain"] < 0, "segment cases run without chains here"
        _run_step(steps[k], n, leaves, arena, steps)
        pos += 1
    root = arena[steps[n - 2]["c_offset"] // 8:]
    oo = bit_offsets(info["root_open_log2"][:info["n_open_bits"]])
    orr = bit_offsets(info["root_res_log2"][:info["n_resident_bits"]])
    return root[oo[:, None] + orr[None, :]]


def _run_desc(D, mem):
    """k_persistent's arithmetic for every item of one descriptor."""
    nb, nm, nn, nk = int(D["nb"]), int(D["nm"]), int(D["nn"]), int(D["nk"])
    o = np.arange(1 << (nb + nm + nn), dtype=np.int64)
    nidx = o & ((1 << nn) - 1)
    m = (o >> nn) & ((1 << nm) - 1)
    b = o >> (nn + nm)

    def scat(idx, s, cnt):
        off = np.zeros_like(idx)
        for j in range(cnt):
            off += ((idx >> j) & 1) << int(s[j])
        return off
    A, a0 = mem(int(D["A"]))
    B, b0 = mem(int(D["B"]))
    C, c0 = mem(int(D["C"]))
    oa = a0 + scat(m, D["sA_m"], nm) + scat(b, D["sA_b"], nb)
    ob = b0 + scat(nidx, D["sB_n"], nn) + scat(b, D["sB_b"], nb)
    k = np.arange(1 << nk, dtype=np.int64)
    acc = (A[oa[:, None] + scat(k, D["sA_k"], nk)[None, :]] *
           B[ob[:, None] + scat(k, D["sB_k"], nk)[None, :]]).sum(1)
    C[c0 + scat(nidx, D["sC_n"], nn) + scat(m, D["sC_m"], nm) + scat(b, D["sC_b"], nb)] = acc


def _run_step(s, n, leaves, arena, steps):
    def src(node):
        if node < n:
            return leaves[node], 0
        return arena, steps[node - n]["c_offset"] // 8
    A, a0 = src(s["a"])
    B, b0 = src(s["b"])
    ia = (a0 + bit_offsets(s["sA_b"])[:, None, None] + bit_offsets(s["sA_m"])[None, :, None]
          + bit_offsets(s["sA_k"])[None, None, :])
    ib = (b0 + bit_offsets(s["sB_b"])[:, None, None] + bit_offsets(s["sB_k"])[None, :, None]
          + bit_offsets(s["sB_n"])[None, None, :])
    c = np.matmul(A[ia], B[ib])
    ic = (s["c_offset"] // 8 + bit_offsets(s["sC_b"])[:, None, None]
          + bit_offsets(s["sC_m"])[None, :, None] + bit_offsets(s["sC_n"])[None, None, :])
    arena[ic] = c


@pytest.mark.parametrize("case", range(3))
def test_segment_tables_small(case):
    name, tn, p, sl, kw = _small_cases()[case]
    pl = Plan(tn.labels, tn.dims, tn.open, p, sl, persistent=True, chains=False, **kw)
    segs, bases = _check_tables(pl, tn)
    if pl.info()["n_outer_bits"]:
        return   # leaf offsets per outer iteration: covered by the table checks above
    vals = _emulate(pl, tn, segs, bases)                   # (outputs, resident slices)
    ref = tn_oracle.contract(tn.tensors, tn.labels, tn.dims, tn.open, p, sl, per_slice=True)
    ref = np.asarray(ref).reshape(len(ref), -1).T          # (outputs, slices)
    info = pl.info()
    # resident slice bit j of the root is bit res_slicebit[j] of the slice id
    sid = np.zeros(1 << info["n_resident_bits"], np.int64)
    for j, b in enumerate(info["res_slicebit"][:info["n_resident_bits"]]):
        sid += ((np.arange(len(sid)) >> j) & 1) << b
    assert np.allclose(vals, ref[:, sid], rtol=1e-10, atol=1e-13 * np.abs(ref).max())


@pytest.mark.slow
def test_segment_tables_30_qubit_workload():
    w = workloads.build("sliced", seed=0)
    for chains in (True, False):
        pl = Plan.from_network(w.tn, w.path, w.sliced, persistent=True, chains=chains,
                               workspace_limit=0)
        _check_tables(pl, w.tn)
