"""CPU executor of a plan's step descriptors (test infrastructure).

Runs the schedule that ``tn_plan_step`` reports exactly as the device does:
every operand is read through its bit strides, results are written into one
flat arena at the plan's offsets (so a liveness mistake that lets two live
results overlap corrupts the answer), and the root's resident slice bits are
summed at the end.  It shares only the network arrays with the oracle.
"""

import numpy as np


def bit_offsets(log2s):
    off = np.zeros(1, dtype=np.int64)
    for s in log2s:
        off = np.concatenate([off, off + (np.int64(1) << np.int64(s))])
    return off


def _chain(ch, X, x0, Bs, Y, y0, dtype):
    """A fused chain as the device runs it: every tile of the passive bits is
    loaded into LDS slots, mapped through each step's small operand, stored."""
    tb = ch["tile_bits"]
    pin, pout = bit_offsets(ch["pas_in"]), bit_offsets(ch["pas_out"])
    nt = len(pin)
    buf = np.full((nt, 1 << tb), np.nan + 0j, dtype=dtype)
    slots_in = bit_offsets(ch["in_slot"])
    buf[:, slots_in] = X[x0 + pin[:, None] + bit_offsets(ch["in_log2"])[None, :]]
    tiles = np.arange(nt, dtype=np.int64)
    for d, (B, b0) in zip(ch["st"], Bs):
        nxt = np.full_like(buf, np.nan + 0j)
        rows = bit_offsets(d["rslot"])
        ko, no = bit_offsets(d["kslot"]), bit_offsets(d["nslot"])
        bb = np.zeros(nt, dtype=np.int64)
        for s_b, q in zip(d["bB"], d["bpas"]):
            bb += ((tiles >> q) & 1) << s_b
        bmat = B[b0 + bb[:, None, None] + bit_offsets(d["kB"])[None, :, None]
                 + bit_offsets(d["nB"])[None, None, :]]            # tile, k, n
        a = buf[:, rows[:, None] | ko[None, :]]                     # tile, row, k
        nxt[:, rows[:, None] | no[None, :]] = np.matmul(a, bmat)
        buf = nxt
    Y[y0 + pout[:, None] + bit_offsets(ch["out_log2"])[None, :]] = \
        buf[:, bit_offsets(ch["out_slot"])]


def execute(plan, leaves, dtype=np.complex128):
    info = plan.info()
    if info["n_outer_bits"] != 0:
        raise NotImplementedError("CPU executor handles all-resident plans only")
    n = plan.n_tensors
    steps = plan.steps()
    arena = np.full(max(info["arena_bytes"] // 8, 1), np.nan + 0j, dtype=dtype)
    flat = [np.asarray(x, dtype).reshape(-1) for x in leaves]

    def src(node):
        if node < n:
            return flat[node], 0
        return arena, steps[node - n]["c_offset"] // 8

    chains = plan.chains() if info.get("n_chains", 0) else []
    order = [k for k in range(n - 1) if steps[k]["phase"] == 0] + \
            [k for k in range(n - 1) if steps[k]["phase"] == 1]
    for k in order:
        s = steps[k]
        stepwise = s["chain"] >= 0 and steps[chains[s["chain"]]["first"]]["c_offset"] != -1 \
            if chains else False
        if s["chain"] >= 0 and not stepwise:
            ch = chains[s["chain"]]
            if k != ch["last"]:
                assert s["c_offset"] == -1
                continue
            X, x0 = src(steps[ch["first"]]["a"])
            Bs = [src(steps[d["step"]]["b"]) for d in ch["st"]]
            assert [d["step"] for d in ch["st"]] == list(range(ch["first"], ch["last"] + 1))
            _chain(ch, X, x0, Bs, arena, s["c_offset"] // 8, dtype)
            continue
        A, a0 = src(s["a"])
        B, b0 = src(s["b"])
        ia = (a0 + bit_offsets(s["sA_b"])[:, None, None] + bit_offsets(s["sA_m"])[None, :, None]
              + bit_offsets(s["sA_k"])[None, None, :])
        ib = (b0 + bit_offsets(s["sB_b"])[:, None, None] + bit_offsets(s["sB_k"])[None, :, None]
              + bit_offsets(s["sB_n"])[None, None, :])
        c = np.matmul(A[ia], B[ib])
        ic = (s["c_offset"] // 8 + bit_offsets(s["sC_b"])[:, None, None]
              + bit_offsets(s["sC_m"])[None, :, None] + bit_offsets(s["sC_n"])[None, None, :])
        assert ic.max() * 8 < info["arena_bytes"] + 8
        arena[ic] = c
    if n == 1:
        root, r0 = flat[0], 0
    else:
        root, r0 = arena, steps[n - 2]["c_offset"] // 8
    oo = bit_offsets(info["root_open_log2"][:info["n_open_bits"]])
    orr = bit_offsets(info["root_res_log2"][:info["n_resident_bits"]])
    vals = root[r0 + oo[:, None] + orr[None, :]]
    return vals.sum(1), vals
