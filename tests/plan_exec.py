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


def execute(plan, leaves, dtype=np.complex128, arena=None, start=0):
    """Runs the schedule from position ``start`` (earlier results are read
    from ``arena``, as left by a previous run: the reuse of invariant
    results).  Returns (sum over resident slices, per-slice values, arena)."""
    info = plan.info()
    if info["n_outer_bits"] != 0:
        raise NotImplementedError("CPU executor handles all-resident plans only")
    n = plan.n_tensors
    steps = plan.steps()
    if arena is None:
        arena = np.full(max(info["arena_bytes"] // 8, 1), np.nan + 0j, dtype=dtype)
    flat = [np.asarray(x, dtype).reshape(-1) for x in leaves]

    def src(node):
        if node < n:
            return flat[node], 0
        return arena, steps[node - n]["c_offset"] // 8

    chains = plan.chains() if info.get("n_chains", 0) else []
    order = plan.schedule()[start:]
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
    return vals.sum(1), vals, arena


def leaf_outer_offsets(plan, tn):
    """Element offset of every leaf's sub-block for each outer iteration:
    offs[t][it] (a leaf with no outer bits: all zero)."""
    info = plan.info()
    n_outer = info["n_outer_bits"]
    # slice-id bit positions: last sliced index least significant
    idbits = []
    for e in reversed(list(plan.sliced)):
        w = int(tn.dims[e]).bit_length() - 1
        for j in range(w):
            idbits.append((e, j))
    outer = [idbits[b] for b in info["outer_slicebit"][:n_outer]]
    offs = []
    for lab in tn.labels:
        lab = list(lab)
        stride = {}
        s = 0
        for ax in reversed(range(len(lab))):
            w = int(tn.dims[lab[ax]]).bit_length() - 1
            for j in range(w):
                stride[(lab[ax], j)] = s + j
            s += w
        o = np.zeros(1 << n_outer, dtype=np.int64)
        for j, key in enumerate(outer):
            if key in stride:
                o += ((np.arange(1 << n_outer) >> j) & 1) << stride[key]
        offs.append(o)
    return offs


def execute_backward(plan, tn, grad_out, slice_ids=None, dtype=np.complex128):
    """tn_contract_backward's sequence, step for step, on the CPU: the
    backward's forward pass (fused chains where the plan says so), zeroed
    frontier gradients, per outer iteration the phase-1 forward, root
    gradient and block adjoints (recompute, then reverse sweep), then the
    phase-0 block adjoints.  Every buffer lives at the plan's offsets in one
    flat workspace, so a liveness mistake corrupts the result.  Returns the
    leaf gradients (PyTorch convention)."""
    info = plan.info()
    n = plan.n_tensors
    steps = plan.steps()
    sched = plan.schedule()
    T = plan.backward_tables()
    chains = plan.chains() if info["n_chains"] else []
    root = 2 * n - 2
    W = np.full(max(info["workspace_backward_bytes"] // 8, 1), np.nan + 0j, dtype=dtype)
    leaves = [np.asarray(x, dtype).reshape(-1) for x in tn.tensors]
    grads = [np.zeros_like(x) for x in leaves]
    offs = leaf_outer_offsets(plan, tn)
    g_out = np.asarray(grad_out, dtype).reshape(-1)
    n_out = 1 << info["n_open_bits"]
    n_res = info["n_resident_bits"]
    if n == 1:
        raise NotImplementedError

    def val(x, it, rec):
        if x < n:
            return leaves[x], int(offs[x][it])
        key = "recompute_off" if rec and T["keep"][x] == 0 else "value_off"
        assert T[key][x] >= 0, (x, key)
        return W, int(T[key][x]) // 8

    def gradp(x, it):
        if x < n:
            return grads[x], int(offs[x][it])
        assert T["grad_off"][x] >= 0, x
        return W, int(T["grad_off"][x]) // 8

    def idx3(o, s1, s2, s3):
        return (o + bit_offsets(s1)[:, None, None] + bit_offsets(s2)[None, :, None]
                + bit_offsets(s3)[None, None, :])

    def fwd_step(s, A, a0, B, b0, C, c0):
        C[idx3(c0, s["sC_b"], s["sC_m"], s["sC_n"])] = np.matmul(
            A[idx3(a0, s["sA_b"], s["sA_m"], s["sA_k"])], B[idx3(b0, s["sB_b"], s["sB_k"], s["sB_n"])])

    def forward(q0, q1, it):
        for q in range(q0, q1):
            k = sched[q]
            s = steps[k]
            fused = s["chain"] >= 0 and bool(T["fuse_chain"][s["chain"]])
            if not fused and n + k == root:
                continue
            if fused:
                ch = chains[s["chain"]]
                if ch["last"] != k:
                    continue
                X, x0 = val(steps[ch["first"]]["a"], it, False)
                Bs = [val(steps[d["step"]]["b"], it, False) for d in ch["st"]]
                _chain(ch, X, x0, Bs, W, int(T["value_off"][n + k]) // 8, dtype)
                continue
            fwd_step(s, *val(s["a"], it, False), *val(s["b"], it, False), W,
                     int(T["value_off"][n + k]) // 8)

    def root_grad(it, sel):
        g0 = int(T["grad_off"][root]) // 8
        oo = bit_offsets(info["root_open_log2"][:info["n_open_bits"]])
        orr = bit_offsets(info["root_res_log2"][:n_res])
        W[g0 + oo[:, None] + orr[None, :]] = 0
        for r, mult in sel.items():
            W[g0 + oo + orr[r]] = mult * g_out

    def adjoint_step(s, it):
        gC, g0 = gradp(s["c"], it)
        gc = gC[idx3(g0, s["sC_b"], s["sC_m"], s["sC_n"])]
        for x, side in ((s["a"], "A"), (s["b"], "B")):
            G, go = gradp(x, it)
            acc = x < n or bool(T["frontier"][x])
            if side == "A":
                Bv, b0 = val(s["b"], it, True)
                bm = Bv[idx3(b0, s["sB_b"], s["sB_k"], s["sB_n"])]
                d = np.matmul(gc, np.conj(np.swapaxes(bm, 1, 2)))
                ig = idx3(go, s["sA_b"], s["sA_m"], s["sA_k"])
            else:
                Av, a0 = val(s["a"], it, True)
                am = Av[idx3(a0, s["sA_b"], s["sA_m"], s["sA_k"])]
                d = np.matmul(np.conj(np.swapaxes(am, 1, 2)), gc)
                ig = idx3(go, s["sB_b"], s["sB_k"], s["sB_n"])
            G[ig] = G[ig] + d if acc else d

    def adjoint(q0, q1, it):
        blk = T["block_of"]
        bl = []
        q = q0
        while q < q1:
            e = q
            while e < q1 and blk[e] == blk[q]:
                e += 1
            bl.append((q, e))
            q = e
        for b0, b1 in reversed(bl):
            for q in range(b0, b1):
                s = steps[sched[q]]
                if T["keep"][s["c"]] == 0:
                    fwd_step(s, *val(s["a"], it, True), *val(s["b"], it, True), W,
                             int(T["recompute_off"][s["c"]]) // 8)
            for q in range(b1 - 1, b0 - 1, -1):
                adjoint_step(steps[sched[q]], it)

    # selected resident slices per iteration (slice id bits -> iteration, r)
    n_it = 1 << info["n_outer_bits"]
    sel = {}
    ids = range(info["n_slices"]) if slice_ids is None else slice_ids
    for sid in ids:
        it = sum(((sid >> b) & 1) << j for j, b in
                 enumerate(info["outer_slicebit"][:info["n_outer_bits"]]))
        r = sum(((sid >> b) & 1) << j for j, b in enumerate(info["res_slicebit"][:n_res]))
        sel.setdefault(it, {}).setdefault(r, 0)
        sel[it][r] += 1
    n0, N = info["n_phase0"], len(sched)
    forward(0, n0, 0)
    if n0 < N:
        for v in range(n, root + 1):
            if T["frontier"][v]:
                g0 = int(T["grad_off"][v]) // 8
                W[g0:g0 + steps[v - n]["c_bytes"] // 8] = 0
        for it in range(n_it):
            if it not in sel:
                continue
            forward(n0, N, it)
            root_grad(it, sel[it])
            adjoint(n0, N, it)
    else:
        if 0 not in sel:
            return grads
        root_grad(0, sel[0])
    adjoint(0, n0, 0)
    del n_out
    return grads
