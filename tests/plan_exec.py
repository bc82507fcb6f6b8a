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

    order = [k for k in range(n - 1) if steps[k]["phase"] == 0] + \
            [k for k in range(n - 1) if steps[k]["phase"] == 1]
    for k in order:
        s = steps[k]
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
