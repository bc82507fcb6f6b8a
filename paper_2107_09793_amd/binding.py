"""ctypes binding of the C ABI in include/tn.h (argument marshalling only).

Every contraction step runs in the HIP library ``libtnmi.so`` built in this
directory; if it is missing, importing the binding raises.  torch supplies
device memory (leaves, outputs, workspace) and the current stream.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# TNMI_LIB_PATH selects another build of the same library (the host-sanitizer
# build that the CPU test suite runs the plan tests against)
LIB_PATH = os.environ.get("TNMI_LIB_PATH") or os.path.join(_HERE, "libtnmi.so")

TN_OK, TN_E_INVALID, TN_E_UNSUPPORTED, TN_E_WORKSPACE, TN_E_OOM, TN_E_HIP = range(6)
TN_C64, TN_SPLIT_BF16 = 0, 1
TN_OUT_SUM, TN_OUT_PER_SLICE = 0, 1
TN_FLAG_NO_REUSE = 1
TN_FLAG_SIMPLE_KERNELS = 2
TN_FLAG_NO_PERSISTENT = 4
TN_FLAG_NO_CHAIN = 8
TN_FLAG_PERSISTENT = 16
TN_FLAG_CHAIN_VALU = 32
TN_FLAG_CHAIN_STEPWISE = 64
TN_FLAG_CHAIN_NO_SINGLE = 128
TN_FLAG_FIT_BACKWARD = 256
TN_FLAG_NO_TINY = 512
TN_FLAG_GEMM_EMBED = 1024
TN_CKPT_AUTO, TN_CKPT_ALL, TN_CKPT_RECOMPUTE = 0, 1, 2
_CKPT = {"auto": TN_CKPT_AUTO, "all": TN_CKPT_ALL, "recompute": TN_CKPT_RECOMPUTE}
KIND_NAMES = {0: "simple", 1: "splitk", 2: "stream", 3: "gemm"}

I8x48 = ctypes.c_int8 * 48


class PlanOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_resident_bits", ctypes.c_int32),
                ("workspace_limit", ctypes.c_int64), ("flags", ctypes.c_uint32),
                ("gemm_config", ctypes.c_int32), ("tune", ctypes.POINTER(ctypes.c_int32)),
                ("n_tune", ctypes.c_int32), ("checkpoint_policy", ctypes.c_int32),
                ("n_variable", ctypes.c_int32),
                ("variable_leaves", ctypes.POINTER(ctypes.c_int32)),
                ("batch", ctypes.c_int32), ("n_batched", ctypes.c_int32),
                ("batched_leaves", ctypes.POINTER(ctypes.c_int32))]


class PlanInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "n_tensors", "n_steps", "n_index", "n_sliced", "n_open_bits", "n_resident_bits",
        "n_outer_bits", "max_log2_per_slice", "max_log2_resident", "n_launches")] + \
        [(n, ctypes.c_int64) for n in (
            "n_slices", "out_elems", "workspace_bytes", "workspace_backward_bytes",
            "arena_bytes", "bytes_no_deletion")] + \
        [(n, ctypes.c_double) for n in (
            "cmac_reuse", "cmac_noreuse", "cmac_exec", "cmac_per_slice", "f_sl",
            "bytes_min_exec")] + \
        [(n, I8x48) for n in ("root_open_log2", "root_res_log2", "res_slicebit",
                              "outer_slicebit")] + \
        [("n_chains", ctypes.c_int32), ("n_segments", ctypes.c_int32),
         ("segment_table_bytes", ctypes.c_int64), ("segment_table_offset", ctypes.c_int64),
         ("n_phase0", ctypes.c_int32), ("backward_policy", ctypes.c_int32),
         ("backward_blocks", ctypes.c_int32), ("n_invariant", ctypes.c_int32),
         ("cmac_backward_recompute", ctypes.c_double), ("cmac_invariant", ctypes.c_double),
         ("n_launches_reuse", ctypes.c_int32), ("reserved_info", ctypes.c_int32)]


class StepInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "a", "b", "c", "phase", "kind", "nb", "nm", "nn", "nk", "inst_bits", "tile")] + \
        [("cmac", ctypes.c_double)] + \
        [(n, I8x48) for n in ("sA_b", "sB_b", "sC_b", "sA_m", "sC_m", "sB_n", "sC_n",
                              "sA_k", "sB_k")] + \
        [("c_offset", ctypes.c_int64), ("c_bytes", ctypes.c_int64),
         ("chain", ctypes.c_int32), ("chunks", ctypes.c_int32), ("tile_run", ctypes.c_int32),
         ("tiny_batch", ctypes.c_int32), ("tiny_level", ctypes.c_int32)]


class ChainStepInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("step", "nrow", "nk", "nn", "nbb")] + \
        [(n, ctypes.c_int8 * 8) for n in ("kslot", "nslot", "kB", "nB")] + \
        [(n, ctypes.c_int8 * 12) for n in ("rslot", "bB", "bpas")]


class ChainInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("first", "last", "phase", "tile_bits", "n_in",
                                              "n_out", "n_passive", "n_steps")] + \
        [(n, ctypes.c_int8 * 12) for n in ("in_slot", "in_log2", "out_slot", "out_log2")] + \
        [(n, ctypes.c_int8 * 40) for n in ("pas_in", "pas_out")] + \
        [("st", ChainStepInfo * 8)]


class SegmentLayout(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("segment", "execution", "n_steps", "n_items",
                                              "first_pos", "reserved")] + \
        [(n, ctypes.c_int64) for n in ("off_desc", "off_items", "off_ctr")]


EXPORTS = ("tn_plan_create", "tn_plan_query", "tn_plan_step", "tn_contract",
           "tn_contract_probe", "tn_contract_backward", "tn_plan_destroy", "tn_last_error",
           "tn_permute", "tn_plan_chain", "tn_plan_schedule", "tn_plan_segment_tables",
           "tn_contract_noalloc", "tn_plan_backward_tables", "tn_contract_ex",
           "tn_graph_create", "tn_graph_launch", "tn_graph_destroy", "tn_graph_create_backward")
TN_CALL_REUSE_INVARIANT = 1
NOALLOC_WORKSPACE_BYTES = 64 << 20

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.tn_plan_create.restype = ctypes.c_int
        L.tn_plan_create.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32, i32p,
                                     ctypes.c_int32, i32p, ctypes.c_int32, i32p, ctypes.c_int32,
                                     i32p, ctypes.POINTER(PlanOptions), ctypes.POINTER(P)]
        L.tn_plan_query.restype = ctypes.c_int
        L.tn_plan_query.argtypes = [P, ctypes.POINTER(PlanInfo)]
        L.tn_plan_step.restype = ctypes.c_int
        L.tn_plan_step.argtypes = [P, ctypes.c_int32, ctypes.POINTER(StepInfo)]
        L.tn_contract.restype = ctypes.c_int
        L.tn_contract.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.c_int64, ctypes.c_int32, P, P, ctypes.c_size_t, P]
        L.tn_contract_ex.restype = ctypes.c_int
        L.tn_contract_ex.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.c_int64, ctypes.c_int32, P, P, ctypes.c_size_t, P,
                                     ctypes.c_uint32]
        L.tn_contract_probe.restype = ctypes.c_int
        L.tn_contract_probe.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_int64),
                                        ctypes.c_int64, ctypes.c_int32, P, P, ctypes.c_size_t, P,
                                        ctypes.c_int32, P, P]
        L.tn_contract_backward.restype = ctypes.c_int
        L.tn_contract_backward.argtypes = [P, ctypes.POINTER(P), P, ctypes.POINTER(P),
                                           ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, P,
                                           ctypes.c_size_t, P]
        L.tn_graph_create.restype = ctypes.c_int
        L.tn_graph_create.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.c_int64, ctypes.c_int32, P, P, ctypes.c_size_t, P,
                                      ctypes.POINTER(P)]
        L.tn_graph_create_backward.restype = ctypes.c_int
        L.tn_graph_create_backward.argtypes = [P, ctypes.POINTER(P), P, ctypes.POINTER(P),
                                               ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, P,
                                               ctypes.c_size_t, P, ctypes.POINTER(P)]
        L.tn_graph_launch.restype = ctypes.c_int
        L.tn_graph_launch.argtypes = [P, P]
        L.tn_graph_destroy.restype = None
        L.tn_graph_destroy.argtypes = [P]
        L.tn_contract_noalloc.restype = ctypes.c_int
        L.tn_contract_noalloc.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_int64),
                                          ctypes.c_int64, ctypes.c_int32, P, P]
        i8p, i64p = ctypes.POINTER(ctypes.c_int8), ctypes.POINTER(ctypes.c_int64)
        L.tn_plan_backward_tables.restype = ctypes.c_int
        L.tn_plan_backward_tables.argtypes = [P, i8p, i8p, i64p, i64p, i64p, i32p, i8p]
        L.tn_plan_schedule.restype = ctypes.c_int
        L.tn_plan_schedule.argtypes = [P, i32p, ctypes.c_int32]
        L.tn_plan_segment_tables.restype = ctypes.c_int
        L.tn_plan_segment_tables.argtypes = [P, ctypes.POINTER(P), P, P, ctypes.c_int64,
                                             ctypes.POINTER(SegmentLayout), ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_int32)]
        L.tn_plan_chain.restype = ctypes.c_int
        L.tn_plan_chain.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ChainInfo)]
        L.tn_plan_destroy.restype = None
        L.tn_plan_destroy.argtypes = [P]
        L.tn_last_error.restype = ctypes.c_char_p
        L.tn_last_error.argtypes = []
        L.tn_permute.restype = ctypes.c_int
        L.tn_permute.argtypes = [P, P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int8),
                                 ctypes.POINTER(ctypes.c_int8), P]
        _lib = L
    return _lib


class TnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tn status {status}: {msg}")
        self.status = status


def _check(status):
    if status != TN_OK:
        raise TnError(status, lib().tn_last_error().decode())


def _i32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


TUNE_PATH = os.path.join(_HERE, "tune", "gfx950.json")


def default_workspace_limit():
    """80 % of the current device's free memory (0 = no limit without a GPU)."""
    try:
        import torch
        if not torch.cuda.is_available():
            return 0
        free, _ = torch.cuda.mem_get_info()
        return int(0.8 * free)
    except Exception:
        return 0


def load_tune_table(path=TUNE_PATH):
    """Autotuned GEMM tile choices: list of [precision, nm, nn, nk, config]."""
    if not os.path.exists(path):
        return []
    import json
    with open(path) as f:
        doc = json.load(f)
    return [list(map(int, e[:5])) for e in doc.get("entries", [])]


class Graph:
    """An instantiated contraction graph (``tn_graph_create``) or adjoint
    graph (``tn_graph_create_backward``).  Holds the plan and every tensor its
    kernels use: leaves, output (or output gradient and leaf gradients) and
    workspace."""

    def __init__(self, handle, plan, leaves, out, ws, keep=()):
        self._h, self.plan, self.leaves, self.out, self._ws = handle, plan, leaves, out, ws
        self._keep = keep

    def launch(self, stream=None):
        """One contraction of the leaves' current contents into ``out`` (an
        adjoint graph adds the leaf gradients into its ``out`` list)."""
        _check(lib().tn_graph_launch(self._h, _stream_ptr(stream)))
        return self.out

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            import torch
            torch.cuda.synchronize()    # no launch of the graph still running
            _lib.tn_graph_destroy(self._h)
            self._h = None


class Plan:
    """A contraction plan (``tn_plan_create``).

    ``labels``: index ids of each leaf (dense ids 0..n_index-1); ``dims``:
    mapping or sequence id -> dimension; ``open_ids``: output indices;
    ``path``: SSA pairs; ``sliced``: sliced index ids.
    """

    def __init__(self, labels, dims, open_ids, path, sliced=(), precision="c64",
                 max_resident_bits=-1, workspace_limit="auto", no_reuse=False, simple=False,
                 gemm_config=-1, tune="default", persistent=False, chains=True,
                 chain_mfma=True, chain_fused=True, chain_single=True, checkpoint="auto",
                 fit_backward=False, variable_leaves=(), batch=1, batched_leaves=(), tiny=True,
                 gauss=True):
        n_index = (max(dims) + 1) if isinstance(dims, dict) else len(dims)
        dim_arr = [dims[i] for i in range(n_index)]
        ranks, r_p = _i32([len(l) for l in labels])
        ids, ids_p = _i32([i for l in labels for i in l] or [0])
        darr, d_p = _i32(dim_arr or [2])
        op, op_p = _i32(list(open_ids) or [0])
        pa, pa_p = _i32([x for pr in path for x in pr] or [0])
        sl, sl_p = _i32(list(sliced) or [0])
        opts = PlanOptions()
        opts.precision = {"c64": TN_C64, "split_bf16": TN_SPLIT_BF16}[precision]
        opts.max_resident_bits = max_resident_bits
        opts.workspace_limit = default_workspace_limit() if workspace_limit == "auto" \
            else int(workspace_limit)
        opts.flags = (TN_FLAG_NO_REUSE if no_reuse else 0) | \
            (TN_FLAG_SIMPLE_KERNELS if simple else 0) | \
            (TN_FLAG_PERSISTENT if persistent else 0) | (0 if chains else TN_FLAG_NO_CHAIN) | \
            (0 if chain_mfma else TN_FLAG_CHAIN_VALU) | \
            (0 if chain_fused else TN_FLAG_CHAIN_STEPWISE) | \
            (0 if chain_single else TN_FLAG_CHAIN_NO_SINGLE) | \
            (TN_FLAG_FIT_BACKWARD if fit_backward else 0) | (0 if tiny else TN_FLAG_NO_TINY) | \
            (0 if gauss else TN_FLAG_GEMM_EMBED)
        opts.gemm_config = gemm_config
        opts.checkpoint_policy = _CKPT[checkpoint]
        varr, v_p = _i32(list(variable_leaves) or [0])
        opts.variable_leaves = v_p
        opts.n_variable = len(variable_leaves)
        barr, b_p = _i32(list(batched_leaves) or [0])
        opts.batch = int(batch)
        opts.batched_leaves = b_p
        opts.n_batched = len(batched_leaves)
        entries = load_tune_table() if tune == "default" else (tune or [])
        tarr, t_p = _i32([x for e in entries for x in e] or [0])
        opts.tune = t_p
        opts.n_tune = len(entries)
        h = ctypes.c_void_p()
        _check(lib().tn_plan_create(len(labels), r_p, ids_p, n_index, d_p, len(open_ids), op_p,
                                    len(path), pa_p, len(sliced), sl_p, ctypes.byref(opts),
                                    ctypes.byref(h)))
        self._h = h
        self.n_tensors = len(labels)
        self.labels = [list(l) for l in labels]
        self.dims = dim_arr
        self.open_ids = list(open_ids)
        if batch > 1:
            # the library's added index (id n_index): leading axis of the
            # batched leaves and leading open index
            bat = set(int(t) for t in batched_leaves)
            self.labels = [([n_index] if t in bat else []) + l for t, l in enumerate(self.labels)]
            self.dims = dim_arr + [int(batch)]
            self.open_ids = [n_index] + self.open_ids
        # elements of each leaf, checked on every call
        self._leaf_numel = [int(np.prod([self.dims[i] for i in l], dtype=np.int64))
                            for l in self.labels]
        self._ptr_array = ctypes.c_void_p * self.n_tensors
        self._info = None         # tn_plan_query, fixed for the plan's life
        self.sliced = list(sliced)
        self.precision = precision
        self.chain_valu = not chain_mfma
        self._ws = None
        self._ws_bwd = None
        self.variable_leaves = sorted(set(int(t) for t in variable_leaves))
        self._inv_key = None      # key of the invariant leaves whose results ws holds
        self._inv_refs = None

    @classmethod
    def from_network(cls, tn, path, sliced=(), **kw):
        return cls(tn.labels, tn.dims, tn.open, path, sliced, **kw)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.tn_plan_destroy(h)
            self._h = None

    def _static_info(self):
        if self._info is None:
            self._info = self.info()
        return self._info

    def info(self):
        inf = PlanInfo()
        _check(lib().tn_plan_query(self._h, ctypes.byref(inf)))
        d = {}
        for name, _ in PlanInfo._fields_:
            v = getattr(inf, name)
            d[name] = list(v) if isinstance(v, ctypes.Array) else v
        return d

    def step(self, k):
        s = StepInfo()
        _check(lib().tn_plan_step(self._h, k, ctypes.byref(s)))
        d = {}
        for name, _ in StepInfo._fields_:
            v = getattr(s, name)
            d[name] = list(v) if isinstance(v, ctypes.Array) else v
        for cls_, keys in (("nb", ("sA_b", "sB_b", "sC_b")), ("nm", ("sA_m", "sC_m")),
                           ("nn", ("sB_n", "sC_n")), ("nk", ("sA_k", "sB_k"))):
            for key in keys:
                d[key] = d[key][:d[cls_]]
        d["kind_name"] = KIND_NAMES.get(d["kind"], "?")
        return d

    def steps(self):
        return [self.step(k) for k in range(self.n_tensors - 1)]

    def chain(self, i):
        """Fused chain ``i`` (``tn_plan_chain``) with lists cut to length."""
        c = ChainInfo()
        _check(lib().tn_plan_chain(self._h, i, ctypes.byref(c)))
        d = {k: getattr(c, k) for k in ("first", "last", "phase", "tile_bits")}
        d["in_slot"] = list(c.in_slot)[:c.n_in]
        d["in_log2"] = list(c.in_log2)[:c.n_in]
        d["out_slot"] = list(c.out_slot)[:c.n_out]
        d["out_log2"] = list(c.out_log2)[:c.n_out]
        d["pas_in"] = list(c.pas_in)[:c.n_passive]
        d["pas_out"] = list(c.pas_out)[:c.n_passive]
        d["st"] = []
        for q in range(c.n_steps):
            t = c.st[q]
            d["st"].append(dict(step=t.step, nrow=t.nrow,
                                kslot=list(t.kslot)[:t.nk], nslot=list(t.nslot)[:t.nn],
                                kB=list(t.kB)[:t.nk], nB=list(t.nB)[:t.nn],
                                rslot=list(t.rslot)[:t.nrow],
                                bB=list(t.bB)[:t.nbb], bpas=list(t.bpas)[:t.nbb]))
        return d

    def chains(self):
        return [self.chain(i) for i in range(self.info()["n_chains"])]

    def schedule(self):
        """Step indices in execution order (``tn_plan_schedule``)."""
        arr = (ctypes.c_int32 * max(self.n_tensors - 1, 1))()
        _check(lib().tn_plan_schedule(self._h, arr, len(arr)))
        return list(arr)[:self.n_tensors - 1]

    def backward_tables(self):
        """Backward schedule (``tn_plan_backward_tables``) as numpy arrays."""
        nodes = 2 * self.n_tensors - 1
        nst = max(self.n_tensors - 1, 1)
        nch = max(self.info()["n_chains"], 1)
        keep = np.zeros(nodes, np.int8)
        front = np.zeros(nodes, np.int8)
        voff = np.zeros(nodes, np.int64)
        roff = np.zeros(nodes, np.int64)
        goff = np.zeros(nodes, np.int64)
        blk = np.zeros(nst, np.int32)
        fuse = np.zeros(nch, np.int8)
        ptr = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))  # noqa: E731
        _check(lib().tn_plan_backward_tables(
            self._h, ptr(keep, ctypes.c_int8), ptr(front, ctypes.c_int8),
            ptr(voff, ctypes.c_int64), ptr(roff, ctypes.c_int64), ptr(goff, ctypes.c_int64),
            ptr(blk, ctypes.c_int32), ptr(fuse, ctypes.c_int8)))
        return dict(keep=keep, frontier=front, value_off=voff, recompute_off=roff,
                    grad_off=goff, block_of=blk[:self.n_tensors - 1], fuse_chain=fuse)

    def segment_tables(self, leaf_ptrs, ws_ptr):
        """Persistent-segment control tables for the given (integer) leaf and
        workspace addresses (``tn_plan_segment_tables``): (bytes, layouts)."""
        inf = self.info()
        nbytes = int(inf["segment_table_bytes"])
        blob = (ctypes.c_char * max(nbytes, 1))()
        arr = (ctypes.c_void_p * self.n_tensors)(*leaf_ptrs)
        n = ctypes.c_int32()
        lay = (SegmentLayout * 4096)()
        _check(lib().tn_plan_segment_tables(self._h, arr, ctypes.c_void_p(ws_ptr), blob, nbytes,
                                            lay, len(lay), ctypes.byref(n)))
        out = []
        for i in range(n.value):
            L = lay[i]
            out.append({k: getattr(L, k) for k, _ in SegmentLayout._fields_})
        return bytes(blob)[:nbytes], out

    def release_workspace(self):
        """Drop the cached device workspaces (allocated again on next use)."""
        self._ws = None
        self._ws_bwd = None
        self._inv_key = self._inv_refs = None

    def _workspace(self, nbytes, device, attr):
        import torch
        ws = getattr(self, attr)
        if ws is None or ws.numel() < nbytes or ws.device != device:
            ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
            setattr(self, attr, ws)
        return ws

    def _leaf_ptrs(self, leaves):
        import torch
        if len(leaves) != self.n_tensors:
            raise ValueError(f"expected {self.n_tensors} leaves, got {len(leaves)}")
        dev = leaves[0].device
        c64, numel = torch.complex64, self._leaf_numel
        ptrs = []
        for t, x in enumerate(leaves):
            if x.dtype != c64 or not x.is_contiguous() or x.device != dev:
                raise ValueError(f"leaf {t} must be a contiguous complex64 tensor on {dev}")
            if x.numel() != numel[t]:
                raise ValueError(f"leaf {t} has {x.numel()} elements, network says otherwise")
            ptrs.append(x.data_ptr())
        return self._ptr_array(*ptrs), dev

    def _grad_ptrs(self, grad_leaves, grad_out):
        """Device pointers of the leaf-gradient buffers (None: skipped), each
        checked against its leaf's size, and of the output gradient."""
        import torch
        if len(grad_leaves) != self.n_tensors:
            raise ValueError(f"expected {self.n_tensors} gradient buffers, got {len(grad_leaves)}")
        for t, x in enumerate(grad_leaves):
            if x is not None and (x.dtype != torch.complex64 or not x.is_contiguous()
                                  or x.numel() != self._leaf_numel[t]):
                raise ValueError(f"gradient buffer {t} must be a contiguous complex64 tensor "
                                 f"of {self._leaf_numel[t]} elements")
        if grad_out.dtype != torch.complex128 or not grad_out.is_contiguous() or \
                grad_out.numel() != self._static_info()["out_elems"]:
            raise ValueError("grad_out must be a contiguous complex128 tensor of the output's size")
        garr = self._ptr_array(*[(x.data_ptr() if x is not None else None) for x in grad_leaves])
        return garr, ctypes.c_void_p(grad_out.data_ptr())

    def _invariant_key(self, leaves, ws):
        """Key of the invariant leaves' contents: each tensor's identity and
        torch's in-place version counter (the tensors are held, so their
        storage cannot be recycled), plus the workspace."""
        var = set(self.variable_leaves)
        inv = [x for t, x in enumerate(leaves) if t not in var]
        return tuple((id(x), x.data_ptr(), x._version) for x in inv) + (ws.data_ptr(),), inv

    def contract(self, leaves, slice_ids=None, per_slice=False, stream=None, out=None,
                 probe=None, reuse_invariant=True):
        """complex128 result: sum over the selected slices, or one row per slice.
        ``probe=(step, start_event, stop_event)`` times one step with the
        given torch.cuda.Event pair (tn_contract_probe).  For a plan with
        variable leaves, the invariant steps are skipped when the invariant
        leaves are the same tensors, unmodified, as in the previous call on
        this workspace (``reuse_invariant``)."""
        import torch
        inf = self._static_info()
        arr, dev = self._leaf_ptrs(leaves)
        ws = self._workspace(inf["workspace_bytes"], dev, "_ws")
        flags = 0
        if self.variable_leaves and probe is None:
            key, inv = self._invariant_key(leaves, ws)
            if reuse_invariant and key == self._inv_key:
                flags = TN_CALL_REUSE_INVARIANT
        shape = [self.dims[i] for i in self.open_ids]
        if slice_ids is not None:
            sids = np.ascontiguousarray(np.asarray(slice_ids, dtype=np.int64))
            sp = sids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            nsel = len(sids)
        else:
            sids, sp, nsel = None, None, 0
        rows = (nsel if nsel else inf["n_slices"]) if per_slice else None
        full = ([rows] if per_slice else []) + shape
        if out is None:
            out = torch.empty(full, dtype=torch.complex128, device=dev)
        mode = TN_OUT_PER_SLICE if per_slice else TN_OUT_SUM
        args = (self._h, arr, sp, nsel, mode, ctypes.c_void_p(out.data_ptr()),
                ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream))
        if probe is None:
            if self.variable_leaves:
                self._inv_key = None
                _check(lib().tn_contract_ex(*args, flags))
                self._inv_key, self._inv_refs = key, inv
            else:
                _check(lib().tn_contract(*args))
        else:
            self._inv_key = None
            step, e0, e1 = probe
            for e in (e0, e1):
                if not e.cuda_event:        # torch creates the HIP event on first record
                    e.record()
            _check(lib().tn_contract_probe(*args, step, ctypes.c_void_p(e0.cuda_event),
                                           ctypes.c_void_p(e1.cuda_event)))
        return out

    def graph(self, leaves, slice_ids=None, per_slice=False):
        """``tn_graph_create``: the contraction of these leaf tensors as a HIP
        graph with its own output (``Graph.out``) on the plan's workspace
        (shared with ``contract``: calls and launches on one stream run in
        order); change the leaves in place and call ``Graph.launch()`` to
        recompute."""
        import torch
        inf = self._static_info()
        arr, dev = self._leaf_ptrs(leaves)
        ws = self._workspace(inf["workspace_bytes"], dev, "_ws")
        self._inv_key = None        # the graph's launches overwrite every result
        shape = [self.dims[i] for i in self.open_ids]
        if slice_ids is not None:
            sids = np.ascontiguousarray(np.asarray(slice_ids, dtype=np.int64))
            sp = sids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            nsel = len(sids)
        else:
            sids, sp, nsel = None, None, 0
        rows = (nsel if nsel else inf["n_slices"]) if per_slice else None
        out = torch.empty(([rows] if per_slice else []) + shape, dtype=torch.complex128,
                          device=dev)
        mode = TN_OUT_PER_SLICE if per_slice else TN_OUT_SUM
        h = ctypes.c_void_p()
        _check(lib().tn_graph_create(self._h, arr, sp, nsel, mode, ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), None,
                                     ctypes.byref(h)))
        return Graph(h, self, list(leaves), out, ws)

    def backward_graph(self, leaves, grad_out, grad_leaves, slice_ids=None):
        """``tn_graph_create_backward``: the adjoint of these leaves as a HIP
        graph on the plan's backward workspace.  ``grad_out`` (complex128,
        the output's shape) and ``grad_leaves`` (complex64 like the leaves, or
        None) are fixed in the graph: change their contents in place; each
        ``Graph.launch()`` adds the leaf gradients into ``grad_leaves``."""
        import torch
        inf = self._static_info()
        arr, dev = self._leaf_ptrs(leaves)
        ws = self._workspace(inf["workspace_backward_bytes"], dev, "_ws_bwd")
        garr, gp = self._grad_ptrs(grad_leaves, grad_out)
        if slice_ids is not None:
            sids = np.ascontiguousarray(np.asarray(slice_ids, dtype=np.int64))
            sp = sids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            nsel = len(sids)
        else:
            sids, sp, nsel = None, None, 0
        h = ctypes.c_void_p()
        _check(lib().tn_graph_create_backward(self._h, arr, gp,
                                              garr, sp, nsel, ctypes.c_void_p(ws.data_ptr()),
                                              ws.numel(), None, ctypes.byref(h)))
        return Graph(h, self, list(leaves), list(grad_leaves), ws, keep=(grad_out,))

    def contract_noalloc(self, leaves, out, slice_ids=None, per_slice=False, stream=None):
        """``tn_contract_noalloc``: the library's own static workspace, the
        caller's ``out`` (complex128, shaped as ``contract`` returns it)."""
        arr, dev = self._leaf_ptrs(leaves)
        if slice_ids is not None:
            sids = np.ascontiguousarray(np.asarray(slice_ids, dtype=np.int64))
            sp = sids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            nsel = len(sids)
        else:
            sids, sp, nsel = None, None, 0
        mode = TN_OUT_PER_SLICE if per_slice else TN_OUT_SUM
        _check(lib().tn_contract_noalloc(self._h, arr, sp, nsel, mode,
                                         ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def backward(self, leaves, grad_out, grad_leaves, slice_ids=None, stream=None):
        """Adds d(loss)/d(leaf) (PyTorch convention) into ``grad_leaves`` for
        the output summed over ``slice_ids`` (None = all slices)."""
        import torch
        inf = self._static_info()
        arr, dev = self._leaf_ptrs(leaves)
        ws = self._workspace(inf["workspace_backward_bytes"], dev, "_ws_bwd")
        g = grad_out.to(torch.complex128).contiguous()
        garr, gp = self._grad_ptrs(grad_leaves, g)
        if slice_ids is not None:
            sids = np.ascontiguousarray(np.asarray(slice_ids, dtype=np.int64))
            sp = sids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            nsel = len(sids)
        else:
            sids, sp, nsel = None, None, 0
        _check(lib().tn_contract_backward(self._h, arr, gp, garr, sp,
                                          nsel, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                          _stream_ptr(stream)))
        return grad_leaves


def permute(x, in_log2, out_log2, out=None, stream=None):
    """Bit permutation of a complex64 device tensor (``tn_permute``)."""
    import torch
    nbits = len(in_log2)
    if x.numel() != (1 << nbits) or x.dtype != torch.complex64 or not x.is_contiguous():
        raise ValueError("x must be a contiguous complex64 tensor of 2^nbits elements")
    if out is None:
        out = torch.empty_like(x)
    a = (ctypes.c_int8 * max(nbits, 1))(*in_log2)
    b = (ctypes.c_int8 * max(nbits, 1))(*out_log2)
    _check(lib().tn_permute(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), nbits,
                            a, b, _stream_ptr(stream)))
    return out
