"""Kernel-family parity on single pairwise contractions (GPU).

Each case is a two-tensor network whose free and batch indices are open, so
the whole product tensor comes back through the C ABI.  Axis orders are
shuffled so the operands' bit strides are scattered, and shapes are chosen
to land on every kernel family (GEMM tile configurations including partial
tiles, split-k, stream, plain).  Reference: the oracle's pairwise step in
complex128.  Tolerances: complex64 1e-5, split-BF16 1e-3 relative (Frobenius)
-- the stated bounds for the two precisions.
"""

import numpy as np
import pytest

from oracle import tn_oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case(rng, nb, nm, nn, nk, d4=0):
    """Index ids: batch, row, column, summed; d4 of the row indices get dim 4."""
    ids = iter(range(1000))
    bat = [next(ids) for _ in range(nb)]
    row = [next(ids) for _ in range(nm)]
    col = [next(ids) for _ in range(nn)]
    summ = [next(ids) for _ in range(nk)]
    dims = {i: 2 for i in bat + row + col + summ}
    for i in row[:d4]:
        dims[i] = 4
    la = list(rng.permutation(bat + row + summ))
    lb = list(rng.permutation(bat + summ + col))
    la = [int(x) for x in la]
    lb = [int(x) for x in lb]
    a = (rng.standard_normal([dims[i] for i in la]) + 1j * rng.standard_normal([dims[i] for i in la]))
    b = (rng.standard_normal([dims[i] for i in lb]) + 1j * rng.standard_normal([dims[i] for i in lb]))
    open_ids = list(rng.permutation(bat + row + col))
    open_ids = [int(x) for x in open_ids]
    return [a, b], [la, lb], dims, open_ids


CASES = [
    # (nb, nm, nn, nk, d4, expected kind)
    (0, 10, 7, 8, 0, "gemm"),      # 128x64 tiles
    (1, 9, 6, 5, 0, "gemm"),
    (0, 10, 5, 6, 0, "gemm"),      # 128x32 tiles
    (2, 8, 4, 7, 0, "gemm"),       # 256x16 tiles
    (0, 5, 3, 5, 0, "gemm"),       # partial row and column tiles
    (0, 5, 6, 3, 0, "gemm"),       # partial row and k tiles (operands swap roles)
    (0, 12, 2, 6, 0, "gemm"),      # many rows, 4 columns: the narrowest tile, partial columns
    (1, 12, 1, 5, 0, "gemm"),
    (0, 6, 9, 9, 1, "gemm"),       # dim-4 rows
    (0, 12, 3, 2, 0, "stream"),
    (2, 10, 2, 4, 1, "stream"),
    (3, 4, 2, 3, 0, "stream"),     # batch bits inside a workgroup's rows: B through the cache
    (0, 7, 4, 4, 0, "stream"),     # fewer rows than a workgroup
    (1, 6, 5, 14, 0, "gemm"),      # few output tiles, long sums: MFMA tiles split over k
    (0, 5, 3, 12, 0, "gemm"),      # ... with partial tiles
    (0, 7, 4, 9, 1, "gemm"),       # ... dim-4 rows
    (0, 10, 8, 12, 0, "gemm"),     # 32 tiles of 128x64 against 2^12 summed: 32 chunks of k
    (0, 2, 2, 14, 0, "splitk"),
    (3, 1, 0, 10, 0, "splitk"),
    (0, 3, 3, 6, 0, "simple"),
]


@pytest.mark.parametrize("precision", ["c64", "split_bf16"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "b%dm%dn%dk%d_%s" % (c[0], c[1], c[2], c[3], c[5]))
def test_pairwise_kernels(case, precision):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_09793_amd import Plan
    nb, nm, nn, nk, d4, kind = case
    rng = np.random.default_rng([nb, nm, nn, nk, d4])
    tensors, labels, dims, open_ids = _case(rng, nb, nm, nn, nk, d4)
    pl = Plan(labels, dims, open_ids, [(0, 1)], precision=precision)
    st = pl.step(0)
    assert st["kind_name"] == kind, st["kind_name"]
    if kind == "gemm":   # split over k: long sums, few output tiles
        out = nb + nm + nn + d4
        few_tiles = out - 13 < 8 and min(10 - max(0, out - 13), nk - 7) >= 1
        assert (st["chunks"] > 1) == (nk >= 8 and (out <= 12 or few_tiles)), st["chunks"]
    dev = torch.device("cuda:0")
    leaves = [torch.from_numpy(t.astype(np.complex64)).to(dev) for t in tensors]
    got = pl.contract(leaves).cpu().numpy()
    ref = tn_oracle.contract([t.astype(np.complex64).astype(np.complex128) for t in tensors],
                             labels, dims, open_ids, [(0, 1)])
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    tol = 1e-5 if (precision == "c64" or kind != "gemm") else 1e-3
    assert err <= tol, err
    if precision == "split_bf16" and kind == "gemm":
        assert err > 1e-9   # really ran in reduced precision
        assert err <= 1e-4  # three-product split: ~2^-16 relative


@pytest.mark.parametrize("shape", [(1, 10, 7, 6), (1, 6, 5, 14)])
def test_gemm_deterministic_run_to_run(shape):
    """Tiles, and partial tiles of a split sum added in a fixed order."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_09793_amd import Plan
    rng = np.random.default_rng(3)
    tensors, labels, dims, open_ids = _case(rng, *shape)
    pl = Plan(labels, dims, open_ids, [(0, 1)])
    dev = torch.device("cuda:0")
    leaves = [torch.from_numpy(t.astype(np.complex64)).to(dev) for t in tensors]
    x = pl.contract(leaves).cpu().numpy()
    y = pl.contract(leaves).cpu().numpy()
    assert np.array_equal(x, y)


@pytest.mark.parametrize("precision", ["c64", "split_bf16"])
@pytest.mark.parametrize("cfg", range(10))
def test_every_gemm_tile_config(cfg, precision):
    """Each compiled tile configuration, forced on a full and a partial tile shape
    (the stream configurations, 8 and 9, do not take these shapes and run them
    with the rule's configuration)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_09793_amd import Plan
    dev = torch.device("cuda:0")
    for shape in ((1, 10, 8, 7, 0), (0, 6, 5, 5, 1), (0, 6, 5, 12, 0)):
        rng = np.random.default_rng([cfg, *shape])
        tensors, labels, dims, open_ids = _case(rng, *shape)
        pl = Plan(labels, dims, open_ids, [(0, 1)], precision=precision, gemm_config=cfg)
        st = pl.step(0)
        assert st["kind_name"] == "gemm" and st["tile"] == cfg
        leaves = [torch.from_numpy(t.astype(np.complex64)).to(dev) for t in tensors]
        got = pl.contract(leaves).cpu().numpy()
        ref = tn_oracle.contract([t.astype(np.complex64).astype(np.complex128) for t in tensors],
                                 labels, dims, open_ids, [(0, 1)])
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= (1e-5 if precision == "c64" else 1e-4), (shape, err)


STREAM_CASES = [
    # (nb, nm, nn, nk, d4): column blocks of 16, 32, 64, 128; several bands per
    # wave; one k tile per band; column tiles; dim-4 rows; K up to 512
    (0, 17, 7, 6, 0),
    (0, 17, 4, 9, 0),   # 2^21 outputs: enough tiles that the sum stays whole
    (0, 16, 5, 8, 0),
    (0, 13, 6, 5, 0),
    (0, 11, 9, 6, 0),
    (0, 10, 7, 4, 1),
    (0, 10, 5, 5, 0),   # fewer bands than waves
    (1, 12, 7, 6, 0),   # batch bit: runs with the rule's configuration
]


@pytest.mark.parametrize("cfg", [8, 9])
@pytest.mark.parametrize("precision", ["c64", "split_bf16"])
@pytest.mark.parametrize("shape", STREAM_CASES, ids=lambda c: "b%dm%dn%dk%dd%d" % c)
def test_stream_gemm(shape, precision, cfg):
    """The stream configuration (B block resident in LDS, 32-row bands) forced,
    against the oracle: complex64 takes every shape but the batch one;
    split-BF16 (B blocks of at most 2^12 entries, k tiles of 32) takes
    m17n7k6 (two column tiles), m16n5k8 (two), m13n6k5, m11n9k6 (eight) and
    m10n5k5; the others run with the rule's configuration.  Configuration 9
    (complex64, three real products per complex product, 5 <= nk <= 7) takes
    m17n7k6 (two column tiles of 64), m13n6k5, m11n9k6 (eight tiles of 64)
    and m10n5k5 (one tile of 32); the others run as configuration 8."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_09793_amd import Plan
    dev = torch.device("cuda:0")
    rng = np.random.default_rng([8, *shape])
    tensors, labels, dims, open_ids = _case(rng, *shape)
    pl = Plan(labels, dims, open_ids, [(0, 1)], precision=precision, gemm_config=cfg)
    st = pl.step(0)
    assert st["kind_name"] == "gemm" and st["tile"] == cfg and st["chunks"] <= 1
    leaves = [torch.from_numpy(t.astype(np.complex64)).to(dev) for t in tensors]
    got = pl.contract(leaves).cpu().numpy()
    x = pl.contract(leaves).cpu().numpy()
    assert np.array_equal(got, x)
    ref = tn_oracle.contract([t.astype(np.complex64).astype(np.complex128) for t in tensors],
                             labels, dims, open_ids, [(0, 1)])
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print("stream", cfg, shape, precision, err)
    assert err <= (1e-5 if precision == "c64" else 1e-4), err
    if precision == "split_bf16":
        assert err > 1e-9   # really ran in reduced precision


@pytest.mark.parametrize("cfg", [8, 9])
@pytest.mark.parametrize("precision", ["c64", "split_bf16"])
@pytest.mark.parametrize("shape", [(0, 12, 6, 6, 0), (0, 11, 8, 5, 0)])
def test_stream_gemm_adjoint(shape, precision, cfg):
    """Leaf gradients of a single product C = A B with the stream configuration
    forced: the adjoint step for A, grad_A = grad_C B^H, is a stream-shaped
    GEMM with B conjugated that adds into the gradient buffer.  Reference: the
    same product in complex128."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_09793_amd import Plan
    dev = torch.device("cuda:0")
    rng = np.random.default_rng([9, *shape])
    tensors, labels, dims, open_ids = _case(rng, *shape)
    pl = Plan(labels, dims, open_ids, [(0, 1)], gemm_config=cfg, precision=precision)
    leaves = [torch.from_numpy(t.astype(np.complex64)).to(dev) for t in tensors]
    out = pl.contract(leaves)
    w = (rng.standard_normal(out.shape) + 1j * rng.standard_normal(out.shape)).astype(np.complex64)
    # backward adds into the gradient buffers: start them non-zero
    g0 = [(rng.standard_normal(t.shape) + 1j * rng.standard_normal(t.shape)).astype(np.complex64)
          for t in tensors]
    grads = [torch.from_numpy(g).to(dev) for g in g0]
    pl.backward(leaves, torch.from_numpy(w).to(dev), grads)
    a, b = [t.astype(np.complex64).astype(np.complex128) for t in tensors]
    la, lb = labels
    sym = {i: chr(97 + n) for n, i in enumerate(sorted(set(la) | set(lb)))}
    sa = "".join(sym[i] for i in la)
    sb = "".join(sym[i] for i in lb)
    so = "".join(sym[i] for i in open_ids)
    wd = w.astype(np.complex128)
    ga = np.einsum(f"{so},{sb}->{sa}", wd, np.conj(b))
    gb = np.einsum(f"{so},{sa}->{sb}", wd, np.conj(a))
    for got, ref, init in ((grads[0], ga, g0[0]), (grads[1], gb, g0[1])):
        got = got.cpu().numpy().astype(np.complex128) - init
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= (1e-5 if precision == "c64" else 1e-4), err


@pytest.mark.parametrize("cfg", [0, 1, 3, 4, 5, 6])
@pytest.mark.parametrize("shape", [(0, 9, 7, 6, 0), (1, 7, 6, 9, 0), (0, 6, 5, 5, 1)])
def test_gemm_three_products_and_embedding(shape, cfg):
    """complex64 tiled GEMM tiles with three real products per complex product
    (the default) and with the real embedding (TN_FLAG_GEMM_EMBED), forced
    tile configuration, against the oracle; full, batched, split-k and
    partial tiles; and the adjoint (conjugated operands, accumulation) of the
    three-product kernel against that of the embedding."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_09793_amd import Plan
    dev = torch.device("cuda:0")
    rng = np.random.default_rng([11, cfg, *shape])
    tensors, labels, dims, open_ids = _case(rng, *shape)
    ref = tn_oracle.contract([t.astype(np.complex64).astype(np.complex128) for t in tensors],
                             labels, dims, open_ids, [(0, 1)])
    leaves = [torch.from_numpy(t.astype(np.complex64)).to(dev) for t in tensors]
    grads = {}
    for gauss in (True, False):
        pl = Plan(labels, dims, open_ids, [(0, 1)], gemm_config=cfg, gauss=gauss)
        assert pl.step(0)["kind_name"] == "gemm" and pl.step(0)["tile_run"] == cfg
        got = pl.contract(leaves).cpu().numpy()
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print("cfg", cfg, shape, "three products" if gauss else "embedding", err)
        assert err <= 1e-5, err
        w = torch.from_numpy(rng.standard_normal(got.shape) + 1j * rng.standard_normal(got.shape)
                             if gauss else grads["w"]).to(dev)
        if gauss:
            grads["w"] = w.cpu().numpy()
        g = [torch.ones_like(x) for x in leaves]
        pl.backward(leaves, w.reshape(-1), g)
        grads[gauss] = [x.cpu().numpy().astype(np.complex128) for x in g]
    for a, b in zip(grads[True], grads[False]):
        assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(b)
