"""Full-size workloads in the benchmark's launch configuration: every row's
length and column sum against the oracle's structure pass, and sampled rows
element by element (the whole C is too large to compare on the host): the
heaviest rows, rows of every kernel class and random rows."""
import numpy as np
import pytest

import oracle
import synth
from helpers import assert_structure_matches_oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2206_06611_amd as brm  # noqa: E402

TOL = 1e-12


def sampled_check(A, C, rows):
    sampled_check_rows(A, A, C, rows)


def sampled_check_rows(A, B, C, rows):
    """Rows `rows` of C = A*B against the oracle and the merge-tree model."""
    rows = np.asarray(sorted(set(int(r) for r in rows)), np.int64)
    rpt = C.rpt[torch.as_tensor(np.concatenate([rows, rows + 1]), device=C.rpt.device)].cpu().numpy()
    lo, hi = rpt[:rows.size], rpt[rows.size:]
    ref = oracle.spgemm(A, B, rows=rows)
    model = oracle.brmerge(A, B, rows=rows)
    assert np.array_equal(hi - lo, np.diff(ref.rpt)), "row lengths differ"
    idx = torch.as_tensor(np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)]), device=C.col.device)
    col = C.col[idx].cpu().numpy()
    val = C.val[idx].cpu().numpy()
    assert np.array_equal(col, ref.col), "columns differ"
    err = np.abs(val - ref.val)
    assert np.all(err <= TOL * ref.absval), "values outside tolerance"
    assert np.array_equal(val.view(np.int64), model.val.view(np.int64)), "values differ from the merge-tree model"


@pytest.mark.timeout(600)
def test_rmat_scale20_sampled():
    print("case: R-MAT scale 20, edge factor 16, seed 3 (full size, sampled rows)", flush=True)
    A = synth.rmat(20, 16, 3)
    nprod = oracle.row_nprod(A, A)
    h = brm.Handle(0)
    dA = brm.DeviceCSR.from_host(A)
    C = h.spgemm(dA, dA)
    torch.cuda.synchronize()
    assert h.stat(brm.STAT_DEVICE_ERR) == 0
    assert h.stat(brm.STAT_NPROD) == int(nprod.sum())
    cls = h.class_rows()
    print("classes", cls, "nnz", C.nnz, flush=True)
    assert cls["heavy"] > 0
    rng = np.random.default_rng(0)
    order = np.argsort(-nprod)
    sample = list(order[:6]) + list(rng.choice(A.rows, 300, replace=False))
    # a few rows from every product-count band
    for lo, hi in [(1, 64), (65, 256), (257, 1024), (1025, 4096), (4097, 10 ** 5), (10 ** 5, 10 ** 9)]:
        band = np.nonzero((nprod >= lo) & (nprod <= hi))[0]
        if band.size:
            sample += list(rng.choice(band, min(20, band.size), replace=False))
    sampled_check(A, C, sample)
    # every row: length and column sum against the oracle's structure pass
    print("whole-C structure check against the oracle", flush=True)
    assert C.rpt[-1].item() == C.nnz
    assert_structure_matches_oracle(A, A, C)
    h.close()


def _stencil_row_lengths(n):
    # the square of the 27-point stencil couples offsets -2..2 in each
    # dimension, clipped at the cube's faces
    x = np.arange(n)
    per = np.minimum(x + 2, n - 1) - np.maximum(x - 2, 0) + 1
    return (per[:, None, None] * per[None, :, None] * per[None, None, :]).reshape(-1)


def test_stencil27_128_full_size():
    print("case: 27-point stencil on a 128^3 cube squared (full size)", flush=True)
    n = 128
    A = synth.stencil_3d_27pt(n)
    h = brm.Handle(0)
    dA = brm.DeviceCSR.from_host(A)
    C = h.spgemm(dA, dA)
    torch.cuda.synchronize()
    assert h.stat(brm.STAT_DEVICE_ERR) == 0
    assert h.stat(brm.STAT_NPROD) == 1489355288
    assert C.nnz == (5 * n - 6) ** 3
    # every row length from the closed form
    lens = np.diff(C.rpt.cpu().numpy())
    assert np.array_equal(lens, _stencil_row_lengths(n))
    rng = np.random.default_rng(5)
    sample = [0, 1, n - 1, n * n + n + 1, A.rows // 2, A.rows - 1] + list(rng.choice(A.rows, 400, replace=False))
    sampled_check(A, C, sample)
    h.close()


@pytest.mark.timeout(900)
def test_rmat_scale21_row_blocks():
    # C has about 2.6e10 entries (over 300 GB): computed in row blocks of at
    # most 2^32 products, each block checked on sampled rows
    print("case: R-MAT scale 21, edge factor 16, seed 5 (full size, row blocks, sampled rows)", flush=True)
    A = synth.rmat(21, 16, 5)
    nprod = oracle.row_nprod(A, A)
    h = brm.Handle(0)
    dA = brm.DeviceCSR.from_host(A)
    dev_nprod = h.row_products(dA, dA).cpu().numpy()
    assert np.array_equal(dev_nprod, nprod)
    blocks = h.row_blocks(dA, dA, 1 << 32)
    assert blocks[0][0] == 0 and blocks[-1][1] == A.rows
    assert all(a[1] == b[0] for a, b in zip(blocks, blocks[1:]))
    rng = np.random.default_rng(1)
    total_nnz = 0
    for b, e in blocks:
        assert nprod[b:e].sum() <= (1 << 32) or e == b + 1
        Ab = synth.row_block(A, b, e)
        C = h.spgemm(dA.row_block(b, e), dA)
        torch.cuda.synchronize()
        assert h.stat(brm.STAT_DEVICE_ERR) == 0
        assert h.stat(brm.STAT_NPROD) == int(nprod[b:e].sum())
        total_nnz += C.nnz
        nb = nprod[b:e]
        sample = list(np.argsort(-nb)[:2]) + list(rng.choice(e - b, min(60, e - b), replace=False))
        print(f"block [{b}, {e}) nnz {C.nnz} classes {h.class_rows()}", flush=True)
        sampled_check_rows(Ab, A, C, sample)
        assert_structure_matches_oracle(Ab, A, C)
        del C
        torch.cuda.empty_cache()
    print("nnz(C)", total_nnz, "nprod", int(nprod.sum()), flush=True)
    assert total_nnz <= int(nprod.sum())
    h.close()


@pytest.mark.parametrize("rows", [4096 * 1024, 4096 * 1024 + 1, 5_000_000])
def test_row_pointer_scan_either_side_of_fused_limit(rows):
    # the row-pointer scan folds its top level into the apply pass up to 4096
    # tiles of 1024 rows and runs three passes beyond: a scaled permutation
    # squared has one entry per row, C[i, p[p[i]]] = a[i] * a[p[i]]
    print(f"case: permutation squared, {rows} rows", flush=True)
    rng = np.random.default_rng(rows)
    p = rng.permutation(rows).astype(np.int32)
    a = rng.uniform(0.5, 2.0, rows)
    empty = rng.random(rows) < 0.25  # a quarter of the rows empty: uneven tiles
    cnt = (~empty).astype(np.int64)
    rpt = np.zeros(rows + 1, np.int64)
    rpt[1:] = np.cumsum(cnt)
    A = synth.CSR(rows, rows, rpt, p[~empty], a[~empty])
    dA = brm.DeviceCSR.from_host(A)
    h = brm.Handle(0)
    try:
        C = h.spgemm(dA, dA)
        torch.cuda.synchronize()
        assert h.stat(brm.STAT_DEVICE_ERR) == 0
        c_rpt = C.rpt.cpu().numpy()
        # row i has an entry iff row i and row p[i] of A are both nonempty
        has = ~empty & ~empty[p]
        exp_rpt = np.zeros(rows + 1, np.int64)
        exp_rpt[1:] = np.cumsum(has)
        assert np.array_equal(c_rpt, exp_rpt)
        assert np.array_equal(C.col.cpu().numpy(), p[p][has])
        assert np.array_equal(C.val.cpu().numpy(), (a * a[p])[has])
    finally:
        h.close()
