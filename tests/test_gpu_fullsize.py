"""Full-size workloads in the benchmark's launch configuration, checked on
sampled rows against the oracle (the whole C is too large to compare on the
host): the heaviest rows, rows of every kernel class and random rows."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2206_06611_amd as brm  # noqa: E402

TOL = 1e-12


def sampled_check(A, C, rows):
    rows = np.asarray(sorted(set(int(r) for r in rows)), np.int64)
    rpt = C.rpt[torch.as_tensor(np.concatenate([rows, rows + 1]), device=C.rpt.device)].cpu().numpy()
    lo, hi = rpt[:rows.size], rpt[rows.size:]
    ref = oracle.spgemm(A, A, rows=rows)
    model = oracle.brmerge(A, A, rows=rows)
    assert np.array_equal(hi - lo, np.diff(ref.rpt)), "row lengths differ"
    idx = torch.as_tensor(np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)]), device=C.col.device)
    col = C.col[idx].cpu().numpy()
    val = C.val[idx].cpu().numpy()
    assert np.array_equal(col, ref.col), "columns differ"
    err = np.abs(val - ref.val)
    assert np.all(err <= TOL * ref.absval), "values outside tolerance"
    assert np.array_equal(val.view(np.int64), model.val.view(np.int64)), "values differ from the merge-tree model"


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
    # properties at full size: rows sorted and in range
    last = C.rpt[-1].item()
    assert last == C.nnz
    h.close()
