"""Shared checks of GPU results against the CPU oracle."""
import numpy as np

TOL = 1e-12  # |C_gpu - C| <= TOL * sum_k |A_ik B_kj| per entry


def to_host(C):
    return (C.rpt.cpu().numpy().astype(np.int64), C.col.cpu().numpy(), C.val.cpu().numpy())


def assert_matches_oracle(C, ref, model=None, rows=None):
    """C: DeviceCSR from the library (all rows); ref: oracle.spgemm result for
    `rows` (all rows when None); model: oracle.brmerge result for the same rows
    (bitwise expectation of the merge tree) or None."""
    rpt, col, val = to_host(C)
    if rows is None:
        assert np.array_equal(rpt, ref.rpt), "row pointers differ"
        assert np.array_equal(col, ref.col), "columns differ"
        gv = val
    else:
        rows = np.asarray(rows, np.int64)
        lens = rpt[rows + 1] - rpt[rows]
        assert np.array_equal(lens, np.diff(ref.rpt)), "row lengths differ"
        idx = np.concatenate([np.arange(rpt[r], rpt[r + 1]) for r in rows]) if rows.size else \
            np.zeros(0, np.int64)
        assert np.array_equal(col[idx], ref.col), "columns differ"
        gv = val[idx]
    err = np.abs(gv - ref.val)
    bad = ~(err <= TOL * ref.absval)
    assert not bad.any(), f"{bad.sum()} values outside tolerance, worst {err[bad].max() if bad.any() else 0}"
    if model is not None:
        assert np.array_equal(gv.view(np.int64), model.val.view(np.int64)), \
            "values differ bitwise from the merge-tree model"
