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


def device_row_colsums(C, chunk=1 << 28):
    """Per row of the device CSR C, the sum of its column indices (int64,
    on the device), in chunks of at most `chunk` entries: a whole-C check
    of the structure against oracle.pattern_sums where C is too large to
    copy to the host."""
    import torch
    rpt_h = C.rpt.cpu().numpy().astype(np.int64)
    M = C.rows
    out = torch.zeros(max(M, 1), dtype=torch.int64, device=C.rpt.device)
    r0 = 0
    while r0 < M:
        e0 = int(rpt_h[r0])
        r1 = int(np.searchsorted(rpt_h, e0 + chunk, side="right")) - 1
        r1 = min(max(r1, r0 + 1), M)
        e1 = int(rpt_h[r1])
        cs = torch.zeros(e1 - e0 + 1, dtype=torch.int64, device=C.col.device)
        if e1 > e0:
            cs[1:] = torch.cumsum(C.col[e0:e1].to(torch.int64), 0)
        idx = C.rpt[r0:r1 + 1] - e0
        out[r0:r1] = cs[idx[1:]] - cs[idx[:-1]]
        del cs
        r0 = r1
    return out[:M]


def assert_structure_matches_oracle(A, B, C):
    """Every row's length and column sum against the oracle's structure pass
    (rows sorted and in range are checked where the columns are read)."""
    import oracle
    cnt, csum = oracle.pattern_sums(A, B)
    lens = np.diff(C.rpt.cpu().numpy().astype(np.int64))
    assert np.array_equal(lens, cnt), f"{int((lens != cnt).sum())} row lengths differ"
    got = device_row_colsums(C).cpu().numpy()
    assert np.array_equal(got, csum), f"{int((got != csum).sum())} row column sums differ"
