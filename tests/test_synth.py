"""The seeded input generators: shapes, counts, sortedness and determinism."""
import numpy as np
import pytest

import synth


def check_csr(A):
    assert A.rpt[0] == 0 and A.rpt.size == A.rows + 1
    assert np.all(np.diff(A.rpt.astype(np.int64)) >= 0)
    assert A.col.dtype == np.int32 and A.val.dtype == np.float64
    assert A.col.size == A.nnz == A.val.size
    if A.nnz:
        assert A.col.min() >= 0 and A.col.max() < A.cols
    r = np.repeat(np.arange(A.rows), A.row_lengths())
    same_row = r[1:] == r[:-1]
    assert np.all(np.diff(A.col.astype(np.int64))[same_row] > 0)


def test_laplacian_counts():
    A = synth.laplacian_2d_5pt(64)
    check_csr(A)
    assert A.rows == 4096 and A.nnz == 20224
    assert set(np.unique(A.val)) == {4.0, -1.0}


def test_stencil27_counts():
    n = 6
    A = synth.stencil_3d_27pt(n)
    check_csr(A)
    assert A.nnz == (3 * n - 2) ** 3
    assert np.all(A.val[A.col == np.repeat(np.arange(n ** 3), A.row_lengths())] == 26.0)


def test_erdos_renyi():
    A = synth.erdos_renyi_rows(5000, 8, 2)
    check_csr(A)
    assert np.all(A.row_lengths() == 8)
    assert A.val.min() >= -1 and A.val.max() < 1
    B = synth.erdos_renyi_rows(5000, 8, 2)
    assert np.array_equal(A.col, B.col) and np.array_equal(A.val, B.val)
    C = synth.erdos_renyi_rows(5000, 8, 3)
    assert not np.array_equal(A.col, C.col)
    # columns are spread over the whole range
    assert abs(A.col.mean() / 5000 - 0.5) < 0.02


def test_rmat():
    A = synth.rmat(12, 16, 3)
    check_csr(A)
    assert A.rows == 4096 and A.nnz <= 16 * 4096
    assert A.val.min() >= 0 and A.val.max() < 1
    lens = A.row_lengths()
    # power-law skew: row 0 collects quadrant a at every level
    assert lens[0] == lens.max() and lens.max() > 20 * lens.mean()
    B = synth.rmat(12, 16, 3)
    assert np.array_equal(A.col, B.col)


def test_aggregation_transpose():
    for n in (4, 5):
        P, Pt = synth.aggregation_p(n), synth.aggregation_pt(n)
        check_csr(P)
        check_csr(Pt)
        T = synth.csr_transpose(P)
        assert np.array_equal(T.rpt, Pt.rpt) and np.array_equal(T.col, Pt.col)
        assert np.all(P.row_lengths() == 1)


def test_amg_batch_edges():
    b = synth.amg_batch(5, 4, 3, 6)
    assert len(b) == 5
    for n, A, P, Pt in b:
        assert 3 <= n <= 6 and A.rows == n ** 3 and P.cols == ((n + 1) // 2) ** 3


def test_row_block_and_transpose():
    A = synth.random_csr(30, 20, 0.3, 1)
    blk = synth.row_block(A, 5, 17)
    check_csr(blk)
    assert np.array_equal(blk.to_dense(), A.to_dense()[5:17])
    assert np.array_equal(synth.csr_transpose(A).to_dense(), A.to_dense().T)
