"""Pins of the CPU oracle against facts fixed by the mathematics and the paper.

The oracle is only trusted once these pass: brute force on tiny inputs
(Eq. (1)), closed forms of stencil products, identity and permutation
products, the transpose identity, a library SpGEMM (scipy) on positive data,
an exactly rounded sum (math.fsum) for ill-conditioned rows, the merge-tree
shape of Algorithm 1 and Eq. (5) against Table II.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_of(res, shape):
    rows = np.repeat(np.arange(len(res.rows)), np.diff(res.rpt))
    pat = np.zeros(shape, bool)
    val = np.zeros(shape)
    pat[rows, res.col] = True
    val[rows, res.col] = res.val
    return pat, val


def check_sorted_distinct(res):
    for i in range(len(res.rows)):
        c = res.col[res.rpt[i]:res.rpt[i + 1]]
        assert np.all(np.diff(c) > 0)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("density", [0.0, 0.05, 0.25, 0.6])
def test_brute_force_integer(seed, density):
    rng = np.random.default_rng(seed)
    M, K, N = rng.integers(1, 40, size=3)
    A = synth.random_csr(M, K, density, seed, integer_values=True, empty_row_frac=0.2)
    B = synth.random_csr(K, N, density, seed + 100, integer_values=True, empty_row_frac=0.2)
    res = oracle.spgemm(A, B)
    pat, val = oracle.brute_force(A.to_dense(), A.to_dense() != 0, B.to_dense(), B.to_dense() != 0)
    gpat, gval = dense_of(res, (M, N))
    assert np.array_equal(gpat, pat)
    assert np.array_equal(gval, val)  # small integers: every order is exact
    check_sorted_distinct(res)
    assert res.nnz == pat.sum()


def test_stored_zeros_and_cancellation_are_kept():
    # A has a stored zero; row 0 of A*B cancels exactly to 0 at column 0
    Ad = np.array([[1.0, 1.0, 0.0], [0.0, 0.0, 2.0]])
    Apat = np.array([[True, True, True], [False, False, True]])
    Bd = np.array([[3.0, 1.0], [-3.0, 0.0], [5.0, 0.0]])
    Bpat = np.array([[True, True], [True, False], [True, False]])
    A = synth.from_dense(Ad, Apat)
    B = synth.from_dense(Bd, Bpat)
    res = oracle.spgemm(A, B)
    pat, val = oracle.brute_force(Ad, Apat, Bd, Bpat)
    gpat, gval = dense_of(res, (2, 2))
    assert np.array_equal(gpat, pat) and pat[0, 0] and val[0, 0] == 0.0
    assert np.array_equal(gval, val)
    # the sum of |products| is 3 + 3 + 0 at (0, 0)
    assert res.absval[0] == 6.0


@pytest.mark.parametrize("seed", range(4))
def test_absval_is_product_of_absolute_values(seed):
    A = synth.random_csr(30, 20, 0.3, seed, integer_values=True)
    B = synth.random_csr(20, 25, 0.3, seed + 7, integer_values=True)
    r = oracle.spgemm(A, B)
    Aabs = synth.CSR(A.rows, A.cols, A.rpt, A.col, np.abs(A.val))
    Babs = synth.CSR(B.rows, B.cols, B.rpt, B.col, np.abs(B.val))
    pat, val = oracle.brute_force(Aabs.to_dense(), A.to_dense() != 0, Babs.to_dense(), B.to_dense() != 0)
    _, absd = dense_of(synth_result_with(r, r.absval), (30, 25))
    assert np.array_equal(absd, val)


def synth_result_with(r, values):
    return oracle.Result(r.rows, r.rpt, r.col, values)


def test_compensated_sum_against_fsum():
    # one output entry whose products are 1e16, 1, -1e16, 1, 3e-17 ...
    a = np.array([1e16, 1.0, -1e16, 1.0, 3e-17, -2.5, 1e-3])
    K = a.size
    A = synth.CSR(1, K, np.array([0, K], np.int32), np.arange(K, dtype=np.int32), a)
    B = synth.CSR(K, 1, np.arange(K + 1, dtype=np.int32), np.zeros(K, np.int32), np.ones(K))
    r = oracle.spgemm(A, B)
    exact = math.fsum(a)
    u = 2.0 ** -53
    bound = 2 * u * abs(exact) + K * K * u * u * math.fsum(np.abs(a))
    assert abs(r.val[0] - exact) <= bound
    naive = 0.0
    for x in a:
        naive += x
    assert abs(naive - exact) > 1e6 * bound  # the uncompensated sum is far off
    assert r.absval[0] == math.fsum(np.abs(a))


@pytest.mark.parametrize("seed", range(5))
def test_compensated_sum_random_rows(seed):
    rng = np.random.default_rng(seed)
    K = 300
    a = rng.standard_normal(K) * 10.0 ** rng.integers(-8, 9, size=K)
    A = synth.CSR(1, K, np.array([0, K], np.int32), np.arange(K, dtype=np.int32), a)
    B = synth.CSR(K, 1, np.arange(K + 1, dtype=np.int32), np.zeros(K, np.int32), np.ones(K))
    r = oracle.spgemm(A, B)
    exact = math.fsum(a)
    u = 2.0 ** -53
    assert abs(r.val[0] - exact) <= 2 * u * abs(exact) + K * K * u * u * math.fsum(np.abs(a))


def _laplacian_square_expected(n):
    """A^2 for A = 4I - (Tx + Ty) on the n x n grid, from
    A^2 = 16I - 8(Tx + Ty) + Tx^2 + Ty^2 + 2 Tx Ty: entries by offset."""
    ent = {}
    for y in range(n):
        for x in range(n):
            i = x + n * y
            degx = (x > 0) + (x < n - 1)
            degy = (y > 0) + (y < n - 1)
            ent[(i, i)] = 16 + degx + degy
            for dx, dy, v in [(1, 0, -8), (-1, 0, -8), (0, 1, -8), (0, -1, -8),
                              (2, 0, 1), (-2, 0, 1), (0, 2, 1), (0, -2, 1),
                              (1, 1, 2), (1, -1, 2), (-1, 1, 2), (-1, -1, 2)]:
                xx, yy = x + dx, y + dy
                if 0 <= xx < n and 0 <= yy < n:
                    ent[(i, xx + n * yy)] = v
    return ent


@pytest.mark.parametrize("n", [1, 2, 3, 5, 64])
def test_laplacian_square_closed_form(n):
    A = synth.laplacian_2d_5pt(n)
    r = oracle.spgemm(A, A)
    ent = _laplacian_square_expected(n)
    assert r.nnz == len(ent)
    if n >= 2:
        assert r.nnz == n * n + 4 * n * (n - 1) + 4 * (n - 1) ** 2 + 4 * n * max(n - 2, 0)
    rows = np.repeat(np.arange(n * n), np.diff(r.rpt))
    got = {(int(i), int(j)): v for i, j, v in zip(rows, r.col, r.val)}
    assert got == ent
    if n == 64:
        assert oracle.row_nprod(A, A).sum() == 100104
        assert r.nnz == 51972
        assert np.diff(r.rpt).max() == 13


@pytest.mark.parametrize("n", [2, 3, 7])
def test_nine_point_from_factors(n):
    S = np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    SI = synth.from_dense(np.kron(np.eye(n), S))   # acts along x (fastest index)
    IS = synth.from_dense(np.kron(S, np.eye(n)))   # acts along y
    r = oracle.spgemm(SI, IS)
    T = synth.tridiag_kron2(n)
    assert np.array_equal(r.rpt, T.rpt.astype(np.int64))
    assert np.array_equal(r.col, T.col)
    assert np.array_equal(r.val, T.val)
    assert r.nnz == (3 * n - 2) ** 2


@pytest.mark.parametrize("seed", range(3))
def test_identity_and_permutation(seed):
    rng = np.random.default_rng(seed)
    B = synth.random_csr(23, 17, 0.3, seed)
    I = synth.identity(23)
    r = oracle.spgemm(I, B)
    assert np.array_equal(r.rpt, B.rpt.astype(np.int64)) and np.array_equal(r.col, B.col)
    assert np.array_equal(r.val, B.val)
    r = oracle.spgemm(B, synth.identity(17))
    assert np.array_equal(r.col, B.col) and np.array_equal(r.val, B.val)
    perm = rng.permutation(23)
    r = oracle.spgemm(synth.permutation(perm), B)
    _, got = dense_of(r, (23, 17))
    assert np.array_equal(got, B.to_dense()[perm])
    pc = rng.permutation(17)
    r = oracle.spgemm(B, synth.permutation(pc))
    _, got = dense_of(r, (23, 17))
    expect = np.zeros((23, 17))
    expect[:, pc] = B.to_dense()
    assert np.array_equal(got, expect)
    check_sorted_distinct(r)


@pytest.mark.parametrize("seed", range(3))
def test_transpose_identity(seed):
    A = synth.random_csr(31, 27, 0.2, seed, integer_values=True)
    B = synth.random_csr(27, 35, 0.2, seed + 50, integer_values=True)
    ab = oracle.spgemm(A, B)
    btat = oracle.spgemm(synth.csr_transpose(B), synth.csr_transpose(A))
    pa, va = dense_of(ab, (31, 35))
    pb, vb = dense_of(btat, (35, 31))
    assert np.array_equal(pa, pb.T) and np.array_equal(va, vb.T)


@pytest.mark.parametrize("seed", range(3))
def test_against_scipy_positive(seed):
    sp = pytest.importorskip("scipy.sparse")
    A = synth.random_csr(300, 400, 0.03, seed, lo=0.5, hi=2.0)
    B = synth.random_csr(400, 350, 0.03, seed + 9, lo=0.5, hi=2.0)
    r = oracle.spgemm(A, B)
    sa = sp.csr_matrix((A.val, A.col, A.rpt), shape=(300, 400))
    sb = sp.csr_matrix((B.val, B.col, B.rpt), shape=(400, 350))
    sc = (sa @ sb).tocsr()
    sc.sort_indices()
    assert np.array_equal(sc.indptr, r.rpt) and np.array_equal(sc.indices, r.col)
    assert np.all(np.abs(sc.data - r.val) <= 1e-13 * r.absval)


@pytest.mark.parametrize("seed", range(3))
def test_nprod_outer_product_count(seed):
    A = synth.random_csr(40, 30, 0.2, seed)
    B = synth.random_csr(30, 50, 0.2, seed + 1)
    col_counts = np.bincount(A.col, minlength=30)
    assert oracle.row_nprod(A, B).sum() == int((col_counts * B.row_lengths()).sum())


def _kron3(m):
    return np.kron(m, np.kron(m, m))


@pytest.mark.parametrize("n", [3, 4, 5])
def test_stencil27_square_closed_form(n):
    A = synth.stencil_3d_27pt(n)
    S = np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    S3 = _kron3(S)
    assert np.array_equal(A.to_dense(), 27 * np.eye(n ** 3) - S3)
    r = oracle.spgemm(A, A)
    pat, val = dense_of(r, (n ** 3, n ** 3))
    expect = 729 * np.eye(n ** 3) - 54 * S3 + _kron3(S @ S)
    assert np.array_equal(pat, _kron3(S @ S) != 0)
    assert np.array_equal(val, expect)
    assert r.nnz == (5 * n - 6) ** 3
    assert oracle.row_nprod(A, A).sum() == (9 * n - 10) ** 3


@pytest.mark.parametrize("n", [4, 5])
def test_galerkin_closed_form(n):
    A = synth.stencil_3d_27pt(n)
    P = synth.aggregation_p(n)
    Pt = synth.aggregation_pt(n)
    m = (n + 1) // 2
    P1 = np.zeros((n, m))
    P1[np.arange(n), np.arange(n) // 2] = 1
    S = np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    assert np.array_equal(P.to_dense(), _kron3(P1))
    assert np.array_equal(Pt.to_dense(), _kron3(P1).T)
    ap = oracle.spgemm(A, P)
    _, apd = dense_of(ap, (n ** 3, m ** 3))
    assert np.array_equal(apd, 27 * _kron3(P1) - _kron3(S @ P1))
    apc = synth.CSR(n ** 3, m ** 3, ap.rpt, ap.col, ap.val)
    g = oracle.spgemm(Pt, apc)
    _, gd = dense_of(g, (m ** 3, m ** 3))
    assert np.array_equal(gd, 27 * _kron3(P1.T @ P1) - _kron3(P1.T @ S @ P1))
    if n % 2 == 0:
        assert set(np.unique(g.val)) <= {152.0, -16.0, -4.0, -1.0}
        assert ap.nnz == (2 * n - 2) ** 3
    else:
        assert ap.nnz == (2 * n - 1) ** 3
    assert g.nnz == (3 * m - 2) ** 3


@pytest.mark.parametrize("shape", [(0, 5, 4), (5, 0, 4), (5, 4, 0), (0, 0, 0)])
def test_empty_shapes(shape):
    M, K, N = shape
    A = synth.random_csr(M, K, 0.5, 1)
    B = synth.random_csr(K, N, 0.5, 2)
    r = oracle.spgemm(A, B)
    assert r.nnz == 0 and r.rpt.size == M + 1
    b = oracle.brmerge(A, B)
    assert b.nnz == 0


# ---- Algorithm 1 (the accumulation method) run on the CPU -------------------

def _tree_value(leaf_vals, nleaves):
    """Value of one output column from the leaves (list positions) holding it,
    by the rounds of Section III-B: every round combines the partial lists
    2p and 2p+1 into list p of the next round (an odd last list passes), and
    a column present in both adds the left value and the right value."""
    cur = [leaf_vals.get(p) for p in range(nleaves)]
    while len(cur) > 1:
        nxt = []
        for p in range(0, len(cur), 2):
            left = cur[p]
            right = cur[p + 1] if p + 1 < len(cur) else None
            nxt.append(right if left is None else left if right is None else left + right)
        cur = nxt
    return cur[0] if cur else None


@pytest.mark.parametrize("seed", range(6))
def test_brmerge_tree_grouping(seed):
    rng = np.random.default_rng(seed)
    A = synth.random_csr(25, 60, rng.uniform(0.05, 0.5), seed)
    B = synth.random_csr(60, 40, rng.uniform(0.05, 0.5), seed + 3, empty_row_frac=0.2)
    b = oracle.brmerge(A, B)
    for i in range(A.rows):
        ks = A.col[A.rpt[i]:A.rpt[i + 1]]
        avals = A.val[A.rpt[i]:A.rpt[i + 1]]
        per_col = {}
        for leaf, (k, a) in enumerate(zip(ks, avals)):
            for q in range(B.rpt[k], B.rpt[k + 1]):
                per_col.setdefault(int(B.col[q]), {})[leaf] = a * B.val[q]
        cols = sorted(per_col)
        got_c = b.col[b.rpt[i]:b.rpt[i + 1]]
        got_v = b.val[b.rpt[i]:b.rpt[i + 1]]
        assert list(got_c) == cols
        for c, v in zip(cols, got_v):
            assert v == _tree_value(per_col[c], len(ks))  # bitwise
        nl = len(ks)
        assert b.rounds[i] == (math.ceil(math.log2(nl)) if nl > 1 else 0)


def test_brmerge_six_lists_three_rounds():
    # six lists merge in ceil(log2 6) = 3 rounds (Fig. 2 of the paper)
    A = synth.CSR(1, 6, np.array([0, 6], np.int32), np.arange(6, dtype=np.int32), np.ones(6))
    B = synth.random_csr(6, 12, 0.4, 4)
    assert oracle.brmerge(A, B).rounds[0] == 3


@pytest.mark.parametrize("seed", range(4))
def test_brmerge_matches_definition(seed):
    A = synth.random_csr(60, 80, 0.15, seed)
    B = synth.random_csr(80, 70, 0.15, seed + 11, empty_row_frac=0.1)
    r = oracle.spgemm(A, B)
    b = oracle.brmerge(A, B)
    assert np.array_equal(r.rpt, b.rpt) and np.array_equal(r.col, b.col)
    depth = max(1, math.ceil(math.log2(max(2, np.diff(A.rpt).max()))))
    assert np.all(np.abs(r.val - b.val) <= depth * 2.0 ** -53 * r.absval * 1.01)


def test_row_subsets_match_full():
    A = synth.random_csr(50, 40, 0.2, 5)
    B = synth.random_csr(40, 30, 0.2, 6)
    full = oracle.spgemm(A, B)
    rows = np.array([3, 0, 49, 17, 17])
    sub = oracle.spgemm(A, B, rows=rows)
    for t, i in enumerate(rows):
        assert np.array_equal(sub.col[sub.rpt[t]:sub.rpt[t + 1]], full.col[full.rpt[i]:full.rpt[i + 1]])
        assert np.array_equal(sub.val[sub.rpt[t]:sub.rpt[t + 1]], full.val[full.rpt[i]:full.rpt[i + 1]])


def test_compression_ratio_table2():
    rows = np.loadtxt(os.path.join(GOLDEN, "table2_compression_ratio.txt"), comments="#")
    assert rows.shape == (26, 6)
    for _id, _rows, _nnz, nprod, nnzc, cr in rows:
        assert round(oracle.compression_ratio(int(nprod), int(nnzc)), 2) == pytest.approx(cr, abs=1e-9)


def test_row_features_small():
    A = synth.random_csr(20, 15, 0.3, 2)
    B = synth.random_csr(15, 30, 0.3, 3, empty_row_frac=0.3)
    f = oracle.row_features(A, B)
    r = oracle.spgemm(A, B)
    nnzc = np.diff(r.rpt)
    assert np.array_equal(f["nprod"], oracle.row_nprod(A, B))
    # every row of C lies between the longest B row used and min(nprod, span)
    assert np.all(nnzc >= f["maxb"])
    assert np.all(nnzc <= np.minimum(f["nprod"], f["span"]))


@pytest.mark.parametrize("seed", range(3))
def test_pattern_sums_match_brute_force(seed):
    # the structure-only pass: entry count and column sum of every row from
    # the boolean product of Eq. (1)
    A = synth.random_csr(30, 40, 0.1 + 0.1 * seed, seed)
    B = synth.random_csr(40, 50, 0.1, seed + 21, empty_row_frac=0.2)
    cnt, csum = oracle.pattern_sums(A, B)
    pat, _ = oracle.brute_force(A.to_dense(), _pattern(A),
                                B.to_dense(), _pattern(B))
    assert np.array_equal(cnt, pat.sum(axis=1))
    assert np.array_equal(csum, (pat * np.arange(B.cols)[None, :]).sum(axis=1))


def _pattern(X):
    p = np.zeros((X.rows, X.cols), bool)
    p[np.repeat(np.arange(X.rows), X.row_lengths()), X.col.astype(np.int64)] = True
    return p
