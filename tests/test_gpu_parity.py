"""GPU parity of the plain two-pass path against the CPU oracle.

Every case compares, through the C ABI, C's row pointers and columns
bit-exactly with the oracle's definition and the values within
1e-12 * sum|products| per entry; where noted also bitwise with the CPU run of
Algorithm 1 (same merge tree).
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import assert_matches_oracle, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2206_06611_amd as brm  # noqa: E402


@pytest.fixture(scope="module")
def handle():
    h = brm.Handle(0)
    h.set_option(brm.OPT_VALIDATE, 1)
    yield h
    h.close()


def run(h, A, B, rpt_dtype=None):
    dA = brm.DeviceCSR.from_host(A, rpt_dtype=rpt_dtype)
    dB = dA if B is A else brm.DeviceCSR.from_host(B, rpt_dtype=rpt_dtype)
    C = h.spgemm(dA, dB)
    torch.cuda.synchronize()
    assert h.stat(brm.STAT_DEVICE_ERR) == 0
    return C


def test_config1_laplacian_exact(handle):
    print("case: 64x64 5-point Laplacian squared", flush=True)
    A = synth.laplacian_2d_5pt(64)
    C = run(handle, A, A)
    ref = oracle.spgemm(A, A)
    rpt, col, val = to_host(C)
    assert C.nnz == 51972
    assert np.array_equal(rpt, ref.rpt) and np.array_equal(col, ref.col)
    assert np.array_equal(val, ref.val)  # integer values: exact
    assert handle.stat(brm.STAT_NPROD) == 100104


@pytest.mark.parametrize("seed", range(8))
def test_random_small(handle, seed):
    rng = np.random.default_rng(seed)
    M, K, N = (int(x) for x in rng.integers(1, 300, size=3))
    dens = float(rng.uniform(0.001, 0.08))
    print(f"case: random seed={seed} M={M} K={K} N={N} density={dens:.4f}", flush=True)
    A = synth.random_csr(M, K, dens, seed, empty_row_frac=0.1)
    B = synth.random_csr(K, N, dens * 2, seed + 1000, empty_row_frac=0.1)
    C = run(handle, A, B)
    assert_matches_oracle(C, oracle.spgemm(A, B), oracle.brmerge(A, B))


@pytest.mark.parametrize("force", [2, 3, 4, 5])
def test_forced_classes_bitwise(handle, force):
    # rows of every size routed to one kernel class must give identical bits
    A = synth.random_csr(300, 200, 0.02, 7, empty_row_frac=0.1)
    B = synth.random_csr(200, 400, 0.02, 8, empty_row_frac=0.1)
    # keep only rows that fit the smallest class (64 products and lists)
    w = np.maximum(oracle.row_nprod(A, B), np.diff(A.rpt))
    d = A.to_dense()
    pat = A.to_dense() != 0
    pat[w > 64] = False
    A = synth.from_dense(np.where(pat, d, 0.0), pat)
    base = to_host(run(handle, A, B))
    handle.set_option(brm.OPT_FORCE_CLASS, force)
    try:
        C = to_host(run(handle, A, B))
        assert handle.stat(brm.STAT_CLASS_ROWS0 + force) > 0
    finally:
        handle.set_option(brm.OPT_FORCE_CLASS, -1)
    for x, y in zip(base, C):
        assert np.array_equal(x.view(np.int64) if x.dtype == np.float64 else x,
                              y.view(np.int64) if y.dtype == np.float64 else y)


def test_row_classes_all_used(handle):
    # rows spanning single lists, <=64, <=256, <=1024, <=4096 products
    rng = np.random.default_rng(3)
    K, N = 400, 6000
    lens = np.concatenate([np.zeros(5, int), np.ones(10, int), rng.integers(2, 6, 30),
                           rng.integers(8, 20, 30), rng.integers(40, 80, 20), rng.integers(100, 180, 10)])
    rows = []
    for i, l in enumerate(lens):
        rows.append(np.sort(rng.choice(K, size=min(l, K), replace=False)))
    rpt = np.zeros(len(rows) + 1, np.int64)
    rpt[1:] = np.cumsum([len(r) for r in rows])
    A = synth.CSR(len(rows), K, rpt.astype(np.int32), np.concatenate(rows).astype(np.int32),
                  rng.uniform(-1, 1, rpt[-1]))
    B = synth.random_csr(K, N, 0.0025, 4)
    ref, model = oracle.spgemm(A, B), oracle.brmerge(A, B)
    try:
        for g in (1, 0):  # with lane windows (wave-small, multi), then LDS only
            handle.set_option(brm.OPT_GROUP_ROWS, g)
            C = run(handle, A, B)
            cls = handle.class_rows()
            print(f"case: mixed row sizes, group rows {g}: {cls}", flush=True)
            assert cls["heavy"] == 0
            assert cls["copy"] > 0 and cls["wave_small"] > 0 and cls["group"] > 0
            assert cls["multi"] > 0 if g == 1 else (cls["multi"] == 0 and cls["wave"] > 0)
            assert_matches_oracle(C, ref, model)
    finally:
        handle.set_option(brm.OPT_GROUP_ROWS, 1)


def test_int64_row_pointers(handle):
    A = synth.random_csr(150, 90, 0.05, 11)
    B = synth.random_csr(90, 140, 0.05, 12)
    C = run(handle, A, B, rpt_dtype=torch.int64)
    assert_matches_oracle(C, oracle.spgemm(A, B), oracle.brmerge(A, B))


@pytest.mark.parametrize("shape", [(0, 5, 4), (5, 0, 4), (5, 4, 0), (0, 0, 0), (7, 3, 9)])
def test_empty_and_degenerate(handle, shape):
    M, K, N = shape
    A = synth.random_csr(M, K, 0.0 if shape == (7, 3, 9) else 0.5, 1)
    B = synth.random_csr(K, N, 0.5, 2)
    C = run(handle, A, B)
    assert C.nnz == 0 and C.rpt.numel() == M + 1
    assert int(C.rpt.abs().sum()) == 0


def test_stored_zeros_kept(handle):
    Ad = np.array([[1.0, 1.0, 0.0], [0.0, 0.0, 2.0]])
    Apat = np.array([[True, True, True], [False, False, True]])
    Bd = np.array([[3.0, 1.0], [-3.0, 0.0], [5.0, 0.0]])
    Bpat = np.array([[True, True], [True, False], [True, False]])
    A, B = synth.from_dense(Ad, Apat), synth.from_dense(Bd, Bpat)
    C = run(handle, A, B)
    assert_matches_oracle(C, oracle.spgemm(A, B), oracle.brmerge(A, B))


def test_errors(handle):
    A = synth.random_csr(20, 10, 0.3, 1)
    B = synth.random_csr(11, 10, 0.3, 2)
    dA, dB = brm.DeviceCSR.from_host(A), brm.DeviceCSR.from_host(B)
    with pytest.raises(brm.SpgError) as e:
        handle.spgemm(dA, dB)
    assert e.value.code == brm.SPG_ERR_DIM
    # unsorted columns are caught by validation
    B = synth.random_csr(10, 10, 0.5, 2)
    bad = synth.CSR(B.rows, B.cols, B.rpt, B.col[::-1].copy(), B.val)
    with pytest.raises(brm.SpgError) as e:
        handle.spgemm(dA, brm.DeviceCSR.from_host(bad))
    assert e.value.code == brm.SPG_ERR_INVALID_CSR
    # numeric without symbolic
    h2 = brm.Handle(0)
    dB = brm.DeviceCSR.from_host(B)
    c_rpt = torch.zeros(21, dtype=torch.int64, device="cuda")
    with pytest.raises(brm.SpgError) as e:
        h2.numeric(dA, dB, c_rpt, torch.empty(1, dtype=torch.int32, device="cuda"),
                   torch.empty(1, dtype=torch.float64, device="cuda"))
    assert e.value.code == brm.SPG_ERR_STATE
    h2.close()


def test_deterministic_repeats(handle):
    A = synth.erdos_renyi_rows(20000, 8, 5)
    outs = [to_host(run(handle, A, A)) for _ in range(3)]
    for o in outs[1:]:
        for x, y in zip(outs[0], o):
            assert np.array_equal(x.view(np.int64) if x.dtype == np.float64 else x,
                                  y.view(np.int64) if y.dtype == np.float64 else y)


def test_config2_erdos_renyi_full(handle):
    print("case: ER 2^20 x 2^20, 8 per row, seed 2 (full compare)", flush=True)
    A = synth.erdos_renyi_rows(1 << 20, 8, 2)
    C = run(handle, A, A)
    assert handle.stat(brm.STAT_NPROD) == 8 * A.nnz
    assert_matches_oracle(C, oracle.spgemm(A, A), oracle.brmerge(A, A))


def test_stencil27_square(handle):
    n = 24
    A = synth.stencil_3d_27pt(n)
    C = run(handle, A, A)
    assert C.nnz == (5 * n - 6) ** 3
    ref = oracle.spgemm(A, A)
    rpt, col, val = to_host(C)
    assert np.array_equal(rpt, ref.rpt) and np.array_equal(col, ref.col)
    assert np.array_equal(val, ref.val)


def _mixed_short_rows(seed):
    # rows of at most 64 products; some with lists too uneven for lane
    # windows (one long list beside short ones), some with many tiny lists
    rng = np.random.default_rng(seed)
    K, N = 500, 3000
    blens = np.where(rng.random(K) < 0.1, rng.integers(20, 40, K), rng.integers(0, 4, K))
    brows = [np.sort(rng.choice(N, size=l, replace=False)) for l in blens]
    brpt = np.zeros(K + 1, np.int64)
    brpt[1:] = np.cumsum(blens)
    B = synth.CSR(K, N, brpt.astype(np.int32), np.concatenate(brows).astype(np.int32),
                  rng.uniform(-1, 1, brpt[-1]))
    long_rows = np.flatnonzero(blens >= 20)
    short_rows = np.flatnonzero(blens < 4)
    rows = []
    for i in range(400):
        kind = i % 4
        if kind == 0:  # one long list and a few short ones: uneven
            r = np.concatenate([rng.choice(long_rows, 1), rng.choice(short_rows, int(rng.integers(2, 6)), replace=False)])
        elif kind == 1:  # many tiny lists
            r = rng.choice(short_rows, int(rng.integers(8, 30)), replace=False)
        elif kind == 2:  # two long lists
            r = rng.choice(long_rows, 2, replace=False)
        else:
            r = rng.choice(K, int(rng.integers(0, 5)), replace=False)
        rows.append(np.unique(r))
    rpt = np.zeros(len(rows) + 1, np.int64)
    rpt[1:] = np.cumsum([len(r) for r in rows])
    A = synth.CSR(len(rows), K, rpt.astype(np.int32), np.concatenate(rows).astype(np.int32),
                  rng.uniform(-1, 1, rpt[-1]))
    return A, B


def test_short_row_kernels_agree(handle):
    # every kernel choice for the wave-small class gives the same bits; with
    # lane windows the rows whose lists do not fit them move to the next class
    A, B = _mixed_short_rows(21)
    ref, model = oracle.spgemm(A, B), oracle.brmerge(A, B)
    outs, classes = {}, {}
    try:
        for g in (0, 1, 2, 4):
            print(f"case: mixed short rows, group rows {g}", flush=True)
            handle.set_option(brm.OPT_GROUP_ROWS, g)
            C = run(handle, A, B)
            assert_matches_oracle(C, ref, model)
            outs[g] = to_host(C)
            classes[g] = handle.class_rows()
    finally:
        handle.set_option(brm.OPT_GROUP_ROWS, 1)
    for g in (1, 2, 4):
        for x, y in zip(outs[0], outs[g]):
            assert np.array_equal(x.view(np.int64) if x.dtype == np.float64 else x,
                                  y.view(np.int64) if y.dtype == np.float64 else y)
    assert classes[1]["wave_small"] > 0
    assert classes[1]["wave_small"] < classes[0]["wave_small"]
    # (the rows that leave it go to the multi-register or the LDS classes)
    assert classes[1]["wave"] + classes[1]["multi"] > classes[0]["wave"]


def test_option_change_between_passes(handle):
    # an option set between the passes voids the symbolic plan (the kernels
    # are tied to its classification); the numeric pass then refuses
    A, B = _mixed_short_rows(22)
    dA, dB = brm.DeviceCSR.from_host(A), brm.DeviceCSR.from_host(B)
    try:
        handle.set_option(brm.OPT_GROUP_ROWS, 0)
        c_rpt, nnz = handle.symbolic(dA, dB)
        handle.set_option(brm.OPT_GROUP_ROWS, 1)
        c_col = torch.empty(nnz, dtype=torch.int32, device="cuda")
        c_val = torch.empty(nnz, dtype=torch.float64, device="cuda")
        with pytest.raises(brm.SpgError) as e:
            handle.numeric(dA, dB, c_rpt, c_col, c_val)
        assert e.value.code == brm.SPG_ERR_STATE
    finally:
        handle.set_option(brm.OPT_GROUP_ROWS, 1)


def test_wide_b_columns(handle):
    # B with 2^26 + 5 columns (beyond the 26-bit keys of the register
    # merges, which are then switched off).  Checked against the oracle on a
    # monotone relabelling of B's columns to a compact range: the product
    # commutes with it.
    A, Bc = _mixed_short_rows(23)
    N = (1 << 26) + 5
    rng = np.random.default_rng(24)
    wide = np.sort(rng.choice(N - 1, size=Bc.cols - 1, replace=False))
    wide = np.append(wide, N - 1).astype(np.int32)  # the last column is used
    Bw = synth.CSR(Bc.rows, N, Bc.rpt, wide[Bc.col], Bc.val)
    ref = oracle.spgemm(A, Bc)
    Cw = run(handle, A, Bw)
    cls_w = handle.class_rows()
    run(handle, A, Bc)
    cls_c = handle.class_rows()
    ref.col = wide[ref.col]
    assert_matches_oracle(Cw, ref)
    assert cls_w["wave_small"] > cls_c["wave_small"]


def test_row_blocks_match_whole_product(handle):
    print("case: R-MAT scale 12 in row blocks of at most 20000 products", flush=True)
    A = synth.rmat(12, 16, 44)
    dA = brm.DeviceCSR.from_host(A)
    nprod = handle.row_products(dA, dA).cpu().numpy()
    assert np.array_equal(nprod, oracle.row_nprod(A, A))
    whole = to_host(handle.spgemm(dA, dA))
    blocks = handle.row_blocks(dA, dA, 20000)
    assert len(blocks) > 10
    parts = []
    for b, e in blocks:
        assert nprod[b:e].sum() <= 20000 or e == b + 1
        parts.append(to_host(handle.spgemm(dA.row_block(b, e), dA)))
    rpt = np.concatenate([[0]] + [p[0][1:] + off for p, off in
                                  zip(parts, np.cumsum([0] + [p[0][-1] for p in parts[:-1]]))])
    assert np.array_equal(rpt, whole[0])
    assert np.array_equal(np.concatenate([p[1] for p in parts]), whole[1])
    assert np.array_equal(np.concatenate([p[2] for p in parts]).view(np.int64), whole[2].view(np.int64))
    # empty and single-row blocks
    C0 = handle.spgemm(dA.row_block(7, 7), dA)
    assert C0.rows == 0 and C0.nnz == 0
    C1 = to_host(handle.spgemm(dA.row_block(0, 1), dA))
    assert np.array_equal(C1[1], whole[1][:whole[0][1]])


def test_column_wise_dual(handle):
    # CSC in, CSC out: column j of C = A*B merges the columns of A selected
    # by column j of B; the same arrays are the row-wise product B^T A^T
    print("case: column-wise product of CSC inputs", flush=True)
    A = synth.random_csr(150, 90, 0.05, 81, empty_row_frac=0.1)
    B = synth.random_csr(90, 200, 0.06, 82, empty_row_frac=0.1)
    dA, dB = brm.DeviceCSC.from_host_csr(A), brm.DeviceCSC.from_host_csr(B)
    assert np.array_equal(dA.row.cpu().numpy(), synth.csr_transpose(A).col)
    C = handle.spgemm_csc(dA, dB)
    torch.cuda.synchronize()
    assert (C.rows, C.cols) == (150, 200)
    Bt, At = synth.csr_transpose(B), synth.csr_transpose(A)
    assert_matches_oracle(C.transposed_csr(), oracle.spgemm(Bt, At), oracle.brmerge(Bt, At))
    # read back as CSR, C is the definition of A*B
    ct = C.transposed_csr()
    Ct = synth.CSR(ct.rows, ct.cols, ct.rpt.cpu().numpy(), ct.col.cpu().numpy(), ct.val.cpu().numpy())
    Cr = synth.csr_transpose(Ct)
    ref = oracle.spgemm(A, B)
    assert np.array_equal(np.asarray(Cr.rpt, np.int64), ref.rpt) and np.array_equal(Cr.col, ref.col)
    assert np.all(np.abs(Cr.val - ref.val) <= 1e-12 * ref.absval)
    with pytest.raises(brm.SpgError):
        handle.spgemm_csc(dA, dA)


def _multi_window_rows(seed, M=500):
    # rows whose lists fit lane windows of 2 to 16 registers per lane: padded
    # total 2^t (t = 7..10) split between list width 2^sw and list count
    rng = np.random.default_rng(seed)
    K, N = 2048, 4096
    blens = rng.integers(0, 1025, K)
    blens[:64] = np.arange(64)  # short rows of every length
    order = np.argsort(blens, kind="stable")
    sl_ = blens[order]
    brows = [np.sort(rng.choice(N, size=int(l), replace=False)) for l in blens]
    brpt = np.zeros(K + 1, np.int64)
    brpt[1:] = np.cumsum(blens)
    B = synth.CSR(K, N, brpt.astype(np.int32), np.concatenate(brows).astype(np.int32), rng.uniform(-1, 1, brpt[-1]))
    rows = []
    for i in range(M):
        t = int(rng.integers(7, 11))
        sw = int(rng.integers(max(t - 6, 0), t + 1))
        L = int(rng.integers((1 << (t - sw - 1)) + 1, (1 << (t - sw)) + 1)) if t - sw > 0 else 1
        L = max(L, 2)
        mx = int(rng.integers((1 << (sw - 1)) + 1, (1 << sw) + 1)) if sw > 0 else 1
        # one list of length mx, the others not longer
        lo, hi = np.searchsorted(sl_, [mx, mx + 1])
        if hi <= lo:
            continue
        first = order[rng.integers(lo, hi)]
        short = order[:np.searchsorted(sl_, mx + 1)]
        rest = rng.choice(short, size=min(L - 1, short.size), replace=False)
        r = np.unique(np.concatenate([[first], rest]))
        rng.shuffle(r)  # any stored order of the lists, columns sorted below
        rows.append(np.sort(r))
    rpt = np.zeros(len(rows) + 1, np.int64)
    rpt[1:] = np.cumsum([len(r) for r in rows])
    A = synth.CSR(len(rows), K, rpt.astype(np.int32), np.concatenate(rows).astype(np.int32),
                  rng.uniform(-1, 1, rpt[-1]))
    return A, B


@pytest.mark.parametrize("seed", [31, 32])
def test_multi_register_windows(handle, seed):
    A, B = _multi_window_rows(seed)
    ref, model = oracle.spgemm(A, B), oracle.brmerge(A, B)
    outs = {}
    try:
        for g, force in ((1, -1), (1, 7), (0, -1)):
            print(f"case: multi-register windows seed {seed}, group rows {g}, force {force}", flush=True)
            handle.set_option(brm.OPT_GROUP_ROWS, g)
            handle.set_option(brm.OPT_FORCE_CLASS, force)
            C = run(handle, A, B)
            cls = handle.class_rows()
            print(cls, flush=True)
            if g == 1:
                assert cls["multi"] > A.rows // 2
            else:
                assert cls["multi"] == 0
            assert_matches_oracle(C, ref, model)
            outs[(g, force)] = to_host(C)
    finally:
        handle.set_option(brm.OPT_FORCE_CLASS, -1)
        handle.set_option(brm.OPT_GROUP_ROWS, 1)
    # the symbolic counts of the multi class are the exact row sizes
    assert np.array_equal(outs[(1, -1)][0], ref.rpt)


def test_multi_register_windows_column_limit(handle):
    # keys hold columns below 2^21: with B that wide the class is not used
    A, B = _multi_window_rows(33, M=120)
    ref = oracle.spgemm(A, B)
    for N, want in ((1 << 21, True), ((1 << 21) + 1, False)):
        Bw = synth.CSR(B.rows, N, B.rpt, (B.col.astype(np.int64) * (N - 1) // (B.cols - 1)).astype(np.int32), B.val)
        refw = oracle.spgemm(A, Bw)
        C = run(handle, A, Bw)
        assert (handle.class_rows()["multi"] > 0) == want
        assert_matches_oracle(C, refw, oracle.brmerge(A, Bw))
    assert ref.nnz > 0


def test_multi_register_windows_int64_row_pointers(handle):
    # the multi-register class with 64-bit row pointers in A and B
    A, B = _multi_window_rows(34, M=150)
    ref, model = oracle.spgemm(A, B), oracle.brmerge(A, B)
    C = run(handle, A, B, rpt_dtype=torch.int64)
    assert handle.class_rows()["multi"] > 0
    assert_matches_oracle(C, ref, model)


@pytest.mark.parametrize("seed", [61, 62])
def test_paired_short_rows(handle, seed):
    # rows whose windows fit 32 lanes share a wavefront in pairs; mixed with
    # rows that need all 64 lanes and a count of rows that is no multiple of
    # 64, so that pairs, single rows and a ragged last chunk all occur
    rng = np.random.default_rng(seed)
    K, N = 3000, 5000
    B = synth.random_csr(K, N, 0.0015, seed + 100)  # B rows of about 7 entries
    rows = []
    for i in range(2000 + seed):
        L = int(rng.choice([1, 2, 3, 4, 5, 6, 8]))
        rows.append(np.sort(rng.choice(K, size=L, replace=False)))
    rpt = np.zeros(len(rows) + 1, np.int64)
    rpt[1:] = np.cumsum([len(r) for r in rows])
    A = synth.CSR(len(rows), K, rpt.astype(np.int32), np.concatenate(rows).astype(np.int32),
                  rng.uniform(-1, 1, rpt[-1]))
    ref, model = oracle.spgemm(A, B), oracle.brmerge(A, B)
    C = run(handle, A, B)
    assert handle.class_rows()["wave_small"] > 500
    assert_matches_oracle(C, ref, model)


def _repeat_heavy_short_rows(seed, ncols=40):
    """Rows of 1..8 lists over B rows whose columns fall in a narrow range
    (many repeated columns per row), mixed widths so that paired and single
    64-lane windows both occur."""
    rng = np.random.default_rng(seed)
    K = 2000
    B = synth.random_csr(K, ncols, 0.15, seed + 300)
    rows = []
    for i in range(3000 + seed):
        L = int(rng.choice([1, 2, 3, 4, 6, 8]))
        rows.append(np.sort(rng.choice(K, size=L, replace=False)))
    rpt = np.zeros(len(rows) + 1, np.int64)
    rpt[1:] = np.cumsum([len(r) for r in rows])
    A = synth.CSR(len(rows), K, rpt.astype(np.int32), np.concatenate(rows).astype(np.int32),
                  rng.uniform(-1, 1, rpt[-1]))
    return A, B


@pytest.mark.parametrize("seed", [0, 1])
def test_stored_order_matches_window_merges(handle, seed):
    # the numeric pass applying the order the symbolic pass kept (default)
    # and the numeric pass merging its windows itself: the same bits, both
    # bitwise Algorithm 1's tree; rows with many repeated columns, paired
    # short rows and full 64-lane rows (ER-8 rows)
    cases = [_repeat_heavy_short_rows(seed), (synth.erdos_renyi_rows(1 << 12, 8, seed + 7),) * 2]
    try:
        for A, B in cases:
            ref, model = oracle.spgemm(A, B), oracle.brmerge(A, B)
            outs = {}
            for so in (1, 0):
                print(f"case: stored order {so}, {A.rows} rows", flush=True)
                handle.set_option(brm.OPT_STORED_ORDER, so)
                C = run(handle, A, B)
                assert handle.class_rows()["wave_small"] > A.rows // 4
                assert_matches_oracle(C, ref, model)
                outs[so] = to_host(C)
            for x, y in zip(outs[0], outs[1]):
                assert np.array_equal(x.view(np.int64) if x.dtype == np.float64 else x,
                                      y.view(np.int64) if y.dtype == np.float64 else y)
    finally:
        handle.set_option(brm.OPT_STORED_ORDER, 1)


def test_stored_order_new_values_between_passes(handle):
    # the kept order is structure only: values changed between the passes
    # (same arrays) are the ones the numeric pass multiplies
    A, B = _repeat_heavy_short_rows(5)
    dA, dB = brm.DeviceCSR.from_host(A), brm.DeviceCSR.from_host(B)
    c_rpt, nnz = handle.symbolic(dA, dB)
    A2 = synth.CSR(A.rows, A.cols, A.rpt, A.col, np.random.default_rng(6).uniform(-2, 2, A.nnz))
    dA.val.copy_(torch.as_tensor(A2.val, device=dA.val.device))
    c_col = torch.empty(nnz, dtype=torch.int32, device="cuda")
    c_val = torch.empty(nnz, dtype=torch.float64, device="cuda")
    handle.numeric(dA, dB, c_rpt, c_col, c_val)
    torch.cuda.synchronize()
    assert handle.stat(brm.STAT_DEVICE_ERR) == 0
    C = brm.DeviceCSR(A.rows, B.cols, c_rpt, c_col, c_val)
    assert_matches_oracle(C, oracle.spgemm(A2, B), oracle.brmerge(A2, B))


def test_stored_order_option_range(handle):
    assert handle.get_option(brm.OPT_STORED_ORDER) == 1
    for bad in (-1, 2):
        with pytest.raises(brm.SpgError):
            handle.set_option(brm.OPT_STORED_ORDER, bad)


def test_csr_struct_follows_replaced_tensors(handle):
    # the binding keeps a matrix's last C struct while its tensors stay the
    # same; a replaced value or row-pointer array is the one the library reads
    A = synth.erdos_renyi_rows(700, 6, 11)
    dA = brm.DeviceCSR.from_host(A)
    assert dA._struct() is dA._struct()
    run_C = handle.spgemm(dA, dA)
    torch.cuda.synchronize()
    assert_matches_oracle(run_C, oracle.spgemm(A, A), oracle.brmerge(A, A))
    A2 = synth.CSR(A.rows, A.cols, A.rpt, A.col, np.random.default_rng(12).uniform(-2, 2, A.nnz))
    old = dA._struct()
    dA.val = torch.as_tensor(A2.val, device=dA.val.device)
    assert dA._struct() is not old and dA._struct().val == dA.val.data_ptr()
    C2 = handle.spgemm(dA, dA)
    torch.cuda.synchronize()
    assert handle.stat(brm.STAT_DEVICE_ERR) == 0
    assert_matches_oracle(C2, oracle.spgemm(A2, A2), oracle.brmerge(A2, A2))
    # the same matrix with 32-bit row pointers: a new rpt tensor, a new width
    dA.rpt = dA.rpt.to(torch.int32)
    assert dA._struct().rpt_bytes == 4
    C3 = handle.spgemm(dA, dA)
    torch.cuda.synchronize()
    assert handle.stat(brm.STAT_DEVICE_ERR) == 0
    assert_matches_oracle(C3, oracle.spgemm(A2, A2), oracle.brmerge(A2, A2))


@pytest.mark.parametrize("rows", [1, 1023, 1024, 1025, 2047, 4097, 65537])
def test_row_pointer_scan_tile_edges(handle, rows):
    # the row-pointer scan works in tiles of 1024 rows: row counts on either
    # side of a tile's end; a scaled permutation squared with a quarter of
    # the rows empty has C[i, p[p[i]]] = a[i] * a[p[i]] where both rows hold
    # an entry
    rng = np.random.default_rng(rows + 7)
    p = rng.permutation(rows).astype(np.int32)
    a = rng.uniform(0.5, 2.0, rows)
    empty = rng.random(rows) < 0.25
    rpt = np.zeros(rows + 1, np.int64)
    rpt[1:] = np.cumsum(~empty)
    A = synth.CSR(rows, rows, rpt, p[~empty], a[~empty])
    C = run(handle, A, A)
    has = ~empty & ~empty[p]
    exp_rpt = np.zeros(rows + 1, np.int64)
    exp_rpt[1:] = np.cumsum(has)
    assert np.array_equal(C.rpt.cpu().numpy(), exp_rpt)
    assert np.array_equal(C.col.cpu().numpy(), p[p][has])
    assert np.array_equal(C.val.cpu().numpy(), (a * a[p])[has])
    assert_matches_oracle(C, oracle.spgemm(A, A), oracle.brmerge(A, A))
