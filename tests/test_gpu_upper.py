"""GPU checks of the upper-bound allocation (every row of C gets a slot of as
many entries as it has products, the numeric pass runs into the slots, the
rows are then copied into C): bitwise equal to the precise path, no
overflow, and row blocks for products whose slots exceed a memory budget."""
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


@pytest.fixture()
def handle():
    h = brm.Handle(0)
    h.set_option(brm.OPT_VALIDATE, 1)
    yield h
    h.close()


def _same(x, y):
    return np.array_equal(x.view(np.int64) if x.dtype == np.float64 else x,
                          y.view(np.int64) if y.dtype == np.float64 else y)


CASES = {
    "er_2e13": lambda: synth.erdos_renyi_rows(1 << 13, 8, 71),
    "rmat_13": lambda: synth.rmat(13, 16, 72),
    "stencil_10": lambda: synth.stencil_3d_27pt(10),
    "laplace_40": lambda: synth.laplacian_2d_5pt(40),
    "random_empty_rows": lambda: synth.random_csr(300, 300, 0.03, 73, empty_row_frac=0.3),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_upper_bound_bitwise_equal_to_precise(handle, name):
    print(f"case: upper-bound allocation, {name}", flush=True)
    A = CASES[name]()
    dA = brm.DeviceCSR.from_host(A)
    base = to_host(handle.spgemm(dA, dA))
    handle.set_option(brm.OPT_ALLOC, brm.ALLOC_UPPER)
    C = handle.spgemm(dA, dA)
    torch.cuda.synchronize()
    assert handle.stat(brm.STAT_DEVICE_ERR) == 0
    assert handle.stat(brm.STAT_OVERFLOW_ROWS) == 0
    nprod = oracle.row_nprod(A, A)
    assert handle.stat(brm.STAT_PRED_TOTAL) == int(nprod.sum())
    got = to_host(C)
    for x, y in zip(base, got):
        assert _same(x, y)
    if name == "rmat_13":
        assert handle.class_rows()["heavy"] > 0
        assert_matches_oracle(C, oracle.spgemm(A, A), oracle.brmerge(A, A))
    handle.set_option(brm.OPT_ALLOC, brm.ALLOC_PRECISE)


def test_upper_bound_empty_and_rectangular(handle):
    handle.set_option(brm.OPT_ALLOC, brm.ALLOC_UPPER)
    for M, K, N in [(0, 5, 7), (5, 0, 7), (5, 7, 0), (1, 1, 1)]:
        print(f"case: upper-bound allocation, {M}x{K} times {K}x{N}", flush=True)
        A = synth.random_csr(M, K, 0.5, 74)
        B = synth.random_csr(K, N, 0.5, 75)
        C = handle.spgemm(brm.DeviceCSR.from_host(A), brm.DeviceCSR.from_host(B))
        torch.cuda.synchronize()
        ref = oracle.spgemm(A, B)
        assert_matches_oracle(C, ref)
    handle.set_option(brm.OPT_ALLOC, brm.ALLOC_PRECISE)


def test_upper_bound_row_blocks(handle):
    # a slot budget of 30000 products: the product runs block by block
    A = synth.rmat(12, 16, 76)
    dA = brm.DeviceCSR.from_host(A)
    whole = to_host(handle.spgemm(dA, dA))
    handle.set_option(brm.OPT_ALLOC, brm.ALLOC_UPPER)
    cols, vals, lens = [], [], []
    for b, e, Cb in handle.spgemm_row_blocks(dA, dA, 30000):
        assert handle.stat(brm.STAT_PRED_TOTAL) <= 30000 or e == b + 1
        r, c, v = to_host(Cb)
        lens.append(np.diff(r))
        cols.append(c)
        vals.append(v)
    assert np.array_equal(np.concatenate(lens), np.diff(whole[0]))
    assert np.array_equal(np.concatenate(cols), whole[1])
    assert _same(np.concatenate(vals), whole[2])
    handle.set_option(brm.OPT_ALLOC, brm.ALLOC_PRECISE)


def _csr_struct(X, with_val=True):
    s = X._struct()
    if not with_val:
        s.val = None
    return s


@pytest.mark.parametrize("alloc", ["upper", "learned"])
def test_slotted_symbolic_needs_values(handle, alloc):
    # learned and upper-bound allocation compute the values in the symbolic
    # call: NULL values are rejected there, before any launch
    import ctypes
    print(f"case: {alloc} allocation, symbolic with NULL values", flush=True)
    A = synth.rmat(10, 8, 77)
    dA = brm.DeviceCSR.from_host(A)
    if alloc == "learned":
        from oracle import mlp
        theta = mlp.init_params(3)
        handle.mlp_set_params(theta, np.r_[np.zeros(6), np.ones(6)], 0.0)
        handle.set_option(brm.OPT_ALLOC, brm.ALLOC_LEARNED)
    else:
        handle.set_option(brm.OPT_ALLOC, brm.ALLOC_UPPER)
    c_rpt = torch.empty(A.rows + 1, dtype=torch.int64, device="cuda")
    nnz = ctypes.c_int64()
    lib = brm.library()
    for a_val, b_val in ((False, True), (True, False)):
        sa, sb = _csr_struct(dA, a_val), _csr_struct(dA, b_val)
        rc = lib.spgemm_symbolic(handle._h, ctypes.byref(sa), ctypes.byref(sb), ctypes.c_void_p(c_rpt.data_ptr()),
                                 ctypes.byref(nnz), brm._stream_ptr(None))
        assert rc == brm.SPG_ERR_ARG
        assert b"val is NULL" in lib.spg_last_error(handle._h)
    # the precise method takes NULL values in the symbolic call
    handle.set_option(brm.OPT_ALLOC, brm.ALLOC_PRECISE)
    sa, sb = _csr_struct(dA, False), _csr_struct(dA, False)
    rc = lib.spgemm_symbolic(handle._h, ctypes.byref(sa), ctypes.byref(sb), ctypes.c_void_p(c_rpt.data_ptr()),
                             ctypes.byref(nnz), brm._stream_ptr(None))
    assert rc == brm.SPG_OK
    assert nnz.value == oracle.spgemm(A, A).nnz


def test_upper_bound_values_taken_at_symbolic_call(handle):
    # under the upper-bound method every row's values are computed by the
    # symbolic call; the numeric call copies them: values changed between
    # the two calls do not reach C (the documented contract)
    print("case: upper-bound allocation, values changed between the calls", flush=True)
    A = synth.rmat(12, 16, 78)
    B = synth.rmat(12, 16, 79)
    dA, dB = brm.DeviceCSR.from_host(A), brm.DeviceCSR.from_host(B)
    handle.set_option(brm.OPT_ALLOC, brm.ALLOC_UPPER)
    c_rpt, nnz = handle.symbolic(dA, dB)
    orig = dB.val.clone()
    dB.val.mul_(-3.0)
    c_col = torch.empty(nnz, dtype=torch.int32, device="cuda")
    c_val = torch.empty(nnz, dtype=torch.float64, device="cuda")
    handle.numeric(dA, dB, c_rpt, c_col, c_val)
    torch.cuda.synchronize()
    assert handle.stat(brm.STAT_OVERFLOW_ROWS) == 0
    C = brm.DeviceCSR(A.rows, B.cols, c_rpt, c_col, c_val)
    assert_matches_oracle(C, oracle.spgemm(A, B), oracle.brmerge(A, B))
    # the precise method reads the values in the numeric call
    handle.set_option(brm.OPT_ALLOC, brm.ALLOC_PRECISE)
    c_rpt, nnz = handle.symbolic(dA, dB)
    dB.val.copy_(orig)
    handle.numeric(dA, dB, c_rpt, c_col, c_val)
    torch.cuda.synchronize()
    assert_matches_oracle(C, oracle.spgemm(A, B), oracle.brmerge(A, B))


def test_row_with_2_31_products_is_rejected(handle):
    # one row of A takes all 65536 rows of B, each of 32769 entries:
    # 2^31 + 2^16 products in one row.  The analysis routes the row to no
    # kernel and the symbolic call fails with SPG_ERR_CAPACITY (values are not
    # read by the precise method: B has no value array).
    import ctypes
    print("case: one row of 2^31 + 2^16 products (B.col 8.6 GB)", flush=True)
    K, blen = 1 << 16, (1 << 15) + 1
    b_rpt = torch.arange(K + 1, dtype=torch.int64, device="cuda") * blen
    b_col = torch.arange(blen, dtype=torch.int32, device="cuda").repeat(K)
    a_rpt = torch.tensor([0, K], dtype=torch.int32, device="cuda")
    a_col = torch.arange(K, dtype=torch.int32, device="cuda")
    sa = brm._Csr(1, K, K, a_rpt.data_ptr(), 4, a_col.data_ptr(), None)
    sb = brm._Csr(K, blen, K * blen, b_rpt.data_ptr(), 8, b_col.data_ptr(), None)
    c_rpt = torch.empty(2, dtype=torch.int64, device="cuda")
    nnz = ctypes.c_int64()
    handle.set_option(brm.OPT_VALIDATE, 0)
    lib = brm.library()
    rc = lib.spgemm_symbolic(handle._h, ctypes.byref(sa), ctypes.byref(sb), ctypes.c_void_p(c_rpt.data_ptr()),
                             ctypes.byref(nnz), brm._stream_ptr(None))
    torch.cuda.synchronize()
    assert rc == brm.SPG_ERR_CAPACITY
    assert b"2^31" in lib.spg_last_error(handle._h)
    # the handle stays usable
    del b_col
    A = synth.laplacian_2d_5pt(16)
    dA = brm.DeviceCSR.from_host(A)
    assert_matches_oracle(handle.spgemm(dA, dA), oracle.spgemm(A, A))
