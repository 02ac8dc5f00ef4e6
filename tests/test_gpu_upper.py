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
