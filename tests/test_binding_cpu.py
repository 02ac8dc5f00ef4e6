"""Host logic of the Python binding (no device calls)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
brm = pytest.importorskip("paper_2206_06611_amd")


@pytest.mark.parametrize("seed", range(5))
def test_cut_row_blocks(seed):
    rng = np.random.default_rng(seed)
    nprod = rng.integers(0, 100, 500) * (rng.random(500) < 0.8)
    nprod[rng.integers(0, 500, 3)] = 5000  # rows above the budget
    budget = int(rng.integers(100, 2000))
    blocks = brm.cut_row_blocks(nprod, budget)
    assert blocks[0][0] == 0 and blocks[-1][1] == 500
    for (b, e), (b2, _) in zip(blocks, blocks[1:]):
        assert e == b2
    for b, e in blocks:
        assert e > b
        assert nprod[b:e].sum() <= budget or e == b + 1
        # greedy: the next row would not have fitted
        if e < 500:
            assert nprod[b:e + 1].sum() > budget
    assert brm.cut_row_blocks(np.zeros(0, np.int64), 10) == []
    assert brm.cut_row_blocks(np.zeros(7, np.int64), 0) == [(0, 7)]


def test_csc_from_host_is_the_transpose():
    A = synth.random_csr(40, 30, 0.1, 3, empty_row_frac=0.2)
    C = brm.DeviceCSC.from_host_csr(A, device="cpu")
    T = synth.csr_transpose(A)
    assert (C.rows, C.cols) == (40, 30)
    assert np.array_equal(C.cpt.numpy().astype(np.int64), np.asarray(T.rpt, np.int64))
    assert np.array_equal(C.row.numpy(), T.col)
    assert np.array_equal(C.val.numpy(), T.val)
    t = C.transposed_csr()
    assert (t.rows, t.cols) == (30, 40)
