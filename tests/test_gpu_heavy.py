"""GPU parity of the heavy-row path (rows beyond one workgroup's LDS):
aligned list ranges merged in LDS, HBM ping-pong merges of tree nodes,
single lists longer than LDS, spill batches."""
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


def run(h, A, B):
    dA = brm.DeviceCSR.from_host(A)
    dB = dA if B is A else brm.DeviceCSR.from_host(B)
    C = h.spgemm(dA, dB)
    torch.cuda.synchronize()
    assert h.stat(brm.STAT_DEVICE_ERR) == 0
    return C


@pytest.fixture(params=[512, 1024])
def handle(request):
    # both heavy kernels (512- and 1024-thread workgroups) on every case
    h = brm.Handle(0)
    h.set_option(brm.OPT_VALIDATE, 1)
    h.set_option(brm.OPT_HEAVY_THREADS, request.param)
    print(f"heavy workgroups of {request.param} threads", flush=True)
    yield h
    h.close()


def _uniform_heavy(nrows, lists, blen, ncols, seed):
    """A (nrows x K) whose rows each take `lists` B rows of `blen` entries:
    every row has lists * blen products (heavy beyond 4096)."""
    rng = np.random.default_rng(seed)
    K = lists * 8
    b_cols = [np.sort(rng.choice(ncols, size=blen, replace=False)) for _ in range(K)]
    B = synth.CSR(K, ncols, np.arange(0, K * blen + 1, blen, dtype=np.int32),
                  np.concatenate(b_cols).astype(np.int32), rng.uniform(-1, 1, K * blen))
    a_cols = [np.sort(rng.choice(K, size=lists, replace=False)) for _ in range(nrows)]
    A = synth.CSR(nrows, K, np.arange(0, nrows * lists + 1, lists, dtype=np.int32),
                  np.concatenate(a_cols).astype(np.int32), rng.uniform(-1, 1, nrows * lists))
    return A, B


def test_heavy_threads_chosen_per_batch():
    # many heavy rows of equal size: 512-thread workgroups; one row far
    # longer than a workgroup's share: 1024-thread workgroups
    h = brm.Handle(0)
    try:
        h.set_option(brm.OPT_VALIDATE, 1)
        A, B = _uniform_heavy(2400, 5, 1000, 20000, 25)
        print("case: 2400 heavy rows of 5000 products", flush=True)
        C = run(h, A, B)
        assert h.stat(brm.STAT_HEAVY_BATCHES) == 1 and h.stat(brm.STAT_HEAVY_WIDE) == 0
        assert_matches_oracle(C, oracle.spgemm(A, B), oracle.brmerge(A, B))
        # one more row taking every list of B: 40000 products
        K = B.rows
        A2 = synth.CSR(A.rows + 1, K, np.concatenate([A.rpt, [A.rpt[-1] + K]]).astype(np.int32),
                       np.concatenate([A.col, np.arange(K)]).astype(np.int32),
                       np.concatenate([A.val, np.ones(K)]))
        print("case: plus one row of 40000 products", flush=True)
        C2 = run(h, A2, B)
        assert h.stat(brm.STAT_HEAVY_BATCHES) == 1 and h.stat(brm.STAT_HEAVY_WIDE) == 1
        assert_matches_oracle(C2, oracle.spgemm(A2, B), oracle.brmerge(A2, B))
    finally:
        h.close()


def test_rmat_all_rows_heavy(handle):
    print("case: R-MAT scale 11, every row forced to the heavy path", flush=True)
    A = synth.rmat(11, 16, 21)
    handle.set_option(brm.OPT_FORCE_CLASS, 6)
    C = run(handle, A, A)
    assert handle.class_rows()["heavy"] == int((oracle.row_nprod(A, A) > 0).sum())
    assert_matches_oracle(C, oracle.spgemm(A, A), oracle.brmerge(A, A))


@pytest.mark.parametrize("lds_max", [64, 500])
def test_rmat_deep_hbm_trees(handle, lds_max):
    print(f"case: R-MAT scale 13, heavy rows with LDS ranges of at most {lds_max}", flush=True)
    A = synth.rmat(13, 16, 22)
    handle.set_option(brm.OPT_HEAVY_LDS_MAX, lds_max)
    C = run(handle, A, A)
    assert handle.class_rows()["heavy"] > 0
    assert_matches_oracle(C, oracle.spgemm(A, A), oracle.brmerge(A, A))


def test_spill_batches(handle):
    print("case: R-MAT scale 13, 1 MB spill budget", flush=True)
    A = synth.rmat(13, 16, 23)
    handle.set_option(brm.OPT_SPILL_BUDGET_MB, 1)
    C = run(handle, A, A)
    assert handle.stat(brm.STAT_HEAVY_BATCHES) > 1
    assert_matches_oracle(C, oracle.spgemm(A, A), oracle.brmerge(A, A))


@pytest.mark.parametrize("budget_mb", [0, 1, 3])
def test_spill_pool_kept_between_calls(handle, budget_mb):
    # the batches of a repeated call fit the pool the first call left, so it
    # is neither freed nor allocated again
    print(f"case: R-MAT scale 13 twice, spill budget {budget_mb} MB", flush=True)
    A = synth.rmat(13, 16, 24)
    handle.set_option(brm.OPT_SPILL_BUDGET_MB, budget_mb)
    dA = brm.DeviceCSR.from_host(A)
    first = to_host(handle.spgemm(dA, dA))
    pool, batches = handle.stat(brm.STAT_SPILL_POOL_BYTES), handle.stat(brm.STAT_HEAVY_BATCHES)
    assert handle.stat(brm.STAT_SPILL_ALLOCS) == 1 and pool > 0
    for _ in range(2):
        again = to_host(handle.spgemm(dA, dA))
        assert handle.stat(brm.STAT_SPILL_ALLOCS) == 1
        assert handle.stat(brm.STAT_SPILL_POOL_BYTES) == pool
        assert handle.stat(brm.STAT_HEAVY_BATCHES) <= batches
        for x, y in zip(first, again):
            assert np.array_equal(x.view(np.int64) if x.dtype == np.float64 else x,
                                  y.view(np.int64) if y.dtype == np.float64 else y)
    assert handle.stat(brm.STAT_DEVICE_ERR) == 0
    assert_matches_oracle(handle.spgemm(dA, dA), oracle.spgemm(A, A), oracle.brmerge(A, A))


def test_long_single_lists(handle):
    # rows whose lists include B rows longer than LDS, odd list counts and
    # empty lists between them
    rng = np.random.default_rng(5)
    K, N = 40, 50000
    lens = rng.integers(0, 300, K)
    lens[[0, 7, 13]] = [9000, 5000, 12000]
    lens[[3, 4]] = 0
    cols = [np.sort(rng.choice(N, size=l, replace=False)) for l in lens]
    rpt = np.zeros(K + 1, np.int64)
    rpt[1:] = np.cumsum(lens)
    B = synth.CSR(K, N, rpt.astype(np.int32), np.concatenate(cols).astype(np.int32),
                  rng.uniform(-1, 1, rpt[-1]))
    rows = [np.arange(K), np.array([0, 3, 4, 7, 13]), np.array([13]), np.array([1, 7, 9, 13, 20, 21, 22]),
            np.arange(0, K, 3)]
    arpt = np.zeros(len(rows) + 1, np.int64)
    arpt[1:] = np.cumsum([len(r) for r in rows])
    A = synth.CSR(len(rows), K, arpt.astype(np.int32), np.concatenate(rows).astype(np.int32),
                  rng.uniform(-1, 1, arpt[-1]))
    for force in (-1, 6):
        handle.set_option(brm.OPT_FORCE_CLASS, force)
        C = run(handle, A, B)
        assert_matches_oracle(C, oracle.spgemm(A, B), oracle.brmerge(A, B))


@pytest.mark.parametrize("split", [2048, 9000, 40000])
def test_split_rows(handle, split):
    # long rows merged as several aligned subtrees (one workgroup each) and
    # the levels above them (one launch per level): bitwise the same tree
    print(f"case: R-MAT scale 13, subtrees of {split} products", flush=True)
    A = synth.rmat(13, 16, 27)
    handle.set_option(brm.OPT_HEAVY_SPLIT, split)
    C = run(handle, A, A)
    assert handle.stat(brm.STAT_HEAVY_SPLIT_ROWS) > 0
    assert_matches_oracle(C, oracle.spgemm(A, A), oracle.brmerge(A, A))


def test_split_every_row_with_spill_batches(handle):
    # every non-empty row heavy and split where it has 2 lists or more, in
    # several spill batches (each with its own top levels)
    print("case: R-MAT scale 12 all heavy, subtrees of 1024 products, 1 MB budget", flush=True)
    A = synth.rmat(12, 16, 28)
    handle.set_option(brm.OPT_FORCE_CLASS, 6)
    handle.set_option(brm.OPT_HEAVY_SPLIT, 1024)
    handle.set_option(brm.OPT_SPILL_BUDGET_MB, 1)
    C = run(handle, A, A)
    assert handle.stat(brm.STAT_HEAVY_SPLIT_ROWS) > 0 and handle.stat(brm.STAT_HEAVY_BATCHES) > 1
    assert_matches_oracle(C, oracle.spgemm(A, A), oracle.brmerge(A, A))


def test_split_with_long_single_lists(handle):
    # subtrees whose nodes include single lists longer than LDS, and odd
    # subtree counts (a promoted node on the way up)
    print("case: long single lists, split rows", flush=True)
    rng = np.random.default_rng(29)
    ncols = 60000
    lens = [9000, 3, 5000, 17, 2, 4500, 1, 64, 7000, 5, 900, 3000, 6, 11, 5200]
    K = len(lens)
    b_cols = [np.sort(rng.choice(ncols, size=n, replace=False)) for n in lens]
    B = synth.CSR(K, ncols, np.concatenate([[0], np.cumsum(lens)]).astype(np.int32),
                  np.concatenate(b_cols).astype(np.int32), rng.uniform(-1, 1, sum(lens)))
    rows = [np.arange(K), np.arange(0, K, 2), np.arange(1, K), np.arange(K - 5)]
    A = synth.CSR(len(rows), K, np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32),
                  np.concatenate(rows).astype(np.int32), rng.uniform(-1, 1, sum(len(r) for r in rows)))
    for split in (3000, 6000):
        handle.set_option(brm.OPT_HEAVY_SPLIT, split)
        C = run(handle, A, B)
        assert handle.stat(brm.STAT_HEAVY_SPLIT_ROWS) > 0
        assert_matches_oracle(C, oracle.spgemm(A, B), oracle.brmerge(A, B))


@pytest.mark.parametrize("alloc", ["upper", "learned_force"])
def test_split_rows_in_slotted_modes(alloc):
    # split rows written into upper-bound slots, or into predicted slots that
    # are too small (every heavy row falls back to the exact path)
    print(f"case: R-MAT scale 13, split rows, {alloc}", flush=True)
    from paper_2206_06611_amd import learned
    A = synth.rmat(13, 16, 30)
    dA = brm.DeviceCSR.from_host(A)
    h = brm.Handle(0)
    try:
        h.set_option(brm.OPT_HEAVY_SPLIT, 4096)
        ref = to_host(h.spgemm(dA, dA))
        if alloc == "upper":
            h.set_option(brm.OPT_ALLOC, brm.ALLOC_UPPER)
        else:
            feats, targets = learned.collect(h, [(dA, dA)])
            learned.train(h, feats, targets, seed=1, epochs=1)
            h.set_option(brm.OPT_ALLOC, brm.ALLOC_LEARNED)
            h.set_option(brm.OPT_LEARNED_FORCE, 1)
        got = to_host(h.spgemm(dA, dA))
        torch.cuda.synchronize()
        assert h.stat(brm.STAT_DEVICE_ERR) == 0
        for x, y in zip(ref, got):
            assert np.array_equal(x.view(np.int64) if x.dtype == np.float64 else x,
                                  y.view(np.int64) if y.dtype == np.float64 else y)
    finally:
        h.close()


def test_split_rows_int64_row_pointers(handle):
    # the 64-bit row-pointer instantiations of the heavy kernel, split rows included
    print("case: R-MAT scale 12, int64 row pointers, subtrees of 3000 products", flush=True)
    A = synth.rmat(12, 16, 31)
    dA = brm.DeviceCSR.from_host(A, rpt_dtype=torch.int64)
    handle.set_option(brm.OPT_HEAVY_SPLIT, 3000)
    C = handle.spgemm(dA, dA)
    torch.cuda.synchronize()
    assert handle.stat(brm.STAT_DEVICE_ERR) == 0
    assert handle.stat(brm.STAT_HEAVY_SPLIT_ROWS) > 0
    assert_matches_oracle(C, oracle.spgemm(A, A), oracle.brmerge(A, A))
