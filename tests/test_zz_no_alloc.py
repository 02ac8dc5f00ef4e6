"""GPU checks of spgemm_batched_noalloc, the allocation-free form of the
batched product (workspace in the library's fixed scratch array, kernels
launched directly): its outputs against spgemm_batched's (bitwise) and the
oracle's, over two calls in a row whose second batch is smaller, and its
errors (workspace beyond the scratch array, arena too small); batches with
heavy rows, whose spill space lies in the arena."""
import ctypes

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

def dev(A, **kw):
    return brm.DeviceCSR.from_host(A, **kw)


def same_bits(x, y):
    for a, b in zip(x, y):
        if a.dtype == np.float64:
            a, b = a.view(np.int64), b.view(np.int64)
        assert np.array_equal(a, b)


def galerkin_batch(edges, seed):
    """Galerkin problems (stage 1: A P, stage 2: P^T (A P)) followed by
    nothing else; plus the host matrices for the oracle."""
    inp = [(synth.stencil_3d_27pt(n), synth.aggregation_p(n), synth.aggregation_pt(n)) for n in edges]
    triples = [(dev(A), dev(P), dev(Pt)) for A, P, Pt in inp]
    return inp, triples


def run(h, probs, arena_bytes, noalloc):
    arena = torch.full((arena_bytes,), 0xA5, dtype=torch.uint8, device="cuda")
    out = torch.full((max(probs.n, 1), 6), -7, dtype=torch.int64, device="cuda")
    rc, req, outs = h.batched(probs, arena, out=out, noalloc=noalloc)
    torch.cuda.synchronize()
    return rc, req, outs, out.cpu().numpy()


def check_batch(h, inp, triples, arena_bytes):
    probs = brm.Handle.galerkin_problems(triples)
    rc0, req0, ref_outs, ref_desc = run(h, probs, arena_bytes, noalloc=False)
    rc1, req1, outs, desc = run(h, probs, arena_bytes, noalloc=True)
    assert rc0 == brm.SPG_OK and rc1 == brm.SPG_OK, brm.library().spg_last_error(h._h)
    assert req1 == req0
    assert np.array_equal(desc, ref_desc), "output descriptors differ from spgemm_batched's"
    n = len(inp)
    for C, R in zip(outs, ref_outs):
        same_bits(to_host(C), to_host(R))
    for (A, P, Pt), ap, g in zip(inp, outs[:n], outs[n:]):
        ref_ap = oracle.spgemm(A, P)
        assert_matches_oracle(ap, ref_ap, oracle.brmerge(A, P))
        apc = synth.CSR(A.rows, P.cols, ref_ap.rpt, ref_ap.col, ref_ap.val)
        assert_matches_oracle(g, oracle.spgemm(Pt, apc), oracle.brmerge(Pt, apc))


def test_noalloc_matches_batched_on_two_calls_second_smaller():
    h = brm.Handle(0)
    try:
        print("case: noalloc galerkin edges [9, 12, 7, 10, 5]", flush=True)
        inp, triples = galerkin_batch([9, 12, 7, 10, 5], 0)
        check_batch(h, inp, triples, 1 << 24)
        print("case: noalloc galerkin edges [6, 4] (smaller)", flush=True)
        inp, triples = galerkin_batch([6, 4], 1)
        check_batch(h, inp, triples, 1 << 22)
        # the spgemm_batched calls only (each batch seen once: launched directly)
        assert h.stat(brm.STAT_BATCHED_DIRECT) == 2 and h.stat(brm.STAT_GRAPH_CAPTURES) == 0
    finally:
        h.close()


def test_noalloc_generic_problems_and_new_handle():
    """Rectangular problems with empty rows, int64 row pointers, from a handle
    that has made no other call; then a smaller batch."""
    rng = np.random.default_rng(7)
    for count, kw in ((7, {"rpt_dtype": torch.int64}), (3, {})):
        host = []
        for i in range(count):
            M, K, N = (int(x) for x in rng.integers(1, 300, 3))
            host.append((synth.random_csr(M, K, 0.04, 300 + i, empty_row_frac=0.1),
                         synth.random_csr(K, N, 0.04, 400 + i)))
        dp = [(dev(A, **kw), dev(B, **kw)) for A, B in host]
        h = brm.Handle(0)
        try:
            print(f"case: noalloc generic, {count} problems {kw}", flush=True)
            rc, req, outs, _ = run(h, brm.BatchedProblems(dp), 1 << 22, noalloc=True)
            assert rc == brm.SPG_OK, brm.library().spg_last_error(h._h)
            assert h.stat(brm.STAT_GRAPH_CAPTURES) == 0
            for (A, B), (dA, dB), C in zip(host, dp, outs):
                assert_matches_oracle(C, oracle.spgemm(A, B), oracle.brmerge(A, B))
                same_bits(to_host(C), to_host(h.spgemm(dA, dB)))
        finally:
            h.close()


def test_noalloc_rejects_workspace_beyond_scratch():
    # a diagonal matrix of 2.5M rows needs 29 B per row + 12 B per entry
    # (~100 MB) of workspace: more than the 64 MiB array
    M = 2_500_000
    D = synth.CSR(M, M, np.arange(M + 1, dtype=np.int64), np.arange(M, dtype=np.int32), np.ones(M))
    dD = dev(D)
    h = brm.Handle(0)
    try:
        # the arena holds C's row pointers, so the workspace is what fails
        arena = torch.empty(1 << 25, dtype=torch.uint8, device="cuda")
        out = torch.full((1, 6), -7, dtype=torch.int64, device="cuda")
        with pytest.raises(brm.SpgError) as e:
            h.batched([(dD, dD)], arena, out=out, noalloc=True)
        assert e.value.code == brm.SPG_ERR_SCRATCH
        assert "allocation-free" in str(e.value)
        torch.cuda.synchronize()
        assert out.cpu().numpy()[0, 0] == -7  # nothing was launched
        # the handle and the array still serve a batch that fits
        inp, triples = galerkin_batch([5, 6], 2)
        check_batch(h, inp, triples, 1 << 22)
    finally:
        h.close()


def test_noalloc_arena_errors_and_heavy_rows_match_batched():
    h = brm.Handle(0)
    try:
        inp, triples = galerkin_batch([8, 5], 3)
        probs = brm.Handle.galerkin_problems(triples)
        # more than the row pointers, less than C: stage 1 (A P) does not fit,
        # so stage 2 computes nothing; with the size then reported stage 1
        # fits and stage 2 may not; the third size fits both
        size = 1 << 14
        for attempt in range(3):
            rc0, req0, _, _ = run(h, probs, size, noalloc=False)
            rc1, req1, _, desc = run(h, probs, size, noalloc=True)
            assert rc1 == rc0 and req1 == req0
            if rc1 == brm.SPG_OK:
                break
            assert rc1 == brm.SPG_ERR_CAPACITY and req1 > size
            assert (desc[:probs.n, 2] == -1).all()
            size = req1
        assert rc1 == brm.SPG_OK and attempt >= 1
        # heavy rows (spill space in the arena): the same need and the same bits
        A = synth.rmat(12, 16, 5)
        p2 = brm.BatchedProblems([(dev(A), dev(A))])
        rc0, req0, _, _ = run(h, p2, 1 << 20, noalloc=False)
        rc1, req1, _, _ = run(h, p2, 1 << 20, noalloc=True)
        assert rc0 == rc1 == brm.SPG_ERR_CAPACITY and req0 == req1 > 1 << 20
        rc0, req0, ref, _ = run(h, p2, req1, noalloc=False)
        rc1, req1, outs, _ = run(h, p2, req1, noalloc=True)
        assert rc0 == rc1 == brm.SPG_OK and req0 == req1
        same_bits(to_host(outs[0]), to_host(ref[0]))
        assert_matches_oracle(outs[0], oracle.spgemm(A, A), oracle.brmerge(A, A))
    finally:
        h.close()


def test_noalloc_symbol_exported():
    assert hasattr(brm.library(), "spgemm_batched_noalloc")
    assert isinstance(brm.library().spgemm_batched_noalloc, ctypes._CFuncPtr)


def test_noalloc_stage_after_overflow_reads_no_stale_arena():
    """The allocation-free call on a chained batch whose arena still holds
    an earlier batch's row pointers where stage 1's C would go."""
    h = brm.Handle(0)
    try:
        first = galerkin_batch([10, 9], 4)[1]
        p1 = brm.Handle.galerkin_problems(first)
        size = 1 << 14
        for _ in range(3):
            rc, req, _, _ = run(h, p1, size, noalloc=True)
            if rc == brm.SPG_OK:
                break
            size = req
        assert rc == brm.SPG_OK
        arena = torch.empty(size, dtype=torch.uint8, device="cuda")
        rc, req, _ = h.batched(p1, arena, noalloc=True)
        assert rc == brm.SPG_OK
        inp, second = galerkin_batch([12, 11], 5)
        p2 = brm.Handle.galerkin_problems(second)
        rc, req, outs = h.batched(p2, arena, noalloc=True)
        torch.cuda.synchronize()
        assert rc == brm.SPG_ERR_CAPACITY and req > size
        check_batch(h, inp, second, 1 << 24)
    finally:
        h.close()
