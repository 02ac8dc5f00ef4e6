"""GPU checks of the batched path: Galerkin triple products P^T (A P) in one
graph-captured call, bitwise equal to separate calls and to the Kronecker
closed forms; arena capacity errors; graph replays interleaved with eager
work; generic problems with mixed row-pointer widths."""
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


@pytest.fixture()
def handle():
    h = brm.Handle(0)
    yield h
    h.close()


def galerkin_inputs(edges):
    return [(n, synth.stencil_3d_27pt(n), synth.aggregation_p(n), synth.aggregation_pt(n)) for n in edges]


def test_galerkin_small_matches_separate_calls_and_closed_form(handle):
    inp = galerkin_inputs([4, 5, 6, 7, 9, 4])
    triples = [(dev(A), dev(P), dev(Pt)) for _, A, P, Pt in inp]
    G, AP, arena = handle.galerkin(triples)
    torch.cuda.synchronize()
    for (n, A, P, Pt), (dA, dP, dPt), g, ap in zip(inp, triples, G, AP):
        ref_ap = oracle.spgemm(A, P)
        apc = synth.CSR(A.rows, P.cols, ref_ap.rpt, ref_ap.col, ref_ap.val)
        ref_g = oracle.spgemm(Pt, apc)
        same_bits(to_host(ap), (ref_ap.rpt, ref_ap.col, ref_ap.val))  # integer values: exact
        same_bits(to_host(g), (ref_g.rpt, ref_g.col, ref_g.val))
        m = (n + 1) // 2
        assert g.nnz == (3 * m - 2) ** 3
        assert ap.nnz == ((2 * n - 2) ** 3 if n % 2 == 0 else (2 * n - 1) ** 3)
        sep_ap = handle.spgemm(dA, dP)
        sep_g = handle.spgemm(dPt, sep_ap)
        same_bits(to_host(ap), to_host(sep_ap))
        same_bits(to_host(g), to_host(sep_g))


def test_generic_problems_mixed_widths(handle):
    rng = np.random.default_rng(4)
    probs, host = [], []
    for i in range(9):
        M, K, N = (int(x) for x in rng.integers(1, 200, 3))
        A = synth.random_csr(M, K, 0.05, 100 + i, empty_row_frac=0.1)
        B = synth.random_csr(K, N, 0.05, 200 + i)
        host.append((A, B))
    # stage 0: int32 A and B for problems 0-4; int64 for 5-8 would need its own
    # call (one width per stage), so use a second call for them
    for chunk, kw in ((host[:5], {}), (host[5:], {"rpt_dtype": torch.int64})):
        dp = [(dev(A, **kw), dev(B, **kw)) for A, B in chunk]
        arena = torch.empty(1 << 22, dtype=torch.uint8, device="cuda")
        rc, req, outs = handle.batched(dp, arena)
        assert rc == brm.SPG_OK
        for (A, B), (dA, dB), C in zip(chunk, dp, outs):
            same_bits(to_host(C), to_host(handle.spgemm(dA, dB)))
            assert_matches_oracle(C, oracle.spgemm(A, B), oracle.brmerge(A, B))


def test_arena_capacity(handle):
    inp = galerkin_inputs([6, 8])
    triples = [(dev(A), dev(P), dev(Pt)) for _, A, P, Pt in inp]
    probs = [(A, P) for A, P, _ in triples] + [(Pt, i) for i, (_, _, Pt) in enumerate(triples)]
    small = torch.empty(64 * 1024, dtype=torch.uint8, device="cuda")
    rc, req, outs = handle.batched(probs, small)
    assert rc == brm.SPG_ERR_CAPACITY and outs is None and req > small.numel()
    arena = torch.empty(req, dtype=torch.uint8, device="cuda")
    rc, req2, outs = handle.batched(probs, arena)
    assert rc == brm.SPG_OK and req2 == req


def test_stage_after_overflow_reads_no_stale_arena(handle):
    """A chained stage after a stage that overflowed computes nothing: here
    the arena still holds an earlier batch's row pointers where the
    overflowed stage's C would have gone, and the call must report the
    capacity error (then succeed once the arena is large enough) without
    reading them as its B."""
    first = galerkin_inputs([10, 9])
    t1 = [(dev(A), dev(P), dev(Pt)) for _, A, P, Pt in first]
    p1 = [(A, P) for A, P, _ in t1] + [(Pt, i) for i, (_, _, Pt) in enumerate(t1)]
    size = 1 << 14
    for _ in range(3):  # an arena of exactly the size the first batch needs
        arena = torch.empty(size, dtype=torch.uint8, device="cuda")
        rc, req, _ = handle.batched(p1, arena)
        if rc == brm.SPG_OK:
            break
        size = req
    assert rc == brm.SPG_OK and req == size
    torch.cuda.synchronize()
    second = galerkin_inputs([12, 11])
    t2 = [(dev(A), dev(P), dev(Pt)) for _, A, P, Pt in second]
    probs = [(A, P) for A, P, _ in t2] + [(Pt, i) for i, (_, _, Pt) in enumerate(t2)]
    rc, req, outs = handle.batched(probs, arena)
    assert rc == brm.SPG_ERR_CAPACITY and req > size
    for _ in range(3):
        arena = torch.empty(req, dtype=torch.uint8, device="cuda")
        rc, req, outs = handle.batched(probs, arena)
        if rc == brm.SPG_OK:
            break
    assert rc == brm.SPG_OK
    for (n, A, P, Pt), g in zip(second, outs[2:]):
        ref_ap = oracle.spgemm(A, P)
        apc = synth.CSR(A.rows, P.cols, ref_ap.rpt, ref_ap.col, ref_ap.val)
        ref_g = oracle.spgemm(Pt, apc)
        same_bits(to_host(g), (ref_g.rpt, ref_g.col, ref_g.val))


def test_graph_replays_with_eager_work_between(handle):
    inp = galerkin_inputs([5, 8, 6])
    triples = [(dev(A), dev(P), dev(Pt)) for _, A, P, Pt in inp]
    G0, AP0, arena = handle.galerkin(triples)
    ref = [to_host(g) for g in G0]
    caps = handle.stat(brm.STAT_GRAPH_CAPTURES)
    other = dev(synth.erdos_renyi_rows(5000, 8, 3))
    for it in range(4):
        eager = handle.spgemm(other, other)  # eager work on the same handle and stream
        x = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        G, AP, arena = handle.galerkin(triples, arena)
        torch.cuda.synchronize()
        for g, r in zip(G, ref):
            same_bits(to_host(g), r)
        assert eager.nnz > 0 and torch.isfinite(x)
    # the first call launched the batch directly, the next one captured it
    assert handle.stat(brm.STAT_BATCHED_DIRECT) >= 1
    assert handle.stat(brm.STAT_GRAPH_CAPTURES) == caps + 1
    assert handle.stat(brm.STAT_GRAPH_LAUNCHES) >= 3


def run_until_fits(handle, problems, size, noalloc=False):
    """Calls the batched product with growing arenas (each failed call
    reports the need of the stages up to the first that did not fit)."""
    for _ in range(4):
        arena = torch.full((size,), 0x5A, dtype=torch.uint8, device="cuda")
        rc, req, outs = handle.batched(problems, arena, noalloc=noalloc)
        torch.cuda.synchronize()
        if rc == brm.SPG_OK:
            return outs, arena, req
        assert rc == brm.SPG_ERR_CAPACITY and req > size
        size = req
    raise AssertionError("arena sizing did not converge")


def host_csr(C):
    rpt, col, val = to_host(C)
    return synth.CSR(C.rows, C.cols, rpt, col, val)


@pytest.mark.parametrize("noalloc", [False, True])
def test_heavy_rows_in_a_batch(handle, noalloc):
    # rows beyond 4096 products (R-MAT squares) beside light problems: the
    # heavy rows take the bitmap count and the spill merge with their spill
    # buffers in the arena; every output bitwise equal to Algorithm 1's model
    print(f"case: batch with heavy rows, noalloc={noalloc}", flush=True)
    mats = [synth.rmat(12, 16, 5), synth.erdos_renyi_rows(3000, 8, 7), synth.rmat(11, 16, 9),
            synth.laplacian_2d_5pt(20)]
    devs = [dev(M) for M in mats]
    outs, arena, req = run_until_fits(handle, [(d, d) for d in devs], 1 << 16, noalloc=noalloc)
    assert handle.stat(brm.STAT_DEVICE_ERR) == 0
    assert handle.stat(brm.STAT_CLASS_ROWS0 + 6) > 0  # heavy rows in the stage
    for M, C in zip(mats, outs):
        assert_matches_oracle(C, oracle.spgemm(M, M), oracle.brmerge(M, M))


@pytest.mark.parametrize("noalloc", [False, True])
def test_heavy_rows_in_both_stages_of_a_chain(handle, noalloc):
    # stage 1: C0 = A A with heavy rows; stage 2: A C0 (B is stage 1's
    # output in the arena, 64-bit row pointers), heavier still
    print(f"case: chained heavy stages, R-MAT scale 10, noalloc={noalloc}", flush=True)
    A = synth.rmat(10, 16, 6)
    dA = dev(A)
    outs, arena, req = run_until_fits(handle, [(dA, dA), (dA, 0)], 1 << 16, noalloc=noalloc)
    assert handle.stat(brm.STAT_DEVICE_ERR) == 0
    assert handle.stat(brm.STAT_CLASS_ROWS0 + 6) > 0
    C0 = host_csr(outs[0])
    assert_matches_oracle(outs[0], oracle.spgemm(A, A), oracle.brmerge(A, A))
    assert_matches_oracle(outs[1], oracle.spgemm(A, C0), oracle.brmerge(A, C0))


@pytest.mark.parametrize("noalloc", [False, True])
def test_every_row_through_the_heavy_kernels(handle, noalloc):
    # forced routing: every non-empty row of both Galerkin stages takes the
    # heavy kernels (one list per row in stage 1, eight in stage 2)
    handle.set_option(brm.OPT_FORCE_CLASS, 6)
    inp = galerkin_inputs([4, 5, 6, 7])
    triples = [(dev(A), dev(P), dev(Pt)) for _, A, P, Pt in inp]
    probs = brm.Handle.galerkin_problems(triples)
    outs, arena, req = run_until_fits(handle, probs, 1 << 16, noalloc=noalloc)
    assert handle.stat(brm.STAT_DEVICE_ERR) == 0
    n = len(inp)
    for (m, A, P, Pt), ap, g in zip(inp, outs[:n], outs[n:]):
        ref_ap = oracle.spgemm(A, P)
        apc = synth.CSR(A.rows, P.cols, ref_ap.rpt, ref_ap.col, ref_ap.val)
        same_bits(to_host(ap), (ref_ap.rpt, ref_ap.col, ref_ap.val))  # integer values: exact
        ref_g = oracle.spgemm(Pt, apc)
        same_bits(to_host(g), (ref_g.rpt, ref_g.col, ref_g.val))


@pytest.mark.parametrize("noalloc", [False, True])
def test_heavy_spill_counts_towards_required_bytes(handle, noalloc):
    # the reported need includes the spill space: with it the call fits, one
    # byte less fails and reports the same need
    A = synth.rmat(11, 16, 9)
    dA = dev(A)
    probs = [(dA, dA)]
    outs, arena, req = run_until_fits(handle, probs, 1 << 16, noalloc=noalloc)
    ref = to_host(outs[0])
    arena = torch.empty(req, dtype=torch.uint8, device="cuda")
    rc, req2, outs = handle.batched(probs, arena, noalloc=noalloc)
    torch.cuda.synchronize()
    assert rc == brm.SPG_OK and req2 == req
    same_bits(to_host(outs[0]), ref)
    c = outs[0]
    c_end = c.val.data_ptr() + 8 * c.nnz - arena.data_ptr()
    assert req > c_end  # the spill space lies beyond C
    arena = torch.empty(req - 1, dtype=torch.uint8, device="cuda")
    rc, req3, outs = handle.batched(probs, arena, noalloc=noalloc)
    torch.cuda.synchronize()
    assert rc == brm.SPG_ERR_CAPACITY and req3 == req and outs is None


def test_row_with_2_31_products_fails_the_batch(handle):
    # one row of 2^20 entries, all in column 0, over a B row of 2049
    # entries: 2^31 + 2^20 products.  The row goes to no kernel and the
    # batch fails with required_bytes = -1 (validation off: the repeated
    # column is the point of the input)
    handle.set_option(brm.OPT_VALIDATE, 0)
    K, blen = 1 << 20, 2049
    A = brm.DeviceCSR(1, 1, torch.tensor([0, K], dtype=torch.int32, device="cuda"),
                      torch.zeros(K, dtype=torch.int32, device="cuda"),
                      torch.ones(K, dtype=torch.float64, device="cuda"))
    B = brm.DeviceCSR(1, blen, torch.tensor([0, blen], dtype=torch.int32, device="cuda"),
                      torch.arange(blen, dtype=torch.int32, device="cuda"),
                      torch.ones(blen, dtype=torch.float64, device="cuda"))
    arena = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    rc, req, outs = handle.batched([(A, B)], arena)
    torch.cuda.synchronize()
    assert rc == brm.SPG_ERR_CAPACITY and req == -1 and outs is None
    assert b"2^31" in brm.library().spg_last_error(handle._h)
    # the handle serves a batch that fits afterwards
    inp = galerkin_inputs([5, 4])
    triples = [(dev(A_), dev(P), dev(Pt)) for _, A_, P, Pt in inp]
    G, _, _ = handle.galerkin(triples)
    for (n, A_, P, Pt), g in zip(inp, G):
        assert g.nnz == (3 * ((n + 1) // 2) - 2) ** 3


def kernel_choice_inputs():
    rng = np.random.default_rng(9)
    host = []
    for i in range(6):
        M, K, N = (int(x) for x in rng.integers(50, 400, 3))
        host.append((synth.random_csr(M, K, 0.04, 300 + i, empty_row_frac=0.1),
                     synth.random_csr(K, N, 0.06, 400 + i)))
    host.append((synth.stencil_3d_27pt(9), synth.stencil_3d_27pt(9)))  # rows of 27 lists of 27
    host.append((synth.laplacian_2d_5pt(20), synth.laplacian_2d_5pt(20)))
    return host


def outputs_in_mode(handle, problems, mode, noalloc=False):
    handle.set_option(brm.OPT_BATCH_ALLOC, mode)
    try:
        outs, arena, req = run_until_fits(handle, problems, 1 << 16, noalloc=noalloc)
        assert handle.stat(brm.STAT_DEVICE_ERR) == 0
        return [to_host(C) for C in outs], req
    finally:
        handle.set_option(brm.OPT_BATCH_ALLOC, brm.BATCH_PRECISE)


@pytest.mark.parametrize("noalloc", [False, True])
def test_upper_bound_stages_match_precise(handle, noalloc):
    # upper-bound slots (numeric into slots, then compaction) against the
    # symbolic pass: Galerkin chains, short rows of every light class, and a
    # chain with heavy rows in both stages -- the same bits
    print(f"case: batched upper-bound slots, noalloc={noalloc}", flush=True)
    inp = galerkin_inputs([4, 5, 6, 7, 9])
    gal = brm.Handle.galerkin_problems([(dev(A), dev(P), dev(Pt)) for _, A, P, Pt in inp])
    host = kernel_choice_inputs()
    light = brm.BatchedProblems([(dev(A), dev(B)) for A, B in host])
    R = synth.rmat(10, 16, 6)
    dR = dev(R)
    heavy = brm.BatchedProblems([(dR, dR), (dR, 0)])
    for name, probs in (("galerkin", gal), ("light", light), ("heavy chain", heavy)):
        x, req_p = outputs_in_mode(handle, probs, brm.BATCH_PRECISE, noalloc)
        y, req_u = outputs_in_mode(handle, probs, brm.BATCH_UPPER, noalloc)
        print(f"  {name}: arena {req_p} (precise), {req_u} (upper)", flush=True)
        assert req_u > req_p
        for a, b in zip(x, y):
            same_bits(a, b)
        if name == "light":
            for (A, B), c in zip(host, y):
                ref, model = oracle.spgemm(A, B), oracle.brmerge(A, B)
                assert np.array_equal(c[0], ref.rpt) and np.array_equal(c[1], ref.col)
                assert np.array_equal(c[2].view(np.int64), model.val.view(np.int64))


@pytest.mark.parametrize("cls", [2, 3, 4, 5, 6, 7])
def test_upper_bound_slots_in_every_class(handle, cls):
    # every row forced into one class: its numeric kernel writes into the
    # slots and records the rows' lengths
    host = kernel_choice_inputs()[:6]
    probs = brm.BatchedProblems([(dev(A), dev(B)) for A, B in host])
    handle.set_option(brm.OPT_FORCE_CLASS, cls)
    x, _ = outputs_in_mode(handle, probs, brm.BATCH_PRECISE)
    y, _ = outputs_in_mode(handle, probs, brm.BATCH_UPPER)
    for (A, B), a, b in zip(host, x, y):
        same_bits(a, b)
        ref = oracle.spgemm(A, B)
        assert np.array_equal(b[0], ref.rpt) and np.array_equal(b[1], ref.col)


def test_upper_bound_required_bytes_and_replays(handle):
    # the reported need covers C at its largest and the slots: it fits, one
    # byte less fails with the same need; graph replays with eager work
    # between give the first replay's bits
    inp = galerkin_inputs([5, 8, 6])
    triples = [(dev(A), dev(P), dev(Pt)) for _, A, P, Pt in inp]
    probs = brm.Handle.galerkin_problems(triples)
    handle.set_option(brm.OPT_BATCH_ALLOC, brm.BATCH_UPPER)
    outs, arena, req = run_until_fits(handle, probs, 1 << 16)
    ref = [to_host(C) for C in outs]
    arena = torch.empty(req - 1, dtype=torch.uint8, device="cuda")
    rc, req2, outs = handle.batched(probs, arena)
    torch.cuda.synchronize()
    assert rc == brm.SPG_ERR_CAPACITY and req2 == req and outs is None
    arena = torch.empty(req, dtype=torch.uint8, device="cuda")
    caps = handle.stat(brm.STAT_GRAPH_CAPTURES)
    other = dev(synth.erdos_renyi_rows(5000, 8, 3))
    for it in range(4):
        eager = handle.spgemm(other, other)
        torch.cuda.synchronize()
        rc, req3, outs = handle.batched(probs, arena)
        torch.cuda.synchronize()
        assert rc == brm.SPG_OK and req3 == req
        for C, r in zip(outs, ref):
            same_bits(to_host(C), r)
        assert eager.nnz > 0
    assert handle.stat(brm.STAT_GRAPH_CAPTURES) == caps + 1
    for (n, A, P, Pt), g in zip(inp, outs[len(inp):]):
        assert g.nnz == (3 * ((n + 1) // 2) - 2) ** 3


def test_config4_full_batch(handle):
    print("case: 48 Galerkin products, cube edges U{16..64}, seed 4", flush=True)
    inp = synth.amg_batch(48, 4)
    triples = [(dev(A), dev(P), dev(Pt)) for _, A, P, Pt in inp]
    G, AP, arena = handle.galerkin(triples)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    for (n, A, P, Pt), g, ap in zip(inp, G, AP):
        m = (n + 1) // 2
        assert g.nnz == (3 * m - 2) ** 3
        assert ap.nnz == ((2 * n - 2) ** 3 if n % 2 == 0 else (2 * n - 1) ** 3)
    # every problem against the oracle, bitwise (all values are integers)
    for i in range(48):
        n, A, P, Pt = inp[i]
        ref_ap = oracle.spgemm(A, P)
        same_bits(to_host(AP[i]), (ref_ap.rpt, ref_ap.col, ref_ap.val))
        ref_g = oracle.spgemm(Pt, synth.CSR(A.rows, P.cols, ref_ap.rpt, ref_ap.col, ref_ap.val))
        same_bits(to_host(G[i]), (ref_g.rpt, ref_g.col, ref_g.val))


def test_kernel_choices_agree_in_batches(handle):
    # short rows under lane windows (one and several registers per lane) and
    # in LDS give the same bits; the window kernels take every row's arrays
    # from its own problem
    host = kernel_choice_inputs()
    dp = [(dev(A), dev(B)) for A, B in host]
    outs, classes = {}, {}
    try:
        for g in (1, 0):
            handle.set_option(brm.OPT_GROUP_ROWS, g)
            arena = torch.empty(1 << 24, dtype=torch.uint8, device="cuda")
            rc, req, res = handle.batched(dp, arena)
            assert rc == brm.SPG_OK
            outs[g] = [to_host(C) for C in res]
            # the last stage's classes: the rows of every problem together
            classes[g] = handle.class_rows()
            print(f"case: batched kernel choices, group rows {g}: {classes[g]}", flush=True)
    finally:
        handle.set_option(brm.OPT_GROUP_ROWS, 1)
    assert classes[1]["multi"] > 0 and classes[1]["wave_small"] > 0
    assert classes[0]["multi"] == 0
    for (A, B), x, y in zip(host, outs[1], outs[0]):
        same_bits(x, y)
        ref, model = oracle.spgemm(A, B), oracle.brmerge(A, B)
        assert np.array_equal(x[0], ref.rpt) and np.array_equal(x[1], ref.col)
        assert np.array_equal(x[2].view(np.int64), model.val.view(np.int64))


def test_amg_hierarchy(handle):
    # coarse operators of several aggregation hierarchies, level by level in
    # batched calls; every level is again a 27-point pattern on the coarse
    # grid, and the integer values make the oracle's sums exact
    edges = [9, 16, 12, 5]
    As = [dev(synth.stencil_3d_27pt(n)) for n in edges]
    levels_h = [synth.amg_levels(n) for n in edges]
    levels = [[(dev(P), dev(Pt)) for _, P, Pt in lv] for lv in levels_h]
    out = handle.amg_hierarchy(As, levels)
    torch.cuda.synchronize()
    for n, lv, got in zip(edges, levels_h, out):
        print(f"case: AMG hierarchy from edge {n}: {len(lv)} levels", flush=True)
        A = synth.stencil_3d_27pt(n)
        assert len(got) == len(lv)
        for (e, P, Pt), g in zip(lv, got):
            ref_ap = oracle.spgemm(A, P)
            ap = synth.CSR(A.rows, P.cols, ref_ap.rpt, ref_ap.col, ref_ap.val)
            ref = oracle.spgemm(Pt, ap)
            same_bits(to_host(g), (ref.rpt, ref.col, ref.val))
            m = (e + 1) // 2
            assert g.rows == m ** 3 and g.nnz == (3 * m - 2) ** 3
            A = synth.CSR(g.rows, g.cols, ref.rpt, ref.col, ref.val)


def test_autotuner_search_and_cache(tmp_path):
    # the coordinate search times every candidate on the caller's batch,
    # checks that none changes the output, keeps the best on the handle, and
    # answers from its cache the second time
    from paper_2206_06611_amd import autotune
    inp = galerkin_inputs([6, 8, 5])
    triples = [(dev(A), dev(P), dev(Pt)) for _, A, P, Pt in inp]
    cache = str(tmp_path / "tune.json")
    h = brm.Handle(0)
    try:
        res = autotune.tune_galerkin(h, triples, reps=1, cache=cache)
        assert not res["cached"] and res["tried"] >= 10
        for k, v in res["options"].items():
            assert v in autotune.SPACE[k]
            assert h.get_option(autotune.KEYS[k]) == v
        G, _, _ = h.galerkin(triples)
        for (n, A, P, Pt), g in zip(inp, G):
            ref_ap = oracle.spgemm(A, P)
            ref_g = oracle.spgemm(Pt, synth.CSR(A.rows, P.cols, ref_ap.rpt, ref_ap.col, ref_ap.val))
            same_bits(to_host(g), (ref_g.rpt, ref_g.col, ref_g.val))
    finally:
        h.close()
    h2 = brm.Handle(0)
    try:
        res2 = autotune.tune_galerkin(h2, triples, reps=1, cache=cache)
        assert res2["cached"] and res2["options"] == res["options"]
    finally:
        h2.close()


def operand_only_cases():
    """(name, problems without flags, index set of the stage-1 problems):
    light chains (stage 2 has rows of one list: the copy class), Galerkin
    chains, and a chain with heavy rows in both stages."""
    rng = np.random.default_rng(12)
    host = kernel_choice_inputs()[:6]
    first = [(dev(A), dev(B)) for A, B in host]
    second = []
    for i, (A, B) in enumerate(host):
        X = synth.random_csr(60, A.rows, 0.05, 500 + i, empty_row_frac=0.1)
        second.append((dev(X), i))
        second.append((dev(synth.permutation(rng.permutation(A.rows))), i))
    light = (first, second)
    inp = galerkin_inputs([4, 5, 6, 7, 9])
    gal = ([(dev(A), dev(P)) for _, A, P, _ in inp], [(dev(Pt), i) for i, (_, _, _, Pt) in enumerate(inp)])
    R = synth.rmat(10, 16, 6)
    dR = dev(R)
    heavy = ([(dR, dR)], [(dR, 0)])
    return [("light", light), ("galerkin", gal), ("heavy chain", heavy)]


def flagged(stages, flags):
    first, second = stages
    return brm.BatchedProblems([(A, B, flags) for A, B in first] + list(second))


@pytest.mark.parametrize("noalloc", [False, True])
def test_operand_only_stage_keeps_its_slots(handle, noalloc):
    # stage-1 outputs marked operand-only stay in their upper-bound slots and
    # stage 2 reads them from there (rows described by start and end): stage
    # 2's outputs are bitwise those of the materialized run; stage 1 reports
    # nnz = -2 and returns nothing
    handle.set_option(brm.OPT_BATCH_ALLOC, brm.BATCH_UPPER)
    for name, stages in operand_only_cases():
        print(f"case: operand-only stage 1, {name}, noalloc={noalloc}", flush=True)
        n1 = len(stages[0])
        ref, _, req_ref = run_until_fits(handle, flagged(stages, 0), 1 << 16, noalloc=noalloc)
        ref = [to_host(C) for C in ref]
        outs, arena, req = run_until_fits(handle, flagged(stages, brm.PROBLEM_OPERAND_ONLY), 1 << 16,
                                          noalloc=noalloc)
        assert handle.stat(brm.STAT_DEVICE_ERR) == 0
        assert all(o is None for o in outs[:n1])
        for a, b in zip(ref[n1:], outs[n1:]):
            same_bits(a, to_host(b))
        print(f"  arena {req_ref} (materialized), {req} (kept)", flush=True)


def test_operand_only_ignored_unless_whole_stage_and_upper(handle):
    # precise sizes, or a stage where one problem is not an operand only:
    # every C is materialized as usual
    name, stages = operand_only_cases()[0]
    first, second = stages
    for mode in (brm.BATCH_PRECISE, brm.BATCH_UPPER):
        handle.set_option(brm.OPT_BATCH_ALLOC, mode)
        ref, _, _ = run_until_fits(handle, flagged(stages, 0), 1 << 16)
        ref = [to_host(C) for C in ref]
        mixed = [(A, B, brm.PROBLEM_OPERAND_ONLY if i else 0) for i, (A, B) in enumerate(first)]
        cases = [brm.BatchedProblems(mixed + list(second))]
        if mode == brm.BATCH_PRECISE:
            cases.append(flagged(stages, brm.PROBLEM_OPERAND_ONLY))
        for probs in cases:
            outs, _, _ = run_until_fits(handle, probs, 1 << 16)
            assert all(o is not None for o in outs)
            for a, b in zip(ref, outs):
                same_bits(a, to_host(b))
    handle.set_option(brm.OPT_BATCH_ALLOC, brm.BATCH_PRECISE)


def test_operand_only_galerkin_graph_replays(handle):
    # the Galerkin call with A P kept in slots: direct launch, capture, replays
    # with eager work between -- every G bitwise the materialized call's
    inp = galerkin_inputs([5, 8, 6, 7])
    triples = [(dev(A), dev(P), dev(Pt)) for _, A, P, Pt in inp]
    handle.set_option(brm.OPT_BATCH_ALLOC, brm.BATCH_UPPER)
    G0, AP0, _ = handle.galerkin(triples)
    ref = [to_host(g) for g in G0]
    probs = brm.Handle.galerkin_problems(triples, ap_operand_only=True)
    arena = None
    caps = handle.stat(brm.STAT_GRAPH_CAPTURES)
    for k in range(4):
        G, AP, arena = handle.galerkin(triples, arena, problems=probs)
        torch.cuda.synchronize()
        assert all(a is None for a in AP)
        for r, g in zip(ref, G):
            same_bits(r, to_host(g))
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
    assert handle.stat(brm.STAT_GRAPH_CAPTURES) >= caps + 1 and handle.stat(brm.STAT_GRAPH_LAUNCHES) >= 2
    handle.set_option(brm.OPT_BATCH_ALLOC, brm.BATCH_PRECISE)
