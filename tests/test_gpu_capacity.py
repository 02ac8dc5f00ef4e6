"""GPU checks at the capacity boundaries of the kernel classes: rows with
exactly as many products (and lists) as a class holds and one more, the
lane-window limits of the register classes, heavy rows whose aligned list
ranges fill an LDS node exactly or overflow it by one product, and the
column slabs of the heavy rows' bitmap count.  Each case compares the whole
C with the oracle (row pointers and columns bit-exact, values within
1e-12 sum|products|) and bitwise with the CPU run of Algorithm 1's tree."""
import numpy as np
import pytest

import oracle
import synth
from helpers import assert_matches_oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2206_06611_amd as brm  # noqa: E402


def lists_matrix(specs, ncols, seed, col_sampler=None):
    """A and B such that row i of A*B merges lists of the lengths specs[i]
    (in that order): every list is a B row of its own, A's row i takes
    consecutive rows of B.  Columns distinct and sorted within each B row."""
    rng = np.random.default_rng(seed)
    lens = np.array([l for s in specs for l in s], np.int64)
    K = int(lens.size)
    b_rpt = np.zeros(K + 1, np.int64)
    np.cumsum(lens, out=b_rpt[1:])
    cols = []
    for l in lens:
        if col_sampler is not None:
            c = col_sampler(rng, int(l))
        else:
            c = rng.choice(ncols, size=int(l), replace=False)
        cols.append(np.sort(c))
    b_col = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    B = synth.CSR(K, ncols, b_rpt.astype(np.int32), b_col, rng.uniform(-1, 1, b_col.size))
    a_len = np.array([len(s) for s in specs], np.int64)
    a_rpt = np.zeros(len(specs) + 1, np.int64)
    np.cumsum(a_len, out=a_rpt[1:])
    A = synth.CSR(len(specs), K, a_rpt.astype(np.int32), np.arange(K, dtype=np.int32),
                  rng.uniform(-1, 1, K))
    return A, B


def boundary_specs():
    s = []
    for cap in (64, 256, 1024, 4096):
        w = 16 if cap >= 256 else 8
        s.append([cap // (cap // w)] * (cap // w))              # exactly cap products
        s.append([cap // (cap // w)] * (cap // w) + [1])        # cap + 1 products
        s.append([1] * cap)                                      # cap lists of one product
        s.append([1] * (cap + 1))                                # cap + 1 lists
    s += [[2048, 2048], [2048, 2049], [4096], [4097]]           # two halves; single lists
    # lane windows of the register classes
    s += [[4] * 16, [4] * 15 + [5], [3] * 21 + [1], [1] * 64, [2] * 64, [2] * 65,
          [16] * 64, [17] * 64, [16] * 64 + [1], [8] * 8, [8] * 8 + [1]]
    # heavy rows: aligned ranges of 128 lists with 2048 products (a 512-thread
    # node exactly), 2049 (one over), ranges of 256 lists with 4096 / 4097
    # (the 1024-thread node), 2048 and 4096 one-product lists per range, more
    # lists than a node holds
    s += [[16] * 1024, ([16] * 127 + [17]) * 8, ([16] * 255 + [17]) * 4, [1] * 8192,
          [1] * 4097 + [3000], [2049] * 3, [4096] * 2 + [1]]
    return s


@pytest.fixture(scope="module")
def boundary():
    A, B = lists_matrix(boundary_specs(), 8192, 41)
    return A, B, oracle.spgemm(A, B), oracle.brmerge(A, B)


@pytest.fixture()
def handle():
    h = brm.Handle(0)
    h.set_option(brm.OPT_VALIDATE, 1)
    yield h
    h.close()


CONFIGS = {
    "default": {},
    "lds_only": {brm.OPT_GROUP_ROWS: 0},
    "force_wave_small": {brm.OPT_FORCE_CLASS: 2},
    "force_wave": {brm.OPT_FORCE_CLASS: 3},
    "force_group": {brm.OPT_FORCE_CLASS: 4},
    "force_block": {brm.OPT_FORCE_CLASS: 5},
    "force_multi": {brm.OPT_FORCE_CLASS: 7},
    "force_heavy_512": {brm.OPT_FORCE_CLASS: 6, brm.OPT_HEAVY_THREADS: 512},
    "force_heavy_1024": {brm.OPT_FORCE_CLASS: 6, brm.OPT_HEAVY_THREADS: 1024},
    "heavy_512": {brm.OPT_HEAVY_THREADS: 512},
    "heavy_1024": {brm.OPT_HEAVY_THREADS: 1024},
}


@pytest.mark.parametrize("name", sorted(CONFIGS))
def test_class_capacity_boundaries(handle, boundary, name):
    A, B, ref, model = boundary
    print(f"case: capacity boundaries, {name}", flush=True)
    for k, v in CONFIGS[name].items():
        handle.set_option(k, v)
    dA, dB = brm.DeviceCSR.from_host(A), brm.DeviceCSR.from_host(B)
    C = handle.spgemm(dA, dB)
    torch.cuda.synchronize()
    assert handle.stat(brm.STAT_DEVICE_ERR) == 0
    cls = handle.class_rows()
    print("classes", cls, flush=True)
    if name == "default":
        assert all(cls[c] > 0 for c in ("copy", "wave_small", "multi", "wave", "group", "block", "heavy"))
    assert_matches_oracle(C, ref, model)


@pytest.mark.parametrize("threads", [512, 1024])
def test_heavy_bitmap_column_slabs(handle, threads):
    # B has 2^21 + 5 columns: the heavy rows' bitmap count runs over three
    # column slabs of 2^20; rows of 1025 to 3000 lists take several chunks
    # of lists; columns fall in every slab, the last five included
    ncols = (1 << 21) + 5
    rng = np.random.default_rng(43)

    def sampler(r, l):
        c = r.choice(ncols - 5, size=l, replace=False)
        if r.random() < 0.3:
            c[0] = ncols - 1 - r.integers(0, 5)
            c = np.unique(c)
        return c

    specs = [list(rng.integers(1, 9, int(n))) for n in (1025, 1500, 2048, 2049, 3000)]
    specs += [[1] * 1025, [5] * 1200]
    A, B = lists_matrix(specs, ncols, 44, sampler)
    print(f"case: heavy bitmap column slabs, {threads} threads, B {B.rows} x {B.cols}", flush=True)
    handle.set_option(brm.OPT_FORCE_CLASS, 6)
    handle.set_option(brm.OPT_HEAVY_THREADS, threads)
    dA, dB = brm.DeviceCSR.from_host(A), brm.DeviceCSR.from_host(B)
    C = handle.spgemm(dA, dB)
    torch.cuda.synchronize()
    assert handle.stat(brm.STAT_DEVICE_ERR) == 0
    assert handle.class_rows()["heavy"] == A.rows
    assert (B.col >= (1 << 21)).any() and ((B.col >= (1 << 20)) & (B.col < (1 << 21))).any()
    assert_matches_oracle(C, oracle.spgemm(A, B), oracle.brmerge(A, B))
