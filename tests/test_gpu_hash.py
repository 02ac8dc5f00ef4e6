"""GPU checks of the hash-accumulator comparator (rows added into an LDS hash
table, then placed by column rank): structure bit-exact and values within
1e-12 * sum|products| of the oracle, for every light class; rows beyond
4096 products keep the BRMerge path.  Its sums are not the merge tree's, so
no bitwise comparison with the tree is made."""
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


CASES = {
    "random": lambda: (synth.random_csr(300, 250, 0.03, 51, empty_row_frac=0.1),
                       synth.random_csr(250, 400, 0.04, 52, empty_row_frac=0.1)),
    "er_2e13": lambda: (synth.erdos_renyi_rows(1 << 13, 8, 53),) * 2,
    "stencil_10": lambda: (synth.stencil_3d_27pt(10),) * 2,
    "laplace_40": lambda: (synth.laplacian_2d_5pt(40),) * 2,
    "rmat_12": lambda: (synth.rmat(12, 16, 54),) * 2,
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("group_rows", [1, 0])
def test_hash_accumulator_matches_oracle(handle, name, group_rows):
    print(f"case: hash accumulator, {name}, group rows {group_rows}", flush=True)
    A, B = CASES[name]()
    dA = brm.DeviceCSR.from_host(A)
    dB = dA if B is A else brm.DeviceCSR.from_host(B)
    handle.set_option(brm.OPT_GROUP_ROWS, group_rows)
    base = to_host(handle.spgemm(dA, dB))
    handle.set_option(brm.OPT_ACCUMULATOR, brm.ACC_HASH)
    try:
        C = handle.spgemm(dA, dB)
        torch.cuda.synchronize()
        assert handle.stat(brm.STAT_DEVICE_ERR) == 0
        assert_matches_oracle(C, oracle.spgemm(A, B))
        got = to_host(C)
        assert np.array_equal(got[0], base[0]) and np.array_equal(got[1], base[1])
    finally:
        handle.set_option(brm.OPT_ACCUMULATOR, brm.ACC_BRMERGE)
        handle.set_option(brm.OPT_GROUP_ROWS, 1)


@pytest.mark.parametrize("force", [2, 3, 4, 5, 7])
def test_hash_accumulator_every_class(handle, force):
    # the rows of the mixed-size case routed to one class at a time
    A, B = CASES["random"]()
    w = np.maximum(oracle.row_nprod(A, B), np.diff(A.rpt))
    d = A.to_dense()
    pat = d != 0
    pat[w > 64] = False
    A = synth.from_dense(np.where(pat, d, 0.0), pat)
    if force == 7:
        A, B = synth.stencil_3d_27pt(8), synth.stencil_3d_27pt(8)
    dA, dB = brm.DeviceCSR.from_host(A), brm.DeviceCSR.from_host(B)
    handle.set_option(brm.OPT_FORCE_CLASS, force)
    handle.set_option(brm.OPT_ACCUMULATOR, brm.ACC_HASH)
    try:
        C = handle.spgemm(dA, dB)
        torch.cuda.synchronize()
        assert handle.stat(brm.STAT_CLASS_ROWS0 + force) > 0
        assert handle.stat(brm.STAT_DEVICE_ERR) == 0
        assert_matches_oracle(C, oracle.spgemm(A, B))
    finally:
        handle.set_option(brm.OPT_ACCUMULATOR, brm.ACC_BRMERGE)
        handle.set_option(brm.OPT_FORCE_CLASS, -1)


def test_accumulator_option_values(handle):
    assert handle.get_option(brm.OPT_ACCUMULATOR) == brm.ACC_BRMERGE
    with pytest.raises(brm.SpgError) as e:
        handle.set_option(brm.OPT_ACCUMULATOR, 2)
    assert e.value.code == brm.SPG_ERR_ARG
