"""Host model of the batched window kernels' accumulating phase (CPU only).

Those kernels sort a row's products once by (column, lane) -- the lanes of
list p hold its entries, so lanes follow list order -- and then add equal
columns level by level: two products of one column from lists a < b meet in
Algorithm 1's merge tree at the level of the lowest common ancestor of a and
b (node (r, q) covers lists [q 2^r, (q+1) 2^r)), the position of the highest
set bit of a ^ b.  Within a column's run of lanes, the lanes joined by
levels below r hold the column's entries of one node of level r-1; at level
r the first lane of each such run adds the first lane of the next run when
the two meet at level r exactly (left + right).  This file replays that
rule on random rows and checks it bitwise against the oracle's run of
Algorithm 1 (round by round, pairs of consecutive lists, the odd last list
passed up), including empty lists, single lists and lists of several
entries."""
import struct

import numpy as np
import pytest

import oracle
import synth


def lca_level(a: int, b: int) -> int:
    return (a ^ b).bit_length()


def tree_adds_row(cols, vals, list_of):
    """cols, vals, list_of: the row's products in (column, lane) order.
    Returns the (column, value) pairs of the row of C."""
    n = len(cols)
    INF = 1 << 30
    lvl = [INF] * n
    for i in range(n - 1):
        if cols[i] == cols[i + 1]:
            lvl[i] = lca_level(list_of[i], list_of[i + 1])
    head = [i == 0 or cols[i - 1] != cols[i] for i in range(n)]
    v = list(vals)
    levels = max([x for x in lvl if x < INF], default=0)
    for r in range(1, levels + 1):
        nv = list(v)
        for j in range(n):
            if not (head[j] or lvl[j - 1] >= r):
                continue  # not the first lane of its run
            e = j
            while lvl[e] < r:
                e += 1  # the run's last lane
            if lvl[e] == r:
                nv[j] = v[j] + v[e + 1]  # left + right
        v = nv
    return [(cols[i], v[i]) for i in range(n) if head[i]]


def model_product(A, B):
    rows = []
    for i in range(A.rows):
        prods = []
        for p, a in enumerate(range(A.rpt[i], A.rpt[i + 1])):
            k = A.col[a]
            for b in range(B.rpt[k], B.rpt[k + 1]):
                prods.append((int(B.col[b]), p, b - B.rpt[k], A.val[a] * B.val[b]))
        # sort by (column, lane): the lane of list p entry o is p * W + o
        prods.sort(key=lambda x: (x[0], x[1], x[2]))
        rows.append(tree_adds_row([x[0] for x in prods], [x[3] for x in prods], [x[1] for x in prods]))
    return rows


def same_bits(x, y):
    return struct.pack('d', x) == struct.pack('d', y)


@pytest.mark.parametrize("seed", range(6))
def test_lca_levels_give_algorithm_1_sums(seed):
    rng = np.random.default_rng(seed)
    M, K = (int(x) for x in rng.integers(20, 120, size=2))
    N = int(rng.choice([3, 7, 40]))  # few columns: many repeated columns per row
    A = synth.random_csr(M, K, float(rng.uniform(0.05, 0.3)), 100 + seed, empty_row_frac=0.1)
    B = synth.random_csr(K, N, float(rng.uniform(0.1, 0.5)), 200 + seed, empty_row_frac=0.2)
    ref = oracle.brmerge(A, B)
    got = model_product(A, B)
    repeats = 0
    for i in range(M):
        exp = list(zip(ref.col[ref.rpt[i]:ref.rpt[i + 1]].tolist(), ref.val[ref.rpt[i]:ref.rpt[i + 1]].tolist()))
        assert [c for c, _ in got[i]] == [c for c, _ in exp], f"row {i}: columns"
        assert all(same_bits(x, y) for (_, x), (_, y) in zip(got[i], exp)), f"row {i}: values"
        nprod = sum(B.rpt[A.col[a] + 1] - B.rpt[A.col[a]] for a in range(A.rpt[i], A.rpt[i + 1]))
        repeats += nprod - len(exp)
    assert repeats > 0  # the rule was exercised


def test_lca_level_of_lists():
    # lists 0 and 1 meet at level 1, 1 and 2 at level 2, 3 and 4 at level 3
    assert [lca_level(0, 1), lca_level(1, 2), lca_level(3, 4), lca_level(5, 6), lca_level(0, 63)] == [1, 2, 3, 2, 6]


def test_three_lists_group_as_the_tree():
    # one column in lists 0, 1 and 2: the tree adds (v0 + v1) + v2; in
    # lists 0, 2, 3 it adds v0 + (v2 + v3).  Values chosen so that the two
    # groupings round differently.
    a, b, c = 1.0, 1e-16, 1e-16
    assert tree_adds_row([5, 5, 5], [a, b, c], [0, 1, 2]) == [(5, (a + b) + c)]
    assert tree_adds_row([5, 5, 5], [a, b, c], [0, 2, 3]) == [(5, a + (b + c))]
    assert (a + b) + c != a + (b + c)
