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


def stored_order_row(lists, avals, bvals):
    """The symbolic and numeric passes of a wave-small row with a stored
    order, as the window kernels lay them out: list p's entry o sits in lane
    p * W0 + o (W0 the next power of two of the longest list, T = W0 times
    the next power of two of the list count, at most 64 lanes).  The
    symbolic pass sorts (column << 6 | lane) keys and keeps, for every
    position t < T, the source lane (bits 0-5) and whether position t + 1
    holds the same column (bit 6), 0xFF for an empty position, and the
    distinct columns in order.  The numeric pass moves the lanes' products
    into that order and adds by levels: a run's first position is live with
    a previous position that does not repeat its column; two positions of
    a column meet at the level of the highest bit of their lists' xor."""
    L = len(lists)
    W0 = 1
    while W0 < max(len(c) for c in lists):
        W0 *= 2
    nl = 1
    while nl < L:
        nl *= 2
    T = W0 * nl
    assert T <= 64
    lsw = W0.bit_length() - 1
    EMPTY = (1 << 32) - 64
    keys, prod = [], {}
    for p, cols in enumerate(lists):
        for o, c in enumerate(cols):
            lane = p * W0 + o
            keys.append((int(c) << 6) | lane)
            prod[lane] = avals[p] * bvals[p][o]
    keys.sort()
    keys += [EMPTY | t for t in range(len(keys), T)]
    # symbolic pass: the kept bytes and distinct columns
    perm, ucol = [], []
    for t in range(T):
        k = keys[t]
        live = k < EMPTY
        same = live and t + 1 < T and keys[t + 1] < EMPTY and (keys[t + 1] >> 6) == (k >> 6)
        perm.append(((k & 63) | (64 if same else 0)) if live else 0xFF)
        head = live and (t == 0 or keys[t - 1] >= EMPTY or (keys[t - 1] >> 6) != (k >> 6))
        if head:
            ucol.append(k >> 6)
    # numeric pass: only the bytes, the distinct columns and the products
    live = [q != 0xFF for q in perm]
    same = [live[t] and bool(perm[t] & 64) for t in range(T)]
    src = [perm[t] & 63 for t in range(T)]
    v = [prod[src[t]] if live[t] else 0.0 for t in range(T)]
    head = [live[t] and (t == 0 or not same[t - 1]) for t in range(T)]
    li = [(src[t] & (T - 1)) >> lsw for t in range(T)]
    INF = 1 << 30
    lvl = [lca_level(li[t], li[t + 1]) if same[t] else INF for t in range(T)]
    for r in range(1, (T.bit_length() - 1) - lsw + 1):
        nv = list(v)
        for j in range(T):
            if not (live[j] and (head[j] or (j > 0 and lvl[j - 1] >= r))):
                continue
            e = j
            while lvl[e] < r:
                e += 1
            if lvl[e] == r:
                nv[j] = v[j] + v[e + 1]
        v = nv
    out = [v[t] for t in range(T) if head[t]]
    assert len(out) == len(ucol)
    return list(zip(ucol, out))


@pytest.mark.parametrize("seed", range(4))
def test_stored_order_bytes_give_algorithm_1_sums(seed):
    # rows of at most 64 products in lane windows, many repeated columns;
    # every row bitwise the oracle's run of Algorithm 1
    rng = np.random.default_rng(40 + seed)
    K, N = 300, int(rng.choice([5, 12, 60]))
    B = synth.random_csr(K, N, float(rng.uniform(0.05, 0.3)), 300 + seed, empty_row_frac=0.1)
    blen = np.diff(B.rpt.astype(np.int64))
    rows = []
    while len(rows) < 150:
        L = int(rng.integers(1, 17))
        lists = np.sort(rng.choice(K, size=L, replace=False))
        W0 = 1 << int(max(1, int(blen[lists].max()))  - 1).bit_length()
        nl = 1 << int(L - 1).bit_length()
        if W0 * nl <= 64 and blen[lists].sum() > 0:
            rows.append(lists)
    rpt = np.zeros(len(rows) + 1, np.int64)
    rpt[1:] = np.cumsum([len(r) for r in rows])
    A = synth.CSR(len(rows), K, rpt.astype(np.int32), np.concatenate(rows).astype(np.int32),
                  rng.uniform(-1, 1, int(rpt[-1])))
    ref = oracle.brmerge(A, B)
    repeats = 0
    for i in range(A.rows):
        lists = [B.col[B.rpt[k]:B.rpt[k + 1]] for k in A.col[A.rpt[i]:A.rpt[i + 1]]]
        bv = [B.val[B.rpt[k]:B.rpt[k + 1]] for k in A.col[A.rpt[i]:A.rpt[i + 1]]]
        got = stored_order_row(lists, A.val[A.rpt[i]:A.rpt[i + 1]], bv)
        exp = list(zip(ref.col[ref.rpt[i]:ref.rpt[i + 1]].tolist(), ref.val[ref.rpt[i]:ref.rpt[i + 1]].tolist()))
        assert [c for c, _ in got] == [c for c, _ in exp], f"row {i}: columns"
        assert all(same_bits(x, y) for (_, x), (_, y) in zip(got, exp)), f"row {i}: values"
        repeats += sum(len(c) for c in lists) - len(exp)
    assert repeats > 0
