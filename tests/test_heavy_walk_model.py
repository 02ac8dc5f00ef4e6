"""Host model of the heavy-row path's index logic, with a bounds assertion
on every global access (CPU only).

The heavy kernel merges one row per workgroup: aligned list ranges (nodes
of Algorithm 1's merge tree) that fit LDS are merged there and written to
one of two spill buffers of nprod entries, a stack of finished nodes
combines two siblings as soon as both exist (a binary counter over the
lists), an unpaired left child is promoted, and two spill nodes are merged
tile by tile into the other buffer or into the region of the right child.
The host cuts the heavy rows into batches whose spill buffers and list
offsets share one pool.  This file replays exactly those decisions -- the
node choice, the action order, the buffer choice, the tile cuts of the
spill merge and the pool layout -- and asserts that every read and write
stays inside its row's buffers, that no write lands on a live node other
than the documented overlap with the right child being consumed, that the
stack and the action guard hold, and that the walk ends with the row.
Node contents are the real column sets of R-MAT rows (small scales), or
their upper bound (every node as long as its products) at larger ones."""
import numpy as np
import pytest

import synth

KMERGE_STEPS = 4
KWIN_PER = 2


class Region:
    def __init__(self, buf, start, length):
        self.buf, self.start, self.length = buf, start, length

    def overlaps(self, buf, lo, hi):
        return buf == self.buf and lo < self.start + self.length and self.start < hi


def merge_tiles(X, Y, T, rx, ry, zcap, same_buffer_as_y):
    """The spill merge of sorted duplicate-free column lists X (left) and Y
    (right) by tiles of at most 2 T entries a side; checks the window reads,
    the steps per thread, the capacity, and (when the output shares Y's
    buffer, starting at rx <= ry) that no write reaches a Y entry that has not
    been read yet.  Returns the merged length."""
    nx, ny = len(X), len(Y)
    win = KWIN_PER * T
    x0 = y0 = out = 0
    tiles = 0
    while x0 < nx or y0 < ny:
        wx, wy = min(nx - x0, win), min(ny - y0, win)
        assert 0 <= wx <= win and 0 <= wy <= win
        cx, cy = wx, wy
        tx, ty = x0 + wx < nx, y0 + wy < ny
        if tx or ty:
            lim = np.iinfo(np.int32).max
            if tx:
                lim = X[x0 + wx - 1]
            if ty and Y[y0 + wy - 1] < lim:
                lim = Y[y0 + wy - 1]
            if not (tx and X[x0 + wx - 1] == lim):
                cx = int(np.searchsorted(X[x0:x0 + wx], lim, side="right"))
            if not (ty and Y[y0 + wy - 1] == lim):
                cy = int(np.searchsorted(Y[y0:y0 + wy], lim, side="right"))
        assert cx + cy >= 1, "a tile must consume an entry"
        assert cx + cy <= KMERGE_STEPS * T, "steps per thread do not cover the tile"
        nx0, ny0 = x0 + cx, y0 + cy
        # the next windows are fetched before this tile writes
        assert nx0 + min(nx - nx0, win) <= nx and ny0 + min(ny - ny0, win) <= ny
        tot = len(np.union1d(X[x0:nx0], Y[y0:ny0]))
        # a column's two entries are never split between tiles
        if nx0 < nx and ny0 > 0:
            assert not (y0 < ny0 and nx0 < nx and X[nx0] == Y[ny0 - 1])
        if ny0 < ny and nx0 > 0:
            assert not (x0 < nx0 and Y[ny0] == X[nx0 - 1])
        assert out + tot <= zcap, "merged row longer than its capacity"
        if same_buffer_as_y:
            # writes end at or before the first Y entry not yet consumed
            assert rx + out + tot <= ry + ny0
        out += tot
        x0, y0 = nx0, ny0
        tiles += 1
    assert out == len(np.union1d(X, Y))
    return out


def heavy_walk(list_cols, lds_cap, T, ccap, exact=True, l_begin=0, l_end=None, writes=None):
    """Replays the walk over one row whose lists have the given column
    arrays (sorted, duplicate-free): the whole row (l_begin = 0, l_end =
    None; its root goes to C), or the aligned subtree [l_begin, l_end) of a
    split row, whose result stays in a spill buffer and is returned as
    (buffer, length, columns).  exact=False models every node as long as its
    products (an upper bound of every length).  `writes` collects the
    (buffer, lo, hi) ranges written to the spill buffers."""
    L = len(list_cols)
    whole = l_end is None
    if whole:
        l_end = L
    lens = np.array([len(c) for c in list_cols], dtype=np.int64)
    leaf = np.zeros(L + 1, dtype=np.int64)
    leaf[1:] = np.cumsum(lens)
    nprod = int(leaf[L])
    assert nprod < 2 ** 31 and L < 2 ** 31  # int32 list offsets
    assert 0 <= l_begin < l_end <= L
    stack = []  # dicts p, h, len, buf, cols
    next_list = l_begin
    guard = 0
    actions = []
    if writes is None:
        writes = []

    def content(a, b):
        if not exact:
            return None
        if b - a == 1:
            return list_cols[a]
        return np.unique(np.concatenate(list_cols[a:b])) if b > a else np.zeros(0, np.int64)

    def live(exclude=()):
        out = []
        for k, nd in enumerate(stack):
            if k in exclude or nd["buf"] == 2:
                continue
            out.append(Region(nd["buf"], int(leaf[nd["p"] << nd["h"]]), nd["len"]))
        return out

    while True:
        guard += 1
        sp = len(stack)
        if guard > 4 * (l_end - l_begin + 64):
            raise AssertionError("walk guard exceeded")
        if sp >= 2 and stack[-2]["h"] == stack[-1]["h"] and (stack[-1]["p"] & 1) and \
                stack[-2]["p"] == stack[-1]["p"] - 1:
            act = "merge"
        elif next_list < l_end:
            act = "node"
        elif sp == 1:
            act = "done" if (not whole or stack[0]["buf"] == 2) else "toC"
        elif sp >= 2 and (stack[-1]["p"] & 1) == 0:
            act = "promote"
        else:
            raise AssertionError(f"no action (stack {[(n['h'], n['p']) for n in stack]})")
        actions.append(act)
        if act == "done":
            break
        if act == "node":
            l = next_list
            h = 0
            while h < 40 and ((l >> h) & 1) == 0 and l + (1 << h) < l_end:
                e = min(l + (1 << (h + 1)), l_end)
                if leaf[e] - leaf[l] <= lds_cap and e - l <= lds_cap:
                    h += 1
                else:
                    break
            l0, l1 = l, min(l + (1 << h), l_end)
            root = whole and l0 == 0 and l1 == L
            r0, np_ = int(leaf[l0]), int(leaf[l1] - leaf[l0])
            if np_ <= lds_cap and l1 - l0 <= lds_cap:
                pass  # LDS node: brmerge_range_lds over lists [l0, l1)
            else:
                assert l1 - l0 == 1, "only a single list may exceed LDS"
            cols = content(l0, l1)
            ln = len(cols) if exact else np_
            assert ln <= np_
            if root:
                assert ln <= ccap
            else:
                # written to buffer 0 at its first list's products
                assert leaf[l_begin] <= r0 and r0 + ln <= leaf[l_end], "node write outside its subtree"
                for rg in live():
                    assert not rg.overlaps(0, r0, r0 + ln), "node write over a live node"
                writes.append((0, r0, r0 + ln))
            assert len(stack) < 64, "node stack overflow"
            stack.append({"p": l0 >> h, "h": h, "len": ln, "buf": 2 if root else 0, "cols": cols})
            next_list = l1
        elif act == "merge":
            x, y = stack[-2], stack[-1]
            root = whole and (y["p"] >> 1) == 0 and (1 << (y["h"] + 1)) >= L
            rx, ry = int(leaf[x["p"] << x["h"]]), int(leaf[y["p"] << y["h"]])
            assert x["len"] <= ry - rx, "left child longer than its products"
            assert ry + y["len"] <= nprod
            ob = 2 if root else (1 - x["buf"] if x["buf"] == y["buf"] else y["buf"])
            assert ob != x["buf"], "the left child is never overwritten"
            cap = ccap if root else nprod - rx
            if exact:
                ln = merge_tiles(x["cols"], y["cols"], T, rx, ry, cap, ob == y["buf"])
                cols = np.union1d(x["cols"], y["cols"])
            else:
                ln = x["len"] + y["len"]
                cols = None
                assert ln <= cap
                if ob == y["buf"]:
                    assert rx + ln <= ry + y["len"]
            if not root:
                assert leaf[l_begin] <= rx and rx + ln <= leaf[l_end], "merge write outside its subtree"
                for rg in live(exclude=(len(stack) - 2, len(stack) - 1)):
                    assert not rg.overlaps(ob, rx, rx + ln), "merge write over a live node"
                writes.append((ob, rx, rx + ln))
            stack[-2:] = [{"p": x["p"] >> 1, "h": x["h"] + 1, "len": ln, "buf": ob, "cols": cols}]
        elif act == "promote":
            stack[-1]["p"] >>= 1
            stack[-1]["h"] += 1
        elif act == "toC":
            assert stack[0]["len"] <= ccap
            stack[0]["buf"] = 2
    assert len(stack) == 1 and stack[0]["h"] >= 0
    if not whole:
        assert stack[0]["buf"] in (0, 1)
        return (stack[0]["buf"], stack[0]["len"], stack[0]["cols"]), actions
    return stack[0]["len"], actions


def plan_split(np_, L, target):
    """run_heavy's cut of a long row: (H, S) subtrees of 2^H lists, or None
    when the row stays whole."""
    if target < 0 or np_ <= 2 * target or L < 2:
        return None
    want = min((np_ + target - 1) // target, 1024)
    H = 0
    while ((L + (1 << (H + 1)) - 1) >> (H + 1)) >= want:
        H += 1
    S = (L + (1 << H) - 1) >> H
    return None if S < 2 else (H, S)


def top_levels(S, H):
    """The merges above S subtrees, level by level: (res_x, res_y or -1,
    root, lx, ly) with result slots relative to the row's first slot."""
    levels = []
    r = 1
    while ((S + (1 << (r - 1)) - 1) >> (r - 1)) > 1:
        nprev = (S + (1 << (r - 1)) - 1) >> (r - 1)
        ncur = (S + (1 << r) - 1) >> r
        lv = []
        for q in range(ncur):
            xq, yq = 2 * q, 2 * q + 1
            root = ncur == 1
            if yq >= nprev and not root:
                continue
            lv.append((xq << (r - 1), (yq << (r - 1)) if yq < nprev else -1, root,
                       (xq << (r - 1)) << H, ((yq << (r - 1)) << H) if yq < nprev else 0))
        levels.append(lv)
        r += 1
    return levels


def split_row(list_cols, lds_cap, T, target, exact=True):
    """A split row end to end: every subtree walk (checked to write only
    inside its own products, so that the subtrees of one launch never
    meet), then the top merges level by level with the kernel's buffer rule
    and bounds checks.  Returns the root's length."""
    L = len(list_cols)
    lens = np.array([len(c) for c in list_cols], dtype=np.int64)
    leaf = np.zeros(L + 1, dtype=np.int64)
    leaf[1:] = np.cumsum(lens)
    nprod = int(leaf[L])
    cut = plan_split(nprod, L, target)
    assert cut is not None
    H, S = cut
    res = {}
    spans = []
    for q in range(S):
        l0, l1 = q << H, min((q + 1) << H, L)
        w = []
        (buf, ln, cols), _ = heavy_walk(list_cols, lds_cap, T, ccap=nprod, exact=exact, l_begin=l0, l_end=l1,
                                        writes=w)
        for b, lo, hi in w:
            assert leaf[l0] <= lo and hi <= leaf[l1]
        spans.append((leaf[l0], leaf[l1]))
        res[q] = (buf, ln, cols)
    for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
        assert a1 <= b0
    root_len = None
    for lv in top_levels(S, H):
        written = []
        for rx_s, ry_s, root, lx, ly in lv:
            xb, xl, xc = res[rx_s]
            rx = int(leaf[lx])
            if ry_s < 0:
                assert root
                root_len = xl
                continue
            yb, yl, yc = res[ry_s]
            ry = int(leaf[ly])
            assert xb in (0, 1) and yb in (0, 1)
            assert rx + xl <= ry and ry + yl <= nprod
            if root:
                root_len = merge_tiles(xc, yc, T, rx, ry, nprod, False) if exact else xl + yl
                continue
            ob = 1 - xb if xb == yb else yb
            if exact:
                ln = merge_tiles(xc, yc, T, rx, ry, nprod - rx, ob == yb)
                cols = np.union1d(xc, yc)
            else:
                ln, cols = xl + yl, None
                if ob == yb:
                    assert rx + ln <= ry + yl
            # the node's products end where the next node of its level begins
            end = int(leaf[min(ly + (ly - lx), L)])
            assert rx + ln <= end
            for b, lo, hi in written:
                assert not (b == ob and lo < rx + ln and rx < hi), "two merges of a level overlap"
            written.append((ob, rx, rx + ln))
            res[rx_s] = (ob, ln, cols)
    assert root_len is not None
    return root_len


def row_lists(A, B, i):
    cols = []
    for p in range(A.rpt[i], A.rpt[i + 1]):
        k = A.col[p]
        cols.append(B.col[B.rpt[k]:B.rpt[k + 1]].astype(np.int64))
    return cols


def heavy_rows(A, threshold):
    lens = np.diff(A.rpt.astype(np.int64))
    blen = np.diff(A.rpt.astype(np.int64))
    nprod = np.zeros(A.rows, np.int64)
    np.add.at(nprod, np.repeat(np.arange(A.rows), lens), blen[A.col])
    return np.nonzero(nprod > threshold)[0], nprod


@pytest.mark.parametrize("T", [512, 1024])
def test_walk_exact_contents_rmat12(T):
    A = synth.rmat(12, 16, 13)
    rows, nprod = heavy_rows(A, 4096)
    assert rows.size > 10
    lds = 4 * T
    for i in rows[:120]:
        lists = row_lists(A, A, i)
        ln, acts = heavy_walk(lists, lds, T, ccap=int(nprod[i]))
        assert ln == len(np.unique(np.concatenate(lists)))
        # small LDS nodes give deep spill trees
        ln2, _ = heavy_walk(lists, 64, T, ccap=int(nprod[i]))
        assert ln2 == ln


@pytest.mark.parametrize("scale,T", [(14, 512), (15, 1024)])
def test_walk_upper_bound_lengths(scale, T):
    A = synth.rmat(scale, 16, 14)
    rows, nprod = heavy_rows(A, 4096)
    for i in rows[np.argsort(-nprod[rows])][:40]:
        lists = row_lists(A, A, i)
        for cap in (4 * T, 2048, 256):
            ln, _ = heavy_walk(lists, cap, T, ccap=int(nprod[i]), exact=False)
            assert ln == nprod[i]


def test_walk_single_lists_beyond_lds():
    # lists longer than LDS alternate with short ones; an odd last list
    rng = np.random.default_rng(3)
    lists = []
    for k in range(37):
        n = int(rng.integers(5000, 9000)) if k % 3 == 0 else int(rng.integers(1, 50))
        lists.append(np.sort(rng.choice(1 << 20, n, replace=False)).astype(np.int64))
    ln, acts = heavy_walk(lists, 2048, 512, ccap=sum(len(c) for c in lists))
    assert ln == len(np.unique(np.concatenate(lists)))
    assert "promote" in acts


def test_merge_tiles_boundaries():
    # equal columns on window edges, one side exhausted, empty sides
    T = 8
    win = KWIN_PER * T
    a = np.arange(0, 4 * win, 2, dtype=np.int64)
    b = np.arange(0, 4 * win, 3, dtype=np.int64)
    for X, Y in ((a, b), (b, a), (a, a), (a[:0], b), (a, b[:0]), (a[:win], b[:win]),
                 (np.arange(win, dtype=np.int64), np.arange(win, 2 * win, dtype=np.int64))):
        n = merge_tiles(X, Y, T, 0, len(X), len(X) + len(Y), True)
        assert n == len(np.union1d(X, Y))


def pool_layout(np_rows, nl_rows, budget):
    """run_heavy's ordering, batching and pool layout for heavy rows with
    product counts np_rows and list counts nl_rows."""
    n = len(np_rows)

    def bucket(v):
        v = max(int(v), 1)
        lg = v.bit_length() - 1
        frac = (v >> (lg - 3)) & 7 if lg >= 3 else (v << (3 - lg)) & 7
        return max(255 - (8 * lg + frac), 0)

    bk = [bucket(v) for v in np_rows]
    order = sorted(range(n), key=lambda i: (bk[i], i))  # counting sort, rows in id order

    def align(x):
        return (x + 255) // 256 * 256

    def pool_bytes(elems, leafs):
        return align(4 * elems) + align(8 * elems) + align(4 * leafs) + 256

    batches, soff, loff = [], [0] * n, [0] * n
    max_e = max_l = elems = leafs = 0
    b0 = 0
    for j, i in enumerate(order):
        np_, nl = int(np_rows[i]), int(nl_rows[i])
        if j > b0 and pool_bytes(max(max_e, elems + 2 * np_), max(max_l, leafs + nl + 1)) > budget:
            batches.append((b0, j))
            b0 = j
            elems = leafs = 0
        soff[j], loff[j] = elems, leafs
        elems += 2 * np_
        leafs += nl + 1
        max_e, max_l = max(max_e, elems), max(max_l, leafs)
    batches.append((b0, n))
    return order, batches, soff, loff, max_e, max_l, pool_bytes(max_e, max_l)


@pytest.mark.parametrize("budget", [1 << 20, 1 << 24, 1 << 30])
def test_pool_layout_bounds(budget):
    A = synth.rmat(14, 16, 15)
    rows, nprod = heavy_rows(A, 4096)
    nl = np.diff(A.rpt.astype(np.int64))[rows]
    npr = nprod[rows]
    order, batches, soff, loff, max_e, max_l, pool = pool_layout(npr, nl, budget)
    assert [r for b in batches for r in range(*b)] == list(range(len(rows)))
    for lo, hi in batches:
        used = []
        for j in range(lo, hi):
            i = order[j]
            assert 0 <= soff[j] and soff[j] + 2 * npr[i] <= max_e
            assert 0 <= loff[j] and loff[j] + nl[i] + 1 <= max_l
            used.append((soff[j], soff[j] + 2 * npr[i]))
        used.sort()
        for (a0, a1), (b0, b1) in zip(used, used[1:]):
            assert a1 <= b0, "two rows of a batch share spill entries"
    # the column, value and list-offset parts fit the pool
    assert ((4 * max_e + 255) // 256 * 256 + (8 * max_e + 255) // 256 * 256 + 4 * max_l) <= pool


@pytest.mark.parametrize("T,target", [(512, 4096), (1024, 15000), (512, 9000)])
def test_split_rows_exact(T, target):
    A = synth.rmat(12, 16, 13)
    rows, nprod = heavy_rows(A, 4096)
    done = 0
    for i in rows[np.argsort(-nprod[rows])][:25]:
        lists = row_lists(A, A, i)
        if plan_split(int(nprod[i]), len(lists), target) is None:
            continue
        ln = split_row(lists, 4 * T, T, target)
        assert ln == len(np.unique(np.concatenate(lists)))
        done += 1
    assert done > 0


def test_split_rows_upper_bound_scale15():
    A = synth.rmat(15, 16, 14)
    rows, nprod = heavy_rows(A, 4096)
    for i in rows[np.argsort(-nprod[rows])][:20]:
        lists = row_lists(A, A, i)
        for target in (4096, 50000):
            if plan_split(int(nprod[i]), len(lists), target) is not None:
                assert split_row(lists, 2048, 512, target, exact=False) == nprod[i]


def test_top_levels_cover_every_subtree():
    for S in range(2, 70):
        levels = top_levels(S, 3)
        alive = set(range(S))
        for lv in levels:
            for x, y, root, lx, ly in lv:
                assert x in alive
                if y >= 0:
                    assert y in alive and y > x
                    alive.discard(y)
        assert alive == {0}
        assert levels[-1][0][2]  # the last level holds the root
