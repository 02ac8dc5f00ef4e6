"""CPU oracle for C = A*B on CSR -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library (``paper_2206_06611_amd``) never imports
it and shares no code with it; both sides consume the same seeded inputs from
``synth``.

Contents
--------
``spgemm``         the plain definition of the row-wise product (Eq. (2),
                   Section II-A.2) with a dense accumulator and compensated
                   sums; returns C and, per entry, the sum of |products|.
``brmerge``        the accumulation method of Section III-B (Algorithm 1) run
                   row by row on the CPU: its values are the bitwise
                   expectation for any implementation that groups additions by
                   the same merge tree.
``pattern_sums``   per row of C the entry count and the sum of its columns
                   (the structure alone, for products too large to hold).
``row_nprod``      products per row (Section II-A.4).
``brute_force``    Eq. (1) on dense arrays, pure Python loops: tiny inputs only.
``compression_ratio``  Eq. (5).
``row_features``   the per-row features the learned size predictor consumes.

The C part lives in ``oracle.c`` and is compiled by :func:`build` with gcc,
OpenMP and -ffp-contract=off.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.oracle_row_nprod.argtypes = [I64, I64, P, P, P, P]
        lib.oracle_spa_counts.argtypes = [I64, I64, I64, P, P, P, P, P, ctypes.c_int]
        lib.oracle_spa_pattern_sums.argtypes = [I64, I64, I64, P, P, P, P, P, P, ctypes.c_int]
        lib.oracle_spa_fill.argtypes = [I64, I64, I64, P, P, P, P, P, P, P, P, P, P, ctypes.c_int]
        lib.oracle_brmerge_rows.argtypes = [I64, I64, P, P, P, P, P, P, P, P, P, P, P, ctypes.c_int]
        lib.oracle_max_threads.argtypes = []
        for f in (lib.oracle_row_nprod, lib.oracle_spa_counts, lib.oracle_spa_pattern_sums, lib.oracle_spa_fill,
                  lib.oracle_brmerge_rows, lib.oracle_max_threads):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return _load().oracle_max_threads()


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Result:
    """Rows of C in CSR form (rpt relative to the first returned row)."""

    rows: np.ndarray  # the row ids of A these rows belong to
    rpt: np.ndarray   # int64, len(rows) + 1
    col: np.ndarray   # int32
    val: np.ndarray   # float64
    absval: np.ndarray | None = None  # float64, sum of |products| per entry
    rounds: np.ndarray | None = None  # int32 merge rounds per row (brmerge only)

    @property
    def nnz(self) -> int:
        return int(self.rpt[-1])


def _prep(A, B, rows):
    """Widen row pointers to int64 and, when a row subset is asked for, gather
    those rows of A into a compact CSR (index reshuffling only)."""
    if A.cols != B.rows:
        raise ValueError("inner dimensions differ")
    a_rpt = np.ascontiguousarray(A.rpt, dtype=np.int64)
    a_col = np.ascontiguousarray(A.col, dtype=np.int32)
    a_val = np.ascontiguousarray(A.val, dtype=np.float64)
    if rows is None:
        rows = np.arange(A.rows, dtype=np.int64)
    else:
        rows = np.asarray(rows, dtype=np.int64)
        lens = a_rpt[rows + 1] - a_rpt[rows]
        idx = np.concatenate([np.arange(a_rpt[r], a_rpt[r + 1]) for r in rows]) if rows.size else \
            np.zeros(0, np.int64)
        idx = idx.astype(np.int64)
        a_rpt = np.zeros(rows.size + 1, np.int64)
        np.cumsum(lens, out=a_rpt[1:])
        a_col = np.ascontiguousarray(a_col[idx])
        a_val = np.ascontiguousarray(a_val[idx])
    b_rpt = np.ascontiguousarray(B.rpt, dtype=np.int64)
    b_col = np.ascontiguousarray(B.col, dtype=np.int32)
    b_val = np.ascontiguousarray(B.val, dtype=np.float64)
    return rows, a_rpt, a_col, a_val, b_rpt, b_col, b_val


def row_nprod(A, B, rows=None) -> np.ndarray:
    lib = _load()
    rows, a_rpt, a_col, _, b_rpt, _, _ = _prep(A, B, rows)
    out = np.zeros(rows.size, np.int64)
    lib.oracle_row_nprod(0, rows.size, _p(a_rpt), _p(a_col), _p(b_rpt), _p(out))
    return out


def pattern_sums(A, B, rows=None, nthreads: int = 0):
    """The structure of C = A*B without its values: per row the number of
    stored entries (distinct columns) and the sum of their column indices
    (int64 arrays).  For products whose C does not fit in host memory."""
    lib = _load()
    rows, a_rpt, a_col, _, b_rpt, b_col, _ = _prep(A, B, rows)
    m = rows.size
    counts = np.zeros(m, np.int64)
    sums = np.zeros(m, np.int64)
    rc = lib.oracle_spa_pattern_sums(B.cols, 0, m, _p(a_rpt), _p(a_col), _p(b_rpt), _p(b_col), _p(counts),
                                     _p(sums), nthreads)
    if rc:
        raise MemoryError(f"oracle_spa_pattern_sums failed ({rc})")
    return counts, sums


def spgemm(A, B, rows=None, nthreads: int = 0) -> Result:
    """The definition of C = A*B (all rows, or the given row ids)."""
    lib = _load()
    rows, a_rpt, a_col, a_val, b_rpt, b_col, b_val = _prep(A, B, rows)
    m = rows.size
    counts = np.zeros(m, np.int64)
    rc = lib.oracle_spa_counts(B.cols, 0, m, _p(a_rpt), _p(a_col), _p(b_rpt), _p(b_col),
                               _p(counts), nthreads)
    if rc:
        raise MemoryError(f"oracle_spa_counts failed ({rc})")
    rpt = np.zeros(m + 1, np.int64)
    np.cumsum(counts, out=rpt[1:])
    nnz = int(rpt[-1])
    col = np.empty(max(nnz, 1), np.int32)
    val = np.empty(max(nnz, 1), np.float64)
    absval = np.empty(max(nnz, 1), np.float64)
    rc = lib.oracle_spa_fill(B.cols, 0, m, _p(a_rpt), _p(a_col), _p(a_val), _p(b_rpt),
                             _p(b_col), _p(b_val), _p(rpt), _p(col), _p(val), _p(absval),
                             nthreads)
    if rc:
        raise MemoryError(f"oracle_spa_fill failed ({rc})")
    return Result(rows, rpt, col[:nnz], val[:nnz], absval[:nnz])


def brmerge(A, B, rows=None, nthreads: int = 0) -> Result:
    """Algorithm 1's accumulation run row by row on the CPU."""
    lib = _load()
    rows, a_rpt, a_col, a_val, b_rpt, b_col, b_val = _prep(A, B, rows)
    m = rows.size
    nprod = np.zeros(m, np.int64)
    lib.oracle_row_nprod(0, m, _p(a_rpt), _p(a_col), _p(b_rpt), _p(nprod))
    # each row's result fits in its product count; compact afterwards
    off = np.zeros(m + 1, np.int64)
    np.cumsum(nprod, out=off[1:])
    tot = int(off[-1])
    col = np.empty(max(tot, 1), np.int32)
    val = np.empty(max(tot, 1), np.float64)
    lens = np.zeros(m, np.int64)
    rounds = np.zeros(m, np.int32)
    rc = lib.oracle_brmerge_rows(0, m, _p(a_rpt), _p(a_col), _p(a_val), _p(b_rpt), _p(b_col),
                                 _p(b_val), _p(off), _p(col), _p(val), _p(lens), _p(rounds),
                                 nthreads)
    if rc:
        raise MemoryError(f"oracle_brmerge_rows failed ({rc})")
    rpt = np.zeros(m + 1, np.int64)
    np.cumsum(lens, out=rpt[1:])
    keep = np.zeros(max(tot, 1), bool)
    starts = off[:-1]
    if tot:
        # mark the first lens[i] slots of every row's region
        marker = np.zeros(tot + 1, np.int64)
        np.add.at(marker, starts, 1)
        np.add.at(marker, starts + lens, -1)
        keep = np.cumsum(marker[:-1]) > 0
    return Result(rows, rpt, col[:tot][keep[:tot]], val[:tot][keep[:tot]], rounds=rounds)


def brute_force(Ad: np.ndarray, Apat: np.ndarray, Bd: np.ndarray, Bpat: np.ndarray):
    """Eq. (1) with explicit loops over dense arrays: C_ij is the sum over k of
    A_ik * B_kj for the k where both entries are stored; (i, j) is stored iff
    such a k exists.  Returns (pattern, values) as dense arrays.  Products are
    summed in increasing k, so compare values exactly only for integer data."""
    M, K = Ad.shape
    K2, N = Bd.shape
    assert K == K2
    pat = np.zeros((M, N), bool)
    vals = np.zeros((M, N), np.float64)
    for i in range(M):
        for j in range(N):
            s = 0.0
            hit = False
            for k in range(K):
                if Apat[i, k] and Bpat[k, j]:
                    s += float(Ad[i, k]) * float(Bd[k, j])
                    hit = True
            pat[i, j] = hit
            vals[i, j] = s
    return pat, vals


def compression_ratio(total_nprod: int, nnz_c: int) -> float:
    """Eq. (5): products per stored entry of C."""
    return float(total_nprod) / float(nnz_c) if nnz_c else math.inf


def row_features(A, B) -> dict:
    """Per-row quantities of a row of C that need no merging: the A row
    length, the product count, the longest and shortest B row used, and the
    column span covered by the B rows used (last column minus first column
    plus one, 0 when there is no product)."""
    a_rpt = np.asarray(A.rpt, np.int64)
    b_rpt = np.asarray(B.rpt, np.int64)
    blen = np.diff(b_rpt)
    nnza = np.diff(a_rpt)
    out = {k: np.zeros(A.rows, np.int64) for k in ("nnza", "nprod", "maxb", "minb", "span")}
    out["nnza"][:] = nnza
    for i in range(A.rows):
        ks = A.col[a_rpt[i]:a_rpt[i + 1]].astype(np.int64)
        if ks.size == 0:
            continue
        lens = blen[ks]
        out["nprod"][i] = lens.sum()
        out["maxb"][i] = lens.max()
        out["minb"][i] = lens.min()
        nz = ks[lens > 0]
        if nz.size:
            first = B.col[b_rpt[nz]].min()
            last = B.col[b_rpt[nz + 1] - 1].max()
            out["span"][i] = int(last) - int(first) + 1
    return out
