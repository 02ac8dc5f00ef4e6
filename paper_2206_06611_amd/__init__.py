"""MI355X (gfx950) row-wise SpGEMM with the BRMerge accumulation.

Thin Python binding of the C ABI in ``include/spgemm.h`` (library
``libbrmspgemm.so`` built from ``csrc/`` by ``build.py``).  Python only
marshals arguments: device memory comes from PyTorch tensors, the stream is
PyTorch's current stream, and every step of the product runs in the HIP
kernels of the library.  There is no fallback: importing this package fails
if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbrmspgemm.so")

# status codes
SPG_OK = 0
SPG_ERR_ARG = -1
SPG_ERR_DIM = -2
SPG_ERR_INVALID_CSR = -3
SPG_ERR_CAPACITY = -4
SPG_ERR_NOMEM = -5
SPG_ERR_HIP = -6
SPG_ERR_NOT_TRAINED = -7
SPG_ERR_STATE = -8
SPG_ERR_SCRATCH = -9

# options
OPT_VALIDATE = 1
OPT_WAVE_SMALL_MAX = 2
OPT_WAVE_MAX = 3
OPT_GROUP_MAX = 4
OPT_BLOCK_MAX = 5
OPT_FORCE_CLASS = 6
OPT_HEAVY_LDS_MAX = 7
OPT_SPILL_BUDGET_MB = 8
OPT_GRID_WAVES = 9
OPT_ALLOC = 10
OPT_LEARNED_FORCE = 11
OPT_GROUP_ROWS = 12
OPT_ACCUMULATOR = 13
OPT_HEAVY_THREADS = 14
OPT_HEAVY_SPLIT = 15
OPT_LEARNED_HEAVY_MARGIN = 16
OPT_BATCH_ALLOC = 17
OPT_STORED_ORDER = 18
PROBLEM_OPERAND_ONLY = 1
BATCH_PRECISE = 0
BATCH_UPPER = 1
ACC_BRMERGE = 0
ACC_HASH = 1
ALLOC_PRECISE = 0
ALLOC_LEARNED = 1
ALLOC_UPPER = 2
MLP_NUM_PARAMS = 4673

# statistics
STAT_NPROD = 1
STAT_NNZ = 2
STAT_CLASS_ROWS0 = 10
STAT_HEAVY_BATCHES = 20
STAT_PRED_TOTAL = 21
STAT_OVERFLOW_ROWS = 22
STAT_PREDICTED_ROWS = 23
STAT_GRAPH_CAPTURES = 24
STAT_GRAPH_LAUNCHES = 25
STAT_SPILL_POOL_BYTES = 26
STAT_SPILL_ALLOCS = 27
STAT_HEAVY_WIDE = 28
STAT_HEAVY_SPLIT_ROWS = 29
STAT_DEVICE_ERR = 30
STAT_OVERFLOW_HEAVY_ROWS = 31
STAT_BATCHED_DIRECT = 32

CLASS_NAMES = ["empty", "copy", "wave_small", "wave", "group", "block", "heavy", "multi"]


class SpgError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"spgemm error {code}: {message}")
        self.code = code


class _Csr(ctypes.Structure):
    _fields_ = [
        ("rows", ctypes.c_int64),
        ("cols", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("rpt", ctypes.c_void_p),
        ("rpt_bytes", ctypes.c_int32),
        ("col", ctypes.c_void_p),
        ("val", ctypes.c_void_p),
    ]


class _Problem(ctypes.Structure):
    _fields_ = [("A", _Csr), ("B", _Csr), ("b_from", ctypes.c_int32), ("flags", ctypes.c_int32)]


class _BatchedOut(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("rows", "cols", "nnz", "rpt_off", "col_off", "val_off")]


def _load_library():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it first (python -m paper_2206_06611_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    PH = ctypes.POINTER(ctypes.c_void_p)
    PCSR = ctypes.POINTER(_Csr)
    sig = {
        "spg_create": ([PH, I32], I32),
        "spg_destroy": ([P], I32),
        "spg_set_option": ([P, I32, I64], I32),
        "spg_get_option": ([P, I32, ctypes.POINTER(I64)], I32),
        "spg_get_stat": ([P, I32, ctypes.POINTER(I64)], I32),
        "spgemm_symbolic": ([P, PCSR, PCSR, P, ctypes.POINTER(I64), P], I32),
        "spgemm_numeric": ([P, PCSR, PCSR, P, P, P, P], I32),
        "spgemm_row_products": ([P, PCSR, PCSR, P, P], I32),
        "spg_last_error": ([P], ctypes.c_char_p),
        "spg_mlp_set_params": ([P, P, P, ctypes.c_float], I32),
        "spg_mlp_get_params": ([P, P, P, P], I32),
        "spg_mlp_features": ([P, PCSR, PCSR, P, P, P, P, P, P, P], I32),
        "spg_mlp_forward": ([P, P, I64, P, P], I32),
        "spg_mlp_gradient": ([P, P, P, I64, P, P, P], I32),
        "spg_mlp_fit_normalization": ([P, P, I64, P], I32),
        "spg_mlp_train": ([P, P, P, I64, I32, I32, ctypes.c_float, P], I32),
        "spg_mlp_loss": ([P, P, P, I64, P, P], I32),
        "spg_mlp_calibrate": ([P, P, P, I64, ctypes.c_double, P, P], I32),
        "spg_mlp_save": ([P, ctypes.c_char_p], I32),
        "spg_mlp_load": ([P, ctypes.c_char_p], I32),
        "spgemm_batched": ([P, I32, ctypes.POINTER(_Problem), P, I64, P, ctypes.POINTER(I64), P], I32),
        "spgemm_batched_noalloc": ([P, I32, ctypes.POINTER(_Problem), P, I64, P, ctypes.POINTER(I64), P], I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load_library()

# every symbol declared in include/spgemm.h
EXPORTED = ("spg_create", "spg_destroy", "spg_set_option", "spg_get_option", "spg_get_stat",
            "spgemm_symbolic", "spgemm_numeric", "spg_last_error", "spg_mlp_set_params",
            "spg_mlp_get_params", "spg_mlp_features", "spg_mlp_forward", "spg_mlp_gradient",
            "spg_mlp_fit_normalization", "spg_mlp_train", "spg_mlp_loss", "spg_mlp_calibrate",
            "spg_mlp_save", "spg_mlp_load", "spgemm_batched", "spgemm_row_products",
            "spgemm_batched_noalloc")


def library():
    return _lib


@dataclass
class DeviceCSR:
    """A CSR matrix whose arrays are device tensors."""

    rows: int
    cols: int
    rpt: torch.Tensor  # int32 or int64, rows + 1
    col: torch.Tensor  # int32
    val: torch.Tensor  # float64

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @classmethod
    def from_host(cls, A, device="cuda", rpt_dtype=None) -> "DeviceCSR":
        """Copy a host CSR (any object with rows, cols, rpt, col, val arrays)."""
        rpt = torch.as_tensor(A.rpt)
        if rpt_dtype is not None:
            rpt = rpt.to(rpt_dtype)
        return cls(int(A.rows), int(A.cols), rpt.to(device),
                   torch.as_tensor(A.col, dtype=torch.int32).to(device),
                   torch.as_tensor(A.val, dtype=torch.float64).to(device))

    def row_block(self, begin: int, end: int) -> "DeviceCSR":
        """Rows [begin, end) as a CSR of their own: the column and value
        arrays are views into this matrix, the row pointers are rebased to
        start at zero (a new array of end - begin + 1 entries)."""
        if not 0 <= begin <= end <= self.rows:
            raise ValueError(f"row block [{begin}, {end}) outside 0..{self.rows}")
        rpt = self.rpt[begin:end + 1]
        lo, hi = (int(x) for x in rpt[[0, -1]].tolist())
        return DeviceCSR(end - begin, self.cols, (rpt - lo).contiguous(), self.col[lo:hi], self.val[lo:hi])

    def _struct(self) -> _Csr:
        # the last struct is kept while the same tensors, at the same
        # addresses and sizes, make up the matrix (rebuilding it costs the
        # checks below on every call)
        rpt, col, val = self.rpt, self.col, self.val
        key = (self.rows, self.cols, rpt.data_ptr(), col.data_ptr(), val.data_ptr(),
               rpt.numel(), col.numel(), val.numel())
        memo = self.__dict__.get("_memo")
        if memo is not None and memo[0] == key and memo[1] is rpt and memo[2] is col and memo[3] is val:
            return memo[4]
        if self.rpt.dtype not in (torch.int32, torch.int64):
            raise TypeError("rpt must be int32 or int64")
        for t in (self.rpt, self.col, self.val):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("CSR arrays must be contiguous device tensors")
        if self.col.dtype != torch.int32 or self.val.dtype != torch.float64:
            raise TypeError("col must be int32 and val float64")
        st = _Csr(self.rows, self.cols, self.nnz, self.rpt.data_ptr(),
                  4 if self.rpt.dtype == torch.int32 else 8,
                  self.col.data_ptr() if self.nnz else None,
                  self.val.data_ptr() if self.nnz else None)
        self.__dict__["_memo"] = (key, rpt, col, val, st)
        return st


@dataclass
class DeviceCSC:
    """A CSC matrix whose arrays are device tensors: cpt[cols + 1] column
    pointers, row indices strictly increasing within each column."""

    rows: int
    cols: int
    cpt: torch.Tensor  # int32 or int64, cols + 1
    row: torch.Tensor  # int32
    val: torch.Tensor  # float64

    @property
    def nnz(self) -> int:
        return int(self.row.numel())

    def transposed_csr(self) -> DeviceCSR:
        """The same arrays read as the CSR of the transpose (no copy)."""
        return DeviceCSR(self.cols, self.rows, self.cpt, self.row, self.val)

    @classmethod
    def from_host_csr(cls, A, device="cuda") -> "DeviceCSC":
        """CSC of a host CSR matrix (transposed on the host, then copied)."""
        import numpy as np
        order = np.lexsort((np.repeat(np.arange(A.rows), np.diff(np.asarray(A.rpt, np.int64))),
                            np.asarray(A.col)))
        counts = np.bincount(np.asarray(A.col), minlength=A.cols)
        cpt = np.zeros(A.cols + 1, np.int64)
        cpt[1:] = np.cumsum(counts)
        rows = np.repeat(np.arange(A.rows, dtype=np.int32), np.diff(np.asarray(A.rpt, np.int64)))[order]
        return cls(int(A.rows), int(A.cols), torch.as_tensor(cpt.astype(np.int32 if cpt[-1] < 2**31 else np.int64),
                                                                device=device),
                   torch.as_tensor(rows, device=device), torch.as_tensor(np.asarray(A.val)[order], device=device))


def cut_row_blocks(row_nprod, max_products: int):
    """Greedy cut of consecutive rows into blocks whose product counts sum to
    at most `max_products` (a row with more is a block of its own)."""
    import numpy as np
    n = len(row_nprod)
    csum = np.concatenate([[0], np.cumsum(np.asarray(row_nprod, np.int64))])
    blocks, r = [], 0
    while r < n:
        e = int(np.searchsorted(csum, csum[r] + max_products, side="right")) - 1
        e = min(max(e, r + 1), n)
        blocks.append((r, e))
        r = e
    return blocks


class BatchedProblems:
    """The problems of a batched call in the C ABI's layout, built once; it
    keeps the matrices it points to alive."""

    def __init__(self, problems):
        """problems: (A, B) or (A, B, flags) tuples (flags: PROBLEM_OPERAND_ONLY or 0)."""
        self.n = len(problems)
        self.arr = (_Problem * max(self.n, 1))()
        self._keep = list(problems)
        for i, prob in enumerate(problems):
            A, B = prob[0], prob[1]
            self.arr[i].flags = prob[2] if len(prob) > 2 else 0
            self.arr[i].A = A._struct()
            if isinstance(B, int):
                self.arr[i].b_from = B
            else:
                self.arr[i].B = B._struct()
                self.arr[i].b_from = -1


def _stream_ptr(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Handle:
    """Owns a library handle (device workspace, options, statistics)."""

    def __init__(self, device: int = 0):
        self._h = ctypes.c_void_p()
        rc = _lib.spg_create(ctypes.byref(self._h), device)
        if rc != SPG_OK:
            raise SpgError(rc, "spg_create failed")
        self.device = device

    def close(self):
        if self._h:
            _lib.spg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != SPG_OK:
            raise SpgError(rc, _lib.spg_last_error(self._h).decode())

    def set_option(self, key: int, value: int):
        self._check(_lib.spg_set_option(self._h, key, int(value)))

    def get_option(self, key: int) -> int:
        v = ctypes.c_int64()
        self._check(_lib.spg_get_option(self._h, key, ctypes.byref(v)))
        return v.value

    def stat(self, key: int) -> int:
        v = ctypes.c_int64()
        self._check(_lib.spg_get_stat(self._h, key, ctypes.byref(v)))
        return v.value

    def class_rows(self) -> dict:
        return {n: self.stat(STAT_CLASS_ROWS0 + i) for i, n in enumerate(CLASS_NAMES)}

    def symbolic(self, A: DeviceCSR, B: DeviceCSR, c_rpt: torch.Tensor | None = None, stream=None):
        """Returns (c_rpt int64 device tensor, nnz)."""
        if c_rpt is None:
            c_rpt = torch.empty(A.rows + 1, dtype=torch.int64, device=A.rpt.device)
        nnz = ctypes.c_int64()
        sa, sb = A._struct(), B._struct()
        self._check(_lib.spgemm_symbolic(self._h, ctypes.byref(sa), ctypes.byref(sb),
                                         ctypes.c_void_p(c_rpt.data_ptr()), ctypes.byref(nnz),
                                         _stream_ptr(stream)))
        return c_rpt, nnz.value

    def numeric(self, A: DeviceCSR, B: DeviceCSR, c_rpt: torch.Tensor, c_col: torch.Tensor,
                c_val: torch.Tensor, stream=None):
        sa, sb = A._struct(), B._struct()
        self._check(_lib.spgemm_numeric(self._h, ctypes.byref(sa), ctypes.byref(sb),
                                        ctypes.c_void_p(c_rpt.data_ptr()),
                                        ctypes.c_void_p(c_col.data_ptr() if c_col.numel() else None),
                                        ctypes.c_void_p(c_val.data_ptr() if c_val.numel() else None),
                                        _stream_ptr(stream)))

    def row_products(self, A: DeviceCSR, B: DeviceCSR, stream=None) -> torch.Tensor:
        """Products of every row of A*B (int64 device tensor of A.rows)."""
        out = torch.empty(max(A.rows, 1), dtype=torch.int64, device=A.rpt.device)
        sa, sb = A._struct(), B._struct()
        self._check(_lib.spgemm_row_products(self._h, ctypes.byref(sa), ctypes.byref(sb),
                                             ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out[:A.rows]

    def row_blocks(self, A: DeviceCSR, B: DeviceCSR, max_products: int, stream=None):
        """Cuts A's rows into consecutive blocks of at most `max_products`
        products each (a row with more forms a block of its own); the
        products bound each block's C.  Returns [(begin, end), ...]."""
        if A.rows == 0:
            return []
        return cut_row_blocks(self.row_products(A, B, stream).cpu().numpy(), max_products)

    def spgemm_row_blocks(self, A: DeviceCSR, B: DeviceCSR, max_products: int, stream=None):
        """C = A*B one row block at a time, for products whose C does not fit
        in device memory at once: yields (begin, end, C_block) with C_block
        the rows [begin, end) of C (each a complete product of its own)."""
        for b, e in self.row_blocks(A, B, max_products, stream):
            yield b, e, self.spgemm(A.row_block(b, e), B, stream)

    # ---- learned size predictor --------------------------------------------
    def mlp_set_params(self, params, norm, delta: float = 0.0):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        n = np.ascontiguousarray(norm, dtype=np.float32)
        if p.size != MLP_NUM_PARAMS or n.size != 12:
            raise ValueError("params must have 4673 entries and norm 12")
        self._check(_lib.spg_mlp_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p),
                                            n.ctypes.data_as(ctypes.c_void_p), float(delta)))

    def mlp_get_params(self):
        import numpy as np
        p = np.zeros(MLP_NUM_PARAMS, np.float32)
        n = np.zeros(12, np.float32)
        d = ctypes.c_float()
        self._check(_lib.spg_mlp_get_params(self._h, p.ctypes.data_as(ctypes.c_void_p),
                                            n.ctypes.data_as(ctypes.c_void_p), ctypes.byref(d)))
        return p, n, d.value

    def mlp_features(self, A: DeviceCSR, B: DeviceCSR, c_rpt: torch.Tensor | None = None, stream=None):
        """Returns (feats [rows, 6], targets or None, predicted int8, lo, hi)."""
        dev = A.rpt.device
        m = A.rows
        feats = torch.empty((max(m, 1), 6), dtype=torch.float32, device=dev)
        pred = torch.empty(max(m, 1), dtype=torch.int8, device=dev)
        lo = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
        hi = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
        tg = torch.empty(max(m, 1), dtype=torch.float32, device=dev) if c_rpt is not None else None
        sa, sb = A._struct(), B._struct()
        self._check(_lib.spg_mlp_features(
            self._h, ctypes.byref(sa), ctypes.byref(sb),
            ctypes.c_void_p(c_rpt.data_ptr()) if c_rpt is not None else None,
            ctypes.c_void_p(feats.data_ptr()), ctypes.c_void_p(tg.data_ptr()) if tg is not None else None,
            ctypes.c_void_p(pred.data_ptr()), ctypes.c_void_p(lo.data_ptr()), ctypes.c_void_p(hi.data_ptr()),
            _stream_ptr(stream)))
        return feats[:m], (tg[:m] if tg is not None else None), pred[:m], lo[:m], hi[:m]

    def mlp_forward(self, feats: torch.Tensor, stream=None) -> torch.Tensor:
        feats = feats.contiguous()
        y = torch.empty(feats.shape[0], dtype=torch.float32, device=feats.device)
        self._check(_lib.spg_mlp_forward(self._h, ctypes.c_void_p(feats.data_ptr()), feats.shape[0],
                                         ctypes.c_void_p(y.data_ptr()), _stream_ptr(stream)))
        return y

    def mlp_gradient(self, feats: torch.Tensor, targets: torch.Tensor, stream=None):
        feats, targets = feats.contiguous(), targets.contiguous()
        g = torch.empty(MLP_NUM_PARAMS, dtype=torch.float32, device=feats.device)
        loss = ctypes.c_float()
        self._check(_lib.spg_mlp_gradient(self._h, ctypes.c_void_p(feats.data_ptr()),
                                          ctypes.c_void_p(targets.data_ptr()), feats.shape[0],
                                          ctypes.c_void_p(g.data_ptr()), ctypes.byref(loss),
                                          _stream_ptr(stream)))
        return g, loss.value

    def mlp_fit_normalization(self, feats: torch.Tensor, stream=None):
        feats = feats.contiguous()
        self._check(_lib.spg_mlp_fit_normalization(self._h, ctypes.c_void_p(feats.data_ptr()),
                                                   feats.shape[0], _stream_ptr(stream)))

    def mlp_train(self, feats, targets, epochs: int, batch: int = 4096, lr: float = 1e-3, stream=None):
        feats, targets = feats.contiguous(), targets.contiguous()
        self._check(_lib.spg_mlp_train(self._h, ctypes.c_void_p(feats.data_ptr()),
                                       ctypes.c_void_p(targets.data_ptr()), feats.shape[0], int(epochs),
                                       int(batch), float(lr), _stream_ptr(stream)))

    def mlp_loss(self, feats, targets, stream=None) -> float:
        feats, targets = feats.contiguous(), targets.contiguous()
        loss = ctypes.c_float()
        self._check(_lib.spg_mlp_loss(self._h, ctypes.c_void_p(feats.data_ptr()),
                                      ctypes.c_void_p(targets.data_ptr()), feats.shape[0],
                                      ctypes.byref(loss), _stream_ptr(stream)))
        return loss.value

    def mlp_calibrate(self, feats, targets, quantile: float = 0.99, stream=None) -> float:
        feats, targets = feats.contiguous(), targets.contiguous()
        d = ctypes.c_float()
        self._check(_lib.spg_mlp_calibrate(self._h, ctypes.c_void_p(feats.data_ptr()),
                                           ctypes.c_void_p(targets.data_ptr()), feats.shape[0],
                                           float(quantile), ctypes.byref(d), _stream_ptr(stream)))
        return d.value

    def mlp_save(self, path: str):
        self._check(_lib.spg_mlp_save(self._h, path.encode()))

    def mlp_load(self, path: str):
        self._check(_lib.spg_mlp_load(self._h, path.encode()))

    # ---- batched products -------------------------------------------------
    def batched(self, problems, arena: torch.Tensor, out: torch.Tensor | None = None, stream=None,
                views: bool = True, noalloc: bool = False):
        """problems: list of (A, B) where B is a DeviceCSR or the index of an
        earlier problem whose C is B, or a BatchedProblems made from such a
        list once (repeated calls then skip the marshalling).  arena: uint8
        device tensor.  Returns (status, required_bytes, outputs); outputs are
        DeviceCSR views into the arena (None when the arena was too small, or
        when views is False: `out` then holds the descriptors).  noalloc:
        call spgemm_batched_noalloc (workspace in the library's fixed
        scratch array) instead of spgemm_batched."""
        bp = problems if isinstance(problems, BatchedProblems) else BatchedProblems(problems)
        n = bp.n
        if out is None:
            out = torch.empty((max(n, 1), 6), dtype=torch.int64, device=arena.device)
        req = ctypes.c_int64()
        fn = _lib.spgemm_batched_noalloc if noalloc else _lib.spgemm_batched
        rc = fn(self._h, n, bp.arr, ctypes.c_void_p(arena.data_ptr()), arena.numel(),
                ctypes.c_void_p(out.data_ptr()), ctypes.byref(req), _stream_ptr(stream))
        if rc not in (SPG_OK, SPG_ERR_CAPACITY):
            self._check(rc)
        if rc != SPG_OK or not views:
            return rc, req.value, None
        desc = out[:n].cpu().tolist()
        outs = []
        for rows, cols, nnz, ro, co, vo in desc:
            if nnz == -2:  # an operand only, kept in slots: not returned
                outs.append(None)
                continue
            rpt = arena[ro:ro + 8 * (rows + 1)].view(torch.int64)
            col = arena[co:co + 4 * nnz].view(torch.int32)
            val = arena[vo:vo + 8 * nnz].view(torch.float64)
            outs.append(DeviceCSR(int(rows), int(cols), rpt, col, val))
        return rc, req.value, outs

    @staticmethod
    def galerkin_problems(triples, ap_operand_only: bool = False) -> "BatchedProblems":
        """The batched problems of galerkin(triples), marshalled once;
        ap_operand_only marks every A_i P_i as an operand only."""
        f = PROBLEM_OPERAND_ONLY if ap_operand_only else 0
        return BatchedProblems([(A, P, f) for A, P, _ in triples] +
                               [(Pt, i) for i, (_, _, Pt) in enumerate(triples)])

    def galerkin(self, triples, arena: torch.Tensor | None = None, stream=None, problems=None,
                 ap_operand_only: bool = False):
        """G_i = P_i^T (A_i P_i) for triples (A_i, P_i, Pt_i) in one batched
        call (stage 1: A_i P_i, stage 2: Pt_i times stage 1's output).  Grows
        the arena when it is too small.  `problems` may be
        galerkin_problems(triples, ap_operand_only), made once.
        ap_operand_only: the A_i P_i are not returned (with upper-bound stage
        sizes they stay in their slots: no compaction).  Returns (G list, AP
        list -- None entries for operands kept in slots --, arena)."""
        n = len(triples)
        probs = problems if problems is not None else self.galerkin_problems(triples, ap_operand_only)
        if arena is None:
            est = sum(8 * (A.rows + 1) + 8 * (Pt.rows + 1) + 12 * 27 * A.rows + 8192 for A, _, Pt in triples)
            arena = torch.empty(est, dtype=torch.uint8, device=triples[0][0].rpt.device)
        # each failed call reports what the stages up to the first one that
        # did not fit need (a later stage's size depends on earlier outputs)
        for _ in range(3):
            rc, req, outs = self.batched(probs, arena, stream=stream)
            if rc == SPG_OK:
                return outs[n:], outs[:n], arena
            if req < 0:
                raise SpgError(rc, _lib.spg_last_error(self._h).decode())
            arena = torch.empty(req, dtype=torch.uint8, device=arena.device)
        raise SpgError(SPG_ERR_CAPACITY, "arena sizing failed")

    def amg_hierarchy(self, As, levels, stream=None):
        """Coarse operators of many aggregation hierarchies, level by level:
        A_{l+1} = P_l^T (A_l P_l), with the products of every hierarchy at
        level l in one batched call (whose two stages chain A_l P_l into
        P_l^T times it); each level's outputs are the next level's A.
        As: the finest operator of every hierarchy; levels: for every
        hierarchy the list of its (P_l, Pt_l) pairs (hierarchies may differ
        in depth).  Returns, per hierarchy, the list [A_1, ..., A_L] of
        DeviceCSR views into the level arenas (kept alive by the views)."""
        cur = list(As)
        out = [[] for _ in As]
        depth = max((len(lv) for lv in levels), default=0)
        for l in range(depth):
            ids = [i for i, lv in enumerate(levels) if l < len(lv)]
            triples = [(cur[i], levels[i][l][0], levels[i][l][1]) for i in ids]
            G, _, _ = self.galerkin(triples, stream=stream, ap_operand_only=True)
            for i, g in zip(ids, G):
                out[i].append(g)
                cur[i] = g
        return out

    def spgemm_csc(self, A: DeviceCSC, B: DeviceCSC, stream=None) -> DeviceCSC:
        """C = A*B with A, B and C in CSC: the column-wise dataflow (column j
        of C merges the columns of A selected by column j of B, Eq. (3)),
        which is the row-wise product of the transposes, C^T = B^T A^T, on
        the same arrays.  The merge tree's leaves are the stored entries of
        column j of B in stored order."""
        if A.cols != B.rows:
            raise SpgError(SPG_ERR_DIM, f"A is {A.rows} x {A.cols} but B has {B.rows} rows")
        Ct = self.spgemm(B.transposed_csr(), A.transposed_csr(), stream)
        return DeviceCSC(A.rows, B.cols, Ct.rpt, Ct.col, Ct.val)

    def spgemm(self, A: DeviceCSR, B: DeviceCSR, stream=None) -> DeviceCSR:
        """C = A*B: symbolic pass, allocation of C, numeric pass."""
        c_rpt, nnz = self.symbolic(A, B, stream=stream)
        dev = A.rpt.device
        c_col = torch.empty(nnz, dtype=torch.int32, device=dev)
        c_val = torch.empty(nnz, dtype=torch.float64, device=dev)
        self.numeric(A, B, c_rpt, c_col, c_val, stream=stream)
        return DeviceCSR(A.rows, B.cols, c_rpt, c_col, c_val)


def spgemm(A: DeviceCSR, B: DeviceCSR, handle: Handle | None = None) -> DeviceCSR:
    h = handle or Handle(A.rpt.device.index or 0)
    return h.spgemm(A, B)
