"""Thin ctypes binding of the C ABI in ``include/swmi.h`` (argument marshalling only).

Every step of a search runs inside ``libswmi.so`` (HIP kernels for gfx950).  There is
no Python or CPU fallback: if the library is missing this module raises on import of
the library, and every call fails loudly with the library's error code.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswmi.so")

SW_OK = 0
SW_EINVAL = -1
SW_ENOMEM = -2
SW_EDEVICE = -3
SW_ENODB = -4

SW_MAX_ALPHABET = 31
SW_MAX_QUERY_LEN = 1 << 24
SW_MAX_GOE = 16383
SW_MAX_ABS_SCORE = 127

SW_KNOB_INTRA_MIN_LEN = 1
SW_KNOB_RECOMPUTE_ALL = 2
SW_KNOB_STRIP_ROWS = 3
SW_KNOB_GRID_WAVES = 4
SW_KNOB_MEM_CAP_MB = 5
SW_KNOB_ROUTE_LEN = 6
SW_KNOB_WIDE_LEN = 7
SW_KNOB_MAX_SEGMENTS = 8
SW_KNOB_INTRA_ROWS = 9
SW_KNOB_INTRA_PAIRS = 10
SW_KNOB_SPIN_LIMIT = 11
SW_KNOB_QUERY_PAIRS = 12
SW_KNOB_MAIN_WAVES = 13
SW_KNOB_PRIO_COLS = 14
SW_KNOB_FLAG_CAP = 15
SW_KNOB_CRIT_ROWS = 16
SW_KNOB_CRIT_SHARE = 17
SW_KNOB_INTRA_PRIO = 18
SW_KNOB_INTRA_CHAIN = 19

# Every entry point declared in include/swmi.h.
SYMBOLS = ("sw_db_load", "sw_db_size", "sw_db_free", "sw_search", "sw_search_async",
           "sw_search_batch", "sw_strerror", "sw_timing_enable", "sw_timing_read",
           "sw_timing_read_kernel", "sw_set_knob", "sw_get_knob", "sw_plan_create",
           "sw_plan_launch", "sw_plan_free", "sw_server_create", "sw_server_submit",
           "sw_server_wait", "sw_server_stats", "sw_server_counters", "sw_server_free",
           "sw_topk", "sw_search_stats", "sw_topk_noalloc")

# sw_search_stats indices
SW_ST_CELLS_INTER16 = 0
SW_ST_CELLS_INTRA32 = 1
SW_ST_CELLS_INTRA16 = 2
SW_ST_CELLS_CRIT = 3
SW_ST_INTRA_ROWS = 4
SW_ST_MAIN_WAVES = 5
SW_ST_ROUTED_GROUPS = 6
SW_ST_STRIP_ROWS = 7
SW_ST_QUERY_PAIRS = 8
SW_ST_BIG_WAVES = 9
SW_SEARCH_NSTATS = 10
SW_ST_NAMES = ("cells_inter16", "cells_intra32", "cells_intra16", "cells_crit", "intra_rows",
               "main_waves", "routed_groups", "strip_rows", "query_pairs", "big_waves")

# sw_server_counters indices
SW_SC_LAUNCHES = 0
SW_SC_MAX_IN_FLIGHT = 1
SW_SC_REFUSED = 2
SW_SC_SESSION_MODE = 3
SW_SC_RECORDS = 4
SW_SC_PAIRED = 5
SW_SC_EXACT_RUNS = 6
SW_SC_WAVES = 7
SW_SC_COPY_US = 8
SW_SERVER_NCOUNTERS = 9
SW_SC_NAMES = ("launches", "max_in_flight", "refused", "session_mode", "records", "paired",
               "exact_runs", "waves", "copy_us")

SW_KERNEL_INTER16 = 0
SW_KERNEL_INTRA_LONG = 1
SW_KERNEL_RECOMPUTE = 2

_u8p = ctypes.POINTER(ctypes.c_uint8)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p

_lib = None


class SwError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


def lib():
    """Load libswmi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        # torch bundles its own HIP runtime with the same soname (libamdhip64.so.7).
        # Loading torch first makes libswmi.so bind to that runtime, so the process has
        # one HIP runtime and torch tensors/streams are valid inside the library.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        L.sw_db_load.restype = ctypes.c_int
        L.sw_db_load.argtypes = [_u8p, _i64p, ctypes.c_int64, ctypes.c_int32,
                                 ctypes.POINTER(_vp)]
        L.sw_db_size.restype = ctypes.c_int64
        L.sw_db_size.argtypes = [_vp]
        L.sw_db_free.restype = None
        L.sw_db_free.argtypes = [_vp]
        L.sw_search.restype = ctypes.c_int
        L.sw_search.argtypes = [_vp, _u8p, ctypes.c_int32, _i32p, ctypes.c_int32,
                                ctypes.c_int32, _i32p]
        L.sw_search_async.restype = ctypes.c_int
        L.sw_search_async.argtypes = [_vp, _u8p, ctypes.c_int32, _i32p, ctypes.c_int32,
                                      ctypes.c_int32, _vp, _vp]
        L.sw_search_batch.restype = ctypes.c_int
        L.sw_search_batch.argtypes = [_vp, _u8p, _i64p, ctypes.c_int64, _i32p, ctypes.c_int32,
                                      ctypes.c_int32, _i32p]
        L.sw_strerror.restype = ctypes.c_char_p
        L.sw_strerror.argtypes = [ctypes.c_int]
        L.sw_timing_enable.restype = ctypes.c_int
        L.sw_timing_enable.argtypes = [_vp, ctypes.c_int32]
        L.sw_timing_read.restype = ctypes.c_int
        L.sw_timing_read.argtypes = [_vp, _i64p, ctypes.POINTER(ctypes.c_double)]
        L.sw_timing_read_kernel.restype = ctypes.c_int
        L.sw_timing_read_kernel.argtypes = [_vp, ctypes.c_int32, _i64p,
                                            ctypes.POINTER(ctypes.c_double)]
        L.sw_plan_create.restype = ctypes.c_int
        L.sw_plan_create.argtypes = [_vp, _u8p, _i64p, ctypes.c_int64, _i32p, ctypes.c_int32,
                                     ctypes.c_int32, _vp, ctypes.POINTER(_vp)]
        L.sw_plan_launch.restype = ctypes.c_int
        L.sw_plan_launch.argtypes = [_vp, _vp]
        L.sw_plan_free.restype = None
        L.sw_plan_free.argtypes = [_vp]
        L.sw_server_create.restype = ctypes.c_int
        L.sw_server_create.argtypes = [_vp, _i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(_vp)]
        L.sw_server_submit.restype = ctypes.c_int
        L.sw_server_submit.argtypes = [_vp, _u8p, ctypes.c_int32, _i32p,
                                       ctypes.POINTER(ctypes.c_uint64)]
        L.sw_server_wait.restype = ctypes.c_int
        L.sw_server_wait.argtypes = [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
        L.sw_server_stats.restype = ctypes.c_int
        L.sw_server_stats.argtypes = [_vp, _i64p, _i64p, _i64p]
        L.sw_server_counters.restype = ctypes.c_int
        L.sw_server_counters.argtypes = [_vp, _i64p, ctypes.c_int32]
        L.sw_server_free.restype = None
        L.sw_server_free.argtypes = [_vp]
        L.sw_topk.restype = ctypes.c_int
        L.sw_topk.argtypes = [_vp, _vp, ctypes.c_int32, _i32p, _i32p, _i32p, _vp]
        L.sw_topk_noalloc.restype = ctypes.c_int
        L.sw_topk_noalloc.argtypes = [_vp, _vp, ctypes.c_int32, _i32p, _i32p, _i32p, _vp]
        L.sw_search_stats.restype = ctypes.c_int
        L.sw_search_stats.argtypes = [_vp, _i64p, ctypes.c_int32]
        L.sw_set_knob.restype = ctypes.c_int
        L.sw_set_knob.argtypes = [ctypes.c_int32, ctypes.c_int64]
        L.sw_get_knob.restype = ctypes.c_int64
        L.sw_get_knob.argtypes = [ctypes.c_int32]
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().sw_strerror(int(code)).decode()


def _check(rc: int, where: str):
    if rc != SW_OK:
        raise SwError(rc, where)


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(_u8p)


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_i32p)


def _i64(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(_i64p)


def _dev_i32(t, need: int, where: str) -> int:
    """Device address of an int32 tensor that can hold ``need`` scores, after checking
    that it is int32, on the GPU, contiguous and large enough (the library writes
    ``need`` elements there, so anything else would be an out-of-bounds device write)."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{where}: scores_dev must be a torch tensor")
    if t.dtype != torch.int32:
        raise ValueError(f"{where}: scores_dev must be int32, not {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{where}: scores_dev must be on the GPU, not {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{where}: scores_dev must be contiguous")
    if t.numel() < need:
        raise ValueError(f"{where}: scores_dev holds {t.numel()} elements, {need} needed")
    return int(t.data_ptr())


def set_knob(knob: int, value: int):
    _check(lib().sw_set_knob(knob, int(value)), "sw_set_knob")


def get_knob(knob: int) -> int:
    return int(lib().sw_get_knob(knob))


def sw_db_load(residues, offsets, alphabet: int) -> "SwDb":
    """Pre-process and upload a database (see sw_db_load in include/swmi.h)."""
    res, pres = _u8(residues)
    offs, poffs = _i64(offsets)
    handle = _vp()
    rc = lib().sw_db_load(pres, poffs, len(offs) - 1, int(alphabet), ctypes.byref(handle))
    _check(rc, "sw_db_load")
    return SwDb(handle, len(offs) - 1, int(alphabet))


class SwDb:
    """Owner of a loaded database handle."""

    def __init__(self, handle, n_seqs: int, alphabet: int):
        self._h = handle
        self.n_seqs = n_seqs
        self.alphabet = alphabet

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise SwError(SW_ENODB, "database")
        return self._h

    def free(self):
        if self._h is not None and self._h.value:
            lib().sw_db_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()

    def size(self) -> int:
        return int(lib().sw_db_size(self.handle))

    def search(self, query, matrix, gap_open: int, gap_extend: int) -> np.ndarray:
        """Scores of one query against every sequence, in the caller's order."""
        q, pq = _u8(query)
        m, pm = _i32(matrix)
        out = np.zeros(self.n_seqs, dtype=np.int32)
        rc = lib().sw_search(self.handle, pq, len(q), pm, int(gap_open), int(gap_extend),
                             out.ctypes.data_as(_i32p))
        _check(rc, "sw_search")
        return out

    def search_async(self, query, matrix, gap_open: int, gap_extend: int, scores_dev,
                     stream=None):
        """Enqueue a search on a torch CUDA(HIP) stream; ``scores_dev`` is an int32
        device tensor of ``n_seqs`` elements."""
        q, pq = _u8(query)
        m, pm = _i32(matrix)
        sptr = 0 if stream is None else int(stream.cuda_stream)
        dptr = _dev_i32(scores_dev, self.n_seqs, "sw_search_async")
        rc = lib().sw_search_async(self.handle, pq, len(q), pm, int(gap_open), int(gap_extend),
                                   _vp(dptr), _vp(sptr))
        _check(rc, "sw_search_async")

    def search_batch(self, queries, matrix, gap_open: int, gap_extend: int) -> np.ndarray:
        """Scores of many queries (a list of code arrays) in one launch: [n_queries, n_seqs]."""
        qs = [np.ascontiguousarray(x, dtype=np.uint8) for x in queries]
        offs = np.zeros(len(qs) + 1, dtype=np.int64)
        np.cumsum([len(x) for x in qs], out=offs[1:])
        cat = np.concatenate(qs) if qs else np.zeros(0, np.uint8)
        if len(cat) == 0:
            cat = np.zeros(1, np.uint8)
        c, pc = _u8(cat)
        o, po = _i64(offs)
        m, pm = _i32(matrix)
        out = np.zeros((len(qs), self.n_seqs), dtype=np.int32)
        rc = lib().sw_search_batch(self.handle, pc, po, len(qs), pm, int(gap_open),
                                   int(gap_extend), out.ctypes.data_as(_i32p))
        _check(rc, "sw_search_batch")
        return out

    def plan(self, queries, matrix, gap_open: int, gap_extend: int, scores_dev) -> "SwPlan":
        """Capture a batched search into a HIP graph; ``scores_dev`` is an int32 device
        tensor of n_queries * n_seqs elements."""
        qs = [np.ascontiguousarray(x, dtype=np.uint8) for x in queries]
        offs = np.zeros(len(qs) + 1, dtype=np.int64)
        np.cumsum([len(x) for x in qs], out=offs[1:])
        cat = np.concatenate(qs) if qs else np.zeros(0, np.uint8)
        if len(cat) == 0:
            cat = np.zeros(1, np.uint8)
        c, pc = _u8(cat)
        o, po = _i64(offs)
        m, pm = _i32(matrix)
        handle = _vp()
        dptr = _dev_i32(scores_dev, len(qs) * self.n_seqs, "sw_plan_create")
        rc = lib().sw_plan_create(self.handle, pc, po, len(qs), pm, int(gap_open),
                                  int(gap_extend), _vp(dptr), ctypes.byref(handle))
        _check(rc, "sw_plan_create")
        return SwPlan(handle, self, scores_dev)

    def topk(self, scores_dev, k: int, stream=None):
        """The k best hits of a search: (database indices, scores), score descending,
        ties by index ascending; ``scores_dev`` is the int32 device tensor of scores."""
        idx = np.zeros(k, dtype=np.int32)
        sc = np.zeros(k, dtype=np.int32)
        nh = ctypes.c_int32(0)
        sptr = 0 if stream is None else int(stream.cuda_stream)
        dptr = _dev_i32(scores_dev, self.n_seqs, "sw_topk")
        rc = lib().sw_topk(self.handle, _vp(dptr), int(k),
                           idx.ctypes.data_as(_i32p), sc.ctypes.data_as(_i32p),
                           ctypes.byref(nh), _vp(sptr))
        _check(rc, "sw_topk")
        return idx[:nh.value], sc[:nh.value]

    def stats(self) -> dict:
        """sw_search_stats of the latest search on this handle, by name."""
        v = np.zeros(len(SW_ST_NAMES), dtype=np.int64)
        _check(lib().sw_search_stats(self.handle, v.ctypes.data_as(_i64p), len(v)),
               "sw_search_stats")
        return {k: int(x) for k, x in zip(SW_ST_NAMES, v)}

    def timing_enable(self, on: bool = True):
        _check(lib().sw_timing_enable(self.handle, 1 if on else 0), "sw_timing_enable")

    def timing_read(self, kernel: int = SW_KERNEL_INTER16):
        """(launches, total device milliseconds) of one kernel since timing_enable."""
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0.0)
        _check(lib().sw_timing_read_kernel(self.handle, int(kernel), ctypes.byref(n),
                                           ctypes.byref(ms)), "sw_timing_read_kernel")
        return int(n.value), float(ms.value)


class SwPlan:
    """A search captured into a HIP graph (see sw_plan_create in include/swmi.h)."""

    def __init__(self, handle, db: SwDb, scores_dev):
        self._h = handle
        self._db = db            # keeps the database alive while the plan exists
        self._scores = scores_dev

    def launch(self, stream=None):
        sptr = 0 if stream is None else int(stream.cuda_stream)
        _check(lib().sw_plan_launch(self._h, _vp(sptr)), "sw_plan_launch")

    def free(self):
        if self._h is not None and self._h.value:
            lib().sw_plan_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()


class SwServer:
    """Continuous-batching search server over a loaded database (see sw_server_create)."""

    def __init__(self, db: SwDb, matrix, gap_open: int, gap_extend: int, slots: int = 2,
                 max_batch: int = 8, mem_budget_bytes: int = 0):
        m, pm = _i32(matrix)
        handle = _vp()
        rc = lib().sw_server_create(db.handle, pm, int(gap_open), int(gap_extend), int(slots),
                                    int(max_batch), int(mem_budget_bytes), ctypes.byref(handle))
        _check(rc, "sw_server_create")
        self._h = handle
        self._db = db
        self._pending = {}   # ticket -> (query array, output array) kept alive until waited

    def submit(self, query) -> int:
        q, pq = _u8(query)
        out = np.zeros(self._db.n_seqs, dtype=np.int32)
        t = ctypes.c_uint64(0)
        rc = lib().sw_server_submit(self._h, pq, len(q), out.ctypes.data_as(_i32p),
                                    ctypes.byref(t))
        _check(rc, "sw_server_submit")
        self._pending[t.value] = (q, out)
        return int(t.value)

    def wait(self, ticket: int):
        """(scores, latency_ms, queue_ms) of a submitted query."""
        lat = ctypes.c_double(0.0)
        qms = ctypes.c_double(0.0)
        rc = lib().sw_server_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(lat),
                                  ctypes.byref(qms))
        q, out = self._pending.pop(ticket)
        _check(rc, "sw_server_wait")
        return out, float(lat.value), float(qms.value)

    def stats(self):
        a, b, c = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
        _check(lib().sw_server_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
               "sw_server_stats")
        return {"launches": a.value, "max_in_flight": b.value, "refused": c.value}

    def counters(self) -> dict:
        """Every counter of sw_server_counters, by name."""
        v = np.zeros(len(SW_SC_NAMES), dtype=np.int64)
        _check(lib().sw_server_counters(self._h, v.ctypes.data_as(_i64p), len(v)),
               "sw_server_counters")
        return {k: int(x) for k, x in zip(SW_SC_NAMES, v)}

    def free(self):
        if self._h is not None and self._h.value:
            lib().sw_server_free(self._h)
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()
