"""CPU oracle for Smith-Waterman database search -- TEST INFRASTRUCTURE ONLY.

Plain int32 Gotoh recurrences (paper, Section 2, Eqs. 1-3) in ``sw_oracle.c``,
loaded through ctypes.  Only the tests, the package smoke check and the benchmark's
CPU-baseline leg may use this package; the library's search path never does.

Parity pins (all in ``tests/test_oracle_pins.py``): brute-force enumeration of every
alignment on tiny inputs, hand-worked examples for the gap convention, closed forms
(single residue, homopolymers, ungapped Kadane limit, longest common substring,
linear-gap special case, saturation boundary) and invariants (score >= 0, symmetry,
self-alignment bound, empty sequences, monotonicity in the penalties).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_u8p = ctypes.POINTER(ctypes.c_uint8)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)

NEG_BORDER = -(1 << 28)  # "minus infinity" border for E/F that cannot overflow int32


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.swo_score_border.restype = ctypes.c_int32
        L.swo_score_border.argtypes = [_u8p, ctypes.c_int32, _u8p, ctypes.c_int32, _i32p,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32]
        L.swo_score.restype = ctypes.c_int32
        L.swo_score.argtypes = [_u8p, ctypes.c_int32, _u8p, ctypes.c_int32, _i32p,
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.swo_search.restype = ctypes.c_int
        L.swo_search.argtypes = [_u8p, ctypes.c_int32, _u8p, _i64p, _i64p, ctypes.c_int64,
                                 _i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                 _i32p, ctypes.c_int32]
        _lib = L
    return _lib


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(_u8p)


def _matrix(sm):
    sm = np.ascontiguousarray(sm, dtype=np.int32)
    assert sm.ndim == 2 and sm.shape[0] == sm.shape[1]
    return sm, sm.ctypes.data_as(_i32p), sm.shape[0]


def score(s1, s2, sm, gap_open: int, gap_extend: int, ef_border: int = 0) -> int:
    """Optimal local alignment score of query ``s1`` against sequence ``s2``."""
    a, pa = _u8(s1)
    b, pb = _u8(s2)
    m, pm, alpha = _matrix(sm)
    r = lib().swo_score_border(pa, len(a), pb, len(b), pm, alpha, gap_open, gap_extend,
                               ef_border)
    if r < 0:
        raise MemoryError("oracle allocation failed")
    return int(r)


def search(query, residues, offsets, sm, gap_open: int, gap_extend: int,
           index=None, threads: int | None = None) -> np.ndarray:
    """Scores of ``query`` against database sequences (all, or ``index`` if given)."""
    q, pq = _u8(query)
    res, pr = _u8(residues)
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    m, pm, alpha = _matrix(sm)
    if index is None:
        idx, pidx, count = None, None, len(offs) - 1
    else:
        idx = np.ascontiguousarray(index, dtype=np.int64)
        pidx, count = idx.ctypes.data_as(_i64p), len(idx)
    out = np.zeros(count, dtype=np.int32)
    if threads is None:
        threads = os.cpu_count() or 1
    rc = lib().swo_search(pq, len(q), pr, offs.ctypes.data_as(_i64p), pidx, count, pm, alpha,
                          gap_open, gap_extend, out.ctypes.data_as(_i32p), int(threads))
    if rc != 0:
        raise RuntimeError("oracle search failed")
    return out
