"""Host-side checks of the C ABI that need no GPU: exports and argument validation."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

from paper_1702_07195_amd import swmi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swmi.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sw_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_symbols():
    assert declared_functions() == sorted(swmi.SYMBOLS)


def test_library_exports_every_declared_symbol():
    lib = swmi.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror_codes():
    for code in (swmi.SW_OK, swmi.SW_EINVAL, swmi.SW_ENOMEM, swmi.SW_EDEVICE, swmi.SW_ENODB):
        assert swmi.strerror(code)
    assert swmi.strerror(-99) == "unknown error"


def _load(res, offs, alpha):
    L = swmi.lib()
    r = np.ascontiguousarray(res, np.uint8)
    o = np.ascontiguousarray(offs, np.int64)
    h = ctypes.c_void_p()
    rc = L.sw_db_load(r.ctypes.data_as(swmi._u8p), o.ctypes.data_as(swmi._i64p), len(o) - 1,
                      alpha, ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("res,offs,alpha", [
    ([0, 1, 2], [0, 2, 3], 0),          # alphabet too small
    ([0, 1, 2], [0, 2, 3], 32),         # alphabet too large
    ([0, 1, 5], [0, 2, 3], 5),          # residue >= alphabet
    ([0, 1, 2], [1, 2, 3], 5),          # offsets[0] != 0
    ([0, 1, 2], [0, 2, 1], 5),          # decreasing offsets
])
def test_db_load_rejects_bad_arguments(res, offs, alpha):
    rc, h = _load(res, offs, alpha)
    assert rc == swmi.SW_EINVAL
    assert not h.value


def test_db_load_null_pointers():
    L = swmi.lib()
    h = ctypes.c_void_p()
    o = np.array([0, 3], np.int64)
    assert L.sw_db_load(None, o.ctypes.data_as(swmi._i64p), 1, 5, ctypes.byref(h)) == swmi.SW_EINVAL
    assert L.sw_db_load(None, None, 1, 5, ctypes.byref(h)) == swmi.SW_EINVAL
    assert L.sw_db_load(None, o.ctypes.data_as(swmi._i64p), 1, 5, None) == swmi.SW_EINVAL


def test_search_without_database():
    L = swmi.lib()
    q = np.zeros(4, np.uint8)
    m = np.zeros(25, np.int32)
    out = np.zeros(4, np.int32)
    rc = L.sw_search(None, q.ctypes.data_as(swmi._u8p), 4, m.ctypes.data_as(swmi._i32p), 10, 2,
                     out.ctypes.data_as(swmi._i32p))
    assert rc == swmi.SW_ENODB
    assert L.sw_db_size(None) == swmi.SW_ENODB
    L.sw_db_free(None)  # no-op


def test_knobs_validate_and_round_trip():
    old = swmi.get_knob(swmi.SW_KNOB_STRIP_ROWS)
    with pytest.raises(swmi.SwError):
        swmi.set_knob(swmi.SW_KNOB_STRIP_ROWS, 12)
    swmi.set_knob(swmi.SW_KNOB_STRIP_ROWS, 16)
    assert swmi.get_knob(swmi.SW_KNOB_STRIP_ROWS) == 16
    swmi.set_knob(swmi.SW_KNOB_STRIP_ROWS, 28)  # a height of the query-pair kernel
    assert swmi.get_knob(swmi.SW_KNOB_STRIP_ROWS) == 28
    swmi.set_knob(swmi.SW_KNOB_STRIP_ROWS, old)
    with pytest.raises(swmi.SwError):
        swmi.set_knob(99, 1)


def test_calibration_library_exports_its_header():
    import torch  # noqa: F401  (the HIP runtime torch ships is the one loaded first)

    header = os.path.join(ROOT, "include", "swmi_calib.h")
    text = re.sub(r"/\*.*?\*/", "", open(header).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(swcal_[a-z_]+)\s*\(", text)))
    assert names == ["swcal_cellmix"]
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1702_07195_amd", "libswmi_calib.so"))
    for name in names:
        assert hasattr(lib, name), name
    f = lib.swcal_cellmix
    f.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    ms, cells = ctypes.c_double(), ctypes.c_double()
    # argument checks run before any device call
    assert f(3, 8, 16, ctypes.byref(ms), ctypes.byref(cells)) == -1
    assert f(0, 0, 16, ctypes.byref(ms), ctypes.byref(cells)) == -1
    assert f(0, 8, 16, None, ctypes.byref(cells)) == -1


def test_intra_rows_knob_takes_only_band_shapes():
    old = swmi.get_knob(swmi.SW_KNOB_INTRA_ROWS)
    try:
        for bad in (1, 3, 12, 32, -4):
            with pytest.raises(swmi.SwError):
                swmi.set_knob(swmi.SW_KNOB_INTRA_ROWS, bad)
        for good in (2, 4, 8, 16, 0):
            swmi.set_knob(swmi.SW_KNOB_INTRA_ROWS, good)
            assert swmi.get_knob(swmi.SW_KNOB_INTRA_ROWS) == good
    finally:
        swmi.set_knob(swmi.SW_KNOB_INTRA_ROWS, old)


def test_intra_pairs_knob_values():
    old = swmi.get_knob(swmi.SW_KNOB_INTRA_PAIRS)
    assert old == 1
    try:
        for bad in (-1, 3):
            with pytest.raises(swmi.SwError):
                swmi.set_knob(swmi.SW_KNOB_INTRA_PAIRS, bad)
        for good in (0, 2, 1):
            swmi.set_knob(swmi.SW_KNOB_INTRA_PAIRS, good)
            assert swmi.get_knob(swmi.SW_KNOB_INTRA_PAIRS) == good
    finally:
        swmi.set_knob(swmi.SW_KNOB_INTRA_PAIRS, old)


@pytest.mark.parametrize("name,bad,good,default", [
    ("SW_KNOB_CRIT_SHARE", (-1, 101), (1, 50, 100, 0), 0),
    ("SW_KNOB_INTRA_PRIO", (-1, 2), (0, 1), 1),
    ("SW_KNOB_INTRA_CHAIN", (-1, 2), (0, 1), 1),
    ("SW_KNOB_CRIT_ROWS", (2, 16, -8), (4, 8, 0), 0),
])
def test_critical_pair_knob_values(name, bad, good, default):
    knob = getattr(swmi, name)
    old = swmi.get_knob(knob)
    assert old == default
    try:
        for v in bad:
            with pytest.raises(swmi.SwError):
                swmi.set_knob(knob, v)
        for v in good:
            swmi.set_knob(knob, v)
            assert swmi.get_knob(knob) == v
    finally:
        swmi.set_knob(knob, old)


def test_spin_limit_knob_range():
    old = swmi.get_knob(swmi.SW_KNOB_SPIN_LIMIT)
    try:
        for bad in (-1, (1 << 24) + 1):
            with pytest.raises(swmi.SwError):
                swmi.set_knob(swmi.SW_KNOB_SPIN_LIMIT, bad)
        swmi.set_knob(swmi.SW_KNOB_SPIN_LIMIT, 1)
        assert swmi.get_knob(swmi.SW_KNOB_SPIN_LIMIT) == 1
    finally:
        swmi.set_knob(swmi.SW_KNOB_SPIN_LIMIT, old)


def test_query_pairs_knob_values():
    old = swmi.get_knob(swmi.SW_KNOB_QUERY_PAIRS)
    assert old == 1  # on by default
    try:
        for bad in (-1, 2):
            with pytest.raises(swmi.SwError):
                swmi.set_knob(swmi.SW_KNOB_QUERY_PAIRS, bad)
        for good in (0, 1):
            swmi.set_knob(swmi.SW_KNOB_QUERY_PAIRS, good)
            assert swmi.get_knob(swmi.SW_KNOB_QUERY_PAIRS) == good
    finally:
        swmi.set_knob(swmi.SW_KNOB_QUERY_PAIRS, old)


def test_main_waves_knob_values():
    old = swmi.get_knob(swmi.SW_KNOB_MAIN_WAVES)
    assert old == 0  # automatic by default
    try:
        for bad in (-1, 1, 2, 16):
            with pytest.raises(swmi.SwError):
                swmi.set_knob(swmi.SW_KNOB_MAIN_WAVES, bad)
        for good in (4, 8, 0):
            swmi.set_knob(swmi.SW_KNOB_MAIN_WAVES, good)
            assert swmi.get_knob(swmi.SW_KNOB_MAIN_WAVES) == good
    finally:
        swmi.set_knob(swmi.SW_KNOB_MAIN_WAVES, old)


def test_binding_constants_match_the_header():
    # every #define of include/swmi.h has the same value in the binding
    text = open(HEADER).read()
    defs = dict(re.findall(r"#define\s+(SW_[A-Z0-9_]+)\s+\(?(-?[0-9]+(?:\s*<<\s*[0-9]+)?)\)?", text))
    assert len(defs) > 20
    for name, expr in defs.items():
        assert hasattr(swmi, name), name
        assert getattr(swmi, name) == eval(expr), name  # literal integers and shifts only


def test_binding_refuses_bad_score_tensors_before_calling_the_library():
    # the checks run before any library call, so they need no GPU: a tensor of the wrong
    # type or on the host is refused with ValueError
    import torch
    with pytest.raises(ValueError):
        swmi._dev_i32(np.zeros(4, np.int32), 4, "t")
    with pytest.raises(ValueError):
        swmi._dev_i32(torch.zeros(4, dtype=torch.int64), 4, "t")
    with pytest.raises(ValueError):
        swmi._dev_i32(torch.zeros(4, dtype=torch.int32), 4, "t")
