"""GPU test of sw_topk_noalloc, the top-k entry point that allocates nothing, against
sw_topk (both called through the C ABI) and against a host sort of the same scores."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

from paper_1702_07195_amd import swmi, synth

pytestmark = pytest.mark.gpu

ALPHA = len(synth.ALPHABET)


def _call(fn, h, scores, k):
    idx = np.full(max(k, 1), -1, np.int32)
    sc = np.full(max(k, 1), -1, np.int32)
    nh = ctypes.c_int32(-1)
    rc = fn(h.handle, ctypes.c_void_p(scores.data_ptr()), int(k),
            idx.ctypes.data_as(swmi._i32p), sc.ctypes.data_as(swmi._i32p), ctypes.byref(nh),
            ctypes.c_void_p(0))
    return rc, idx[: max(nh.value, 0)], sc[: max(nh.value, 0)]


def test_topk_noalloc_equals_topk_on_two_calls_the_second_smaller():
    import torch

    L = swmi.lib()
    rng = np.random.Generator(np.random.PCG64(4096))
    # the largest selection (k = 4096 of 20,000 scores), then a smaller one (k = 50 of 900)
    for n, k in ((20_000, 4096), (900, 50)):
        db = synth.db_from_lengths(rng, synth.lognormal_lengths(rng, n, 120, 0.9, 1, 600))
        q = synth.residues(rng, 100)
        with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
            out = torch.zeros(n, dtype=torch.int32, device="cuda")
            h.search_async(q, synth.BLOSUM62, 10, 2, out)
            torch.cuda.synchronize()
            print(f"top-k without allocation: n={n} k={k}", flush=True)
            rc0, want_i, want_s = _call(L.sw_topk, h, out, k)
            rc1, got_i, got_s = _call(L.sw_topk_noalloc, h, out, k)
            assert rc0 == swmi.SW_OK and rc1 == swmi.SW_OK
            assert np.array_equal(got_i, want_i) and np.array_equal(got_s, want_s)
            scores = out.cpu().numpy()
            order = np.lexsort((np.arange(n), -scores.astype(np.int64)))[: min(k, n)]
            assert np.array_equal(got_i, order) and np.array_equal(got_s, scores[order])
            # beyond the array's limit: refused, outputs untouched
            rc, _, _ = _call(L.sw_topk_noalloc, h, out, 4097)
            assert rc == swmi.SW_EINVAL
