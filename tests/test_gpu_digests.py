"""Full-size parity: every score of the large workloads against the oracle.

The oracle's scores of the full-scale search (6,000,000 sequences x 6 queries), the
long-sequence mix (10,000 x 2) and the batched workload (200,000 x 64 queries, two
matrix/gap settings) were computed once on the CPU by ``tests/golden/make_digests.py``
(oracle + seeded inputs only) and stored as SHA-256 digests of consecutive slices of
each query's int32 score vector in the caller's order (``tests/golden/digests.txt``),
with the slice's sum, maximum and a score histogram.  Here the GPU path recomputes the
same score vectors, in the configuration bench.py times (device-resident searches, and
one batched launch for the batched workload), and every slice must hash to the oracle's
digest: parity over every sequence, not a sample.
"""
from __future__ import annotations

import hashlib
import os

import numpy as np
import pytest

from paper_1702_07195_amd import swmi, synth

pytestmark = pytest.mark.gpu

ALPHA = len(synth.ALPHABET)
DIGESTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "digests.txt")
HIST_EDGES = (0, 1, 20, 40, 80, 160, 320, 640, 1280, 32767)
WORKLOADS = {"full_scale": synth.FULL_SCALE, "long_mix": synth.LONG_MIX,
             "batched": synth.BATCHED}


def _say(msg):
    print(msg, flush=True)


def _lines(workload):
    out = []
    with open(DIGESTS) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            w = line.split()
            if len(w) != 12 or w[0] != workload:  # (a line still being written is skipped)
                continue
            out.append(dict(matrix=w[1], go=int(w[2]), ge=int(w[3]), query=int(w[4]),
                            qlen=int(w[5]), begin=int(w[6]), end=int(w[7]), sha=w[8],
                            sum=int(w[9]), max=int(w[10]), hist=w[11]))
    return out


def _check_slices(lines, scores_of):
    bad = []
    for d in lines:
        s = np.ascontiguousarray(scores_of(d)[d["begin"]:d["end"]], dtype="<i4")
        if hashlib.sha256(s.tobytes()).hexdigest() != d["sha"]:
            hist = ",".join(str(int(c)) for c in
                            np.histogram(s, bins=list(HIST_EDGES) + [1 << 31])[0])
            bad.append((d["matrix"], d["go"], d["ge"], d["query"], d["begin"], d["end"],
                        f"sum {int(s.sum(dtype=np.int64))} vs {d['sum']}",
                        f"max {int(s.max())} vs {d['max']}", f"hist {hist} vs {d['hist']}"))
    assert not bad, f"{len(bad)} slices differ from the oracle, first: {bad[:3]}"


@pytest.mark.parametrize("workload", ["long_mix", "full_scale"])
def test_every_score_of_the_search_workloads(workload):
    lines = _lines(workload)
    if not lines:
        pytest.skip(f"no oracle digests of {workload} yet")
    import torch

    w = WORKLOADS[workload]
    _say(f"generate {workload} database")
    db = w.make_db()
    queries = w.make_queries()
    qidx = sorted({d["query"] for d in lines})
    got = {}
    with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
        out = torch.zeros(db.n_seqs, dtype=torch.int32, device="cuda")
        for qi in qidx:
            assert len(queries[qi]) == next(d["qlen"] for d in lines if d["query"] == qi)
            _say(f"{workload}: search m={len(queries[qi])}")
            h.search_async(queries[qi], w.matrix_values, w.gap_open, w.gap_extend, out)
            torch.cuda.synchronize()
            got[qi] = out.cpu().numpy()
    n_full = sum(1 for d in lines if d["begin"] == 0)
    _say(f"{workload}: {len(lines)} slices of {len(qidx)} queries ({n_full} starting at 0)")
    _check_slices(lines, lambda d: got[d["query"]])


def test_every_score_of_the_batched_workload():
    lines = _lines("batched")
    if not lines:
        pytest.skip("no oracle digests of the batched workload yet")
    w = synth.BATCHED
    db = w.make_db()
    qs = synth.batched_queries(64)
    settings = sorted({(d["matrix"], d["go"], d["ge"]) for d in lines})
    got = {}
    with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
        for mat, go, ge in settings:
            _say(f"batched: 64 queries, {mat} {go}/{ge}")
            got[(mat, go, ge)] = h.search_batch(qs, synth.MATRICES[mat], go, ge)
    _say(f"batched: {len(lines)} slices")
    _check_slices(lines, lambda d: got[(d["matrix"], d["go"], d["ge"])][d["query"]])
