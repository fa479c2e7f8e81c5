"""GPU tests of the search server (continuous batching).

On a database that fills the device several times over, the server runs sessions: one
persistent launch whose work list grows as queries are admitted, so a query that
arrives while others are on the device joins them in the same launch.  Every served
query's scores must equal those of the same query searched alone (sw_search), which the
other tests pin to the oracle, and a sample is checked against the oracle directly.
"""
from __future__ import annotations

import time

import numpy as np
import pytest

import oracle
from paper_1702_07195_amd import swmi, synth

pytestmark = pytest.mark.gpu

ALPHA = len(synth.ALPHABET)


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def session_db():
    # 1,000,000 short sequences: 15,625 groups of 64, more than four times the session
    # kernel's wave slots, and none long enough for the intra-task kernel
    rng = np.random.Generator(np.random.PCG64(61))
    db = synth.db_from_lengths(rng, synth.lognormal_lengths(rng, 1_000_000, 30, 0.5, 5, 100))
    _say(f"load session database: {db.n_seqs} sequences")
    h = swmi.sw_db_load(db.residues, db.offsets, ALPHA)
    yield db, h
    h.free()


def _serve(h, qs, pause_after=None, pause_s=0.0, **kw):
    """Submit the queries (pausing once after `pause_after` of them); returns the results,
    the submission times and the server's counters."""
    with swmi.SwServer(h, synth.BLOSUM62, 10, 2, **kw) as sv:
        sub, tickets = [], []
        for k, q in enumerate(qs):
            sub.append(time.perf_counter())
            tickets.append(sv.submit(q))
            if pause_after is not None and k + 1 == pause_after:
                time.sleep(pause_s)
        results = [sv.wait(t) for t in tickets]
        counters = sv.counters()
    return results, sub, counters


def test_session_admits_queries_while_others_run(session_db):
    db, h = session_db
    rng = np.random.Generator(np.random.PCG64(62))
    qs = [synth.residues(rng, m) for m in (1500, 200, 900, 60, 700, 1200, 300, 50, 1000)]
    alone = [h.search(q, synth.BLOSUM62, 10, 2) for q in qs]
    _say("session: staggered arrivals")
    results, sub, c = _serve(h, qs, pause_after=3, pause_s=0.004, slots=2, max_batch=1)
    assert c["session_mode"] == 1
    for k, (scores, lat, qms) in enumerate(results):
        assert np.array_equal(scores, alone[k]), k
        assert lat >= qms >= 0
    # admission (publication to the device) and completion of each query, host clock
    start = [sub[k] + results[k][2] / 1e3 for k in range(len(qs))]
    end = [sub[k] + results[k][1] / 1e3 for k in range(len(qs))]
    joined = [(j, k) for k in range(len(qs)) for j in range(len(qs))
              if j != k and start[j] <= start[k] < end[j]]
    assert joined, "no query was admitted while another was on the device"
    assert c["max_in_flight"] >= 2
    assert c["launches"] < len(qs)  # several queries shared a launch
    assert c["records"] == len(qs) and c["paired"] == 0
    idx = np.linspace(0, db.n_seqs - 1, 300).astype(np.int64)
    for k in (0, 3, 8):
        want = oracle.search(qs[k], db.residues, db.offsets, synth.BLOSUM62, 10, 2, index=idx)
        assert np.array_equal(results[k][0][idx], want), k


def test_session_pairs_queries_of_similar_length(session_db):
    db, h = session_db
    rng = np.random.Generator(np.random.PCG64(63))
    qs = [synth.residues(rng, m) for m in (480, 470, 475, 200, 480, 90, 460, 485, 300)]
    alone = [h.search(q, synth.BLOSUM62, 10, 2) for q in qs]
    _say("session: queries submitted together, paired by length")
    results, _, c = _serve(h, qs, slots=2, max_batch=2)
    for k, (scores, _, _) in enumerate(results):
        assert np.array_equal(scores, alone[k]), k
    assert c["session_mode"] == 1 and c["paired"] >= 2
    assert c["records"] + c["paired"] == len(qs)
    idx = np.linspace(0, db.n_seqs - 1, 200).astype(np.int64)
    want = oracle.search(qs[1], db.residues, db.offsets, synth.BLOSUM62, 10, 2, index=idx)
    assert np.array_equal(results[1][0][idx], want)


def test_session_sends_saturated_and_very_long_queries_to_the_exact_path():
    # SM(A, A) = 7: A^4682 against itself scores 32774, above the int16 range, so the
    # session reports its record saturated and the server searches the query again
    # exactly; a query longer than a session takes (16,384) goes to the standard search
    # directly.  The other queries stay in sessions.
    rng = np.random.Generator(np.random.PCG64(64))
    lengths = synth.lognormal_lengths(rng, 1_000_000, 30, 0.5, 5, 100)
    db = synth.db_from_lengths(rng, lengths)
    homo = np.zeros(4682, np.uint8)  # code 0 is A
    res = np.concatenate([db.residues[: db.offsets[500_000]], homo, db.residues[db.offsets[500_000]:]])
    offs = np.concatenate([db.offsets[:500_001], db.offsets[500_000:] + len(homo)])
    db = synth.SeqDB(res, offs)
    sm = synth.BLOSUM62.copy()
    sm[0, 0] = 7
    qs = [homo, synth.residues(rng, 300), synth.residues(rng, 16400), synth.residues(rng, 120)]
    with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
        alone = [h.search(q, sm, 10, 2) for q in qs]
        assert alone[0][500_000] == 7 * 4682
        _say("session: saturated and long queries")
        with swmi.SwServer(h, sm, 10, 2, slots=2, max_batch=1) as sv:
            results = [sv.wait(t) for t in [sv.submit(q) for q in qs]]
            c = sv.counters()
    for k, (scores, _, _) in enumerate(results):
        assert np.array_equal(scores, alone[k]), k
    assert c["session_mode"] == 1 and c["exact_runs"] == 2
    idx = np.concatenate([np.linspace(0, db.n_seqs - 1, 60).astype(np.int64), [500_000]])
    want = oracle.search(qs[0], db.residues, db.offsets, sm, 10, 2, index=idx)
    assert np.array_equal(results[0][0][idx], want)


def test_session_empty_query_and_back_to_back_sessions(session_db):
    # an empty query scores 0 without a record; a second burst after the server went
    # idle (the first session closed) opens another launch
    db, h = session_db
    rng = np.random.Generator(np.random.PCG64(65))
    qs = [synth.residues(rng, 150), np.zeros(0, np.uint8), synth.residues(rng, 90)]
    alone = [h.search(q, synth.BLOSUM62, 10, 2) for q in qs]
    with swmi.SwServer(h, synth.BLOSUM62, 10, 2, slots=2, max_batch=2) as sv:
        first = [sv.wait(t) for t in [sv.submit(q) for q in qs]]
        time.sleep(0.05)
        second = [sv.wait(t) for t in [sv.submit(q) for q in qs]]
        c = sv.counters()
    for k in range(len(qs)):
        assert np.array_equal(first[k][0], alone[k]) and np.array_equal(second[k][0], alone[k])
    assert not first[1][0].any()
    assert c["launches"] >= 2 and c["records"] == 4


def test_batch_server_reports_a_wait_that_gave_up():
    # Batch mode (a small database): a spin limit of one poll makes the waits between the
    # segments of split pairs give up; the request fails with SW_EDEVICE instead of
    # returning partial scores, and the next one (default limit) is exact.
    rng = np.random.Generator(np.random.PCG64(88))
    lengths = np.concatenate([rng.integers(2000, 3000, 8), rng.integers(1, 900, 20)])
    db = synth.db_from_lengths(rng, lengths)
    q = synth.residues(rng, 17000)
    knobs = (swmi.SW_KNOB_ROUTE_LEN, swmi.SW_KNOB_SPIN_LIMIT, swmi.SW_KNOB_INTRA_PAIRS)
    old = [swmi.get_knob(k) for k in knobs]
    try:
        swmi.set_knob(swmi.SW_KNOB_ROUTE_LEN, 1)
        swmi.set_knob(swmi.SW_KNOB_INTRA_PAIRS, 0)
        with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
            with swmi.SwServer(h, synth.BLOSUM62, 10, 2, slots=1, max_batch=1) as sv:
                assert sv.counters()["session_mode"] == 0
                swmi.set_knob(swmi.SW_KNOB_SPIN_LIMIT, 1)
                _say("server request with a one-poll segment wait")
                t = sv.submit(q)
                with pytest.raises(swmi.SwError) as e:
                    sv.wait(t)
                assert e.value.code == swmi.SW_EDEVICE
                swmi.set_knob(swmi.SW_KNOB_SPIN_LIMIT, 0)
                got = sv.wait(sv.submit(q))[0]
    finally:
        for k, v in zip(knobs, old):
            swmi.set_knob(k, v)
    idx = np.arange(db.n_seqs)
    assert np.array_equal(got, oracle.search(q, db.residues, db.offsets, synth.BLOSUM62, 10, 2,
                                             index=idx))
