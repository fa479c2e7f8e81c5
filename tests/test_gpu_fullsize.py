"""GPU parity at the full workload sizes, in the launch configuration bench.py times.

The oracle cannot score 6e6 x 6 pairs in a test, so each check compares a seeded,
length-stratified sample of sequences (including the longest) with the oracle computed
pair by pair, plus properties that hold at any size (every score in [0, max possible],
scores of identical sequences identical).
"""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
from paper_1702_07195_amd import swmi, synth

pytestmark = pytest.mark.gpu

ALPHA = len(synth.ALPHABET)


def _say(msg):
    print(msg, flush=True)


def _sample(db, n, seed):
    lengths = db.lengths
    order = np.argsort(lengths, kind="stable")
    rng = np.random.Generator(np.random.PCG64(seed))
    strat = order[np.linspace(0, len(order) - 1, n // 2).astype(np.int64)]
    rand = rng.choice(len(order), size=n - n // 2 - 8, replace=False)
    return np.unique(np.concatenate([strat, rand, order[-8:]]))


def _check(db, h, queries, sm, go, ge, n_sample, seed, budget_cells=4e9):
    idx = _sample(db, n_sample, seed)
    for q in queries:
        _say(f"search m={len(q)} on {db.n_seqs} sequences")
        got = h.search(q, sm, go, ge)
        assert got.min() >= 0
        cells = len(q) * int(db.lengths[idx].sum())
        sub = idx if cells <= budget_cells else idx[: max(16, int(len(idx) * budget_cells / cells))]
        want = oracle.search(q, db.residues, db.offsets, sm, go, ge, index=sub)
        assert np.array_equal(got[sub], want), f"m={len(q)}"


def test_full_scale_sampled():
    w = synth.FULL_SCALE
    _say("generate full-scale database")
    db = w.make_db()
    queries = w.make_queries()
    with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
        _check(db, h, queries, w.matrix_values, w.gap_open, w.gap_extend, 600, 1)


def test_plain_config_full():
    w = synth.PLAIN
    db = w.make_db()
    q = w.make_queries()[0]
    with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
        _say("plain search")
        got = h.search(q, w.matrix_values, w.gap_open, w.gap_extend)
    want = oracle.search(q, db.residues, db.offsets, w.matrix_values, w.gap_open, w.gap_extend)
    assert np.array_equal(got, want)


def test_long_mix_sampled():
    w = synth.LONG_MIX
    _say("generate long-mix database")
    db = w.make_db()
    queries = w.make_queries()
    lengths = db.lengths
    long_idx = np.nonzero(lengths >= 10_000)[0]
    assert len(long_idx) == 100
    with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
        for q in queries:
            _say(f"long-mix search m={len(q)}")
            got = h.search(q, w.matrix_values, w.gap_open, w.gap_extend)
            rng = np.random.Generator(np.random.PCG64(len(q)))
            short = rng.choice(np.nonzero(lengths < 10_000)[0], size=200, replace=False)
            # the shortest long sequences keep the oracle within seconds
            longs = long_idx[np.argsort(lengths[long_idx])][:3 if len(q) < 10_000 else 1]
            sub = np.concatenate([short, longs])
            want = oracle.search(q, db.residues, db.offsets, w.matrix_values, w.gap_open,
                                 w.gap_extend, index=sub)
            assert np.array_equal(got[sub], want), f"m={len(q)}"


def test_batched_config_sampled():
    w = synth.BATCHED
    db = w.make_db()
    qs = synth.batched_queries(64)
    sm = synth.BLOSUM50
    with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
        _say("batched search of 64 queries")
        got = h.search_batch(qs, sm, 11, 1)
    idx = _sample(db, 24, 7)
    for k in (0, 17, 63):
        want = oracle.search(qs[k], db.residues, db.offsets, sm, 11, 1, index=idx)
        assert np.array_equal(got[k][idx], want), k


def test_long_mix_longest_pairs():
    # The longest sequence of the mix against both queries: these pairs are split across
    # workgroups (4-band segments for the 5478-residue query, 8-band segments for the
    # 35000-residue one), so this checks the split path at the full workload size.
    from concurrent.futures import ThreadPoolExecutor

    w = synth.LONG_MIX
    db = w.make_db()
    queries = w.make_queries()
    longest = int(np.argmax(db.lengths))
    _say(f"long-mix longest pair: n={int(db.lengths[longest])}")
    with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
        got = [int(h.search(q, w.matrix_values, w.gap_open, w.gap_extend)[longest])
               for q in queries]
    # one oracle call per query, in parallel (each scores one pair on one host thread)
    with ThreadPoolExecutor(max_workers=len(queries)) as ex:
        want = list(ex.map(lambda q: int(oracle.score(q, db.seq(longest), w.matrix_values,
                                                      w.gap_open, w.gap_extend)), queries))
    assert got == want


def test_served_config_sampled():
    # The served configuration: the 4.35e6-sequence database resident, queries of the
    # served length law submitted to the server in the configuration bench.py times
    # (2 stream slots, batches of up to 8, 64 GiB budget); sampled scores of three of
    # them against the oracle, all six complete.
    w = synth.SERVED
    _say("generate served database")
    db = w.make_db()
    qs = synth.served_queries(6)
    with swmi.sw_db_load(db.residues, db.offsets, ALPHA) as h:
        with swmi.SwServer(h, synth.BLOSUM62, 10, 2, slots=2, max_batch=8,
                           mem_budget_bytes=64 << 30) as sv:
            _say("served queries " + ", ".join(str(len(q)) for q in qs))
            results = [sv.wait(t) for t in [sv.submit(q) for q in qs]]
    idx = _sample(db, 200, 11)
    for k in (0, 3, 5):
        want = oracle.search(qs[k], db.residues, db.offsets, synth.BLOSUM62, 10, 2, index=idx)
        assert np.array_equal(results[k][0][idx], want), k
    assert all(r[0].min() >= 0 for r in results)
